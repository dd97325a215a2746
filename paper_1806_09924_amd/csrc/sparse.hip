// Block SELL-C sparse kernels (HBM-streaming, one thread per block row, lanes of a wave
// read consecutive slots), the fused coupled-Jacobian product, Chebyshev smoothing steps
// and small deterministic device primitives (scan, dot, casts).
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "profile.h"
#include "system.h"

namespace fr {
namespace {

// Column of a slot of row r: stored as an int32 index, or as an int16 offset from the row
// (meshes whose node numbering keeps every neighbour within 32767 of the node: 2 bytes
// instead of 4 per stored block on the finest level).
__device__ __forceinline__ int64_t col_at(const int32_t* __restrict__ col, int64_t slot, int64_t) {
    return col[slot];
}
__device__ __forceinline__ int64_t col_at(const int16_t* __restrict__ col, int64_t slot, int64_t r) {
    return r + col[slot];
}

// acc += (row r of A) x over the w slots of the row starting at `slot` (stride C).  The
// entries are taken U at a time with every load of a group issued before its products, so
// a lane keeps several gathers in flight; the summation order stays entry by entry.
template <typename T, int BR, int BC, int U, typename CI>
__device__ __forceinline__ void row_product(int w, int C, int64_t slot, int64_t r, const CI* __restrict__ col,
                                            const T* __restrict__ val, const T* __restrict__ x, T* acc) {
    constexpr int BB = BR * BC;
    int k = 0;
    for (; k + U <= w; k += U, slot += int64_t(U) * C) {
        int64_t c[U];
#pragma unroll
        for (int u = 0; u < U; ++u) c[u] = col_at(col, slot + int64_t(u) * C, r);
        T xv[U][BC];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int j = 0; j < BC; ++j) xv[u][j] = x[c[u] * BC + j];
        T v[U][BB];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int e = 0; e < BB; ++e) v[u][e] = val[(slot + int64_t(u) * C) * BB + e];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int i = 0; i < BR; ++i)
#pragma unroll
                for (int j = 0; j < BC; ++j) acc[i] += v[u][i * BC + j] * xv[u][j];
    }
    for (; k < w; ++k, slot += C) {
        const int64_t c = col_at(col, slot, r);
        const T* v = val + slot * BB;
        T xv[BC];
#pragma unroll
        for (int j = 0; j < BC; ++j) xv[j] = x[c * BC + j];
#pragma unroll
        for (int i = 0; i < BR; ++i)
#pragma unroll
            for (int j = 0; j < BC; ++j) acc[i] += v[i * BC + j] * xv[j];
    }
}

// With G > 1 lanes per row (small levels, long rows: few rows would leave most of the chip
// idle), lane g of a group takes entries g, g+G, ... and the group combines its partial sums
// by an xor butterfly, which leaves the same total on every lane of the group.
template <typename T, int BR, int BC, int G, int U, typename CI>
__device__ __forceinline__ void row_product_g(int w, int C, int64_t slot0, int64_t r, int g, const CI* __restrict__ col,
                                              const T* __restrict__ val, const T* __restrict__ x, T* acc) {
    if constexpr (G == 1) {
        row_product<T, BR, BC, U>(w, C, slot0, r, col, val, x, acc);
    } else {
        constexpr int BB = BR * BC;
        for (int k = g; k < w; k += G) {
            const int64_t slot = slot0 + int64_t(k) * C;
            const int64_t c = col_at(col, slot, r);
            const T* v = val + slot * BB;
            T xv[BC];
#pragma unroll
            for (int j = 0; j < BC; ++j) xv[j] = x[c * BC + j];
#pragma unroll
            for (int i = 0; i < BR; ++i)
#pragma unroll
                for (int j = 0; j < BC; ++j) acc[i] += v[i * BC + j] * xv[j];
        }
#pragma unroll
        for (int o = G / 2; o > 0; o >>= 1)
#pragma unroll
            for (int i = 0; i < BR; ++i) acc[i] += __shfl_xor(acc[i], o, kWave);
    }
}

// Lanes per row for a SELL matrix: 1, 4, 16 or 64, growing while the launch would have
// fewer than 2^20 lanes and an average row still has an entry for every lane.
inline int lanes_per_row(const SellStruct& S) {
    const int64_t avg = S.n_rows > 0 ? S.nnz / S.n_rows : 0;
    int G = 1;
    while (G < 64 && S.n_rows * G < (int64_t(1) << 20) && 4 * G <= avg) G *= 4;
    return G;
}

// MODE 0: y = A x; 1: y = b - A x; 2: y += A x
template <typename T, int BR, int BC, int MODE, int G, typename CI>
__global__ void __launch_bounds__(256) k_spmv(int64_t n_rows, int C, const int32_t* __restrict__ slice_ptr,
                                              const CI* __restrict__ col, const T* __restrict__ val,
                                              const T* __restrict__ x, const T* __restrict__ b, T* __restrict__ y) {
    constexpr int U = BR * BC == 1 ? 8 : 2;   // block rows: two entries in flight (measured fastest for 2x2)
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t r = t / G;
    const int g = int(t % G);
    if (r >= n_rows) return;   // whole groups leave together
    const int64_t s = r / C;
    const int lane = int(r - s * C);
    const int32_t p0 = slice_ptr[s];
    const int w = (slice_ptr[s + 1] - p0) / C;
    // the row's b (mode 1) or y (mode 2) is loaded before the product, in flight with it
    T own[BR];
    if (MODE != 0 && (G == 1 || g == 0)) {
#pragma unroll
        for (int i = 0; i < BR; ++i) own[i] = MODE == 1 ? b[r * BR + i] : y[r * BR + i];
    }
    T acc[BR];
#pragma unroll
    for (int i = 0; i < BR; ++i) acc[i] = T(0);
    row_product_g<T, BR, BC, G, U>(w, C, int64_t(p0) + lane, r, g, col, val, x, acc);
    if (g != 0) return;
#pragma unroll
    for (int i = 0; i < BR; ++i) {
        if (MODE == 0) y[r * BR + i] = acc[i];
        else if (MODE == 1) y[r * BR + i] = own[i] - acc[i];
        else y[r * BR + i] = own[i] + acc[i];
    }
}

// Chebyshev step: r = b - A x_old; d = alpha d + beta D^-1 r; x_new = x_old + d
template <typename T, int B, int G, typename CI>
__global__ void __launch_bounds__(256) k_cheb(int64_t n_rows, int C, const int32_t* __restrict__ slice_ptr,
                                              const CI* __restrict__ col, const T* __restrict__ val,
                                              const T* __restrict__ invd, const T* __restrict__ x_old,
                                              const T* __restrict__ b, T* __restrict__ d, T* __restrict__ x_new,
                                              T alpha, T beta) {
    constexpr int U = B == 1 ? 8 : (B == 6 ? 1 : 2);
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t r = t / G;
    const int g = int(t % G);
    if (r >= n_rows) return;
    const int64_t s = r / C;
    const int lane = int(r - s * C);
    const int32_t p0 = slice_ptr[s];
    const int w = (slice_ptr[s + 1] - p0) / C;
    // the row's own vector entries are loaded before the product, so that they are in flight
    // together with the matrix stream
    T bv[B], dv[B], iv[B], xo[B];
    if (G == 1 || g == 0) {
#pragma unroll
        for (int i = 0; i < B; ++i) {
            const int64_t e = r * B + i;
            bv[i] = b[e];
            dv[i] = alpha != T(0) ? d[e] : T(0);
            iv[i] = invd[e];
            xo[i] = x_old[e];
        }
    }
    T acc[B];
#pragma unroll
    for (int i = 0; i < B; ++i) acc[i] = T(0);
    row_product_g<T, B, B, G, U>(w, C, int64_t(p0) + lane, r, g, col, val, x_old, acc);
    if (g != 0) return;
#pragma unroll
    for (int i = 0; i < B; ++i) {
        const int64_t e = r * B + i;
        const T res = bv[i] - acc[i];
        const T dn = (alpha != T(0) ? alpha * dv[i] : T(0)) + beta * iv[i] * res;
        d[e] = dn;
        x_new[e] = xo[i] + dn;
    }
}

// One power-iteration step of the smoother bounds, y = D^-1 A x: the products of the Chebyshev
// step with b = 0 (same order, so the same values), as a kernel of its own so that the setup's
// launches are told apart from the smoother's in a kernel trace, and without the vectors the
// smoother needs (b, d, x_new).
template <int B, int G, typename CI>
__global__ void __launch_bounds__(256) k_power_step(int64_t n_rows, int C, const int32_t* __restrict__ slice_ptr,
                                                    const CI* __restrict__ col, const double* __restrict__ val,
                                                    const double* __restrict__ invd, const double* __restrict__ x,
                                                    double* __restrict__ y) {
    constexpr int U = B == 1 ? 8 : (B == 6 ? 1 : 2);
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t r = t / G;
    const int g = int(t % G);
    if (r >= n_rows) return;
    const int64_t s = r / C;
    const int lane = int(r - s * C);
    const int32_t p0 = slice_ptr[s];
    const int w = (slice_ptr[s + 1] - p0) / C;
    double acc[B];
#pragma unroll
    for (int i = 0; i < B; ++i) acc[i] = 0.0;
    row_product_g<double, B, B, G, U>(w, C, int64_t(p0) + lane, r, g, col, val, x, acc);
    if (g != 0) return;
#pragma unroll
    for (int i = 0; i < B; ++i) y[r * B + i] = invd[r * B + i] * acc[i];
}

template <typename T>
__global__ void k_cheb_first(int64_t n, const T* __restrict__ invd, const T* __restrict__ b, T* __restrict__ d,
                             T* __restrict__ x, T beta) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const T v = beta * invd[i] * b[i];
    d[i] = v;
    x[i] = v;
}

// y = J x over the coupled system (u rows: M_uu; phi rows: M_phiu and M_phiphi).  x is FP64,
// or FP32 (widened exactly on load); the arithmetic is FP64.
template <int D, typename TX, typename CI>
__global__ void __launch_bounds__(256) k_jspmv(int64_t nf, int C, const int32_t* __restrict__ slice_ptr,
                                               const CI* __restrict__ col, const double* __restrict__ uu,
                                               const double* __restrict__ pu, const double* __restrict__ pp,
                                               const TX* __restrict__ x, double* __restrict__ y,
                                               TX* __restrict__ xcopy, const int* __restrict__ jp,
                                               int64_t xstride) {
    const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= nf) return;
    const int64_t s = r / C;
    const int lane = int(r - s * C);
    const int32_t p0 = slice_ptr[s];
    const int w = (slice_ptr[s + 1] - p0) / C;
    const TX* xp = x + D * nf;
    double au[D], ap = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) au[i] = 0.0;
    int64_t slot = int64_t(p0) + lane;
    for (int k = 0; k < w; ++k, slot += C) {
        const int64_t c = col_at(col, slot, r);
        double xu[D];
#pragma unroll
        for (int j = 0; j < D; ++j) xu[j] = double(x[c * D + j]);
        const double xph = double(xp[c]);
        const double* vu = uu + slot * (D * D);
        const double* vp = pu + slot * D;
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int j = 0; j < D; ++j) au[i] += vu[i * D + j] * xu[j];
#pragma unroll
        for (int j = 0; j < D; ++j) ap += vp[j] * xu[j];
        ap += pp[slot] * xph;
    }
#pragma unroll
    for (int i = 0; i < D; ++i) y[r * D + i] = au[i];
    y[D * nf + r] = ap;
    if (xcopy) {   // the row's own entries of x, kept (the vector x is a scratch copy)
        TX* xc = jp ? xcopy + int64_t(*jp) * xstride : xcopy;   // Z_j of the device's Krylov index
#pragma unroll
        for (int i = 0; i < D; ++i) xc[r * D + i] = x[r * D + i];
        xc[D * nf + r] = xp[r];
    }
}

// ---- scan ---------------------------------------------------------------------------------
constexpr int kScanT = 256, kScanI = 8, kScanTile = kScanT * kScanI;

__device__ inline int32_t block_excl_scan(int32_t v, int32_t* sh, int32_t& total) {
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    int32_t x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int32_t t = __shfl_up(x, o);
        if (lane >= o) x += t;
    }
    if (lane == kWave - 1) sh[w] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t a = 0;
        for (int i = 0; i < int(blockDim.x / kWave); ++i) { const int32_t t = sh[i]; sh[i] = a; a += t; }
        sh[16] = a;
    }
    __syncthreads();
    const int32_t r = x - v + sh[w];
    total = sh[16];
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(kScanT) k_tile_sums(const int32_t* __restrict__ in, int64_t n, int32_t* __restrict__ sums) {
    __shared__ int32_t sh[32];
    const int64_t base = int64_t(blockIdx.x) * kScanTile + int64_t(threadIdx.x) * kScanI;
    int32_t t = 0;
#pragma unroll
    for (int i = 0; i < kScanI; ++i)
        if (base + i < n) t += in[base + i];
    int32_t tot;
    block_excl_scan(t, sh, tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(1024) k_scan_sums(int32_t* __restrict__ sums, int64_t nb) {
    __shared__ int32_t sh[32];
    __shared__ int32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t b0 = 0; b0 < nb; b0 += blockDim.x) {
        const int64_t i = b0 + threadIdx.x;
        const int32_t v = i < nb ? sums[i] : 0;
        int32_t tot;
        const int32_t ex = block_excl_scan(v, sh, tot);
        if (i < nb) sums[i] = ex + carry;
        __syncthreads();
        if (threadIdx.x == 0) carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[nb] = carry;
}

__global__ void __launch_bounds__(kScanT) k_tile_scan(const int32_t* __restrict__ in, int64_t n,
                                                      const int32_t* __restrict__ sums, int32_t* __restrict__ out) {
    __shared__ int32_t sh[32];
    const int64_t base = int64_t(blockIdx.x) * kScanTile + int64_t(threadIdx.x) * kScanI;
    int32_t loc[kScanI];
    int32_t t = 0;
#pragma unroll
    for (int i = 0; i < kScanI; ++i) {
        loc[i] = (base + i < n) ? in[base + i] : 0;
        t += loc[i];
    }
    int32_t tot;
    int32_t run = block_excl_scan(t, sh, tot) + sums[blockIdx.x];
#pragma unroll
    for (int i = 0; i < kScanI; ++i) {
        if (base + i < n) out[base + i] = run;
        run += loc[i];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = sums[gridDim.x];
}

// ---- reductions, casts --------------------------------------------------------------------
constexpr int kDotBlocks = 512;

__global__ void __launch_bounds__(256) k_dot_parts(const double* __restrict__ x, const double* __restrict__ y, int64_t n,
                                                   double* __restrict__ part) {
    __shared__ double sh[16];
    double acc = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        acc += x[i] * y[i];
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(256) k_sum_parts(const double* __restrict__ part, int n, double* __restrict__ out) {
    __shared__ double sh[16];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) acc += part[i];
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) *out = s;
}

template <typename A, typename B>
__global__ void k_cast(const A* __restrict__ x, B* __restrict__ y, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) y[i] = B(x[i]);
}

__global__ void k_fill(double* __restrict__ y, double v, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) y[i] = v;
}

__global__ void k_slice_width(const int32_t* __restrict__ row_len, int64_t n_rows, int C, int64_t n_slices,
                              int32_t* __restrict__ wC) {
    const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s >= n_slices) return;
    int w = 0;
    for (int64_t r = s * C; r < std::min<int64_t>(n_rows, (s + 1) * C); ++r) w = max(w, row_len[r]);
    wC[s] = w * C;
}

inline int nblk(int64_t n, int t) { return int(ceil_div(n, t)); }

}  // namespace

void scan_exclusive_async(const int32_t* in, int32_t* out, int64_t n, hipStream_t s) {
    const int64_t nb = std::max<int64_t>(1, ceil_div(n, kScanTile));
    DBuf<int32_t> sums;
    sums.alloc(size_t(nb) + 1, s);
    k_tile_sums<<<int(nb), kScanT, 0, s>>>(in, n, sums.p);
    FR_LAUNCH_CHECK();
    k_scan_sums<<<1, 1024, 0, s>>>(sums.p, nb);
    FR_LAUNCH_CHECK();
    k_tile_scan<<<int(nb), kScanT, 0, s>>>(in, n, sums.p, out);
    FR_LAUNCH_CHECK();
}

int64_t scan_exclusive(const int32_t* in, int32_t* out, int64_t n, hipStream_t s) {
    scan_exclusive_async(in, out, n, s);
    return int64_t(download1(out + n, s));
}

void dev_dot(const double* x, const double* y, int64_t n, double* dres, DBuf<double>& scratch, hipStream_t s) {
    scratch.reserve(kDotBlocks, s);
    k_dot_parts<<<kDotBlocks, 256, 0, s>>>(x, y, n, scratch.p);
    FR_LAUNCH_CHECK();
    k_sum_parts<<<1, 256, 0, s>>>(scratch.p, kDotBlocks, dres);
    FR_LAUNCH_CHECK();
}

double host_norm2(const double* x, int64_t n, DBuf<double>& scratch, hipStream_t s) {
    scratch.reserve(kDotBlocks + 1, s);
    k_dot_parts<<<kDotBlocks, 256, 0, s>>>(x, x, n, scratch.p);
    FR_LAUNCH_CHECK();
    k_sum_parts<<<1, 256, 0, s>>>(scratch.p, kDotBlocks, scratch.p + kDotBlocks);
    FR_LAUNCH_CHECK();
    return std::sqrt(download1(scratch.p + kDotBlocks, s));
}

void cast_f64_f32(const double* x, float* y, int64_t n, hipStream_t s) {
    if (n) k_cast<double, float><<<nblk(n, 256), 256, 0, s>>>(x, y, n);
    FR_LAUNCH_CHECK();
}

void cast_f32_f64(const float* x, double* y, int64_t n, hipStream_t s) {
    if (n) k_cast<float, double><<<nblk(n, 256), 256, 0, s>>>(x, y, n);
    FR_LAUNCH_CHECK();
}

void vec_copy(const double* x, double* y, int64_t n, hipStream_t s) {
    if (n) FR_HIP(hipMemcpyAsync(y, x, size_t(n) * sizeof(double), hipMemcpyDeviceToDevice, s));
}

void vec_fill(double* y, double v, int64_t n, hipStream_t s) {
    if (n) k_fill<<<nblk(n, 256), 256, 0, s>>>(y, v, n);
    FR_LAUNCH_CHECK();
}

// total slots, nnz and longest row of a structure (and an optional flag word) in one
// device record, so that building a structure costs a single host round trip
__global__ void __launch_bounds__(256) k_struct_stats(const int32_t* __restrict__ len, int64_t n,
                                                      const int32_t* __restrict__ slots_total,
                                                      const int* __restrict__ flag,
                                                      unsigned long long* __restrict__ out) {
    __shared__ unsigned long long sh_s[16];
    __shared__ int sh_m[16];
    unsigned long long sum = 0;
    int mx = 0;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
        sum += (unsigned long long)len[i];
        mx = max(mx, len[i]);
    }
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        sum += __shfl_xor(sum, o);
        mx = max(mx, __shfl_xor(mx, o));
    }
    const int w = threadIdx.x / kWave;
    if (threadIdx.x % kWave == 0) { sh_s[w] = sum; sh_m[w] = mx; }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        int m = 0;
        for (int i = 0; i < int(blockDim.x / kWave); ++i) { t += sh_s[i]; m = max(m, sh_m[i]); }
        atomicAdd(&out[1], t);
        atomicMax(&out[2], (unsigned long long)m);
        if (blockIdx.x == 0) {
            out[0] = (unsigned long long)(*slots_total);
            out[3] = flag ? (unsigned long long)(*flag) : 0ull;
        }
    }
}

void layout_from_lengths(SellStruct& S, hipStream_t s, const int* flag, int* flag_out) {
    S.n_slices = ceil_div(S.n_rows, S.C);
    DBuf<int32_t> wc;
    wc.alloc(size_t(S.n_slices) + 1, s);
    if (S.n_slices) k_slice_width<<<nblk(S.n_slices, 256), 256, 0, s>>>(S.row_len, S.n_rows, S.C, S.n_slices, wc.p);
    FR_LAUNCH_CHECK();
    S.own_slice.alloc(size_t(S.n_slices) + 1, s);
    S.slice_ptr = S.own_slice.p;
    scan_exclusive_async(wc.p, S.slice_ptr, S.n_slices, s);
    DBuf<unsigned long long> st;
    st.alloc(4, s);
    st.zero(s);
    const int g = int(std::max<int64_t>(1, std::min<int64_t>(1024, ceil_div(S.n_rows, 256))));
    k_struct_stats<<<g, 256, 0, s>>>(S.row_len, S.n_rows, S.slice_ptr + S.n_slices, flag, st.p);
    FR_LAUNCH_CHECK();
    auto h = download(st.p, 4, s);
    S.n_slots = int64_t(h[0]);
    S.nnz = int64_t(h[1]);
    S.max_len = int(h[2]);
    if (flag_out) *flag_out = int(h[3]);
    if (S.n_slots >= (int64_t(1) << 31)) fail(FR_EINTERNAL, "sell: more than 2^31 slots");
}

#define FR_BLOCK_DISPATCH(BR_, BC_, CALL)                                                         \
    if (br == BR_ && bc == BC_) { CALL(BR_, BC_); return; }

#define FR_ALL_BLOCKS(CALL)                                                                       \
    FR_BLOCK_DISPATCH(1, 1, CALL)                                                                 \
    FR_BLOCK_DISPATCH(2, 2, CALL)                                                                 \
    FR_BLOCK_DISPATCH(2, 3, CALL)                                                                 \
    FR_BLOCK_DISPATCH(3, 2, CALL)                                                                 \
    FR_BLOCK_DISPATCH(3, 3, CALL)                                                                 \
    FR_BLOCK_DISPATCH(3, 6, CALL)                                                                 \
    FR_BLOCK_DISPATCH(6, 3, CALL)                                                                 \
    FR_BLOCK_DISPATCH(6, 6, CALL)                                                                 \
    fail(FR_EINTERNAL, "spmv: unsupported block shape");

int launch_lanes(const SellStruct& S) { return S.G > 0 ? S.G : lanes_per_row(S); }

template <typename T, int MODE>
static void spmv_launch(const BMat<T>& A, int G, const T* x, const T* b, T* y, hipStream_t s) {
    const int br = A.br, bc = A.bc;
    const SellStruct& S = *A.S;
    const int gg = nblk(S.n_rows * G, 256);
#define FR_SPMV_G(BR_, BC_, G_)                                                                      \
    k_spmv<T, BR_, BC_, MODE, G_, int32_t><<<gg, 256, 0, s>>>(S.n_rows, S.C, S.slice_ptr, S.col, A.val, x, b, y);
#define FR_SPMV_CALL(BR_, BC_)                                                                       \
    switch (G) {                                                                                     \
        case 1:                                                                                      \
            if (S.col16)                                                                             \
                k_spmv<T, BR_, BC_, MODE, 1, int16_t><<<gg, 256, 0, s>>>(S.n_rows, S.C, S.slice_ptr,  \
                                                                       S.col16, A.val, x, b, y);     \
            else                                                                                     \
                FR_SPMV_G(BR_, BC_, 1)                                                               \
            break;                                                                                   \
        case 4: FR_SPMV_G(BR_, BC_, 4) break;                                                        \
        case 16: FR_SPMV_G(BR_, BC_, 16) break;                                                      \
        default: FR_SPMV_G(BR_, BC_, 64) break;                                                      \
    }                                                                                                \
    FR_LAUNCH_CHECK();
    FR_ALL_BLOCKS(FR_SPMV_CALL)
#undef FR_SPMV_CALL
#undef FR_SPMV_G
}

// Profile names: one per kernel instantiation, with the hierarchy level when the caller gives it
// ("_l<level>"), so that a level's launches are told apart from another's of the same kernel.
static void level_suffix(char* name, size_t cap, int level) {
    if (level < 0) return;
    const size_t n = std::strlen(name);
    if (n < cap) std::snprintf(name + n, cap - n, "_l%d", level);
}

template <typename T, int MODE>
static void spmv_mode(const BMat<T>& A, const T* x, const T* b, T* y, hipStream_t s, int level) {
    const int br = A.br, bc = A.bc;
    const SellStruct& S = *A.S;
    if (S.n_rows == 0) return;
    const int G = launch_lanes(S);
    // one profile scope per kernel instantiation (block shape, mode, lanes per row)
    char name[48];
    // one name per kernel instantiation (int16 column offsets are a separate one)
    if (G == 1) std::snprintf(name, sizeof(name), "spmv_%s_%dx%d_m%d%s", sizeof(T) == 8 ? "f64" : "f32", br, bc, MODE,
                              S.col16 ? "_i16" : "");
    else std::snprintf(name, sizeof(name), "spmv_%s_%dx%d_m%d_g%d", sizeof(T) == 8 ? "f64" : "f32", br, bc, MODE, G);
    level_suffix(name, sizeof(name), level);
    const double ib = (S.col16 && G == 1) ? 2.0 : 4.0;   // index bytes per stored block
    const double bytes = double(S.nnz) * (br * bc * sizeof(T) + ib) + double(S.n_cols) * bc * sizeof(T) +
                         double(S.n_rows) * br * sizeof(T) * (MODE == 0 ? 1 : 2);
    ProfScope ps(name, s, bytes);
    spmv_launch<T, MODE>(A, G, x, b, y, s);
}

template <typename T>
void spmv(const BMat<T>& A, const T* x, T* y, hipStream_t s, int level) {
    spmv_mode<T, 0>(A, x, nullptr, y, s, level);
}
template <typename T>
void spmv_residual(const BMat<T>& A, const T* x, const T* b, T* y, hipStream_t s, int level) {
    spmv_mode<T, 1>(A, x, b, y, s, level);
}
template <typename T>
void spmv_add(const BMat<T>& A, const T* x, T* y, hipStream_t s, int level) {
    spmv_mode<T, 2>(A, x, nullptr, y, s, level);
}

template <typename T>
static void cheb_launch(const BMat<T>& A, int G, const T* invd, const T* x_old, const T* b, T* d, T* x_new, T alpha,
                        T beta, hipStream_t s) {
    const SellStruct& S = *A.S;
    const int gg = nblk(S.n_rows * G, 256);
#define FR_CHEB_G(B_, G_)                                                                            \
    k_cheb<T, B_, G_, int32_t><<<gg, 256, 0, s>>>(S.n_rows, S.C, S.slice_ptr, S.col, A.val, invd, x_old, b, d, \
                                                  x_new, alpha, beta);
#define FR_CHEB_CALL(B_)                                                                             \
    switch (G) {                                                                                     \
        case 1:                                                                                      \
            if (S.col16)                                                                             \
                k_cheb<T, B_, 1, int16_t><<<gg, 256, 0, s>>>(S.n_rows, S.C, S.slice_ptr, S.col16, A.val, invd, \
                                                              x_old, b, d, x_new, alpha, beta);      \
            else                                                                                     \
                FR_CHEB_G(B_, 1)                                                                     \
            break;                                                                                   \
        case 4: FR_CHEB_G(B_, 4) break;                                                              \
        case 16: FR_CHEB_G(B_, 16) break;                                                            \
        default: FR_CHEB_G(B_, 64) break;                                                            \
    }
    switch (A.br) {
        case 1: FR_CHEB_CALL(1) break;
        case 2: FR_CHEB_CALL(2) break;
        case 3: FR_CHEB_CALL(3) break;
        case 6: FR_CHEB_CALL(6) break;
        default: fail(FR_EINTERNAL, "cheb: unsupported block size");
    }
#undef FR_CHEB_CALL
#undef FR_CHEB_G
    FR_LAUNCH_CHECK();
}

template <typename T>
void cheb_step(const BMat<T>& A, const T* invd, const T* x_old, const T* b, T* d, T* x_new, T alpha, T beta,
               hipStream_t s, int level) {
    const SellStruct& S = *A.S;
    if (S.n_rows == 0) return;
    const int G = launch_lanes(S);
    // one profile scope per kernel instantiation (block size, lanes per row)
    char name[48];
    if (G == 1) std::snprintf(name, sizeof(name), "cheb_%s_b%d%s", sizeof(T) == 8 ? "f64" : "f32", A.br,
                              S.col16 ? "_i16" : "");
    else std::snprintf(name, sizeof(name), "cheb_%s_b%d_g%d", sizeof(T) == 8 ? "f64" : "f32", A.br, G);
    level_suffix(name, sizeof(name), level);
    // matrix once (index bytes 2 with row offsets), x gathered once, b, d, D^-1 read, d and
    // x_new written
    const double ib = (S.col16 && G == 1) ? 2.0 : 4.0;
    const double bytes = double(S.nnz) * (A.br * A.bc * sizeof(T) + ib) + double(S.n_rows) * A.br * sizeof(T) * 6;
    ProfScope ps(name, s, bytes);
    cheb_launch<T>(A, G, invd, x_old, b, d, x_new, alpha, beta, s);
}

// Row offsets of a SELL structure's columns as int16 (rows beyond n_rows in the last slice
// get 0); *misfit is set when an offset does not fit.
__global__ void k_col16(int64_t n_rows, int C, const int32_t* __restrict__ sp, const int32_t* __restrict__ col,
                        int16_t* __restrict__ col16, int* __restrict__ misfit) {
    const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t n_pad = ((n_rows + C - 1) / C) * C;
    if (r >= n_pad) return;
    const int64_t s0 = r / C;
    const int lane = int(r - s0 * C);
    const int w = (sp[s0 + 1] - sp[s0]) / C;
    bool bad = false;
    for (int k = 0; k < w; ++k) {
        const int64_t slot = int64_t(sp[s0]) + int64_t(k) * C + lane;
        const int64_t off = r < n_rows ? int64_t(col[slot]) - r : 0;
        bad = bad || off < -32768 || off > 32767;
        col16[slot] = int16_t(bad ? 0 : off);
    }
    if (bad) atomicOr(misfit, 1);
}

void make_col16(SellStruct& S, hipStream_t s) {
    if (S.n_rows == 0 || S.n_slots == 0) return;
    S.own_col16.alloc(size_t(S.n_slots), s);
    DBuf<int> misfit;
    misfit.alloc(1, s);
    misfit.zero(s);
    const int64_t n_pad = ceil_div(S.n_rows, S.C) * S.C;
    k_col16<<<nblk(n_pad, 256), 256, 0, s>>>(S.n_rows, S.C, S.slice_ptr, S.col, S.own_col16.p, misfit.p);
    FR_LAUNCH_CHECK();
    if (download1(misfit.p, s) == 0) {
        S.col16 = S.own_col16.p;
    } else {
        S.own_col16.release();
        S.col16 = nullptr;
    }
}

// y = D^-1 A x (the Chebyshev kernel with b = 0, alpha = 0, beta = -1; xn receives x + y),
// in the matrix's launch shape (a refreshed hierarchy's levels carry tuned shapes, so its
// estimates can differ from the build's in the last bits)
void diag_scaled_matvec(const BMat<double>& A, const double* invd, const double* x, double* y, hipStream_t s) {
    const SellStruct& S = *A.S;
    if (S.n_rows == 0) return;
    const int G = launch_lanes(S);
    const int gg = nblk(S.n_rows * G, 256);
#define FR_POW_G(B_, G_) \
    k_power_step<B_, G_, int32_t><<<gg, 256, 0, s>>>(S.n_rows, S.C, S.slice_ptr, S.col, A.val, invd, x, y);
#define FR_POW_CALL(B_)                                                                                         \
    switch (G) {                                                                                                \
        case 1:                                                                                                 \
            if (S.col16)                                                                                        \
                k_power_step<B_, 1, int16_t><<<gg, 256, 0, s>>>(S.n_rows, S.C, S.slice_ptr, S.col16, A.val, invd, x, y); \
            else                                                                                                \
                FR_POW_G(B_, 1)                                                                                 \
            break;                                                                                              \
        case 4: FR_POW_G(B_, 4) break;                                                                          \
        case 16: FR_POW_G(B_, 16) break;                                                                        \
        default: FR_POW_G(B_, 64) break;                                                                        \
    }
    switch (A.br) {
        case 1: FR_POW_CALL(1) break;
        case 2: FR_POW_CALL(2) break;
        case 3: FR_POW_CALL(3) break;
        case 6: FR_POW_CALL(6) break;
        default: fail(FR_EINTERNAL, "power step: unsupported block size");
    }
#undef FR_POW_CALL
#undef FR_POW_G
    FR_LAUNCH_CHECK();
}

// ---- launch-shape tuner ---------------------------------------------------------------------
// Copy of a block SELL matrix in another slice height (C = 1 stores each row contiguously, so
// that the lanes of a row read consecutive slots); padding repeats the row's first column
// with zero blocks.
struct SellRef {
    int C;
    int64_t n_rows;
    const int32_t* sp;
    const int32_t* len;
    const int32_t* col;
};

__device__ __forceinline__ int64_t slot_at(const SellRef& A, int64_t r, int k) {
    return int64_t(A.sp[r / A.C]) + int64_t(k) * A.C + (r % A.C);
}

template <int BB>
__global__ void k_relayout(SellRef A, const double* __restrict__ av, SellRef O, int32_t* __restrict__ ocol,
                           double* __restrict__ ov) {
    const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= O.n_rows) return;
    const int len = A.len[r];
    const int64_t s0 = r / O.C;
    const int width = (O.sp[s0 + 1] - O.sp[s0]) / O.C;
    const int32_t c0 = len > 0 ? A.col[slot_at(A, r, 0)] : 0;
    for (int k = 0; k < width; ++k) {
        const int64_t os = slot_at(O, r, k);
        if (k < len) {
            const int64_t as = slot_at(A, r, k);
            ocol[os] = A.col[as];
            for (int e = 0; e < BB; ++e) ov[os * BB + e] = av[as * BB + e];
        } else {
            ocol[os] = c0;
            for (int e = 0; e < BB; ++e) ov[os * BB + e] = 0.0;
        }
    }
}

BMat<double> relayout(const BMat<double>& A, int C, hipStream_t s) {
    const SellStruct& S = *A.S;
    BMat<double> O;
    O.br = A.br;
    O.bc = A.bc;
    auto N = std::make_shared<SellStruct>();
    N->C = C;
    N->n_rows = S.n_rows;
    N->n_cols = S.n_cols;
    N->own_len.alloc(size_t(std::max<int64_t>(1, S.n_rows)), s);
    N->row_len = N->own_len.p;
    if (S.n_rows) FR_HIP(hipMemcpyAsync(N->row_len, S.row_len, size_t(S.n_rows) * sizeof(int32_t),
                                        hipMemcpyDeviceToDevice, s));
    if (C == 1) {
        // one row per slice: the slice pointers are the row offsets and every statistic is
        // the source's, so no host round trip is needed
        N->n_slices = S.n_rows;
        N->own_slice.alloc(size_t(S.n_rows) + 1, s);
        N->slice_ptr = N->own_slice.p;
        scan_exclusive_async(N->row_len, N->slice_ptr, S.n_rows, s);
        N->n_slots = S.nnz;
        N->nnz = S.nnz;
        N->max_len = S.max_len;
    } else {
        layout_from_lengths(*N, s, nullptr, nullptr);
    }
    N->own_col.alloc(size_t(std::max<int64_t>(1, N->n_slots)), s);
    N->col = N->own_col.p;
    const int BB = A.br * A.bc;
    O.own_val.alloc(size_t(std::max<int64_t>(1, N->n_slots)) * BB, s);
    O.val = O.own_val.p;
    const SellRef av{S.C, S.n_rows, S.slice_ptr, S.row_len, S.col};
    const SellRef ov{N->C, N->n_rows, N->slice_ptr, N->row_len, N->col};
    const int g = nblk(std::max<int64_t>(1, S.n_rows), 256);
#define FR_RL(BB_) case BB_: k_relayout<BB_><<<g, 256, 0, s>>>(av, A.val, ov, N->col, O.val); break;
    switch (BB) {
        FR_RL(1) FR_RL(4) FR_RL(6) FR_RL(9) FR_RL(18) FR_RL(36)
        default: fail(FR_EINTERNAL, "relayout: unsupported block shape");
    }
#undef FR_RL
    FR_LAUNCH_CHECK();
    O.S = N;
    return O;
}

namespace {
struct TuneKey {
    int op, br, bc, lg_rows, avg_len, f32;
    bool operator<(const TuneKey& o) const {
        return std::tie(op, br, bc, lg_rows, avg_len, f32) < std::tie(o.op, o.br, o.bc, o.lg_rows, o.avg_len, o.f32);
    }
};
std::mutex g_tune_mu;
std::map<TuneKey, std::pair<int, int>> g_tune;   // -> (slice height, lanes per row)

// best of five timed launches (after one warm-up) of each candidate shape, in precision T
template <typename T>
std::pair<int, int> time_shapes(const BMat<double>& M, int op, hipStream_t s) {
    const SellStruct& S = *M.S;
    const int64_t nr = S.n_rows * M.br, nc = S.n_cols * M.bc;
    DBuf<T> x, y, b, d, iv;
    x.alloc(size_t(std::max<int64_t>(1, nc)), s);
    y.alloc(size_t(std::max<int64_t>(1, nr)), s);
    b.alloc(size_t(std::max<int64_t>(1, nr)), s);
    d.alloc(size_t(std::max<int64_t>(1, nr)), s);
    iv.alloc(size_t(std::max<int64_t>(1, nr)), s);
    x.zero(s);
    y.zero(s);
    b.zero(s);
    d.zero(s);
    iv.zero(s);
    // the matrix in both slice heights, values in precision T
    BMat<double> alt;
    DBuf<float> v32[2];
    auto as_t = [&](const BMat<double>& A, int which) {
        BMat<T> t;
        t.br = A.br;
        t.bc = A.bc;
        t.S = A.S;
        if constexpr (sizeof(T) == 8) {
            t.val = A.val;
        } else {
            const int64_t n = A.S->n_slots * A.br * A.bc;
            v32[which].alloc(size_t(std::max<int64_t>(1, n)), s);
            cast_f64_f32(A.val, v32[which].p, n, s);
            t.val = v32[which].p;
        }
        return t;
    };
    const BMat<T> m0 = as_t(M, 0);
    BMat<T> m1;
    hipEvent_t e0, e1;
    FR_HIP(hipEventCreate(&e0));
    FR_HIP(hipEventCreate(&e1));
    const std::pair<int, int> cands[] = {{S.C, 1}, {S.C, 4}, {S.C, 16}, {1, 1}, {1, 4}, {1, 16}, {1, 64}};
    const int G0 = lanes_per_row(S);
    double best = 1e30, base = 1e30;
    std::pair<int, int> pick{0, 0};
    std::vector<std::pair<std::pair<int, int>, float>> times;
    for (const auto& cg : cands) {
        if (cg.first != S.C && alt.rows() == 0) {
            alt = relayout(M, cg.first, s);
            m1 = as_t(alt, 1);
        }
        const BMat<T>& A = cg.first == S.C ? m0 : m1;
        auto run = [&]() {
            if (op == 0) cheb_launch<T>(A, cg.second, iv.p, x.p, b.p, d.p, y.p, T(0), T(1), s);
            else if (op == 1) spmv_launch<T, 0>(A, cg.second, x.p, nullptr, y.p, s);
            else spmv_launch<T, 2>(A, cg.second, x.p, nullptr, y.p, s);
        };
        run();
        float t = 1e30f;
        for (int rep = 0; rep < 5; ++rep) {
            FR_HIP(hipEventRecord(e0, s));
            run();
            FR_HIP(hipEventRecord(e1, s));
            FR_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            FR_HIP(hipEventElapsedTime(&ms, e0, e1));
            t = std::min(t, ms);
        }
        if (cg.first == S.C && cg.second == G0) base = t;
        times.push_back({cg, t});
        best = std::min(best, double(t));
    }
    FR_HIP(hipEventDestroy(e0));
    FR_HIP(hipEventDestroy(e1));
    // near ties (within 3 % of the fastest, below the timing noise) go to the shape with the
    // most lanes per row, then to contiguous rows (no padding): fewer dependent loads per lane
    // and fewer bytes, which hold up better beside the other cycle's traffic, and the same
    // choice from run to run
    for (const auto& [cg, t] : times)
        if (t <= 1.03 * best &&
            (pick.first == 0 || cg.second > pick.second || (cg.second == pick.second && cg.first < pick.first)))
            pick = cg;
    if (base < 1e30 && best > 0.95 * base) pick = {S.C, G0};
    return pick;
}
}  // namespace

void tune_clear() {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
}

int tune_entries() {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    return int(g_tune.size());
}

// One line per cached choice: "op br bc lg_rows avg_len f32 C G".
std::string tune_export() {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    std::string out;
    char line[96];
    for (const auto& [k, v] : g_tune) {
        std::snprintf(line, sizeof(line), "%d %d %d %d %d %d %d %d\n", k.op, k.br, k.bc, k.lg_rows, k.avg_len, k.f32,
                      v.first, v.second);
        out += line;
    }
    return out;
}

// Parses the whole text before it touches the cache, so a malformed table changes nothing.
// Entries replace cached choices with the same key.
void tune_import(const char* text) {
    std::vector<std::pair<TuneKey, std::pair<int, int>>> rows;
    const char* p = text;
    int line_no = 0;
    while (*p) {
        const char* e = std::strchr(p, '\n');
        const size_t n = e ? size_t(e - p) : std::strlen(p);
        std::string line(p, n);
        p += n + (e ? 1 : 0);
        ++line_no;
        if (line.find_first_not_of(" \t\r") == std::string::npos) continue;
        TuneKey k{};
        int C = 0, G = 0, used = 0;
        const int got = std::sscanf(line.c_str(), "%d %d %d %d %d %d %d %d %n", &k.op, &k.br, &k.bc, &k.lg_rows,
                                    &k.avg_len, &k.f32, &C, &G, &used);
        if (got != 8 || line.find_first_not_of(" \t\r", size_t(used)) != std::string::npos)
            fail(FR_EINVAL, "tune table line " + std::to_string(line_no) + ": expected 8 integers");
        if (k.op < 0 || k.op > 2 || k.br < 1 || k.br > 6 || k.bc < 1 || k.bc > 6 || k.lg_rows < 0 || k.lg_rows > 62 ||
            k.avg_len < 0 || (k.f32 != 0 && k.f32 != 1))
            fail(FR_EINVAL, "tune table line " + std::to_string(line_no) + ": key out of range");
        if ((C != 1 && C != kWave) || (G != 1 && G != 4 && G != 16 && G != 64))
            fail(FR_EINVAL, "tune table line " + std::to_string(line_no) + ": slice height must be 1 or " +
                                std::to_string(kWave) + ", lanes per row 1, 4, 16 or 64");
        rows.push_back({k, {C, G}});
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto& r : rows) g_tune[r.first] = r.second;
}

// op 0: Chebyshev step (smoother of A), 1: y = M x (restriction), 2: y += M x (prolongation),
// timed in the precision the V-cycle runs in (f32).  Candidates: slice height 64 with 1, 4,
// 16 lanes per row and contiguous rows (C = 1) with 1, 4, 16, 64 lanes.  Each is timed (one
// warm-up, best of five) on the matrix itself; among shapes within 3 % of the fastest the one
// with the most lanes per row (then contiguous rows) is taken, and the heuristic shape is kept
// unless that one is at least 5 % faster.  Choices are cached per process by (op, block shape, log2 rows,
// mean row length, precision), so later setups of similar levels reuse them without timing.
// Large operators are tuned too: the finest prolongator's rows (1 to ~5 blocks) pad a slice
// of 64 to its longest row, which contiguous rows avoid.
void tune_layout(BMat<double>& M, int op, bool f32, hipStream_t s) {
    SellStruct& S = *M.S;
    if (S.n_rows == 0) return;
    const int64_t avg = S.nnz / S.n_rows;
    int lg = 0;
    while ((int64_t(1) << (lg + 1)) <= S.n_rows) ++lg;
    const TuneKey key{op, M.br, M.bc, lg, int(avg), f32 ? 1 : 0};
    std::pair<int, int> choice{0, 0};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) choice = it->second;
    }
    if (choice.first == 0) {
        choice = f32 ? time_shapes<float>(M, op, s) : time_shapes<double>(M, op, s);
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune.emplace(key, choice);
    }
    if (choice.first != S.C) M = relayout(M, choice.first, s);
    M.S->G = choice.second;
}

template <typename T>
void cheb_first(const T* invd, const T* b, T* d, T* x, T beta, int64_t n, hipStream_t s, int level) {
    if (n == 0) return;
    // D^-1 and b read, d and x written
    char name[48];
    std::snprintf(name, sizeof(name), "cheb_first_%s", sizeof(T) == 8 ? "f64" : "f32");
    level_suffix(name, sizeof(name), level);
    ProfScope ps(name, s, double(n) * sizeof(T) * 4);
    k_cheb_first<T><<<nblk(n, 256), 256, 0, s>>>(n, invd, b, d, x, beta);
    FR_LAUNCH_CHECK();
}

template <typename TX>
static void jspmv_t(const DevSystem& sys, const TX* x, double* y, hipStream_t s, TX* xcopy = nullptr,
                    const int* jp = nullptr, int64_t xstride = 0) {
    const SellStruct& S = *sys.Juu.S;
    const int g = nblk(S.n_rows, 256);
    const int D = sys.mesh->dim;
    const double ib = S.col16 ? 2.0 : 4.0;
    const double bytes = double(S.nnz) * ((D * D + D + 1) * 8 + ib) + double(S.n_rows) * (D + 1) * (sizeof(TX) + 8);
    char name[32];
    std::snprintf(name, sizeof(name), "jspmv_d%d%s", D, sizeof(TX) == 4 ? "_x32" : "");
    ProfScope ps(name, s, bytes);
#define FR_JSPMV(D_, CI_, COL_)                                                                        \
    k_jspmv<D_, TX, CI_><<<g, 256, 0, s>>>(S.n_rows, S.C, S.slice_ptr, COL_, sys.Juu.val, sys.Jpu.val, sys.Jpp.val, \
                                           x, y, xcopy, jp, xstride);
    if (D == 2) {
        if (S.col16) { FR_JSPMV(2, int16_t, S.col16) }
        else { FR_JSPMV(2, int32_t, S.col) }
    } else {
        if (S.col16) { FR_JSPMV(3, int16_t, S.col16) }
        else { FR_JSPMV(3, int32_t, S.col) }
    }
#undef FR_JSPMV
    FR_LAUNCH_CHECK();
}

void jspmv(const DevSystem& sys, const double* x, double* y, hipStream_t s) { jspmv_t<double>(sys, x, y, s); }
void jspmv(const DevSystem& sys, const float* x, double* y, hipStream_t s) { jspmv_t<float>(sys, x, y, s); }
void jspmv_copy(const DevSystem& sys, const double* x, double* y, double* xcopy, const int* jp, int64_t xstride,
                hipStream_t s) {
    jspmv_t<double>(sys, x, y, s, xcopy, jp, xstride);
}
void jspmv_copy(const DevSystem& sys, const float* x, double* y, float* xcopy, const int* jp, int64_t xstride,
                hipStream_t s) {
    jspmv_t<float>(sys, x, y, s, xcopy, jp, xstride);
}

void system_matvec(DevSystem& sys, const double* x, double* y) { jspmv(sys, x, y, sys.stream); }

template void spmv<double>(const BMat<double>&, const double*, double*, hipStream_t, int);
template void spmv<float>(const BMat<float>&, const float*, float*, hipStream_t, int);
template void spmv_residual<double>(const BMat<double>&, const double*, const double*, double*, hipStream_t, int);
template void spmv_residual<float>(const BMat<float>&, const float*, const float*, float*, hipStream_t, int);
template void spmv_add<double>(const BMat<double>&, const double*, double*, hipStream_t, int);
template void spmv_add<float>(const BMat<float>&, const float*, float*, hipStream_t, int);
template void cheb_step<double>(const BMat<double>&, const double*, const double*, const double*, double*, double*,
                                double, double, hipStream_t, int);
template void cheb_step<float>(const BMat<float>&, const float*, const float*, const float*, float*, float*, float,
                               float, hipStream_t, int);
template void cheb_first<double>(const double*, const double*, double*, double*, double, int64_t, hipStream_t, int);
template void cheb_first<float>(const float*, const float*, float*, float*, float, int64_t, hipStream_t, int);

}  // namespace fr
