// Flexible GMRES (right preconditioned, restarted) for the masked Newton system of Section 3,
// FP64 throughout.  Arnoldi orthogonalisation is classical Gram-Schmidt with one
// re-orthogonalisation pass (CGS2): a multi-vector dot kernel and a multi-vector update
// kernel stream the basis once each per pass; the small Hessenberg least-squares problem
// (Givens rotations) is solved on the host from the j+2 coefficients copied back per
// iteration, which is also the convergence check.
#include <cmath>
#include <vector>

#include "profile.h"
#include "system.h"

namespace fr {
namespace {

constexpr int kGroup = 8;        // basis vectors per multidot block row
constexpr int kRowBlocks = 256;  // blocks per group along the vector

// part[(v) * kRowBlocks + bx] = sum over this block's rows of V_v[i] w[i], v in [v0, v0+kGroup)
__global__ void __launch_bounds__(256) k_multidot(const double* __restrict__ V, int64_t n, int nv,
                                                  const double* __restrict__ w, double* __restrict__ part) {
    __shared__ double sh[16];
    const int v0 = blockIdx.y * kGroup;
    double acc[kGroup];
#pragma unroll
    for (int g = 0; g < kGroup; ++g) acc[g] = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
        const double wi = w[i];
#pragma unroll
        for (int g = 0; g < kGroup; ++g)
            if (v0 + g < nv) acc[g] += V[int64_t(v0 + g) * n + i] * wi;
    }
#pragma unroll
    for (int g = 0; g < kGroup; ++g) {
        const double s = block_sum(acc[g], sh);
        if (threadIdx.x == 0 && v0 + g < nv) part[int64_t(v0 + g) * gridDim.x + blockIdx.x] = s;
    }
}

// Multi-vector dot, one pass over the basis: each thread holds kE elements of w in
// registers and streams V_0..V_{nv-1}; per vector a wave reduction and a per-block LDS
// row give part[v * gridDim.x + block].
constexpr int kE = 4;

__device__ __forceinline__ void block_store_parts(double (*sh)[4], int nv, double* __restrict__ part) {
    __syncthreads();
    for (int v = threadIdx.x; v < nv; v += blockDim.x)
        part[int64_t(v) * gridDim.x + blockIdx.x] = sh[v][0] + sh[v][1] + sh[v][2] + sh[v][3];
}

__global__ void __launch_bounds__(256) k_multidot2(const double* __restrict__ V, int64_t n, int nv,
                                                   const double* __restrict__ w, double* __restrict__ part) {
    __shared__ double sh[128][4];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int64_t base = int64_t(blockIdx.x) * (256 * kE) + threadIdx.x;
    double wv[kE];
#pragma unroll
    for (int e = 0; e < kE; ++e) {
        const int64_t i = base + 256 * e;
        wv[e] = i < n ? w[i] : 0.0;
    }
    for (int v = 0; v < nv; ++v) {
        const double* Vv = V + int64_t(v) * n;
        double acc = 0.0;
#pragma unroll
        for (int e = 0; e < kE; ++e) {
            const int64_t i = base + 256 * e;
            if (i < n) acc += Vv[i] * wv[e];
        }
        acc = wave_sum(acc);
        if (lane == 0) sh[v][wave] = acc;
    }
    block_store_parts(sh, nv, part);
}

// w -= sum_k c[k] V_k, then the dots of the updated w with the same vectors (the second
// sweep re-reads the block's slice of V while it is still in cache).
__global__ void __launch_bounds__(256) k_update_dot(const double* __restrict__ V, int64_t n, int nv,
                                                    const double* __restrict__ c, double* __restrict__ w,
                                                    double* __restrict__ part) {
    __shared__ double sh[128][4];
    __shared__ double cs[128];
    for (int k = threadIdx.x; k < nv; k += blockDim.x) cs[k] = c[k];
    __syncthreads();
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int64_t base = int64_t(blockIdx.x) * (256 * kE) + threadIdx.x;
    double wv[kE];
#pragma unroll
    for (int e = 0; e < kE; ++e) {
        const int64_t i = base + 256 * e;
        wv[e] = i < n ? w[i] : 0.0;
    }
    for (int v = 0; v < nv; ++v) {
        const double* Vv = V + int64_t(v) * n;
        const double cv = cs[v];
#pragma unroll
        for (int e = 0; e < kE; ++e) {
            const int64_t i = base + 256 * e;
            if (i < n) wv[e] -= cv * Vv[i];
        }
    }
#pragma unroll
    for (int e = 0; e < kE; ++e) {
        const int64_t i = base + 256 * e;
        if (i < n) w[i] = wv[e];
    }
    for (int v = 0; v < nv; ++v) {
        const double* Vv = V + int64_t(v) * n;
        double acc = 0.0;
#pragma unroll
        for (int e = 0; e < kE; ++e) {
            const int64_t i = base + 256 * e;
            if (i < n) acc += Vv[i] * wv[e];
        }
        acc = wave_sum(acc);
        if (lane == 0) sh[v][wave] = acc;
    }
    block_store_parts(sh, nv, part);
}

// h[v] (+)= sum_bx part[v * nb + bx]
__global__ void __launch_bounds__(256) k_reduce_parts(const double* __restrict__ part, int nb,
                                                      double* __restrict__ h, int accumulate) {
    __shared__ double sh[16];
    const int v = blockIdx.x;
    double acc = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) acc += part[int64_t(v) * nb + i];
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) h[v] = accumulate ? h[v] + s : s;
}

// w -= sum_k c[k] V_k; optional partial sums of the squared result
__global__ void __launch_bounds__(256) k_update(const double* __restrict__ V, int64_t n, int nv,
                                                const double* __restrict__ c, double* __restrict__ w,
                                                double* __restrict__ part) {
    __shared__ double sh[16];
    __shared__ double cs[128];
    for (int k = threadIdx.x; k < nv && k < 128; k += blockDim.x) cs[k] = c[k];
    __syncthreads();
    double acc = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
        double t = w[i];
        for (int k = 0; k < nv; ++k) t -= (k < 128 ? cs[k] : c[k]) * V[int64_t(k) * n + i];
        w[i] = t;
        acc += t * t;
    }
    if (part) {
        const double s = block_sum(acc, sh);
        if (threadIdx.x == 0) part[blockIdx.x] = s;
    }
}

// y = x / ||x|| with ||x||^2 read from the device
__global__ void k_scale_copy(int64_t n, const double* __restrict__ x, const double* __restrict__ nrm2,
                             double* __restrict__ y) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) {
        const double v = *nrm2;
        y[i] = v > 0.0 ? x[i] / sqrt(v) : 0.0;
    }
}

// x += sum_j y[j] Z_j
__global__ void __launch_bounds__(256) k_combine(const double* __restrict__ Z, int64_t n, int nz,
                                                 const double* __restrict__ y, double* __restrict__ x) {
    __shared__ double ys[128];
    for (int k = threadIdx.x; k < nz && k < 128; k += blockDim.x) ys[k] = y[k];
    __syncthreads();
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
        double t = x[i];
        for (int k = 0; k < nz; ++k) t += (k < 128 ? ys[k] : y[k]) * Z[int64_t(k) * n + i];
        x[i] = t;
    }
}

// r = F - r (r holds J x on entry); partial sums of r^2
__global__ void __launch_bounds__(256) k_resid(int64_t n, const double* __restrict__ F, double* __restrict__ r,
                                               double* __restrict__ part) {
    __shared__ double sh[16];
    double acc = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
        const double t = F[i] - r[i];
        r[i] = t;
        acc += t * t;
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

}  // namespace

fr_status fgmres(DevSystem& sys, DevAmg& amg, const fr_solve_opts& o, double* du, fr_solve_stats& st, DevKrylov& ws,
                 hipStream_t s) {
    const int64_t n = sys.n_solve;
    const int m = std::max(1, std::min(o.restart, 120));
    if (ws.n != n || ws.m < m) {
        ws.n = n;
        ws.m = m;
        ws.V.alloc(size_t(m + 1) * size_t(n), s);
        ws.Z.alloc(size_t(m) * size_t(n), s);
        ws.w.alloc(size_t(n), s);
        ws.r.alloc(size_t(n), s);
        ws.h.alloc(1024, s);
        ws.part.alloc(size_t(std::max<int64_t>(kRowBlocks, ceil_div(n, 256 * kE))) * 128 + 1024, s);
    }
    const int gridN = int(std::min<int64_t>(1024, ceil_div(n, 256)));
    const int nbE = int(ceil_div(n, 256 * kE));
    double* part = ws.part.p;
    double* h = ws.h.p;          // [0, 122): Hessenberg column of the current iteration
    double* h2 = ws.h.p + 256;   // [256, 378): re-orthogonalisation coefficients
    double* yv = ws.h.p + 512;   // [512, 633): combination coefficients
    double* nrm = ws.h.p + 768;  // squared norm scratch

    auto reduce_to = [&](double* out, int nb) {
        k_reduce_parts<<<1, 256, 0, s>>>(part, nb, out, 0);
        FR_LAUNCH_CHECK();
    };

    // ||F||
    k_update<<<gridN, 256, 0, s>>>(ws.V.p, n, 0, h, sys.F.p, part);   // nv = 0: only the norm of F
    FR_LAUNCH_CHECK();
    reduce_to(nrm, gridN);
    const double bnorm = std::sqrt(download1(nrm, s));
    FR_HIP(hipMemsetAsync(du, 0, size_t(n) * sizeof(double), s));
    st.iters = 0;
    st.relres = 0.0;
    st.status = FR_OK;
    if (!(bnorm > 0.0)) {
        if (std::isnan(bnorm)) { st.status = FR_ENAN; return FR_ENAN; }
        return FR_OK;
    }
    const double target = o.rtol * bnorm;
    int total = 0;
    bool first = true;
    const size_t ms = static_cast<size_t>(m);
    std::vector<double> H((ms + 1) * ms, 0.0), cs(ms, 0.0), sn(ms, 0.0), g(ms + 1, 0.0);
    while (true) {
        // r = F - J x
        double beta;
        if (first) {
            vec_copy(sys.F.p, ws.w.p, n, s);
            beta = bnorm;
            dev_dot(ws.w.p, ws.w.p, n, nrm, ws.part, s);
        } else {
            jspmv(sys, du, ws.w.p, s);
            k_resid<<<gridN, 256, 0, s>>>(n, sys.F.p, ws.w.p, part);
            FR_LAUNCH_CHECK();
            reduce_to(nrm, gridN);
            beta = std::sqrt(download1(nrm, s));
        }
        first = false;
        st.relres = beta / bnorm;
        if (beta <= target) break;
        if (total >= o.maxit) { st.status = FR_ENOCONV; break; }
        k_scale_copy<<<int(ceil_div(n, 256)), 256, 0, s>>>(n, ws.w.p, nrm, ws.V.p);
        FR_LAUNCH_CHECK();
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int j = 0;
        bool breakdown = false;
        for (; j < m && total < o.maxit; ++j) {
            double* Vj = ws.V.p + int64_t(j) * n;
            double* Zj = ws.Z.p + int64_t(j) * n;
            amg_precondition(amg, Vj, Zj, s);
            jspmv(sys, Zj, ws.w.p, s);
            const int nv = j + 1;
            const double md_bytes = double(nv + 1) * double(n) * 8.0;
            const double up_bytes = double(nv + 2) * double(n) * 8.0;
            // pass 1: h = V^T w
            {
                ProfScope ps("gs_multidot", s, md_bytes);
                k_multidot2<<<nbE, 256, 0, s>>>(ws.V.p, n, nv, ws.w.p, part);
                FR_LAUNCH_CHECK();
            }
            k_reduce_parts<<<nv, 256, 0, s>>>(part, nbE, h, 0);
            FR_LAUNCH_CHECK();
            // w -= V h and, in the same sweep, h2 = V^T w (re-orthogonalisation coefficients)
            {
                ProfScope ps("gs_update_dot", s, up_bytes);
                k_update_dot<<<nbE, 256, 0, s>>>(ws.V.p, n, nv, h, ws.w.p, part);
                FR_LAUNCH_CHECK();
            }
            k_reduce_parts<<<nv, 256, 0, s>>>(part, nbE, h2, 0);
            FR_LAUNCH_CHECK();
            // w -= V h2 and ||w||^2
            {
                ProfScope ps("gs_update", s, up_bytes);
                k_update<<<gridN, 256, 0, s>>>(ws.V.p, n, nv, h2, ws.w.p, part);
                FR_LAUNCH_CHECK();
            }
            reduce_to(h + nv, gridN);       // ||w||^2 in h[j+1]
            k_scale_copy<<<int(ceil_div(n, 256)), 256, 0, s>>>(n, ws.w.p, h + nv, ws.V.p + int64_t(j + 1) * n);
            FR_LAUNCH_CHECK();
            std::vector<double> hh = download(h, size_t(nv + 1), s);
            std::vector<double> hc = download(h2, size_t(nv), s);
            for (int i = 0; i < nv; ++i) hh[size_t(i)] += hc[size_t(i)];
            hh[size_t(nv)] = std::sqrt(hh[size_t(nv)]);
            ++total;
            if (!std::isfinite(hh[size_t(nv)])) { st.status = FR_ENAN; breakdown = true; }
            // Givens
            for (int i = 0; i < j; ++i) {
                const double a = hh[size_t(i)], b = hh[size_t(i + 1)];
                hh[size_t(i)] = cs[size_t(i)] * a + sn[size_t(i)] * b;
                hh[size_t(i + 1)] = -sn[size_t(i)] * a + cs[size_t(i)] * b;
            }
            const double a = hh[size_t(j)], b = hh[size_t(j + 1)];
            const double rr = std::hypot(a, b);
            cs[size_t(j)] = rr > 0 ? a / rr : 1.0;
            sn[size_t(j)] = rr > 0 ? b / rr : 0.0;
            hh[size_t(j)] = rr;
            hh[size_t(j + 1)] = 0.0;
            g[size_t(j + 1)] = -sn[size_t(j)] * g[size_t(j)];
            g[size_t(j)] = cs[size_t(j)] * g[size_t(j)];
            for (int i = 0; i <= j; ++i) H[size_t(i) * m + j] = hh[size_t(i)];
            if (breakdown) { ++j; break; }
            if (std::fabs(g[size_t(j + 1)]) <= target) { ++j; break; }
            if (hh[size_t(j)] == 0.0) { ++j; break; }
        }
        // back substitution H y = g
        std::vector<double> y(size_t(j), 0.0);
        for (int i = j - 1; i >= 0; --i) {
            double t = g[size_t(i)];
            for (int k = i + 1; k < j; ++k) t -= H[size_t(i) * m + k] * y[size_t(k)];
            const double d = H[size_t(i) * m + i];
            y[size_t(i)] = d != 0.0 ? t / d : 0.0;
        }
        if (j > 0) {
            FR_HIP(hipMemcpyAsync(yv, y.data(), size_t(j) * sizeof(double), hipMemcpyHostToDevice, s));
            k_combine<<<gridN, 256, 0, s>>>(ws.Z.p, n, j, yv, du);
            FR_LAUNCH_CHECK();
        }
        if (st.status == FR_ENAN) break;
    }
    st.iters = total;
    if (st.status == FR_OK && st.relres > o.rtol) st.status = FR_ENOCONV;
    return fr_status(st.status);
}

}  // namespace fr
