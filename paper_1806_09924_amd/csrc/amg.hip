// Smoothed-aggregation AMG for the two diagonal blocks of the Newton Jacobian (Section 3:
// P^-1 = diag(M_uu~^-1, M_phiphi~^-1), each applied as one multigrid V-cycle).  Setup runs
// on the GPU: strength graph, deterministic MIS(2) aggregation, tentative prolongator by a
// per-aggregate QR of the near-null space (rigid-body modes for the displacement block,
// constants for the phase field), damped-Jacobi prolongator smoothing, Galerkin R A P by a
// two-phase hashed SpGEMM, a power-iteration estimate of lambda_max(D^-1 A) for the
// Chebyshev smoother and a dense inverse of the coarsest operator.  Every kernel
// accumulates in a fixed order, so the hierarchy is bitwise reproducible.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <exception>
#include <functional>
#include <string>
#include <thread>
#include <type_traits>

#include <hipcub/hipcub.hpp>

#include "profile.h"
#include "system.h"

namespace fr {
namespace {

constexpr int kWavesPerBlock = 4;  // 256-thread blocks
constexpr int kDenseMax = 4096;    // largest coarsest level inverted densely

inline int nblk(int64_t n, int t) { return int(ceil_div(n, t)); }

__device__ __forceinline__ int64_t sslot(const int32_t* slice_ptr, int C, int64_t r, int k) {
    return int64_t(slice_ptr[r / C]) + int64_t(k) * C + (r % C);
}

// ---- diagonal information ----------------------------------------------------------------
template <int B>
__global__ void k_diag(int64_t n, int C, const int32_t* __restrict__ sp, const int32_t* __restrict__ len,
                       const int32_t* __restrict__ col, const double* __restrict__ val, double* __restrict__ invd,
                       double* __restrict__ dnorm) {
    const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= n) return;
    double nr = 0.0;
    double dg[B];
    for (int i = 0; i < B; ++i) dg[i] = 0.0;
    for (int k = 0; k < len[r]; ++k) {
        const int64_t s = sslot(sp, C, r, k);
        if (col[s] == r) {
            for (int i = 0; i < B * B; ++i) nr += val[s * B * B + i] * val[s * B * B + i];
            for (int i = 0; i < B; ++i) dg[i] = val[s * B * B + i * B + i];
        }
    }
    dnorm[r] = sqrt(nr);
    for (int i = 0; i < B; ++i) invd[r * B + i] = dg[i] != 0.0 ? 1.0 / dg[i] : 0.0;
}

// strong[slot] = |A_ij|_F^2 >= theta^2 |A_ii|_F |A_jj|_F (i != j, A_ij != 0)
template <int B>
__global__ void k_strength(int64_t n, int C, const int32_t* __restrict__ sp, const int32_t* __restrict__ len,
                           const int32_t* __restrict__ col, const double* __restrict__ val,
                           const double* __restrict__ dnorm, double theta, uint8_t* __restrict__ strong,
                           uint8_t* __restrict__ isolated) {
    const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int64_t s0 = r / C;
    const int w = (sp[s0 + 1] - sp[s0]) / C;
    int cnt = 0;
    for (int k = 0; k < w; ++k) {
        const int64_t s = sslot(sp, C, r, k);
        uint8_t st = 0;
        if (k < len[r]) {
            const int64_t c = col[s];
            if (c != r) {
                double a = 0.0;
                for (int i = 0; i < B * B; ++i) a += val[s * B * B + i] * val[s * B * B + i];
                st = (a > 0.0 && a >= theta * theta * dnorm[r] * dnorm[c]) ? 1 : 0;
            }
        }
        strong[s] = st;
        cnt += st;
    }
    isolated[r] = cnt == 0 ? 1 : 0;
}

// ---- MIS(2) aggregation ----------------------------------------------------------------------
// key = state (2 bits: 2 root, 1 undecided, 0 out) | 30-bit hash | 32-bit index
__device__ __forceinline__ uint64_t mis_key(uint32_t state, int64_t i) {
    return (uint64_t(state) << 62) | (uint64_t(hash32(uint32_t(i) * 2654435761u + 97u) & 0x3fffffffu) << 32) |
           uint64_t(uint32_t(i));
}

__global__ void k_mis_init(int64_t n, const uint8_t* __restrict__ isolated, uint8_t* __restrict__ state,
                           uint64_t* __restrict__ key) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint8_t st = isolated[i] ? 0 : 1;
    state[i] = st;
    key[i] = mis_key(st, i);
}

// m = max(m, in[c]) over the strong slots of row r.  Every slot of the row's slice is visited:
// padding slots are never strong and their columns are valid indices, so each chunk's column,
// flag and gathered value are loaded before any test and the gathers are in flight together.
__device__ __forceinline__ uint64_t strong_max(const int32_t* __restrict__ sp, int C, int64_t r,
                                               const int32_t* __restrict__ col, const uint8_t* __restrict__ strong,
                                               const uint64_t* __restrict__ in, uint64_t m) {
    constexpr int U = 4;
    const int64_t s0 = r / C;
    const int64_t base = int64_t(sp[s0]) + (r - s0 * C);
    const int w = (sp[s0 + 1] - sp[s0]) / C;
    int k = 0;
    for (; k + U <= w; k += U) {
        int32_t c[U];
        uint8_t st[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t sl = base + int64_t(k + u) * C;
            c[u] = col[sl];
            st[u] = strong[sl];
        }
        uint64_t v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = in[c[u]];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (st[u]) m = max(m, v[u]);
    }
    for (; k < w; ++k) {
        const int64_t sl = base + int64_t(k) * C;
        const uint64_t v = in[col[sl]];
        if (strong[sl]) m = max(m, v);
    }
    return m;
}

__global__ void k_mis_prop(int64_t n, int C, const int32_t* __restrict__ sp, const int32_t* __restrict__ col,
                           const uint8_t* __restrict__ strong, const uint64_t* __restrict__ in,
                           uint64_t* __restrict__ out) {
    const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= n) return;
    out[r] = strong_max(sp, C, r, col, strong, in, in[r]);
}

// Second hop fused with the state update: m2 = max of m1 over the row and its strong
// neighbours; an undecided row whose own key is that maximum becomes a root, one that sees a
// root within two hops drops out.  (The first hop of the round has finished, and this kernel
// reads only m1, so the rows' key and state can be updated in place.)
__global__ void __launch_bounds__(256) k_mis_prop_update(int64_t n, int C, const int32_t* __restrict__ sp,
                                                         const int32_t* __restrict__ col,
                                                         const uint8_t* __restrict__ strong,
                                                         const uint64_t* __restrict__ m1, uint8_t* __restrict__ state,
                                                         uint64_t* __restrict__ key, int32_t* __restrict__ undecided) {
    __shared__ int sh[4];
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    int und = 0;
    if (i < n && state[i] == 1) {
        const uint64_t m2 = strong_max(sp, C, i, col, strong, m1, m1[i]);
        if (m2 == key[i]) {
            state[i] = 2;
            key[i] = mis_key(2, i);
        } else if ((m2 >> 62) == 2) {
            state[i] = 0;
            key[i] = mis_key(0, i);
        } else {
            und = 1;
        }
    }
    if (!undecided) return;
    // one atomic per block (the count only decides termination)
    und = wave_sum_int(und);
    if (threadIdx.x % kWave == 0) sh[threadIdx.x / kWave] = und;
    __syncthreads();
    if (threadIdx.x == 0) {
        const int t = sh[0] + sh[1] + sh[2] + sh[3];
        if (t) atomicAdd(undecided, t);
    }
}


__global__ void k_root_flags(int64_t n, const uint8_t* __restrict__ state, int32_t* __restrict__ flag) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) flag[i] = state[i] == 2 ? 1 : 0;
}

// phase 1: roots take their rank; neighbours of roots join the adjacent root with the largest key
__global__ void k_agg_phase1(int64_t n, int C, const int32_t* __restrict__ sp, const int32_t* __restrict__ len,
                             const int32_t* __restrict__ col, const uint8_t* __restrict__ strong,
                             const uint8_t* __restrict__ state, const uint64_t* __restrict__ key,
                             const int32_t* __restrict__ rank, int32_t* __restrict__ agg) {
    const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= n) return;
    if (state[r] == 2) { agg[r] = rank[r]; return; }
    uint64_t best = 0;
    int32_t a = -1;
    for (int k = 0; k < len[r]; ++k) {
        const int64_t s = sslot(sp, C, r, k);
        const int32_t c = col[s];
        if (strong[s] && state[c] == 2 && key[c] > best) { best = key[c]; a = rank[c]; }
    }
    agg[r] = a;
}

// phase 2: remaining non-isolated nodes join the phase-1 neighbour with the largest key
__global__ void k_agg_phase2(int64_t n, int C, const int32_t* __restrict__ sp, const int32_t* __restrict__ len,
                             const int32_t* __restrict__ col, const uint8_t* __restrict__ strong,
                             const uint8_t* __restrict__ isolated, const uint64_t* __restrict__ key,
                             const int32_t* __restrict__ agg1, int32_t* __restrict__ agg2) {
    const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= n) return;
    int32_t a = agg1[r];
    if (a < 0 && !isolated[r]) {
        uint64_t best = 0;
        for (int k = 0; k < len[r]; ++k) {
            const int64_t s = sslot(sp, C, r, k);
            const int32_t c = col[s];
            const uint64_t kc = key[c] & 0x3fffffffffffffffull;
            if (strong[s] && agg1[c] >= 0 && kc >= best) { best = kc; a = agg1[c]; }
        }
    }
    agg2[r] = a;
}

__global__ void k_orphan_flags(int64_t n, const uint8_t* __restrict__ isolated, const int32_t* __restrict__ agg,
                               int32_t* __restrict__ flag) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) flag[i] = (agg[i] < 0 && !isolated[i]) ? 1 : 0;
}

__global__ void k_orphan_assign(int64_t n, const int32_t* __restrict__ flag, const int32_t* __restrict__ rank,
                                int32_t base, int32_t* __restrict__ agg) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n && flag[i]) agg[i] = base + rank[i];
}

// Aggregate member lists by a stable sort of the nodes by aggregate (nodes of no aggregate
// take the key n_agg and sort last): each list comes out in increasing node order.
__global__ void k_agg_keys(int64_t n, const int32_t* __restrict__ agg, int64_t n_agg, uint32_t* __restrict__ key,
                           int32_t* __restrict__ node) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    key[i] = uint32_t(agg[i] >= 0 ? agg[i] : n_agg);
    node[i] = int32_t(i);
}

// ---- tentative prolongator ----------------------------------------------------------------
// Near-null-space row (dof c of node i) at level 0 in aggregate-centred coordinates.
template <int BR, int NS>
__device__ __forceinline__ double nullspace0(int c, int j, const double* x, const double* xc) {
    if (NS == 1) return 1.0;
    if (j < BR) return c == j ? 1.0 : 0.0;
    if (BR == 2) {   // rotation about z: (-(y - yc), x - xc)
        return c == 0 ? -(x[1] - xc[1]) : (x[0] - xc[0]);
    }
    // 3d: rot_z (-y, x, 0), rot_x (0, -z, y), rot_y (z, 0, -x), centred
    const double dx = x[0] - xc[0], dy = x[1] - xc[1], dz = x[2] - xc[2];
    if (j == 3) return c == 0 ? -dy : (c == 1 ? dx : 0.0);
    if (j == 4) return c == 0 ? 0.0 : (c == 1 ? -dz : dy);
    return c == 0 ? dz : (c == 1 ? 0.0 : -dx);
}

// One thread per aggregate: QR (classical Gram-Schmidt, twice) of the aggregate's
// near-null-space rows.  Q goes to the tentative prolongator, R (times the change of
// basis back to global coordinates at level 0) is the coarse near-null space.
template <int BR, int NS, bool LEVEL0>
__global__ void k_tentative(int64_t na, const int32_t* __restrict__ aptr, const int32_t* __restrict__ anodes,
                            const double* __restrict__ coords, int dim, const double* __restrict__ Bf,
                            int C, const int32_t* __restrict__ psp, double* __restrict__ pval,
                            double* __restrict__ Bc, double* __restrict__ ainfo) {
    const int64_t a = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (a >= na) return;
    const int32_t b0 = aptr[a], b1 = aptr[a + 1];
    double xc[3] = {0, 0, 0};
    if (LEVEL0 && NS > 1) {
        for (int32_t t = b0; t < b1; ++t)
            for (int k = 0; k < dim; ++k) xc[k] += coords[int64_t(anodes[t]) * dim + k];
        for (int k = 0; k < dim; ++k) xc[k] /= double(b1 - b0);
    }
    // Cholesky QR, twice: G = B^T B = R1^T R1, then the Gram matrix of B R1^-1 gives R2,
    // Q = B (R2 R1)^-1, R = R2 R1.  The aggregate's rows are regenerated on every pass
    // (from the coordinates at level 0), so Q is written once.  A column whose remaining
    // norm falls below 1e-10 of its own norm is dependent and dropped (zero in Q and R).
    auto brow = [&](int64_t node, int c, double* v) {
        for (int j = 0; j < NS; ++j)
            v[j] = LEVEL0 ? nullspace0<BR, NS>(c, j, coords + node * dim, xc) : Bf[(node * BR + c) * NS + j];
    };
    double Ri[NS][NS];   // accumulated R^-1 (upper triangular)
    double Rm[NS][NS];   // accumulated R
    for (int i = 0; i < NS; ++i)
        for (int j = 0; j < NS; ++j) Ri[i][j] = Rm[i][j] = (i == j) ? 1.0 : 0.0;
    bool drop[NS];
    for (int j = 0; j < NS; ++j) drop[j] = false;
    for (int pass = 0; pass < 2; ++pass) {
        double G[NS][NS];
        for (int i = 0; i < NS; ++i)
            for (int j = 0; j < NS; ++j) G[i][j] = 0.0;
        for (int32_t t = b0; t < b1; ++t) {
            const int64_t node = anodes[t];
            for (int c = 0; c < BR; ++c) {
                double v[NS], q[NS];
                brow(node, c, v);
                for (int j = 0; j < NS; ++j) {
                    double s = 0.0;
                    for (int k = 0; k <= j; ++k) s += v[k] * Ri[k][j];
                    q[j] = s;
                }
                for (int i = 0; i < NS; ++i)
                    for (int j = i; j < NS; ++j) G[i][j] += q[i] * q[j];
            }
        }
        // R = chol(G) (upper), dependent columns dropped
        double Rp[NS][NS];
        for (int i = 0; i < NS; ++i)
            for (int j = 0; j < NS; ++j) Rp[i][j] = 0.0;
        for (int j = 0; j < NS; ++j) {
            if (drop[j]) continue;
            double d = G[j][j];
            for (int k = 0; k < j; ++k) d -= Rp[k][j] * Rp[k][j];
            if (!(d > 1e-20 * G[j][j]) || !(G[j][j] > 0.0)) {
                drop[j] = true;
                continue;
            }
            Rp[j][j] = sqrt(d);
            for (int k = j + 1; k < NS; ++k) {
                double s = G[j][k];
                for (int i = 0; i < j; ++i) s -= Rp[i][j] * Rp[i][k];
                Rp[j][k] = s / Rp[j][j];
            }
        }
        // inverse of this pass's factor (dropped rows/columns stay zero)
        double Pi[NS][NS];
        for (int i = 0; i < NS; ++i)
            for (int j = 0; j < NS; ++j) Pi[i][j] = 0.0;
        for (int j = 0; j < NS; ++j) {
            if (drop[j]) continue;
            Pi[j][j] = 1.0 / Rp[j][j];
            for (int i = j - 1; i >= 0; --i) {
                if (drop[i]) continue;
                double s = 0.0;
                for (int k = i + 1; k <= j; ++k) s += Rp[i][k] * Pi[k][j];
                Pi[i][j] = -s / Rp[i][i];
            }
        }
        // Ri <- Ri Pi, Rm <- Rp Rm
        double T1[NS][NS], T2[NS][NS];
        for (int i = 0; i < NS; ++i)
            for (int j = 0; j < NS; ++j) {
                double a1 = 0.0, a2 = 0.0;
                for (int k = 0; k < NS; ++k) {
                    a1 += Ri[i][k] * Pi[k][j];
                    a2 += Rp[i][k] * Rm[k][j];
                }
                T1[i][j] = a1;
                T2[i][j] = a2;
            }
        for (int i = 0; i < NS; ++i)
            for (int j = 0; j < NS; ++j) {
                Ri[i][j] = drop[j] ? 0.0 : T1[i][j];
                Rm[i][j] = drop[i] ? 0.0 : T2[i][j];
            }
    }
    // Q = B R^-1 into the tentative prolongator (one block per node, at its aggregate)
    for (int32_t t = b0; t < b1; ++t) {
        const int64_t node = anodes[t];
        double* q = pval + (int64_t(psp[node / C]) + (node % C)) * (BR * NS);
        for (int c = 0; c < BR; ++c) {
            double v[NS];
            brow(node, c, v);
            for (int j = 0; j < NS; ++j) {
                double s = 0.0;
                for (int k = 0; k < NS; ++k) s += v[k] * Ri[k][j];
                q[c * NS + j] = s;
            }
        }
    }
    // the aggregate's factors of the tentative rows (R^-1 and the centroid), for the matrix-free
    // transfers of the finest 2d displacement level
    if constexpr (LEVEL0 && NS == 3) {
        if (ainfo) {
            double* o = ainfo + a * kAggInfo;
            for (int i = 0; i < NS; ++i)
                for (int j = 0; j < NS; ++j) o[i * NS + j] = Ri[i][j];
            o[9] = xc[0];
            o[10] = xc[1];
        }
    }
    // coarse near-null space: R T (T maps centred to global rotations at level 0)
    double T[NS][NS];
    for (int i = 0; i < NS; ++i)
        for (int j = 0; j < NS; ++j) T[i][j] = i == j ? 1.0 : 0.0;
    if constexpr (LEVEL0 && NS == 3) {
        T[0][2] = -xc[1];
        T[1][2] = xc[0];
    } else if constexpr (LEVEL0 && NS == 6) {
        T[0][3] = -xc[1]; T[1][3] = xc[0];
        T[1][4] = -xc[2]; T[2][4] = xc[1];
        T[0][5] = xc[2];  T[2][5] = -xc[0];
    }
    for (int i = 0; i < NS; ++i)
        for (int j = 0; j < NS; ++j) {
            double v = 0.0;
            for (int k = 0; k < NS; ++k) v += Rm[i][k] * T[k][j];
            Bc[(a * NS + i) * NS + j] = v;
        }
}

__global__ void k_ptent_struct(int64_t n, const int32_t* __restrict__ agg, int32_t* __restrict__ len) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) len[i] = agg[i] >= 0 ? 1 : 0;
}

__global__ void k_ptent_cols(int64_t n, int C, const int32_t* __restrict__ sp, const int32_t* __restrict__ agg,
                             int32_t* __restrict__ col, double* __restrict__ val, int bb) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t s0 = i / C;
    const int w = (sp[s0 + 1] - sp[s0]) / C;
    for (int k = 0; k < w; ++k) {
        const int64_t s = sslot(sp, C, i, k);
        col[s] = (k == 0 && agg[i] >= 0) ? agg[i] : 0;
        for (int e = 0; e < bb; ++e) val[s * bb + e] = 0.0;
    }
}

// ---- SpGEMM ----------------------------------------------------------------------------------
struct SellV {
    int C;
    int64_t n_rows;
    const int32_t* sp;
    const int32_t* len;
    const int32_t* col;
};

SellV sv(const SellStruct& S) { return SellV{S.C, S.n_rows, S.slice_ptr, S.row_len, S.col}; }

// Hashed SpGEMM symbolic phase.  A group of G lanes (G in {8,16,32,64}) owns one output
// row and an LDS hash set of HS slots (16 G, or 64 G for the rows that overflow that); a
// wave holds 64/G rows.  The set of columns is deterministic, the order of the table is not,
// so the fill kernel ranks the entries.
template <int HS>
__device__ __forceinline__ bool hash_insert(int32_t* tab, int32_t c, int& cnt) {
    uint32_t h = hash32(uint32_t(c)) & (HS - 1);
    for (int probe = 0; probe < HS; ++probe) {
        const int32_t old = atomicCAS(&tab[h], -1, c);
        if (old == -1) { cnt++; return true; }
        if (old == c) return true;
        h = (h + 1) & (HS - 1);
    }
    return false;
}

template <int G>
__device__ __forceinline__ int group_sum(int v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// LDS visibility among the lanes of one wave (each wave works on its own LDS slice)
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Builds the hash set of the columns of row r of A*B in this group's LDS table.
template <int G, int HS>
__device__ void spgemm_row_set(const SellV& A, const SellV& B, int64_t r, int32_t* tab, int lg, int& added,
                               int* overflow) {
    for (int i = lg; i < HS; i += G) tab[i] = -1;
    wave_sync();
    if (r < A.n_rows) {
        const int la = A.len[r];
        bool full = false;
        // each lane takes two of A's entries per round (ka and ka + G) and loads the first U of
        // B's columns of both rows before any insert, so the dependent loads (A's column, B's
        // row start, B's columns) of both are in flight together
        constexpr int U = 8;
        for (int ka = lg; ka < la && !full; ka += 2 * G) {
            const bool two = ka + G < la;
            const int64_t k0 = A.col[sslot(A.sp, A.C, r, ka)];
            const int64_t k1 = two ? A.col[sslot(A.sp, A.C, r, ka + G)] : k0;
            const int lb0 = B.len[k0];
            const int lb1 = two ? B.len[k1] : 0;
            const int64_t b00 = sslot(B.sp, B.C, k0, 0);
            const int64_t b01 = sslot(B.sp, B.C, k1, 0);
            int32_t c0[U], c1[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                c0[u] = u < lb0 ? B.col[b00 + int64_t(u) * B.C] : -1;
                c1[u] = u < lb1 ? B.col[b01 + int64_t(u) * B.C] : -1;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (c0[u] >= 0 && !full && !hash_insert<HS>(tab, c0[u], added)) full = true;
                if (c1[u] >= 0 && !full && !hash_insert<HS>(tab, c1[u], added)) full = true;
            }
            // the rest of long rows of B, U columns at a time
            for (int h = 0; h < 2 && !full; ++h) {
                const int lb = h ? lb1 : lb0;
                const int64_t b0 = h ? b01 : b00;
                for (int kb = U; kb < lb && !full; kb += U) {
                    int32_t c[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) c[u] = kb + u < lb ? B.col[b0 + int64_t(kb + u) * B.C] : -1;
#pragma unroll
                    for (int u = 0; u < U; ++u)
                        if (c[u] >= 0 && !full && !hash_insert<HS>(tab, c[u], added)) full = true;
                }
            }
        }
        if (full) atomicOr(overflow, 1);
    }
    wave_sync();
}

// With `stage` (HS * 3 / 4 slots per row, the most a row may hold before it overflows), the
// row's columns are also written there, unordered, so that the fill needs no second pass over
// A and B (k_spgemm_place).
template <int G, int HS>
__global__ void __launch_bounds__(256) k_spgemm_count(SellV A, SellV B, int32_t* __restrict__ clen,
                                                      int* __restrict__ overflow, int32_t* __restrict__ stage) {
    constexpr int RPW = kWave / G, SW = (HS * 3) / 4;
    __shared__ int32_t tab[kWavesPerBlock][RPW * HS];
    __shared__ int32_t nl[kWavesPerBlock][RPW];
    const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave, gi = lane / G, lg = lane % G;
    const int64_t r = (int64_t(blockIdx.x) * kWavesPerBlock + w) * RPW + gi;
    int added = 0;
    if (lg == 0) nl[w][gi] = 0;
    int32_t* mytab = &tab[w][gi * HS];
    spgemm_row_set<G, HS>(A, B, r, mytab, lg, added, overflow);
    const int tot = group_sum<G>(added);
    if (r < A.n_rows && lg == 0) {
        clen[r] = tot;
        if (tot > SW) atomicOr(overflow, 1);
    }
    if (stage && r < A.n_rows && tot <= SW) {
        for (int i = lg; i < HS; i += G) {
            const int32_t v = mytab[i];
            if (v >= 0) stage[r * SW + atomicAdd(&nl[w][gi], 1)] = v;
        }
    }
}

// The fill from the staged columns: each row's columns ranked (the set is the count's; the
// staged order is not, the ranks are), padding repeats the smallest.  G lanes per row, the
// row's list copied to LDS for the ranking.
template <int G, int HS>
__global__ void __launch_bounds__(256) k_spgemm_place(SellV Cm, const int32_t* __restrict__ stage,
                                                      int32_t* __restrict__ ccol) {
    constexpr int RPW = kWave / G, SW = (HS * 3) / 4;
    __shared__ int32_t lst[kWavesPerBlock][RPW * SW];
    const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave, gi = lane / G, lg = lane % G;
    const int64_t r = (int64_t(blockIdx.x) * kWavesPerBlock + w) * RPW + gi;
    int32_t* mylst = &lst[w][gi * SW];
    const int n = r < Cm.n_rows ? Cm.len[r] : 0;
    for (int i = lg; i < n; i += G) mylst[i] = stage[r * SW + i];
    wave_sync();
    if (r >= Cm.n_rows) return;
    const int64_t s0 = r / Cm.C;
    const int width = (Cm.sp[s0 + 1] - Cm.sp[s0]) / Cm.C;
    int32_t first = -1;
    for (int i = lg; i < n; i += G) {
        const int32_t v = mylst[i];
        int rk = 0;
        for (int j = 0; j < n; ++j) rk += mylst[j] < v;
        ccol[sslot(Cm.sp, Cm.C, r, rk)] = v;
        if (rk == 0) first = v;
    }
    int32_t f = first;
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) f = max(f, __shfl_xor(f, o));
    if (f < 0) f = 0;
    for (int k = n + lg; k < width; k += G) ccol[sslot(Cm.sp, Cm.C, r, k)] = f;
}

template <int G, int HS>
__global__ void __launch_bounds__(256) k_spgemm_fill(SellV A, SellV B, SellV Cm, int32_t* __restrict__ ccol,
                                                     int* __restrict__ overflow) {
    constexpr int RPW = kWave / G;
    __shared__ int32_t tab[kWavesPerBlock][RPW * HS];
    __shared__ int32_t lst[kWavesPerBlock][RPW * HS];
    __shared__ int32_t nl[kWavesPerBlock][RPW];
    const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave, gi = lane / G, lg = lane % G;
    const int64_t r = (int64_t(blockIdx.x) * kWavesPerBlock + w) * RPW + gi;
    int32_t* mytab = &tab[w][gi * HS];
    int32_t* mylst = &lst[w][gi * HS];
    int added = 0;
    if (lg == 0) nl[w][gi] = 0;
    spgemm_row_set<G, HS>(A, B, r, mytab, lg, added, overflow);
    for (int i = lg; i < HS; i += G) {
        const int32_t v = mytab[i];
        if (v >= 0) mylst[atomicAdd(&nl[w][gi], 1)] = v;
    }
    wave_sync();
    if (r >= A.n_rows) return;
    const int n = nl[w][gi];
    const int64_t s0 = r / Cm.C;
    const int width = (Cm.sp[s0 + 1] - Cm.sp[s0]) / Cm.C;
    int32_t first = -1;
    for (int i = lg; i < n; i += G) {
        const int32_t v = mylst[i];
        int rk = 0;
        for (int j = 0; j < n; ++j) rk += mylst[j] < v;
        ccol[sslot(Cm.sp, Cm.C, r, rk)] = v;
        if (rk == 0) first = v;
    }
    // padding slots repeat the first column
    int32_t f = first;
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) f = max(f, __shfl_xor(f, o));
    if (f < 0) f = 0;
    for (int k = n + lg; k < width; k += G) ccol[sslot(Cm.sp, Cm.C, r, k)] = f;
}

// Symbolic phase for few, long rows over few columns (coarse levels): a workgroup per output
// row marks the reached columns in an LDS bitmap (bitwise or, so the set does not depend on
// the order of the marks), then counts them, or writes them in increasing order from
// per-thread chunks of words placed by a prefix sum over the threads.  Padding slots repeat
// the smallest column, as in the hashed kernels.
template <bool FILL>
__global__ void __launch_bounds__(256) k_spgemm_bitmap(SellV A, SellV B, SellV Cm, int32_t* __restrict__ clen,
                                                       int32_t* __restrict__ ccol, int n_words) {
    extern __shared__ uint32_t bits[];
    __shared__ int32_t part[256];
    __shared__ int32_t first_sh[256];
    const int64_t r = blockIdx.x;
    const int t = threadIdx.x, nt = blockDim.x;
    for (int i = t; i < n_words; i += nt) bits[i] = 0u;
    __syncthreads();
    const int la = A.len[r];
    for (int ka = 0; ka < la; ++ka) {
        const int64_t k = A.col[sslot(A.sp, A.C, r, ka)];
        const int lb = B.len[k];
        for (int kb = t; kb < lb; kb += nt) {
            const int32_t c = B.col[sslot(B.sp, B.C, k, kb)];
            atomicOr(&bits[c >> 5], 1u << (c & 31));
        }
    }
    __syncthreads();
    const int per = (n_words + nt - 1) / nt;
    const int w0 = min(n_words, t * per), w1 = min(n_words, w0 + per);
    int cnt = 0, first = 0x7fffffff;
    for (int w = w0; w < w1; ++w) {
        const uint32_t m = bits[w];
        if (m && first == 0x7fffffff) first = w * 32 + __builtin_ctz(m);
        cnt += __builtin_popcount(m);
    }
    part[t] = cnt;
    first_sh[t] = first;
    __syncthreads();
    // inclusive scan of the counts and minimum of the first columns (Hillis-Steele)
    for (int o = 1; o < nt; o <<= 1) {
        const int a = t >= o ? part[t - o] : 0;
        const int f = t >= o ? first_sh[t - o] : 0x7fffffff;
        __syncthreads();
        part[t] += a;
        first_sh[t] = min(first_sh[t], f);
        __syncthreads();
    }
    const int total = part[nt - 1];
    if (!FILL) {
        if (t == 0) clen[r] = total;
        return;
    }
    int pos = part[t] - cnt;
    for (int w = w0; w < w1; ++w) {
        uint32_t m = bits[w];
        while (m) {
            ccol[sslot(Cm.sp, Cm.C, r, pos++)] = w * 32 + __builtin_ctz(m);
            m &= m - 1u;
        }
    }
    const int32_t f = total > 0 ? first_sh[nt - 1] : 0;
    const int64_t s0 = r / Cm.C;
    const int width = (Cm.sp[s0 + 1] - Cm.sp[s0]) / Cm.C;
    for (int k = total + t; k < width; k += nt) ccol[sslot(Cm.sp, Cm.C, r, k)] = f;
}

// Where the one block of each row of B sits (bslot, -1 for an empty row) and its column
// (bcol, -1): the one-block-per-row products then reach B's block in one step from A's column.
__global__ void k_single_index(SellV B, int64_t* __restrict__ bslot, int32_t* __restrict__ bcol) {
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= B.n_rows) return;
    const bool has = B.len[k] > 0;
    const int64_t bs = has ? sslot(B.sp, B.C, k, 0) : -1;
    bslot[k] = bs;
    bcol[k] = has ? B.col[bs] : -1;
}

// Symbolic phase of A B when every row of B has at most one block (a tentative prolongator):
// the columns of row r are the distinct B columns of the rows A's row r touches (bcol[k]: the
// column of B's row k, -1 when the row is empty).  G lanes
// per row (G >= the longest row of A), lane g takes entry g; the group sorts its values by a
// bitonic network over lanes, marks the first of each run of equal values and places it by a
// prefix count: row lengths to clen, the sorted columns to stage (G slots per row), which
// k_single_place moves into C's layout once the layout is known.
template <int G>
__global__ void __launch_bounds__(256) k_spgemm_single(SellV A, const int32_t* __restrict__ bcol, SellV Cm,
                                                       int32_t* __restrict__ clen, int32_t* __restrict__ stage) {
    constexpr int RPW = kWave / G;
    constexpr int32_t kNone = 0x7fffffff;
    const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave, gi = lane / G, lg = lane % G;
    const int64_t r = (int64_t(blockIdx.x) * kWavesPerBlock + w) * RPW + gi;
    const bool row_ok = r < A.n_rows;
    const int la = row_ok ? A.len[r] : 0;
    int32_t v = kNone;
    if (lg < la) {
        const int32_t c = bcol[A.col[sslot(A.sp, A.C, r, lg)]];
        if (c >= 0) v = c;
    }
    // ascending bitonic sort of the group's G values
#pragma unroll
    for (int k = 2; k <= G; k <<= 1)
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            const int32_t o = __shfl_xor(v, j);
            const bool up = (lg & k) == 0, lower = (lg & j) == 0;
            v = (lower == up) ? min(v, o) : max(v, o);
        }
    const int32_t prev = __shfl_up(v, 1);
    const int first = (v != kNone && (lg == 0 || prev != v)) ? 1 : 0;
    // inclusive prefix count of the run heads within the group
    int pos = first;
#pragma unroll
    for (int o = 1; o < G; o <<= 1) {
        const int t = __shfl_up(pos, o);
        if (lg >= o) pos += t;
    }
    const int count = __shfl(pos, lane - lg + G - 1);
    if (!row_ok) return;
    if (lg == 0) clen[r] = count;
    if (first) stage[r * G + pos - 1] = v;
}

// Moves the sorted columns staged by k_spgemm_single (G per row) into C's layout; padding
// repeats the smallest column (0 in an empty row).
__global__ void k_single_place(SellV Cm, int G, const int32_t* __restrict__ stage, int32_t* __restrict__ ccol) {
    const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= Cm.n_rows) return;
    const int n = Cm.len[r];
    const int64_t s0 = r / Cm.C;
    const int width = (Cm.sp[s0 + 1] - Cm.sp[s0]) / Cm.C;
    const int32_t f = n > 0 ? stage[r * G] : 0;
    for (int k = 0; k < width; ++k) ccol[sslot(Cm.sp, Cm.C, r, k)] = k < n ? stage[r * G + k] : f;
}

__device__ __forceinline__ int find_sorted(const SellV& B, int64_t row, int32_t c) {
    int lo = 0, hi = B.len[row] - 1;
    while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        const int32_t v = B.col[sslot(B.sp, B.C, row, mid)];
        if (v == c) return mid;
        if (v < c) lo = mid + 1;
        else hi = mid - 1;
    }
    return -1;
}

// C = A B (MODE 0) or C = B - omega D^-1 A B with B indexed by A's rows (MODE 1, smoothing),
// one output block per lane (G lanes per row), each summing over A's row with a binary search
// in B's rows: for output rows too long for LDS over many columns.
template <int BRA, int BCA, int BCB, int MODE, int G>
__global__ void __launch_bounds__(256) k_spgemm_numeric(SellV A, const double* __restrict__ av, SellV B,
                                                        const double* __restrict__ bv, SellV Cm,
                                                        double* __restrict__ cv, const double* __restrict__ invd,
                                                        double omega) {
    constexpr int RPW = kWave / G;
    const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave, gi = lane / G, lg = lane % G;
    const int64_t r = (int64_t(blockIdx.x) * kWavesPerBlock + w) * RPW + gi;
    if (r >= Cm.n_rows) return;
    const int lc = Cm.len[r];
    const int64_t s0 = r / Cm.C;
    const int width = (Cm.sp[s0 + 1] - Cm.sp[s0]) / Cm.C;
    const int la = A.len[r];
    for (int kc = lg; kc < width; kc += G) {
        const int64_t cs = sslot(Cm.sp, Cm.C, r, kc);
        double acc[BRA][BCB];
        for (int i = 0; i < BRA; ++i)
            for (int j = 0; j < BCB; ++j) acc[i][j] = 0.0;
        if (kc < lc) {
            const int32_t c = Cm.col[cs];
            for (int ka = 0; ka < la; ++ka) {
                const int64_t as = sslot(A.sp, A.C, r, ka);
                const int64_t k = A.col[as];
                const int kb = find_sorted(B, k, c);
                if (kb < 0) continue;
                const double* ab = av + as * (BRA * BCA);
                const double* bb = bv + sslot(B.sp, B.C, k, kb) * (BCA * BCB);
                for (int i = 0; i < BRA; ++i)
                    for (int t = 0; t < BCA; ++t) {
                        const double x = ab[i * BCA + t];
                        for (int j = 0; j < BCB; ++j) acc[i][j] += x * bb[t * BCB + j];
                    }
            }
            if (MODE == 1) {
                const int kb = find_sorted(B, r, c);
                for (int i = 0; i < BRA; ++i) {
                    const double dsc = omega * invd[r * BRA + i];
                    for (int j = 0; j < BCB; ++j) {
                        const double own = kb >= 0 ? bv[sslot(B.sp, B.C, r, kb) * (BCA * BCB) + i * BCB + j] : 0.0;
                        acc[i][j] = own - dsc * acc[i][j];
                    }
                }
            }
        }
        for (int i = 0; i < BRA; ++i)
            for (int j = 0; j < BCB; ++j) cv[cs * (BRA * BCB) + i * BCB + j] = acc[i][j];
    }
}

// ---- transpose -------------------------------------------------------------------------------
// Values of R = P^T into an existing structure (G lanes per row of R, over its entries):
// entry (r, c) of R is entry (c, r) of P, found by binary search in P's sorted row c.
template <int BR, int BC, int G>
__global__ void __launch_bounds__(256) k_transpose_values(SellV P, const double* __restrict__ pv, SellV Rm,
                                                          double* __restrict__ rv) {
    const int64_t r = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / G;
    const int lg = threadIdx.x % G;
    if (r >= Rm.n_rows) return;
    const int n = Rm.len[r];
    const int64_t s0 = r / Rm.C;
    const int width = (Rm.sp[s0 + 1] - Rm.sp[s0]) / Rm.C;
    for (int k = lg; k < width; k += G) {
        const int64_t rs = sslot(Rm.sp, Rm.C, r, k);
        const int kp = k < n ? find_sorted(P, Rm.col[rs], int32_t(r)) : -1;
        const double* pb = kp >= 0 ? pv + sslot(P.sp, P.C, Rm.col[rs], kp) * (BR * BC) : nullptr;
        for (int i = 0; i < BR; ++i)
            for (int j = 0; j < BC; ++j) rv[rs * (BR * BC) + j * BR + i] = pb ? pb[i * BC + j] : 0.0;
    }
}

// Transpose by a stable sort of P's entries by column: the entries listed in row order (key:
// the column; value: the row in the high word, the slot in the low word), sorted, are R's
// entries row by row with the columns (P's rows) ascending, so they are placed without
// atomics and without a per-row ranking.
__global__ void k_tr_entries(SellV P, const int32_t* __restrict__ roff, uint32_t* __restrict__ key,
                             uint64_t* __restrict__ ent) {
    const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= P.n_rows) return;
    const int n = P.len[r];
    const int64_t b = roff[r];
    for (int k = 0; k < n; ++k) {
        const int64_t ps = sslot(P.sp, P.C, r, k);
        key[b + k] = uint32_t(P.col[ps]);
        ent[b + k] = (uint64_t(uint32_t(r)) << 32) | uint64_t(uint32_t(ps));
    }
}

// Lower bounds in sorted keys: start[a] = the first position whose key is >= a, and len[a]
// (when asked for) the number of keys equal to a.  Row a of R holds the sorted entries
// [start[a], start[a] + len[a]).
__global__ void k_tr_bounds(const uint32_t* __restrict__ key, int64_t nnz, int64_t n_rows, int32_t* __restrict__ start,
                            int32_t* __restrict__ len) {
    const int64_t a = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (a >= n_rows) return;
    auto lower = [&](uint32_t v) {
        int64_t lo = 0, hi = nnz;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (key[mid] < v) lo = mid + 1;
            else hi = mid;
        }
        return lo;
    };
    const int64_t b = lower(uint32_t(a)), e = lower(uint32_t(a) + 1u);
    start[a] = int32_t(b);
    if (len) len[a] = int32_t(e - b);
}

template <int BR, int BC>
__global__ void k_tr_place(const uint32_t* __restrict__ key, const uint64_t* __restrict__ ent, int64_t nnz,
                           const int32_t* __restrict__ start, const double* __restrict__ pv, SellV Rm,
                           int32_t* __restrict__ rcol, double* __restrict__ rv) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= nnz) return;
    const int64_t a = key[t];
    const uint64_t e = ent[t];
    const int64_t ps = int64_t(uint32_t(e));
    const int64_t rs = sslot(Rm.sp, Rm.C, a, int(t - start[a]));
    rcol[rs] = int32_t(e >> 32);
    for (int i = 0; i < BR; ++i)
        for (int j = 0; j < BC; ++j) rv[rs * (BR * BC) + j * BR + i] = pv[ps * (BR * BC) + i * BC + j];
}

// padding slots of R's rows repeat the row's smallest column (0 in an empty row) with zero blocks
__global__ void k_tr_pad(const uint64_t* __restrict__ ent, const int32_t* __restrict__ start, SellV Rm,
                         int32_t* __restrict__ rcol, double* __restrict__ rv, int bb) {
    const int64_t a = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (a >= Rm.n_rows) return;
    const int n = Rm.len[a];
    const int64_t s0 = a / Rm.C;
    const int width = (Rm.sp[s0 + 1] - Rm.sp[s0]) / Rm.C;
    const int32_t f = n > 0 ? int32_t(ent[start[a]] >> 32) : 0;
    for (int k = n; k < width; ++k) {
        const int64_t rs = sslot(Rm.sp, Rm.C, a, k);
        rcol[rs] = f;
        for (int b = 0; b < bb; ++b) rv[rs * bb + b] = 0.0;
    }
}

// ---- power iteration for lambda_max(D^-1 A) ------------------------------------------------
__global__ void k_power_init(int64_t n, double* __restrict__ x) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) x[i] = 0.5 + double(hash32(uint32_t(i) ^ 0x9e3779b9u) & 0xffffu) / 65536.0;
}


// ---- dense coarsest level ------------------------------------------------------------------
template <int B>
__global__ void k_to_dense(SellV A, const double* __restrict__ av, int64_t n, double* __restrict__ dense) {
    const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= A.n_rows) return;
    for (int k = 0; k < A.len[r]; ++k) {
        const int64_t s = sslot(A.sp, A.C, r, k);
        const int64_t c = A.col[s];
        for (int i = 0; i < B; ++i)
            for (int j = 0; j < B; ++j) dense[(r * B + i) * n + c * B + j] += av[s * B * B + i * B + j];
    }
}

// rows and columns that are entirely zero (rank-deficient coarse DoFs) get a unit diagonal
__global__ void k_fix_zero_rows(int64_t n, double* __restrict__ dense) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double m = 0.0;
    for (int64_t j = 0; j < n; ++j) m = fmax(m, fabs(dense[i * n + j]));
    if (m == 0.0) dense[i * n + i] = 1.0;
}

// In-place Gauss-Jordan inversion of a symmetric positive (semi)definite matrix without
// pivoting, one workgroup, matrix in global memory (L2 resident for the sizes used here).
// Waves walk rows, lanes walk columns, so every pass is coalesced; the pivot row and
// column are staged in LDS.
__global__ void __launch_bounds__(1024) k_gauss_jordan(int64_t n, double* __restrict__ a) {
    __shared__ double rowk[kDenseMax];
    __shared__ double colk[kDenseMax];
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave, nw = blockDim.x / kWave;
    for (int64_t k = 0; k < n; ++k) {
        const double p = a[k * n + k];
        const double ip = p != 0.0 ? 1.0 / p : 0.0;
        for (int64_t j = threadIdx.x; j < n; j += blockDim.x) {
            rowk[j] = (j == k) ? ip : a[k * n + j] * ip;
            colk[j] = a[j * n + k];
        }
        __syncthreads();
        for (int64_t i = wave; i < n; i += nw) {
            if (i == k) {
                for (int64_t j = lane; j < n; j += kWave) a[i * n + j] = rowk[j];
                continue;
            }
            const double f = colk[i];
            if (f == 0.0) continue;
            for (int64_t j = lane; j < n; j += kWave) {
                if (j == k) a[i * n + j] = -f * ip;
                else a[i * n + j] -= f * rowk[j];
            }
        }
        __syncthreads();
    }
}

// x = Ainv b (dense, FP64 arithmetic; vectors in T)
template <typename T>
__global__ void __launch_bounds__(256) k_dense_gemv(int64_t n, const double* __restrict__ ainv, const T* __restrict__ b,
                                                    T* __restrict__ x) {
    __shared__ double sh[16];
    const int64_t i = blockIdx.x;
    double acc = 0.0;
    for (int64_t j = threadIdx.x; j < n; j += blockDim.x) acc += ainv[i * n + j] * double(b[j]);
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) x[i] = T(s);
}

// ---- host-side helpers ---------------------------------------------------------------------

std::shared_ptr<SellStruct> new_struct(int64_t n_rows, int64_t n_cols, hipStream_t s) {
    auto S = std::make_shared<SellStruct>();
    S->C = kWave;
    S->n_rows = n_rows;
    S->n_cols = n_cols;
    S->own_len.alloc(size_t(std::max<int64_t>(1, n_rows)), s);
    S->row_len = S->own_len.p;
    return S;
}

void finish_struct(SellStruct& S, hipStream_t s, const int* flag = nullptr, int* flag_out = nullptr) {
    layout_from_lengths(S, s, flag, flag_out);
    S.own_col.alloc(size_t(std::max<int64_t>(1, S.n_slots)), s);
    S.col = S.own_col.p;
}

// Row-merge numeric phase: a group of G lanes owns one output row; the row's sorted columns
// and its accumulator blocks sit in LDS.  For every entry A_ik (in column order) the lanes
// walk row k of B, find each column's position in the output row by binary search in LDS
// and add A_ik B_kc there; within one A entry the columns are distinct, so no two lanes
// touch the same accumulator, and the summation order is fixed.
template <int BRA, int BCA, int BCB, int MODE, int G>
__global__ void __launch_bounds__(256) k_spgemm_merge(SellV A, const double* __restrict__ av, SellV B,
                                                      const double* __restrict__ bv, SellV Cm, double* __restrict__ cv,
                                                      const double* __restrict__ invd, double omega, int LC) {
    extern __shared__ double smem[];
    constexpr int RPW = kWave / G, BB = BRA * BCB;
    const int RPB = int(blockDim.x / kWave) * RPW;
    const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave, gi = lane / G, lg = lane % G;
    const int slot_in_block = w * RPW + gi;
    double* acc = smem + size_t(slot_in_block) * LC * BB;
    int32_t* cols = reinterpret_cast<int32_t*>(smem + size_t(RPB) * LC * BB) + slot_in_block * LC;
    const int64_t r = int64_t(blockIdx.x) * RPB + slot_in_block;
    if (r >= Cm.n_rows) return;
    const int lc = Cm.len[r];
    for (int k = lg; k < lc; k += G) {
        cols[k] = Cm.col[sslot(Cm.sp, Cm.C, r, k)];
        for (int e = 0; e < BB; ++e) acc[k * BB + e] = 0.0;
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const int la = A.len[r];
    const int base = lane - lg;   // the group's first lane in the wave
    for (int j0 = 0; j0 < la; j0 += G) {
        // lane lg loads A's entry j0 + lg (its block, and where row k of B starts and how long
        // it is), so the loads of up to G entries are in flight together; the group then takes
        // the entries in column order from the lane that holds each
        const int ja = j0 + lg;
        double abj[BRA * BCA];
        int32_t lbj = 0, b0lo = 0, b0hi = 0;
        for (int e = 0; e < BRA * BCA; ++e) abj[e] = 0.0;
        if (ja < la) {
            const int64_t as = sslot(A.sp, A.C, r, ja);
            const int64_t k = A.col[as];
            for (int e = 0; e < BRA * BCA; ++e) abj[e] = av[as * (BRA * BCA) + e];
            lbj = B.len[k];
            const int64_t b0 = sslot(B.sp, B.C, k, 0);
            b0lo = int32_t(uint32_t(uint64_t(b0)));
            b0hi = int32_t(uint32_t(uint64_t(b0) >> 32));
        }
        const int nj = min(G, la - j0);
        for (int tj = 0; tj < nj; ++tj) {
            const int src = base + tj;
            const int lb = __shfl(lbj, src, kWave);
            const int64_t b0 = int64_t((uint64_t(uint32_t(__shfl(b0hi, src, kWave))) << 32) |
                                       uint64_t(uint32_t(__shfl(b0lo, src, kWave))));
            double ab[BRA * BCA];
            for (int e = 0; e < BRA * BCA; ++e) ab[e] = __shfl(abj[e], src, kWave);
            for (int kb = lg; kb < lb; kb += G) {
                const int64_t bs = b0 + int64_t(kb) * B.C;
                const int32_t c = B.col[bs];
                // B's block is loaded with its column, before the search, so the two loads
                // are in flight together (the output row holds every column of the product)
                double bb[BCA * BCB];
                for (int e = 0; e < BCA * BCB; ++e) bb[e] = bv[bs * (BCA * BCB) + e];
                int lo = 0, hi = lc - 1, p = -1;
                while (lo <= hi) {
                    const int mid = (lo + hi) >> 1;
                    const int32_t v = cols[mid];
                    if (v == c) { p = mid; break; }
                    if (v < c) lo = mid + 1;
                    else hi = mid - 1;
                }
                if (p < 0) continue;
                for (int i = 0; i < BRA; ++i)
                    for (int j = 0; j < BCB; ++j) {
                        double t = 0.0;
                        for (int q = 0; q < BCA; ++q) t += ab[i * BCA + q] * bb[q * BCB + j];
                        acc[p * BB + i * BCB + j] += t;
                    }
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
    }
    const int64_t s0 = r / Cm.C;
    const int width = (Cm.sp[s0 + 1] - Cm.sp[s0]) / Cm.C;
    for (int kc = lg; kc < width; kc += G) {
        const int64_t cs = sslot(Cm.sp, Cm.C, r, kc);
        if (kc < lc) {
            if (MODE == 1) {
                const int kb = find_sorted(B, r, cols[kc]);
                for (int i = 0; i < BRA; ++i) {
                    const double dsc = omega * invd[r * BRA + i];
                    for (int j = 0; j < BCB; ++j) {
                        const double own = kb >= 0 ? bv[sslot(B.sp, B.C, r, kb) * (BCA * BCB) + i * BCB + j] : 0.0;
                        cv[cs * BB + i * BCB + j] = own - dsc * acc[kc * BB + i * BCB + j];
                    }
                }
            } else {
                for (int e = 0; e < BB; ++e) cv[cs * BB + e] = acc[kc * BB + e];
            }
        } else {
            for (int e = 0; e < BB; ++e) cv[cs * BB + e] = 0.0;
        }
    }
}

__device__ __forceinline__ double read_lane(double x, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), l);
    return __hiloint2double(hi, lo);
}

// Numeric phase when every row of B has at most one block (B a tentative prolongator): entry
// A_rk lands in column B.col[k] only.  G lanes own a row; lane j loads A's entry j of the
// current chunk of G and forms its product block with row k_j of B; then every output column
// (one per lane) adds, in A's column order, the products that land on it, read from the
// owning lanes (readlane for a whole wave, shuffles within smaller groups).  Every group
// walks the same number of chunks (the wave's longest row), so the shuffles of a group
// always read lanes of that group in the same step.
template <int G>
__device__ __forceinline__ double group_read(double x, int base, int t) {
    if constexpr (G == kWave) return read_lane(x, t);
    else return __shfl(x, base + t, kWave);
}
template <int G>
__device__ __forceinline__ int32_t group_read(int32_t x, int base, int t) {
    if constexpr (G == kWave) return __builtin_amdgcn_readlane(x, t);
    else return __shfl(x, base + t, kWave);
}

template <int BRA, int BCA, int BCB, int MODE, int G>
__global__ void __launch_bounds__(256) k_spgemm_numeric_single(SellV A, const double* __restrict__ av,
                                                               const int64_t* __restrict__ bslot,
                                                               const int32_t* __restrict__ bcol,
                                                               const double* __restrict__ bv, SellV Cm,
                                                               double* __restrict__ cv,
                                                               const double* __restrict__ invd, double omega) {
    constexpr int BB = BRA * BCB, RPW = kWave / G;
    const int wl = threadIdx.x % kWave, lane = wl % G, base = wl - lane;
    const int64_t r = (int64_t(blockIdx.x) * kWavesPerBlock + threadIdx.x / kWave) * RPW + wl / G;
    const bool live = r < Cm.n_rows;
    const int la = live ? A.len[r] : 0, lc = live ? Cm.len[r] : 0;
    const int64_t s0 = live ? r / Cm.C : 0;
    const int width = live ? (Cm.sp[s0 + 1] - Cm.sp[s0]) / Cm.C : 0;
    // loop bounds shared by the whole wave
    int la_w = la, width_w = width;
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        la_w = max(la_w, __shfl_xor(la_w, o, kWave));
        width_w = max(width_w, __shfl_xor(width_w, o, kWave));
    }
    for (int kc0 = 0; kc0 < width_w; kc0 += G) {
        const int kc = kc0 + lane;
        const int64_t cs = kc < width ? sslot(Cm.sp, Cm.C, r, kc) : 0;
        const int32_t c = kc < lc ? Cm.col[cs] : -1;
        double acc[BB];
#pragma unroll
        for (int e = 0; e < BB; ++e) acc[e] = 0.0;
        for (int j0 = 0; j0 < la_w; j0 += G) {
            const int j = j0 + lane;
            int32_t cj = -1;
            double pj[BB];
#pragma unroll
            for (int e = 0; e < BB; ++e) pj[e] = 0.0;
            if (j < la) {
                const int64_t as = sslot(A.sp, A.C, r, j);
                const int64_t k = A.col[as];
                const int64_t bs = bslot[k];
                if (bs >= 0) {
                    cj = bcol[k];
                    const double* ab = av + as * (BRA * BCA);
                    const double* bb = bv + bs * (BCA * BCB);
#pragma unroll
                    for (int i = 0; i < BRA; ++i)
#pragma unroll
                        for (int jj = 0; jj < BCB; ++jj) {
                            double x = 0.0;
#pragma unroll
                            for (int q = 0; q < BCA; ++q) x += ab[i * BCA + q] * bb[q * BCB + jj];
                            pj[i * BCB + jj] = x;
                        }
                }
            }
            const int nj = min(G, la_w - j0);
            for (int t = 0; t < nj; ++t) {
                const int32_t ct = group_read<G>(cj, base, t);
                double pt[BB];
#pragma unroll
                for (int e = 0; e < BB; ++e) pt[e] = group_read<G>(pj[e], base, t);
                if (ct == c) {
#pragma unroll
                    for (int e = 0; e < BB; ++e) acc[e] += pt[e];
                }
            }
        }
        if (live && kc < width) {
            if (kc < lc) {
                if (MODE == 1) {
                    double ob[BB];
#pragma unroll
                    for (int e = 0; e < BB; ++e) ob[e] = 0.0;
                    const int64_t os = bslot[r];
                    if (os >= 0) {
                        if (bcol[r] == c) {
#pragma unroll
                            for (int e = 0; e < BB; ++e) ob[e] = bv[os * BB + e];
                        }
                    }
#pragma unroll
                    for (int i = 0; i < BRA; ++i) {
                        const double dsc = omega * invd[r * BRA + i];
#pragma unroll
                        for (int jj = 0; jj < BCB; ++jj)
                            cv[cs * BB + i * BCB + jj] = ob[i * BCB + jj] - dsc * acc[i * BCB + jj];
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < BB; ++e) cv[cs * BB + e] = acc[e];
                }
            } else {
#pragma unroll
                for (int e = 0; e < BB; ++e) cv[cs * BB + e] = 0.0;
            }
        }
    }
}

// Dense-row numeric phase for few, long output rows (coarse levels, where C has few block
// columns): a workgroup owns one output row and accumulates it over all of C's columns in
// LDS.  For every entry A_ik in turn the lanes walk row k of B (distinct columns, so no two
// lanes add to one accumulator) and a barrier separates the entries, so the summation order
// of every output block is A's column order, as in the row-merge kernel.
// Columns are taken in windows [c0, c0 + n_cols) of what fits in LDS, one launch per window
// (only the first window writes the padding slots); the order of the additions into every
// output block is the same for any window size.
template <int BRA, int BCA, int BCB, int MODE>
__global__ void __launch_bounds__(256) k_spgemm_dense_row(SellV A, const double* __restrict__ av, SellV B,
                                                          const double* __restrict__ bv, SellV Cm,
                                                          double* __restrict__ cv, const double* __restrict__ invd,
                                                          double omega, int c0, int n_cols) {
    extern __shared__ double acc[];
    constexpr int BB = BRA * BCB;
    const int64_t r = blockIdx.x;
    const int t = threadIdx.x, nt = blockDim.x;
    for (int i = t; i < n_cols * BB; i += nt) acc[i] = 0.0;
    __syncthreads();
    const int la = A.len[r];
    for (int ka = 0; ka < la; ++ka) {
        const int64_t as = sslot(A.sp, A.C, r, ka);
        const int64_t k = A.col[as];
        double ab[BRA * BCA];
        for (int e = 0; e < BRA * BCA; ++e) ab[e] = av[as * (BRA * BCA) + e];
        const int lb = B.len[k];
        for (int kb = t; kb < lb; kb += nt) {
            const int64_t bs = sslot(B.sp, B.C, k, kb);
            const int32_t c = B.col[bs] - c0;
            if (c < 0 || c >= n_cols) continue;
            const double* bb = bv + bs * (BCA * BCB);
            for (int i = 0; i < BRA; ++i)
                for (int j = 0; j < BCB; ++j) {
                    double x = 0.0;
                    for (int q = 0; q < BCA; ++q) x += ab[i * BCA + q] * bb[q * BCB + j];
                    acc[c * BB + i * BCB + j] += x;
                }
        }
        __syncthreads();
    }
    const int lc = Cm.len[r];
    const int64_t s0 = r / Cm.C;
    const int width = (Cm.sp[s0 + 1] - Cm.sp[s0]) / Cm.C;
    for (int kc = t; kc < width; kc += nt) {
        const int64_t cs = sslot(Cm.sp, Cm.C, r, kc);
        if (kc < lc) {
            const int32_t cg = Cm.col[cs], c = cg - c0;
            if (c < 0 || c >= n_cols) continue;
            if (MODE == 1) {
                const int kb = find_sorted(B, r, cg);
                for (int i = 0; i < BRA; ++i) {
                    const double dsc = omega * invd[r * BRA + i];
                    for (int j = 0; j < BCB; ++j) {
                        const double own = kb >= 0 ? bv[sslot(B.sp, B.C, r, kb) * (BCA * BCB) + i * BCB + j] : 0.0;
                        cv[cs * BB + i * BCB + j] = own - dsc * acc[c * BB + i * BCB + j];
                    }
                }
            } else {
                for (int e = 0; e < BB; ++e) cv[cs * BB + e] = acc[c * BB + e];
            }
        } else if (c0 == 0) {
            for (int e = 0; e < BB; ++e) cv[cs * BB + e] = 0.0;
        }
    }
}

static void single_index(const BMat<double>& B, DBuf<int64_t>& bslot, DBuf<int32_t>& bcol, hipStream_t s) {
    const int64_t nb = B.rows();
    bslot.alloc(size_t(std::max<int64_t>(1, nb)), s);
    bcol.alloc(size_t(std::max<int64_t>(1, nb)), s);
    if (nb == 0) return;
    k_single_index<<<nblk(nb, 256), 256, 0, s>>>(sv(*B.S), bslot.p, bcol.p);
    FR_LAUNCH_CHECK();
}

template <int BRA, int BCA, int BCB, int MODE>
void spgemm_numeric(const BMat<double>& A, const BMat<double>& B, BMat<double>& Cm, const double* invd, double omega,
                    hipStream_t s) {
    const int ml = Cm.S->max_len;
    const int64_t rows = std::max<int64_t>(1, A.rows());
    // B with one block per row (tentative prolongators): products handed to the output
    // columns within lane groups; otherwise a dense LDS row for few columns and long B rows,
    // the LDS row merge (8, 16 or 64 lanes per row) while the output rows fit, and beyond
    // that the dense row over a few column windows or one output block per lane
    if (B.S->max_len <= 1) {
        // B with one block per row: G lanes per row by A's mean row length (a wave for the
        // long 3d / coarse rows, 16 or 8 lanes for 2d rows)
        const int64_t avg_a = A.S->nnz / std::max<int64_t>(1, rows);
        DBuf<int64_t> bslot;
        DBuf<int32_t> bcol;
        single_index(B, bslot, bcol, s);
#define FR_NSINGLE(G_)                                                                                 \
    k_spgemm_numeric_single<BRA, BCA, BCB, MODE, G_><<<nblk(rows, kWavesPerBlock * (kWave / G_)), 256, 0, s>>>( \
        sv(*A.S), A.val, bslot.p, bcol.p, B.val, sv(*Cm.S), Cm.val, invd, omega);
        if (avg_a >= 16) { FR_NSINGLE(64) }
        else if (avg_a > 8) { FR_NSINGLE(16) }
        else { FR_NSINGLE(8) }
#undef FR_NSINGLE
        FR_LAUNCH_CHECK();
        return;
    } else {
        constexpr int BB = BRA * BCB;
        constexpr size_t kLds = 64 * 1024;
        // few long rows over few columns (coarse levels): a workgroup per row, dense in LDS
        const int64_t nc = Cm.cols();
        const int64_t avg_b = B.S->nnz / std::max<int64_t>(1, B.rows());
        if (size_t(nc) * BB * sizeof(double) <= kLds && avg_b >= 64 && A.rows() > 0) {
            k_spgemm_dense_row<BRA, BCA, BCB, MODE><<<int(A.rows()), 256, size_t(nc) * BB * sizeof(double), s>>>(
                sv(*A.S), A.val, sv(*B.S), B.val, sv(*Cm.S), Cm.val, invd, omega, 0, int(nc));
            FR_LAUNCH_CHECK();
            return;
        }
        // LDS slots per output row (a stride only: the merge walks each row's own length): the
        // longest row rounded up to a power of two, or, for the 8-lane merge, to a multiple of
        // four where that lets more workgroups share a CU's 160 KiB of LDS (the finest
        // displacement A P: 2.95 -> 2.39 ms; where occupancy is not gained the tighter stride
        // measured slower)
        int LC = 8;
        while (LC < ml) LC <<= 1;
        const size_t per_row = size_t(LC) * (BB * sizeof(double) + sizeof(int32_t));
        constexpr int RPB8 = kWavesPerBlock * (kWave / 8);
        const int LC8t = std::max(8, (ml + 3) & ~3);
        const size_t per_row8t = size_t(LC8t) * (BB * sizeof(double) + sizeof(int32_t));
        auto per_cu = [](size_t block_bytes) {
            return block_bytes > kLds ? size_t(0) : std::min<size_t>(8, size_t(160 * 1024) / block_bytes);
        };
        const bool tight8 = per_cu(RPB8 * per_row8t) > per_cu(RPB8 * per_row);
        const int LC8 = tight8 ? LC8t : LC;
        const size_t per_row8 = tight8 ? per_row8t : per_row;
        if (avg_b <= 8 && ml <= 128 && RPB8 * per_row8 <= kLds) {
            // short rows of B (smoothed prolongators): 8 lanes per row, 32 rows per block
            k_spgemm_merge<BRA, BCA, BCB, MODE, 8><<<nblk(rows, RPB8), 256, RPB8 * per_row8, s>>>(
                sv(*A.S), A.val, sv(*B.S), B.val, sv(*Cm.S), Cm.val, invd, omega, LC8);
            FR_LAUNCH_CHECK();
            return;
        }
        constexpr int RPB16 = kWavesPerBlock * (kWave / 16);
        if (ml <= 256 && RPB16 * per_row <= kLds) {
            // 16 lanes per row, 16 rows per block
            k_spgemm_merge<BRA, BCA, BCB, MODE, 16><<<nblk(rows, RPB16), 256, RPB16 * per_row, s>>>(
                sv(*A.S), A.val, sv(*B.S), B.val, sv(*Cm.S), Cm.val, invd, omega, LC);
            FR_LAUNCH_CHECK();
            return;
        }
        if (per_row <= kLds) {
            // a wave per row: four rows per block when they fit, else one
            const int wpb = kWavesPerBlock * per_row <= kLds ? kWavesPerBlock : 1;
            k_spgemm_merge<BRA, BCA, BCB, MODE, kWave><<<nblk(rows, wpb), wpb * kWave, wpb * per_row, s>>>(
                sv(*A.S), A.val, sv(*B.S), B.val, sv(*Cm.S), Cm.val, invd, omega, LC);
            FR_LAUNCH_CHECK();
            return;
        }
    }
    {
        // output rows too long for the LDS merge: the dense-row kernel over a few column
        // windows, else one output block per lane
        constexpr int BB = BRA * BCB;
        const int64_t win = int64_t(48 * 1024) / (BB * int64_t(sizeof(double)));
        const int64_t nc = Cm.cols();
        if (A.rows() > 0 && ceil_div(nc, win) <= 8) {
            for (int64_t c0 = 0; c0 < nc; c0 += win) {
                const int w = int(std::min<int64_t>(win, nc - c0));
                k_spgemm_dense_row<BRA, BCA, BCB, MODE><<<int(A.rows()), 256, size_t(w) * BB * sizeof(double), s>>>(
                    sv(*A.S), A.val, sv(*B.S), B.val, sv(*Cm.S), Cm.val, invd, omega, int(c0), w);
                FR_LAUNCH_CHECK();
            }
            return;
        }
    }
#define FR_NUM_G(G_)                                                                                          \
    k_spgemm_numeric<BRA, BCA, BCB, MODE, G_><<<nblk(rows, kWavesPerBlock * (kWave / G_)), 256, 0, s>>>(      \
        sv(*A.S), A.val, sv(*B.S), B.val, sv(*Cm.S), Cm.val, invd, omega);
    if (ml <= 8) { FR_NUM_G(8) }
    else if (ml <= 16) { FR_NUM_G(16) }
    else if (ml <= 32) { FR_NUM_G(32) }
    else { FR_NUM_G(64) }
#undef FR_NUM_G
    FR_LAUNCH_CHECK();
}

#define FR_SPGEMM_CASE(BRA_, BCA_, BCB_)                                        \
    if (A.br == BRA_ && A.bc == BCA_ && B.bc == BCB_) {                         \
        spgemm_numeric<BRA_, BCA_, BCB_, MODE>(A, B, Cm, invd, omega, s);       \
        return;                                                                 \
    }

// Values of C = A B (MODE 0) or C = B - omega D^-1 A B (MODE 1) into C's existing structure.
template <int MODE>
void spgemm_values(const BMat<double>& A, const BMat<double>& B, BMat<double>& Cm, const double* invd, double omega,
                   hipStream_t s) {
    if (A.bc != B.br || A.cols() != B.rows() || Cm.rows() != A.rows() || Cm.br != A.br || Cm.bc != B.bc)
        fail(FR_EINTERNAL, "spgemm: shape mismatch");
    FR_SPGEMM_CASE(1, 1, 1)
    FR_SPGEMM_CASE(2, 2, 3)
    FR_SPGEMM_CASE(3, 2, 3)
    FR_SPGEMM_CASE(3, 3, 3)
    FR_SPGEMM_CASE(3, 3, 6)
    FR_SPGEMM_CASE(6, 3, 6)
    FR_SPGEMM_CASE(6, 6, 6)
    fail(FR_EINTERNAL, "spgemm: unsupported block shapes");
}
#undef FR_SPGEMM_CASE

template <int G, int HS>
void spgemm_symbolic(const BMat<double>& A, const BMat<double>& B, BMat<double>& Cm, int* ovf, hipStream_t s,
                     bool fill, int32_t* stage = nullptr) {
    const int g = nblk(std::max<int64_t>(1, A.rows()), kWavesPerBlock * (kWave / G));
    if (!fill) k_spgemm_count<G, HS><<<g, 256, 0, s>>>(sv(*A.S), sv(*B.S), Cm.S->row_len, ovf, stage);
    else if (stage) k_spgemm_place<G, HS><<<g, 256, 0, s>>>(sv(*Cm.S), stage, Cm.S->col);
    else k_spgemm_fill<G, HS><<<g, 256, 0, s>>>(sv(*A.S), sv(*B.S), sv(*Cm.S), Cm.S->col, ovf);
    FR_LAUNCH_CHECK();
}

// `errs` collects overflow flags that are checked once at the end of the setup
template <int MODE>
BMat<double> spgemm(const BMat<double>& A, const BMat<double>& B, const double* invd, double omega, int* errs,
                    hipStream_t s) {
    if (A.bc != B.br || A.cols() != B.rows()) fail(FR_EINTERNAL, "spgemm: shape mismatch");
    BMat<double> Cm;
    Cm.br = A.br;
    Cm.bc = B.bc;
    Cm.S = new_struct(A.rows(), B.cols(), s);
    DBuf<int> ovf;
    ovf.alloc(1, s);
    ovf.zero(s);
    if (B.S->max_len <= 1 && A.S->max_len <= kWave) {
        // B has one block per row: columns by lane ranking, no hash sets
        DBuf<int64_t> bslot;
        DBuf<int32_t> bcol;
        single_index(B, bslot, bcol, s);
        int G = 8;
        while (G < A.S->max_len) G <<= 1;
        const int g = nblk(std::max<int64_t>(1, A.rows()), kWavesPerBlock * (kWave / G));
        // one pass: row lengths, and each row's sorted columns staged at G per row
        DBuf<int32_t> stage;
        stage.alloc(size_t(std::max<int64_t>(1, A.rows())) * G, s);
#define FR_SINGLE(G_) k_spgemm_single<G_><<<g, 256, 0, s>>>(sv(*A.S), bcol.p, sv(*Cm.S), Cm.S->row_len, stage.p);
        switch (G) {
            case 8: FR_SINGLE(8) break;
            case 16: FR_SINGLE(16) break;
            case 32: FR_SINGLE(32) break;
            default: FR_SINGLE(64) break;
        }
#undef FR_SINGLE
        FR_LAUNCH_CHECK();
        finish_struct(*Cm.S, s);
        if (A.rows() > 0) {
            k_single_place<<<nblk(A.rows(), 256), 256, 0, s>>>(sv(*Cm.S), G, stage.p, Cm.S->col);
            FR_LAUNCH_CHECK();
        }
        Cm.own_val.alloc(size_t(std::max<int64_t>(1, Cm.S->n_slots)) * Cm.br * Cm.bc, s);
        Cm.val = Cm.own_val.p;
        spgemm_values<MODE>(A, B, Cm, invd, omega, s);
        return Cm;
    }
    const int64_t avg_b = B.S->nnz / std::max<int64_t>(1, B.rows());
    const int n_words = int(ceil_div(std::max<int64_t>(1, B.cols()), 32));
    auto bitmap_product = [&]() {
        // a workgroup per row with a column bitmap over all of C's columns
        const int g = int(A.rows());
        const size_t lds = size_t(n_words) * sizeof(uint32_t);
        k_spgemm_bitmap<false><<<g, 256, lds, s>>>(sv(*A.S), sv(*B.S), sv(*Cm.S), Cm.S->row_len, nullptr, n_words);
        FR_LAUNCH_CHECK();
        finish_struct(*Cm.S, s);
        k_spgemm_bitmap<true><<<g, 256, lds, s>>>(sv(*A.S), sv(*B.S), sv(*Cm.S), nullptr, Cm.S->col, n_words);
        FR_LAUNCH_CHECK();
        Cm.own_val.alloc(size_t(std::max<int64_t>(1, Cm.S->n_slots)) * Cm.br * Cm.bc, s);
        Cm.val = Cm.own_val.p;
        spgemm_values<MODE>(A, B, Cm, invd, omega, s);
    };
    if (avg_b >= 64 && n_words <= 8192 && A.rows() > 0) {
        // long rows of B over few columns
        bitmap_product();
        return Cm;
    }
    // small hash sets first (8 rows per wave: 32 slots for the short rows of the finest level's
    // A P, else 128); when a row does not fit, all rows rerun with the next size (128 slots, a
    // wave per row with 1024 slots, then 4096 slots)
    int over = 0;
    int tier = 0;
    // the counting pass stages each row's columns (3/4 of the tier's slots per row) when that
    // takes at most 1 GiB; the fill then only ranks them
    DBuf<int32_t> stage;
    int32_t* st = nullptr;
    auto stage_for = [&](int hs) {
        const size_t need = size_t(std::max<int64_t>(1, A.rows())) * size_t(hs * 3 / 4);
        st = nullptr;
        if (need * sizeof(int32_t) > (size_t(1) << 30)) return;
        stage.alloc(need, s);
        st = stage.p;
    };
    const bool short_rows = int64_t(A.S->max_len) * B.S->max_len <= 96;
    if (short_rows) {
        tier = -1;
        stage_for(32);
        spgemm_symbolic<8, 32>(A, B, Cm, ovf.p, s, false, st);
        layout_from_lengths(*Cm.S, s, ovf.p, &over);
    }
    if (!short_rows || over) {
        tier = 0;
        ovf.zero(s);
        stage_for(128);
        spgemm_symbolic<8, 128>(A, B, Cm, ovf.p, s, false, st);
        layout_from_lengths(*Cm.S, s, ovf.p, &over);
    }
    if (over) {
        tier = 1;
        ovf.zero(s);
        stage_for(1024);
        spgemm_symbolic<64, 1024>(A, B, Cm, ovf.p, s, false, st);
        layout_from_lengths(*Cm.S, s, ovf.p, &over);
    }
    if (over) {
        tier = 2;
        ovf.zero(s);
        stage_for(4096);
        spgemm_symbolic<64, 4096>(A, B, Cm, ovf.p, s, false, st);
        layout_from_lengths(*Cm.S, s, ovf.p, &over);
        if (over) {
            // rows beyond the largest hash set: the column bitmap, when C's columns fit in LDS
            if (n_words > 8192) fail(FR_EINTERNAL, "spgemm: a row of the product has more than 3072 block columns");
            bitmap_product();
            return Cm;
        }
    }
    Cm.S->own_col.alloc(size_t(std::max<int64_t>(1, Cm.S->n_slots)), s);
    Cm.S->col = Cm.S->own_col.p;
    if (tier == -1) spgemm_symbolic<8, 32>(A, B, Cm, errs, s, true, st);
    else if (tier == 0) spgemm_symbolic<8, 128>(A, B, Cm, errs, s, true, st);
    else if (tier == 1) spgemm_symbolic<64, 1024>(A, B, Cm, errs, s, true, st);
    else spgemm_symbolic<64, 4096>(A, B, Cm, errs, s, true, st);
    Cm.own_val.alloc(size_t(std::max<int64_t>(1, Cm.S->n_slots)) * Cm.br * Cm.bc, s);
    Cm.val = Cm.own_val.p;
    spgemm_values<MODE>(A, B, Cm, invd, omega, s);
    return Cm;
}

void transpose_values(const BMat<double>& P, BMat<double>& Rm, hipStream_t s) {
    if (Rm.rows() != P.cols() || Rm.cols() != P.rows() || Rm.br != P.bc || Rm.bc != P.br)
        fail(FR_EINTERNAL, "transpose: shape mismatch");
    // lanes per row of R from its mean length (coarse levels have few, long rows)
    const int64_t avg = Rm.S->nnz / std::max<int64_t>(1, Rm.rows());
    const int G = avg >= 48 ? 64 : (avg >= 6 ? 8 : 1);
    const int g = nblk(std::max<int64_t>(1, Rm.rows()) * G, 256);
#define FR_TV_G(BR_, BC_, G_) k_transpose_values<BR_, BC_, G_><<<g, 256, 0, s>>>(sv(*P.S), P.val, sv(*Rm.S), Rm.val);
#define FR_TV_CASE(BR_, BC_)                                                                  \
    if (P.br == BR_ && P.bc == BC_) {                                                         \
        if (G == 64) { FR_TV_G(BR_, BC_, 64) }                                                \
        else if (G == 8) { FR_TV_G(BR_, BC_, 8) }                                             \
        else { FR_TV_G(BR_, BC_, 1) }                                                         \
        FR_LAUNCH_CHECK();                                                                    \
        return;                                                                               \
    }
    FR_TV_CASE(1, 1)
    FR_TV_CASE(2, 3)
    FR_TV_CASE(3, 3)
    FR_TV_CASE(3, 6)
    FR_TV_CASE(6, 6)
#undef FR_TV_CASE
#undef FR_TV_G
    fail(FR_EINTERNAL, "transpose: unsupported block shape");
}

BMat<double> transpose(const BMat<double>& P, hipStream_t s) {
    const SellStruct& PS = *P.S;
    if (PS.n_rows >= (int64_t(1) << 31) || PS.n_slots >= (int64_t(1) << 31) || PS.nnz >= (int64_t(1) << 31))
        fail(FR_EINTERNAL, "transpose: more than 2^31 rows, slots or entries");
    BMat<double> Rm;
    Rm.br = P.bc;
    Rm.bc = P.br;
    Rm.S = new_struct(P.cols(), P.rows(), s);
    const int64_t nnz = PS.nnz, nr = P.cols();
    const size_t ne = size_t(std::max<int64_t>(1, nnz));
    DBuf<int32_t> roff, start;
    DBuf<uint32_t> key[2];
    DBuf<uint64_t> ent[2];
    roff.alloc(size_t(P.rows()) + 1, s);
    scan_exclusive_async(PS.row_len, roff.p, P.rows(), s);
    for (int i = 0; i < 2; ++i) {
        key[i].alloc(ne, s);
        ent[i].alloc(ne, s);
    }
    if (P.rows() > 0) {
        k_tr_entries<<<nblk(P.rows(), 256), 256, 0, s>>>(sv(PS), roff.p, key[0].p, ent[0].p);
        FR_LAUNCH_CHECK();
    }
    // keys below the number of R's rows: only their bits are sorted
    int bits = 1;
    while (bits < 32 && (int64_t(1) << bits) < nr) ++bits;
    size_t tmp_bytes = 0;
    FR_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, key[0].p, key[1].p, ent[0].p, ent[1].p, int(nnz), 0,
                                             bits, s));
    DBuf<char> tmp;
    tmp.alloc(std::max<size_t>(1, tmp_bytes), s);
    if (nnz > 0)
        FR_HIP(hipcub::DeviceRadixSort::SortPairs(tmp.p, tmp_bytes, key[0].p, key[1].p, ent[0].p, ent[1].p, int(nnz), 0,
                                                 bits, s));
    start.alloc(size_t(std::max<int64_t>(1, nr)), s);
    if (nr > 0) {
        k_tr_bounds<<<nblk(nr, 256), 256, 0, s>>>(key[1].p, nnz, nr, start.p, Rm.S->row_len);
        FR_LAUNCH_CHECK();
    }
    finish_struct(*Rm.S, s);
    const size_t nvals = size_t(std::max<int64_t>(1, Rm.S->n_slots)) * Rm.br * Rm.bc;
    Rm.own_val.alloc(nvals, s);
    Rm.val = Rm.own_val.p;
#define FR_TR_CASE(BR_, BC_)                                                                                     \
    if (P.br == BR_ && P.bc == BC_) {                                                                            \
        if (nnz > 0) {                                                                                           \
            k_tr_place<BR_, BC_><<<nblk(nnz, 256), 256, 0, s>>>(key[1].p, ent[1].p, nnz, start.p, P.val, sv(*Rm.S), \
                                                                Rm.S->col, Rm.val);                              \
            FR_LAUNCH_CHECK();                                                                                   \
        }                                                                                                        \
        if (nr > 0) {                                                                                            \
            k_tr_pad<<<nblk(nr, 256), 256, 0, s>>>(ent[1].p, start.p, sv(*Rm.S), Rm.S->col, Rm.val, BR_ * BC_);  \
            FR_LAUNCH_CHECK();                                                                                   \
        }                                                                                                        \
        return Rm;                                                                                               \
    }
    FR_TR_CASE(1, 1)
    FR_TR_CASE(2, 3)
    FR_TR_CASE(3, 3)
    FR_TR_CASE(3, 6)
    FR_TR_CASE(6, 6)
#undef FR_TR_CASE
    fail(FR_EINTERNAL, "transpose: unsupported block shape");
}

// Largest eigenvalue of D^-1 A by ten power steps from a fixed positive start vector.  The
// iterates are not normalised between steps (D^-1 A has eigenvalues of order one, so ten
// steps stay far inside the double range); the estimate is |x_10| / |x_9|.  power_start
// enqueues the steps on a stream and power_finish waits for the estimate, so that other work
// can run in between (the buffers live in the PowerEst until then).  With `mf` the steps apply
// the fine level's block matrix-free (the same operator up to rounding, fewer bytes).
struct PowerEst {
    DBuf<double> v[2], scr, nrm;
    int64_t n = 0;
    hipStream_t st = nullptr;
};

void power_start(PowerEst& pe, const BMat<double>& A, const double* invd, hipStream_t s, const MfState* mf = nullptr,
                 int blk = 0) {
    const int64_t n = A.rows() * A.br;
    pe.n = n;
    pe.st = s;
    if (n == 0) return;
    pe.v[0].alloc(size_t(n), s);
    pe.v[1].alloc(size_t(n), s);
    pe.scr.alloc(1024, s);
    pe.nrm.alloc(2, s);
    k_power_init<<<nblk(n, 256), 256, 0, s>>>(n, pe.v[0].p);
    FR_LAUNCH_CHECK();
    const int iters = 10;
    for (int it = 0; it < iters; ++it) {
        if (mf) mf_power_step(*mf, blk, invd, pe.v[it & 1].p, pe.v[(it + 1) & 1].p, s);
        else diag_scaled_matvec(A, invd, pe.v[it & 1].p, pe.v[(it + 1) & 1].p, s);
    }
    dev_dot(pe.v[iters & 1].p, pe.v[iters & 1].p, n, pe.nrm.p, pe.scr, s);
    dev_dot(pe.v[(iters - 1) & 1].p, pe.v[(iters - 1) & 1].p, n, pe.nrm.p + 1, pe.scr, s);
}

double power_finish(PowerEst& pe) {
    if (pe.n == 0) return 1.0;
    const auto h = download(pe.nrm.p, 2, pe.st);
    const double lam = h[1] > 0 ? std::sqrt(h[0] / h[1]) : 0.0;
    return lam > 0 && std::isfinite(lam) ? lam : 1.0;
}

double lambda_max(const BMat<double>& A, const double* invd, hipStream_t s, const MfState* mf = nullptr,
                  int blk = 0) {
    PowerEst pe;
    power_start(pe, A, invd, s, mf, blk);
    return power_finish(pe);
}

}  // namespace

// ---- setup ----------------------------------------------------------------------------------

static void diag_info(const BMat<double>& A, DBuf<double>& invd, DBuf<double>& dnorm, hipStream_t s) {
    const SellStruct& S = *A.S;
    invd.alloc(size_t(std::max<int64_t>(1, S.n_rows * A.br)), s);
    dnorm.alloc(size_t(std::max<int64_t>(1, S.n_rows)), s);
    const int g = nblk(S.n_rows, 256);
    switch (A.br) {
        case 1: k_diag<1><<<g, 256, 0, s>>>(S.n_rows, S.C, S.slice_ptr, S.row_len, S.col, A.val, invd.p, dnorm.p); break;
        case 2: k_diag<2><<<g, 256, 0, s>>>(S.n_rows, S.C, S.slice_ptr, S.row_len, S.col, A.val, invd.p, dnorm.p); break;
        case 3: k_diag<3><<<g, 256, 0, s>>>(S.n_rows, S.C, S.slice_ptr, S.row_len, S.col, A.val, invd.p, dnorm.p); break;
        case 6: k_diag<6><<<g, 256, 0, s>>>(S.n_rows, S.C, S.slice_ptr, S.row_len, S.col, A.val, invd.p, dnorm.p); break;
        default: fail(FR_EINTERNAL, "diag: unsupported block size");
    }
    FR_LAUNCH_CHECK();
}

// Aggregation of the block rows of A; returns the number of aggregates, agg[n] (-1 = none).
// `before_wait` (may be empty) is called once, after the first round is enqueued and before
// the host first waits for the stream: work the caller enqueues there overlaps the rounds.
static int64_t aggregate(const BMat<double>& A, const double* dnorm, double theta, DBuf<int32_t>& agg, hipStream_t s,
                         const std::function<void()>& before_wait = {}) {
    const SellStruct& S = *A.S;
    const int64_t n = S.n_rows;
    const int g = nblk(n, 256);
    DBuf<uint8_t> strong, isolated, state;
    DBuf<uint64_t> key, m1;
    strong.alloc(size_t(std::max<int64_t>(1, S.n_slots)), s);
    isolated.alloc(size_t(n), s);
    state.alloc(size_t(n), s);
    key.alloc(size_t(n), s);
    m1.alloc(size_t(n), s);
    switch (A.br) {
        case 1: k_strength<1><<<g, 256, 0, s>>>(n, S.C, S.slice_ptr, S.row_len, S.col, A.val, dnorm, theta, strong.p, isolated.p); break;
        case 2: k_strength<2><<<g, 256, 0, s>>>(n, S.C, S.slice_ptr, S.row_len, S.col, A.val, dnorm, theta, strong.p, isolated.p); break;
        case 3: k_strength<3><<<g, 256, 0, s>>>(n, S.C, S.slice_ptr, S.row_len, S.col, A.val, dnorm, theta, strong.p, isolated.p); break;
        case 6: k_strength<6><<<g, 256, 0, s>>>(n, S.C, S.slice_ptr, S.row_len, S.col, A.val, dnorm, theta, strong.p, isolated.p); break;
        default: fail(FR_EINTERNAL, "strength: unsupported block size");
    }
    FR_LAUNCH_CHECK();
    k_mis_init<<<g, 256, 0, s>>>(n, isolated.p, state.p, key.p);
    FR_LAUNCH_CHECK();
    DBuf<int32_t> und;
    und.alloc(1, s);
    // rounds once decided are no-ops: large levels check termination every round (a round
    // costs more than the host round trip), small ones every third round
    const int every = n >= (int64_t(1) << 18) ? 1 : 3;
    for (int round = 0; round < 240; ++round) {
        k_mis_prop<<<g, 256, 0, s>>>(n, S.C, S.slice_ptr, S.col, strong.p, key.p, m1.p);
        const bool check = round % every == every - 1;
        if (check) und.zero(s);
        k_mis_prop_update<<<g, 256, 0, s>>>(n, S.C, S.slice_ptr, S.col, strong.p, m1.p, state.p, key.p,
                                             check ? und.p : nullptr);
        FR_LAUNCH_CHECK();
        if (check && before_wait && round + 1 == every) before_wait();
        if (check && download1(und.p, s) == 0) break;
        if (round == 239) fail(FR_EINTERNAL, "aggregation: MIS(2) did not terminate");
    }
    DBuf<int32_t> flag, rank, agg1;
    flag.alloc(size_t(n), s);
    rank.alloc(size_t(n) + 1, s);
    agg1.alloc(size_t(n), s);
    agg.alloc(size_t(n), s);
    k_root_flags<<<g, 256, 0, s>>>(n, state.p, flag.p);
    FR_LAUNCH_CHECK();
    int64_t n_agg = scan_exclusive(flag.p, rank.p, n, s);
    k_agg_phase1<<<g, 256, 0, s>>>(n, S.C, S.slice_ptr, S.row_len, S.col, strong.p, state.p, key.p, rank.p, agg1.p);
    FR_LAUNCH_CHECK();
    k_agg_phase2<<<g, 256, 0, s>>>(n, S.C, S.slice_ptr, S.row_len, S.col, strong.p, isolated.p, key.p, agg1.p, agg.p);
    FR_LAUNCH_CHECK();
    k_orphan_flags<<<g, 256, 0, s>>>(n, isolated.p, agg.p, flag.p);
    FR_LAUNCH_CHECK();
    const int64_t n_orph = scan_exclusive(flag.p, rank.p, n, s);
    if (n_orph > 0) {
        k_orphan_assign<<<g, 256, 0, s>>>(n, flag.p, rank.p, int32_t(n_agg), agg.p);
        FR_LAUNCH_CHECK();
        n_agg += n_orph;
    }
    return n_agg;
}

// Tentative prolongator (one block per aggregated row) and the coarse near-null space.
static BMat<double> tentative(const BMat<double>& A, const DBuf<int32_t>& agg, int64_t n_agg, int ns, bool level0,
                              const double* coords, int dim, const double* Bf, DBuf<double>& Bc, hipStream_t s,
                              AggTransfer* keep = nullptr) {
    const int64_t n = A.rows();
    const int br = A.br;
    BMat<double> P;
    P.br = br;
    P.bc = ns;
    P.S = new_struct(n, n_agg, s);
    k_ptent_struct<<<nblk(n, 256), 256, 0, s>>>(n, agg.p, P.S->row_len);
    FR_LAUNCH_CHECK();
    finish_struct(*P.S, s);
    P.own_val.alloc(size_t(std::max<int64_t>(1, P.S->n_slots)) * br * ns, s);
    P.val = P.own_val.p;
    k_ptent_cols<<<nblk(n, 256), 256, 0, s>>>(n, P.S->C, P.S->slice_ptr, agg.p, P.S->col, P.val, br * ns);
    FR_LAUNCH_CHECK();
    // aggregate member lists: nodes[ptr[a] .. ptr[a + 1]) are aggregate a's, ascending
    if (n >= (int64_t(1) << 31)) fail(FR_EINTERNAL, "tentative: more than 2^31 rows");
    DBuf<int32_t> ptr, nodes, node_in;
    DBuf<uint32_t> key[2];
    const size_t nn = size_t(std::max<int64_t>(1, n));
    ptr.alloc(size_t(n_agg) + 1, s);
    nodes.alloc(nn, s);
    node_in.alloc(nn, s);
    key[0].alloc(nn, s);
    key[1].alloc(nn, s);
    if (n > 0) {
        k_agg_keys<<<nblk(n, 256), 256, 0, s>>>(n, agg.p, n_agg, key[0].p, node_in.p);
        FR_LAUNCH_CHECK();
    }
    int bits = 1;
    while (bits < 32 && (int64_t(1) << bits) <= n_agg) ++bits;
    size_t tmp_bytes = 0;
    FR_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, key[0].p, key[1].p, node_in.p, nodes.p, int(n), 0,
                                             bits, s));
    DBuf<char> tmp;
    tmp.alloc(std::max<size_t>(1, tmp_bytes), s);
    if (n > 0)
        FR_HIP(hipcub::DeviceRadixSort::SortPairs(tmp.p, tmp_bytes, key[0].p, key[1].p, node_in.p, nodes.p, int(n), 0,
                                                 bits, s));
    k_tr_bounds<<<nblk(n_agg + 1, 256), 256, 0, s>>>(key[1].p, n, n_agg + 1, ptr.p, nullptr);
    FR_LAUNCH_CHECK();
    Bc.alloc(size_t(std::max<int64_t>(1, n_agg)) * ns * ns, s);
    double* ainfo = nullptr;
    if (keep) {
        keep->n_agg = n_agg;
        keep->info.alloc(size_t(std::max<int64_t>(1, n_agg)) * kAggInfo, s);
        ainfo = keep->info.p;
    }
    const int g = nblk(n_agg, 64);
    const int C = P.S->C;
    // level 0 builds the near-null space from coordinates; coarser levels read the R
    // factors of the level above, which must exist
    if (!level0 && Bf == nullptr) fail(FR_EINTERNAL, "tentative: coarse level without a near-null space");
    if (level0 && br == 2 && ns == 3)
        k_tentative<2, 3, true><<<g, 64, 0, s>>>(n_agg, ptr.p, nodes.p, coords, dim, Bf, C, P.S->slice_ptr, P.val, Bc.p, ainfo);
    else if (level0 && br == 3 && ns == 6)
        k_tentative<3, 6, true><<<g, 64, 0, s>>>(n_agg, ptr.p, nodes.p, coords, dim, Bf, C, P.S->slice_ptr, P.val, Bc.p, ainfo);
    else if (level0 && br == 1 && ns == 1)
        k_tentative<1, 1, true><<<g, 64, 0, s>>>(n_agg, ptr.p, nodes.p, coords, dim, Bf, C, P.S->slice_ptr, P.val, Bc.p, ainfo);
    else if (level0)
        fail(FR_EINTERNAL, "tentative: unsupported level-0 block shape");
    else if (br == 1 && ns == 1)
        k_tentative<1, 1, false><<<g, 64, 0, s>>>(n_agg, ptr.p, nodes.p, coords, dim, Bf, C, P.S->slice_ptr, P.val, Bc.p, ainfo);
    else if (br == 3 && ns == 3)
        k_tentative<3, 3, false><<<g, 64, 0, s>>>(n_agg, ptr.p, nodes.p, coords, dim, Bf, C, P.S->slice_ptr, P.val, Bc.p, ainfo);
    else if (br == 6 && ns == 6)
        k_tentative<6, 6, false><<<g, 64, 0, s>>>(n_agg, ptr.p, nodes.p, coords, dim, Bf, C, P.S->slice_ptr, P.val, Bc.p, ainfo);
    else
        fail(FR_EINTERNAL, "tentative: unsupported block shape");
    FR_LAUNCH_CHECK();
    if (keep) {
        keep->aptr = std::move(ptr);
        keep->anodes = std::move(nodes);
    }
    return P;
}

static void make_f32(AmgLevel& L, bool coarsest, hipStream_t s) {
    auto cp = [&](const BMat<double>& a, BMat<float>& b) {
        if (!a.S) return;
        b.br = a.br;
        b.bc = a.bc;
        b.S = a.S;
        const int64_t nv = a.S->n_slots * a.br * a.bc;
        b.own_val.alloc(size_t(std::max<int64_t>(1, nv)), s);
        b.val = b.own_val.p;
        cast_f64_f32(a.val, b.val, nv, s);
    };
    cp(L.A, L.A32);
    // a level with matrix-free transfers (L.mt) keeps its stored P and R for the Galerkin
    // product only: no FP32 copies
    if (!coarsest && !L.mt) {
        cp(L.P, L.P32);
        cp(L.R, L.R32);
    }
    const int64_t n = L.A.rows() * L.A.br;
    L.invd32.alloc(size_t(std::max<int64_t>(1, n)), s);
    cast_f64_f32(L.invd.p, L.invd32.p, n, s);
}

static void alloc_vectors(AmgLevel& L, int precision, hipStream_t s) {
    const size_t n = size_t(std::max<int64_t>(1, L.A.rows() * L.A.br));
    if (precision == 32) {
        L.fb.alloc(n, s); L.fx0.alloc(n, s); L.fx1.alloc(n, s); L.fd.alloc(n, s); L.fr.alloc(n, s);
    } else {
        L.vb.alloc(n, s); L.vx0.alloc(n, s); L.vx1.alloc(n, s); L.vd.alloc(n, s); L.vr.alloc(n, s);
    }
}

// Coarsest level: dense inverse when small enough.
static void coarse_inverse(Hierarchy& H, hipStream_t s) {
    AmgLevel& Lc = *H.lv.back();
    const int64_t nc = Lc.A.rows() * Lc.A.br;
    H.n_coarse = nc;
    if (nc <= kDenseMax) {
        H.dense_inv.reserve(size_t(std::max<int64_t>(1, nc * nc)), s);
        H.dense_inv.zero(s);
        const int g = nblk(Lc.A.rows(), 256);
        switch (Lc.A.br) {
            case 1: k_to_dense<1><<<g, 256, 0, s>>>(sv(*Lc.A.S), Lc.A.val, nc, H.dense_inv.p); break;
            case 2: k_to_dense<2><<<g, 256, 0, s>>>(sv(*Lc.A.S), Lc.A.val, nc, H.dense_inv.p); break;
            case 3: k_to_dense<3><<<g, 256, 0, s>>>(sv(*Lc.A.S), Lc.A.val, nc, H.dense_inv.p); break;
            case 6: k_to_dense<6><<<g, 256, 0, s>>>(sv(*Lc.A.S), Lc.A.val, nc, H.dense_inv.p); break;
            default: fail(FR_EINTERNAL, "dense: unsupported block size");
        }
        FR_LAUNCH_CHECK();
        k_fix_zero_rows<<<nblk(nc, 256), 256, 0, s>>>(nc, H.dense_inv.p);
        FR_LAUNCH_CHECK();
        k_gauss_jordan<<<1, 1024, 0, s>>>(nc, H.dense_inv.p);
        FR_LAUNCH_CHECK();
    } else {
        H.dense_inv.release();
    }
}

// `keep` stores the tentative prolongators and the products A P so that the values can later
// be recomputed for a new matrix with the same sparsity (refresh_hierarchy).
// The power iteration of a level runs on `aux` beside the aggregation and the tentative
// prolongator (which do not need it) and is waited for before the prolongator smoothing.
static void build_hierarchy(Hierarchy& H, BMat<double> A0, int ns0, const double* coords, int dim,
                            const fr_amg_opts& o, bool keep, hipStream_t s, hipStream_t aux, const char* tag,
                            const MfState* mf0 = nullptr, int blk = 0) {
    // profile names of the setup phases, per hierarchy (u / phi)
    const std::string t(tag);
    const std::string nm_lambda = "setup_lambda_" + t, nm_agg = "setup_aggregate_" + t,
                      nm_tent = "setup_tentative_" + t, nm_smooth = "setup_smooth_p_" + t, nm_rap = "setup_rap_" + t,
                      nm_coarse = "setup_coarse_" + t, nm_tune = "setup_tune_" + t, nm_all = "setup_hierarchy_" + t;
    ProfScope ps_all(nm_all.c_str(), s, 0.0);
    H.lv.clear();
    H.refreshable = keep;
    struct Ev {
        hipEvent_t e = nullptr;
        Ev() { FR_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming)); }
        ~Ev() { if (e) (void)hipEventDestroy(e); }
    } ev_holder;
    const hipEvent_t ev_aux = ev_holder.e;
    DBuf<int> errs;    // capacity overflows of the SpGEMM fills, read once at the end
    errs.alloc(1, s);
    errs.zero(s);
    DBuf<double> Bf;   // near-null space of the current level (levels >= 1)
    BMat<double> A = std::move(A0);
    int ns = ns0;
    for (int l = 0;; ++l) {
        auto L = std::make_unique<AmgLevel>();
        L->A.br = A.br;
        L->A.bc = A.bc;
        L->A.S = A.S;
        L->A.val = A.val;
        L->A.own_val = std::move(A.own_val);
        DBuf<double> dnorm;
        {
            ProfScope ps(nm_lambda.c_str(), s, 0.0);
            diag_info(L->A, L->invd, dnorm, s);
        }
        // the power iteration waits for the diagonal only; its launches are enqueued on `aux`
        // while the first aggregation round runs, so the stream is not idle meanwhile
        PowerEst pe;
        FR_HIP(hipEventRecord(ev_aux, s));
        bool power_started = false;
        auto start_power = [&]() {
            if (power_started) return;
            power_started = true;
            FR_HIP(hipStreamWaitEvent(aux, ev_aux, 0));
            ProfScope ps(nm_lambda.c_str(), aux, 0.0);
            power_start(pe, L->A, L->invd.p, aux, l == 0 ? mf0 : nullptr, blk);
        };
        const int64_t nrows = L->A.rows() * L->A.br;
        const bool last = nrows <= o.coarse_max || l + 1 >= o.max_levels;
        if (last) start_power();
        if (!last) {
            DBuf<int32_t> agg;
            int64_t n_agg = 0;
            {
                ProfScope ps(nm_agg.c_str(), s, 0.0);
                // strength threshold: negative selects the measured default per dimension
                const double theta = o.theta >= 0 ? o.theta : (dim == 2 ? 0.08 : 0.02);
                n_agg = aggregate(L->A, dnorm.p, theta, agg, s, start_power);
            }
            start_power();   // aggregation without a host wait in its rounds
            if (n_agg == 0 || n_agg * ns >= nrows) {
                L->lmax = power_finish(pe);
                H.lv.push_back(std::move(L));
                break;   // coarsening stalled: this level is the coarsest
            }
            DBuf<double> Bc;
            BMat<double> Pt, AP, Ac;
            // the finest displacement level of a uniform 2d mesh keeps its aggregation for the
            // matrix-free transfers
            const bool mt = l == 0 && mf0 && blk == 0 && dim == 2 && ns == 3 && (o.fine_matrix_free & 4);
            if (mt) L->mt = std::make_unique<AggTransfer>();
            {
                ProfScope ps(nm_tent.c_str(), s, 0.0);
                Pt = tentative(L->A, agg, n_agg, ns, l == 0, coords, dim, Bf.p, Bc, s, L->mt.get());
            }
            L->lmax = power_finish(pe);
            if (mt) {
                L->mt->agg = std::move(agg);
                L->mt->omega = 4.0 / (3.0 * L->lmax);
                L->mt->w.alloc(size_t(std::max<int64_t>(1, n_agg)) * 3, s);
                if (o.precision == 32) {
                    const int64_t ni = n_agg * kAggInfo;
                    L->mt->info32.alloc(size_t(std::max<int64_t>(1, ni)), s);
                    cast_f64_f32(L->mt->info.p, L->mt->info32.p, ni, s);
                    L->mt->w32.alloc(size_t(std::max<int64_t>(1, n_agg)) * 3, s);
                }
            }
            {
                ProfScope ps(nm_smooth.c_str(), s, 0.0);
                const double omega = 4.0 / (3.0 * L->lmax);
                L->omega = omega;
                L->P = spgemm<1>(L->A, Pt, L->invd.p, omega, errs.p, s);
                L->R = transpose(L->P, s);
            }
            {
                ProfScope ps(nm_rap.c_str(), s, 0.0);
                AP = spgemm<0>(L->A, L->P, nullptr, 0.0, errs.p, s);
                Ac = spgemm<0>(L->R, AP, nullptr, 0.0, errs.p, s);
            }
            L->ns = ns;
            if (keep) {
                L->Pt = std::move(Pt);
                L->AP = std::move(AP);
            }
            Bf = std::move(Bc);
            A = std::move(Ac);
            H.lv.push_back(std::move(L));
            continue;
        }
        L->lmax = power_finish(pe);
        H.lv.push_back(std::move(L));
        break;
    }
    {
        ProfScope ps(nm_coarse.c_str(), s, 0.0);
        coarse_inverse(H, s);
    }
    if (o.autotune) {
        // launch shapes of the smoothers and transfers below the finest level (level 0's
        // matrix is the system's own)
        ProfScope ps(nm_tune.c_str(), s, 0.0);
        for (size_t l = 0; l + 1 < H.lv.size(); ++l) {
            AmgLevel& L = *H.lv[l];
            const bool f32 = o.precision == 32;
            if (l > 0) tune_layout(L.A, 0, f32, s);
            if (L.mt) continue;   // its transfers are matrix-free: P and R are not launched
            tune_layout(L.R, 1, f32, s);
            tune_layout(L.P, 2, f32, s);
        }
    }
    for (size_t l = 0; l < H.lv.size(); ++l) {
        if (o.precision == 32) make_f32(*H.lv[l], l + 1 == H.lv.size(), s);
        alloc_vectors(*H.lv[l], o.precision, s);
    }
    if (download1(errs.p, s)) fail(FR_EINTERNAL, "amg setup: a row exceeded the SpGEMM LDS capacity");
}

// Same aggregates, tentative prolongators and sparsity; new values from the level-0 matrix
// at a0 (whose structure is the one the hierarchy was built on).
static void refresh_hierarchy(Hierarchy& H, double* a0, const fr_amg_opts& o, hipStream_t s, hipStream_t aux,
                              const MfState* mf0 = nullptr, int blk = 0) {
    const size_t nl = H.lv.size();
    H.lv[0]->A.val = a0;
    // refresh_phi 2: the finest level's diagonal and lambda_max only (coarse levels and the
    // transfers stay those of the build: a lagged preconditioner)
    if (o.refresh_phi == 2) {
        AmgLevel& L = *H.lv[0];
        DBuf<double> dnorm;
        diag_info(L.A, L.invd, dnorm, s);
        L.lmax = lambda_max(L.A, L.invd.p, s, mf0, blk);
        if (o.precision == 32) make_f32(L, nl == 1, s);
        return;
    }
    // Every level's new values; the prolongators are smoothed with the build's weights, so
    // each level's lambda_max (the smoother's bound) is estimated on `aux` beside the products
    // instead of ahead of them, and read once at the end.
    struct Ev {
        hipEvent_t e = nullptr;
        Ev() { FR_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming)); }
        ~Ev() { if (e) (void)hipEventDestroy(e); }
    } ev;
    std::vector<PowerEst> pe(nl);
    for (size_t l = 0; l < nl; ++l) {
        AmgLevel& L = *H.lv[l];
        DBuf<double> dnorm;
        diag_info(L.A, L.invd, dnorm, s);
        FR_HIP(hipEventRecord(ev.e, s));
        FR_HIP(hipStreamWaitEvent(aux, ev.e, 0));
        power_start(pe[l], L.A, L.invd.p, aux, l == 0 ? mf0 : nullptr, blk);
        if (l + 1 == nl) break;
        spgemm_values<1>(L.A, L.Pt, L.P, L.invd.p, L.omega, s);
        transpose_values(L.P, L.R, s);
        spgemm_values<0>(L.A, L.P, L.AP, nullptr, 0.0, s);
        spgemm_values<0>(L.R, L.AP, H.lv[l + 1]->A, nullptr, 0.0, s);
    }
    coarse_inverse(H, s);
    if (o.precision == 32)
        for (size_t l = 0; l < nl; ++l) make_f32(*H.lv[l], l + 1 == nl, s);
    for (size_t l = 0; l < nl; ++l) H.lv[l]->lmax = power_finish(pe[l]);
}

static void ensure_side(DevAmg& amg) {
    if (amg.side) return;
    FR_HIP(hipStreamCreateWithFlags(&amg.side, hipStreamNonBlocking));
    for (auto& a : amg.aux) FR_HIP(hipStreamCreateWithFlags(&a, hipStreamNonBlocking));
    FR_HIP(hipEventCreateWithFlags(&amg.ev_fork, hipEventDisableTiming));
    FR_HIP(hipEventCreateWithFlags(&amg.ev_join, hipEventDisableTiming));
}

// The displacement hierarchy lives on the caller's stream, the phase-field hierarchy on the
// side stream (its buffers are allocated, used and freed there).  When both are built from
// scratch the phase-field setup runs in a second host thread, so that the host round trips
// of one setup overlap the device work of the other.
void amg_build(DevAmg& amg, DevSystem& sys, const fr_amg_opts& o, hipStream_t s) {
    const bool keep_u = o.reuse_u_block && amg.sys == &sys && !amg.h[0].lv.empty() &&
                        amg.opts.precision == o.precision && amg.h[0].lv[0]->A.val == sys.Juu.val;
    const bool same_shape = amg.opts.precision == o.precision && amg.opts.theta == o.theta &&
                            amg.opts.coarse_max == o.coarse_max && amg.opts.max_levels == o.max_levels;
    const bool refresh_phi = o.refresh_phi && amg.sys == &sys && !amg.h[1].lv.empty() && amg.h[1].refreshable &&
                             same_shape && amg.h[1].lv[0]->A.S == sys.Jpp.S;
    // graphs captured over the old hierarchy's buffers and coefficients are stale from here on
    amg.epoch = next_epoch();
    amg.sys = &sys;
    amg.opts = o;
    amg.stream = s;
    ensure_side(amg);
    amg.h[1].mf = nullptr;
    DevMesh& m = *sys.mesh;
    // fork: the side stream follows everything enqueued on s so far (the Jacobian, and
    // every earlier use of the buffers that the phase-field setup frees)
    FR_HIP(hipEventRecord(amg.ev_fork, s));
    FR_HIP(hipStreamWaitEvent(amg.side, amg.ev_fork, 0));
    const hipStream_t side = amg.side;
    // the fine levels' power steps apply the blocks matrix-free where the V-cycle will
    const MfState* mf_u = ((o.fine_matrix_free & 1) && sys.mf.valid) ? &sys.mf : nullptr;
    const MfState* mf_p = ((o.fine_matrix_free & 2) && sys.mf.valid) ? &sys.mf : nullptr;
    auto phi_setup = [&amg, &sys, &m, o, refresh_phi, side, mf_p]() {
        if (refresh_phi) {
            ProfScope ps("setup_refresh_phi", side, 0.0);
            refresh_hierarchy(amg.h[1], sys.Jpp.val, o, side, amg.aux[1], mf_p, 1);
        } else {
            BMat<double> Ap;
            Ap.br = Ap.bc = 1;
            Ap.S = sys.Jpp.S;
            Ap.val = sys.Jpp.val;
            build_hierarchy(amg.h[1], std::move(Ap), 1, m.coords_free.p, m.dim, o, o.refresh_phi != 0, side,
                            amg.aux[1], "phi", mf_p, 1);
        }
    };
    auto u_setup = [&]() {
        BMat<double> Au;
        Au.br = Au.bc = m.dim;
        Au.S = sys.Juu.S;
        Au.val = sys.Juu.val;
        build_hierarchy(amg.h[0], std::move(Au), m.dim == 2 ? 3 : 6, m.coords_free.p, m.dim, o, false, s, amg.aux[0],
                        "u", mf_u, 0);
    };
    if (keep_u) {
        phi_setup();
    } else {
        int dev = 0;
        FR_HIP(hipGetDevice(&dev));
        std::exception_ptr phi_err;
        std::thread worker([&]() {
            try {
                FR_HIP(hipSetDevice(dev));
                phi_setup();
            } catch (...) {
                phi_err = std::current_exception();
            }
        });
        std::exception_ptr u_err;
        try {
            u_setup();
        } catch (...) {
            u_err = std::current_exception();
        }
        worker.join();
        if (u_err) std::rethrow_exception(u_err);
        if (phi_err) std::rethrow_exception(phi_err);
    }
    // join
    FR_HIP(hipEventRecord(amg.ev_join, side));
    FR_HIP(hipStreamWaitEvent(s, amg.ev_join, 0));
    amg.sys_version = sys.version;
    // the fine levels apply M_uu (bit 0) and M_phiphi (bit 1) matrix-free where the mesh allows it
    amg.h[0].blk = 0;
    amg.h[1].blk = 1;
    amg.h[0].mf = ((o.fine_matrix_free & 1) && sys.mf.valid) ? &sys.mf : nullptr;
    amg.h[1].mf = ((o.fine_matrix_free & 2) && sys.mf.valid) ? &sys.mf : nullptr;
}

// ---- V-cycle ---------------------------------------------------------------------------------

template <typename T>
struct LevelOps {
    static const BMat<T>& A(const AmgLevel& L);
    static const BMat<T>& P(const AmgLevel& L);
    static const BMat<T>& R(const AmgLevel& L);
    static const T* invd(const AmgLevel& L);
    static T* b(AmgLevel& L);
    static T* x0(AmgLevel& L);
    static T* x1(AmgLevel& L);
    static T* d(AmgLevel& L);
    static T* r(AmgLevel& L);
};

template <>
struct LevelOps<double> {
    static const BMat<double>& A(const AmgLevel& L) { return L.A; }
    static const BMat<double>& P(const AmgLevel& L) { return L.P; }
    static const BMat<double>& R(const AmgLevel& L) { return L.R; }
    static const double* invd(const AmgLevel& L) { return L.invd.p; }
    static double* b(AmgLevel& L) { return L.vb.p; }
    static double* x0(AmgLevel& L) { return L.vx0.p; }
    static double* x1(AmgLevel& L) { return L.vx1.p; }
    static double* d(AmgLevel& L) { return L.vd.p; }
    static double* r(AmgLevel& L) { return L.vr.p; }
};

template <>
struct LevelOps<float> {
    static const BMat<float>& A(const AmgLevel& L) { return L.A32; }
    static const BMat<float>& P(const AmgLevel& L) { return L.P32; }
    static const BMat<float>& R(const AmgLevel& L) { return L.R32; }
    static const float* invd(const AmgLevel& L) { return L.invd32.p; }
    static float* b(AmgLevel& L) { return L.fb.p; }
    static float* x0(AmgLevel& L) { return L.fx0.p; }
    static float* x1(AmgLevel& L) { return L.fx1.p; }
    static float* d(AmgLevel& L) { return L.fd.p; }
    static float* r(AmgLevel& L) { return L.fr.p; }
};

// Chebyshev smoothing of A x = b on [lmax/ratio, 1.1 lmax] starting from x (zero if
// from_zero).  Returns the buffer holding the result: x0 or x1 of the level, or `out` when
// given (the last step writes there).
template <typename T>
static T* chebyshev(const AmgLevel& Lc, AmgLevel& L, const T* b, bool from_zero, T* x, T* other, int degree,
                    double ratio, hipStream_t s, T* out = nullptr, const MfState* mf = nullptr, int blk = 0,
                    int lvl = -1) {
    using O = LevelOps<T>;
    const double hi = 1.1 * Lc.lmax, lo = hi / ratio;
    const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
    double rho = 1.0 / sigma;
    const int64_t n = Lc.A.rows() * Lc.A.br;
    T* d = O::d(L);
    int k0 = 1;
    if (from_zero && mf && degree >= 2) {
        // matrix-free fine level: the first step (x = D^-1 b / theta) is formed inside the second
        const double rn = 1.0 / (2.0 * sigma - rho);
        T* dst = (degree == 2 && out) ? out : other;
        mf_cheb_first2<T>(*mf, blk, O::invd(Lc), b, d, dst, T(1.0 / theta), T(rn * rho), T(2.0 * rn / delta), s);
        rho = rn;
        if (dst == out) return out;
        std::swap(x, other);
        k0 = 2;
    } else if (from_zero) {
        cheb_first<T>(O::invd(Lc), b, d, (degree == 1 && out) ? out : x, T(1.0 / theta), n, s, lvl);
        if (degree == 1 && out) return out;
    } else {
        T* dst = (degree == 1 && out) ? out : other;
        if (mf) mf_cheb_step<T>(*mf, blk, O::invd(Lc), x, b, d, dst, T(0), T(1.0 / theta), s);
        else cheb_step<T>(O::A(Lc), O::invd(Lc), x, b, d, dst, T(0), T(1.0 / theta), s, lvl);
        if (dst == out) return out;
        std::swap(x, other);
    }
    for (int k = k0; k < degree; ++k) {
        const double rn = 1.0 / (2.0 * sigma - rho);
        T* dst = (k + 1 == degree && out) ? out : other;
        if (mf) mf_cheb_step<T>(*mf, blk, O::invd(Lc), x, b, d, dst, T(rn * rho), T(2.0 * rn / delta), s);
        else cheb_step<T>(O::A(Lc), O::invd(Lc), x, b, d, dst, T(rn * rho), T(2.0 * rn / delta), s, lvl);
        rho = rn;
        if (dst == out) return out;
        std::swap(x, other);
    }
    return x;
}

// One V-cycle from level l for A_l x = b; the result is returned (a level buffer, or `out`
// when given: the last smoothing step of level l writes there).
template <typename T>
static T* vcycle(Hierarchy& H, size_t l, const T* b, const fr_amg_opts& o, hipStream_t s, T* out = nullptr) {
    using O = LevelOps<T>;
    AmgLevel& L = *H.lv[l];
    const int64_t n = L.A.rows() * L.A.br;
    if (l + 1 == H.lv.size()) {
        T* x = out ? out : O::x0(L);
        if (H.dense_inv.p) {
            if (n) k_dense_gemv<T><<<int(n), 256, 0, s>>>(n, H.dense_inv.p, b, x);
            FR_LAUNCH_CHECK();
            return x;
        }
        // large coarsest level: a longer smoothing sweep stands in for the exact solve
        return chebyshev<T>(L, L, b, true, O::x0(L), O::x1(L), 4 * o.cheb_degree, o.cheb_ratio, s, out, nullptr, 0,
                            int(l));
    }
    // the fine level of a uniform 2d mesh applies its block (M_uu or M_phiphi) matrix-free
    const MfState* mf = (l == 0 && H.mf && H.mf->valid) ? H.mf : nullptr;
    const int lv = int(l);
    T* x = chebyshev<T>(L, L, b, true, O::x0(L), O::x1(L), o.cheb_degree, o.cheb_ratio, s, nullptr, mf, H.blk, lv);
    T* other = (x == O::x0(L)) ? O::x1(L) : O::x0(L);
    if (mf) mf_residual<T>(*mf, H.blk, x, b, O::r(L), s);
    else spmv_residual<T>(O::A(L), x, b, O::r(L), s, lv);
    AmgLevel& Ln = *H.lv[l + 1];
    // the finest displacement level's transfers matrix-free where its aggregation was kept (the
    // smoother's d is free between the two smoothings: the restriction's scratch)
    const AggTransfer* mt = (mf && L.mt) ? L.mt.get() : nullptr;
    if (mt) mf_restrict<T>(*mf, *mt, O::invd(L), O::r(L), O::d(L), O::b(Ln), s);
    else spmv<T>(O::R(L), O::r(L), O::b(Ln), s, lv);
    T* xc = vcycle<T>(H, l + 1, O::b(Ln), o, s);
    if (mt) mf_prolong<T>(*mf, *mt, O::invd(L), xc, x, s);
    else spmv_add<T>(O::P(L), xc, x, s, lv);
    return chebyshev<T>(L, L, b, false, x, other, o.cheb_degree, o.cheb_ratio, s, out, mf, H.blk, lv);
}

// z = M^-1 r with M^-1 = diag(V-cycle(M_uu), V-cycle(M_phiphi)).  The phi block's cycle
// runs on the side stream, the u block's on the caller's; the u cycle is enqueued first: its
// level-0 sweeps keep the device busy while the host enqueues the phi cycle, whose small
// levels then run beside the u work.  ZT is double, or float for the FP32 hierarchy (whose
// result is FP32 anyway: keeping it so loses nothing).
template <typename ZT>
static void precondition(DevAmg& amg, const double* r, ZT* z, hipStream_t s) {
    DevSystem& sys = *amg.sys;
    const int64_t nu = sys.n_u;
    const int64_t nb[2] = {nu, sys.n_solve - nu};
    const int64_t off[2] = {0, nu};
    ensure_side(amg);
    FR_HIP(hipEventRecord(amg.ev_fork, s));
    FR_HIP(hipStreamWaitEvent(amg.side, amg.ev_fork, 0));
    for (int blk = 0; blk <= 1; ++blk) {
        Hierarchy& H = amg.h[blk];
        const hipStream_t st = blk == 1 ? amg.side : s;
        ProfScope ps(blk == 0 ? "vcycle_u" : "vcycle_phi", st, 0.0);
        if constexpr (std::is_same<ZT, float>::value) {
            AmgLevel& L0 = *H.lv[0];
            if (r) cast_f64_f32(r + off[blk], L0.fb.p, nb[blk], st);   // else staged by the caller
            vcycle<float>(H, 0, L0.fb.p, amg.opts, st, z + off[blk]);
        } else {
            vcycle<double>(H, 0, r + off[blk], amg.opts, st, z + off[blk]);
        }
    }
    FR_HIP(hipEventRecord(amg.ev_join, amg.side));
    FR_HIP(hipStreamWaitEvent(s, amg.ev_join, 0));
}

void amg_precondition(DevAmg& amg, const double* r, double* z, hipStream_t s) {
    if (amg.opts.precision == 32) {
        // FP32 hierarchy, FP64 output
        DevSystem& sys = *amg.sys;
        amg.z32.reserve(size_t(std::max<int64_t>(1, sys.n_solve)), s);
        precondition<float>(amg, r, amg.z32.p, s);
        cast_f32_f64(amg.z32.p, z, sys.n_solve, s);
    } else {
        precondition<double>(amg, r, z, s);
    }
}

void amg_precondition32(DevAmg& amg, const double* r, float* z, hipStream_t s) {
    if (amg.opts.precision != 32) fail(FR_EINTERNAL, "amg_precondition32: the hierarchy is FP64");
    precondition<float>(amg, r, z, s);
}

uint64_t next_epoch() {
    static std::atomic<uint64_t> e{0};
    return ++e;
}

void* amg_graph_input(DevAmg& amg) {
    const int64_t n = std::max<int64_t>(1, amg.sys->n_solve);
    if (amg.opts.precision == 32) {
        if (amg.vin32.n < size_t(n)) { amg.epoch = next_epoch(); amg.vin32.reserve(size_t(n), amg.stream); }
        return amg.vin32.p;
    }
    if (amg.vin64.n < size_t(n)) { amg.epoch = next_epoch(); amg.vin64.reserve(size_t(n), amg.stream); }
    return amg.vin64.p;
}

void* amg_graph_output(DevAmg& amg) {
    const int64_t n = std::max<int64_t>(1, amg.sys->n_solve);
    if (amg.opts.precision == 32) {
        if (amg.vout32.n < size_t(n)) { amg.epoch = next_epoch(); amg.vout32.reserve(size_t(n), amg.stream); }
        return amg.vout32.p;
    }
    if (amg.vout64.n < size_t(n)) { amg.epoch = next_epoch(); amg.vout64.reserve(size_t(n), amg.stream); }
    return amg.vout64.p;
}

void amg_precondition_staged(DevAmg& amg, hipStream_t s) {
    ensure_side(amg);
    DevSystem& sys = *amg.sys;
    const int64_t off[2] = {0, sys.n_u};
    void* vin = amg_graph_input(amg);
    void* vout = amg_graph_output(amg);
    FR_HIP(hipEventRecord(amg.ev_fork, s));
    FR_HIP(hipStreamWaitEvent(amg.side, amg.ev_fork, 0));
    for (int blk = 0; blk <= 1; ++blk) {
        const hipStream_t st = blk == 1 ? amg.side : s;
        ProfScope ps(blk == 0 ? "vcycle_u" : "vcycle_phi", st, 0.0);
        if (amg.opts.precision == 32)
            vcycle<float>(amg.h[blk], 0, static_cast<float*>(vin) + off[blk], amg.opts, st,
                          static_cast<float*>(vout) + off[blk]);
        else
            vcycle<double>(amg.h[blk], 0, static_cast<double*>(vin) + off[blk], amg.opts, st,
                           static_cast<double*>(vout) + off[blk]);
    }
    FR_HIP(hipEventRecord(amg.ev_join, amg.side));
    FR_HIP(hipStreamWaitEvent(s, amg.ev_join, 0));
}

float* amg_input32(DevAmg& amg, int blk) {
    if (amg.opts.precision != 32 || amg.h[blk].lv.empty()) fail(FR_EINTERNAL, "amg_input32: no FP32 hierarchy");
    return amg.h[blk].lv[0]->fb.p;
}

void amg_level_export(DevAmg& amg, int blk, int level, int which, int64_t& n_rows, int64_t& n_cols,
                      std::vector<int64_t>& rp, std::vector<int32_t>& ci, std::vector<double>& vv, hipStream_t s) {
    Hierarchy& H = amg.h[blk];
    if (level < 0 || size_t(level) >= H.lv.size()) fail(FR_EINVAL, "amg_level_csr: level out of range");
    AmgLevel& L = *H.lv[size_t(level)];
    const BMat<double>* M = which == 0 ? &L.A : (which == 1 ? &L.P : &L.R);
    if (!M->S) fail(FR_EINVAL, "amg_level_csr: operator absent on this level");
    const SellStruct& S = *M->S;
    auto sp = download(S.slice_ptr, size_t(S.n_slices) + 1, s);
    auto len = download(S.row_len, size_t(S.n_rows), s);
    auto col = download(S.col, size_t(S.n_slots), s);
    auto val = download(M->val, size_t(S.n_slots) * M->br * M->bc, s);
    const int br = M->br, bc = M->bc;
    n_rows = S.n_rows * br;
    n_cols = S.n_cols * bc;
    rp.assign(size_t(n_rows) + 1, 0);
    ci.clear();
    vv.clear();
    for (int64_t r = 0; r < S.n_rows; ++r)
        for (int i = 0; i < br; ++i) {
            for (int k = 0; k < len[size_t(r)]; ++k) {
                const int64_t sl = int64_t(sp[size_t(r / S.C)]) + int64_t(k) * S.C + r % S.C;
                for (int j = 0; j < bc; ++j) {
                    ci.push_back(col[size_t(sl)] * bc + j);
                    vv.push_back(val[size_t(sl * br * bc + i * bc + j)]);
                }
            }
            rp[size_t(r * br + i) + 1] = int64_t(ci.size());
        }
}

void amg_level_shape(DevAmg& amg, int blk, int level, int which, int& C, int& G) {
    Hierarchy& H = amg.h[blk];
    if (level < 0 || size_t(level) >= H.lv.size()) fail(FR_EINVAL, "amg_level_shape: level out of range");
    AmgLevel& L = *H.lv[size_t(level)];
    const BMat<double>* M = which == 0 ? &L.A : (which == 1 ? &L.P : &L.R);
    if (!M->S) fail(FR_EINVAL, "amg_level_shape: operator absent on this level");
    C = M->S->C;
    G = launch_lanes(*M->S);
}

void amg_info(DevAmg& amg, int blk, int level, int& n_levels, int64_t& rows, int& bsize, int64_t& nnzb, double& lmax,
              hipStream_t s) {
    Hierarchy& H = amg.h[blk];
    n_levels = int(H.lv.size());
    if (level < 0 || size_t(level) >= H.lv.size()) return;
    AmgLevel& L = *H.lv[size_t(level)];
    rows = L.A.rows();
    bsize = L.A.br;
    (void)s;
    nnzb = L.A.S->nnz;
    lmax = L.lmax;
}

}  // namespace fr
