// Matrix-free application of the displacement block M_uu (Section 3, "Linear iterative
// solution": the Jacobian block of equation E22ATW in the displacement) on uniform 2d meshes.
//
// On a uniform mesh every cell is the same square, so the Q1 element stiffness at a Gauss point
// depends on the cell only through the degradation g_q = (1 - kappa) phi_tilde_q^2 + kappa, and
// in 2d the factor w|J| |grad N|^2 is independent of the edge h.  M_uu x is therefore
//     (M_uu x)_(a,c) = sum over the cells e of node a, over the Gauss points q of e of
//                      g_q sum_k sigma_q(x)[c][k] dN_a/dxi_k(q),
//     sigma = 2 mu eps + lambda tr(eps) I,  eps = sym(H),  H[c][k] = sum_b x_(b,c) dN_b/dxi_k(q)
// (reference gradients, the h factors cancel), with the Dirichlet columns left out (x_b = 0 on
// the boundary) and the Dirichlet rows replaced by their diagonal entry: exactly the masked
// M_uu the assembly stores, summed in another order.  Reading the nodal phi_tilde (8 bytes per
// node) and x instead of the 2x2 blocks of nine stored neighbours (306 bytes per node) is what
// makes the fine level's smoother, residual and the J-SpMV's displacement rows cheaper: they
// are bound by HBM bandwidth, and the arithmetic (about 200 FMAs per node) stays far below the
// FP64 vector rate.
//
// A workgroup works on a 31 x 7 tile of nodes (lexicographic numbering, x fastest): it reads the
// tile's patch of x and phi_tilde once into LDS, computes each of the 32 x 8 cells around the
// tile once (one thread per cell: the Gauss-point stresses and the contributions to the cell's
// four vertices), and every node sums the contributions of its four cells.
#include "profile.h"
#include "system.h"

namespace fr {
namespace {

// 1d Q1 factors at the 2-point Gauss abscissae: (1 +- 1/sqrt(3)) / 2
constexpr double kP = 0.78867513459481288225;
constexpr double kM = 0.21132486540518711775;

// N_b at Gauss point q (bit k of b / q: upper side along axis k)
__device__ __forceinline__ constexpr double nq(int q, int b) {
    return ((b & 1) == (q & 1) ? kP : kM) * (((b >> 1) & 1) == ((q >> 1) & 1) ? kP : kM);
}

// dN_b / dxi_k at Gauss point q on the reference square [-1, 1]^2
__device__ __forceinline__ constexpr double gq(int q, int b, int k) {
    const int o = 1 - k;   // the other axis
    return (((b >> k) & 1) ? 0.5 : -0.5) * (((b >> o) & 1) == ((q >> o) & 1) ? kP : kM);
}

// Tiles: a workgroup of 256 threads owns the nodes i0 .. i0 + 30 of rows j0 .. j0 + 6 (31 x 7)
// and computes, one thread per cell, the 32 x 8 cells around them (the node tile grown by one
// cell to the left and below) from the 33 x 9 patch of nodes it reads once into LDS.  Each cell
// leaves the contributions to its four vertices in LDS; a node sums those of its four cells.
constexpr int kTX = 31, kTY = 7;                 // nodes per tile
constexpr int kCX = kTX + 1, kCY = kTY + 1;      // cells per tile (kCX * kCY = 256 threads)
constexpr int kPX = kTX + 2, kPY = kTY + 2;      // patch nodes per tile
static_assert(kCX * kCY == 256, "one cell per thread");

// x of the patch (zero on the boundary: the eliminated Dirichlet columns, and outside the mesh)
// and phi_tilde of the patch (zero outside the mesh), in LDS.
template <typename TA>
struct Patch {
    TA x[2][kPY][kPX];                           // component-major: consecutive lanes, consecutive words
    TA p[kPY][kPX];
    TA c[4][2][kCY][kCX];                        // cell contributions to vertex a, component c
};

template <typename TA, typename TX, typename TP>
__device__ __forceinline__ void load_patch(const MfGrid& g, const TP* __restrict__ pt, const TX* __restrict__ x,
                                           int64_t i0, int64_t j0, Patch<TA>& P) {
    for (int t = threadIdx.x; t < kPX * kPY; t += blockDim.x) {
        const int px = t % kPX, py = t / kPX;
        const int64_t bi = i0 - 1 + px, bj = j0 - 1 + py;
        const bool in = bi >= 0 && bj >= 0 && bi <= g.nx && bj <= g.ny;
        const bool interior = bi > 0 && bj > 0 && bi < g.nx && bj < g.ny;
        const int64_t nb = bi + bj * g.n1;
        P.p[py][px] = in ? TA(pt[nb]) : TA(0);
        P.x[0][py][px] = interior ? TA(x[2 * nb]) : TA(0);
        P.x[1][py][px] = interior ? TA(x[2 * nb + 1]) : TA(0);
    }
}

// Thread t's cell (i0 - 1 + t % kCX, j0 - 1 + t / kCX): its contributions to its four vertices,
// sum over the Gauss points of g_q sigma_q(x) grad N_a(q) (zero for a cell outside the mesh).
// The tensor-product structure of Q1 with 2 x 2 Gauss points is used: with f(b, q) = kP when the
// vertex and the Gauss point lie on the same side of the axis (else kM),
//   d/dxi of the x at Gauss point q  = (f(0, q_y) (x_1 - x_0) + f(1, q_y) (x_3 - x_2)) / 2,
//   d/deta                            = (f(0, q_x) (x_2 - x_0) + f(1, q_x) (x_3 - x_1)) / 2,
// and the vertex contributions need only the stresses summed along one axis:
//   c_(a, comp) = s_x(a) X_comp[a_y] + s_y(a) Y_comp[a_x],
//   X_comp[a_y] = (f(a_y, 0) Sx_comp[0] + f(a_y, 1) Sx_comp[1]) / 2, Sx_comp[q_y] = sum over q_x
//   of sigma[comp][0], and Y the same along the other axis with sigma[comp][1].
template <typename TA>
__device__ __forceinline__ void cell_contrib(const MfGrid& g, int64_t i0, int64_t j0, Patch<TA>& P) {
    const int cx = threadIdx.x % kCX, cy = threadIdx.x / kCX;
    const int64_t ci = i0 - 1 + cx, cj = j0 - 1 + cy;
    TA out[4][2];
#pragma unroll
    for (int a = 0; a < 4; ++a) out[a][0] = out[a][1] = TA(0);
    if (ci >= 0 && cj >= 0 && ci < g.nx && cj < g.ny) {
        const TA mu = TA(g.mu), lam = TA(g.lam), kap = TA(g.kappa), omk = TA(1.0 - g.kappa);
        const TA fP = TA(kP), fM = TA(kM), half = TA(0.5);
        // vertex values: b = 0 (lower left), 1 (lower right), 2 (upper left), 3 (upper right)
        TA xv[2][4], pv[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            pv[b] = P.p[cy + (b >> 1)][cx + (b & 1)];
            xv[0][b] = P.x[0][cy + (b >> 1)][cx + (b & 1)];
            xv[1][b] = P.x[1][cy + (b >> 1)][cx + (b & 1)];
        }
        // reference gradients: Hx[comp][q_y] = d x_comp / dxi, Hy[comp][q_x] = d x_comp / deta
        TA Hx[2][2], Hy[2][2];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const TA dx0 = xv[c][1] - xv[c][0], dx1 = xv[c][3] - xv[c][2];
            const TA dy0 = xv[c][2] - xv[c][0], dy1 = xv[c][3] - xv[c][1];
            Hx[c][0] = half * (fP * dx0 + fM * dx1);
            Hx[c][1] = half * (fM * dx0 + fP * dx1);
            Hy[c][0] = half * (fP * dy0 + fM * dy1);
            Hy[c][1] = half * (fM * dy0 + fP * dy1);
        }
        // phi_tilde at the Gauss points: along x in both vertex rows, then along y
        TA pr[2][2];
#pragma unroll
        for (int by = 0; by < 2; ++by) {
            pr[by][0] = fP * pv[2 * by] + fM * pv[2 * by + 1];
            pr[by][1] = fM * pv[2 * by] + fP * pv[2 * by + 1];
        }
        TA Sx[2][2] = {{TA(0), TA(0)}, {TA(0), TA(0)}}, Sy[2][2] = {{TA(0), TA(0)}, {TA(0), TA(0)}};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int qx = q & 1, qy = q >> 1;
            const TA ph = qy ? fM * pr[0][qx] + fP * pr[1][qx] : fP * pr[0][qx] + fM * pr[1][qx];
            const TA gg = omk * ph * ph + kap;
            const TA h00 = Hx[0][qy], h01 = Hy[0][qx], h10 = Hx[1][qy], h11 = Hy[1][qx];
            const TA tr = h00 + h11;
            const TA s00 = gg * (TA(2) * mu * h00 + lam * tr);
            const TA s11 = gg * (TA(2) * mu * h11 + lam * tr);
            const TA s01 = gg * (mu * (h01 + h10));
            Sx[0][qy] += s00;                    // sigma[0][0]
            Sx[1][qy] += s01;                    // sigma[1][0]
            Sy[0][qx] += s01;                    // sigma[0][1]
            Sy[1][qx] += s11;                    // sigma[1][1]
        }
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const TA X0 = half * (fP * Sx[c][0] + fM * Sx[c][1]), X1 = half * (fM * Sx[c][0] + fP * Sx[c][1]);
            const TA Y0 = half * (fP * Sy[c][0] + fM * Sy[c][1]), Y1 = half * (fM * Sy[c][0] + fP * Sy[c][1]);
            out[0][c] = -X0 - Y0;                // a = (0, 0)
            out[1][c] = X0 - Y1;                 // a = (1, 0)
            out[2][c] = -X1 + Y0;                // a = (0, 1)
            out[3][c] = X1 + Y1;                 // a = (1, 1)
        }
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        P.c[a][0][cy][cx] = out[a][0];
        P.c[a][1][cy][cx] = out[a][1];
    }
}

// Original diagonal entries of a Dirichlet node's two rows (the node of thread tile position
// (tx, ty)): sum over its cells of g_q (mu (|grad N_a|^2 + (d_c N_a)^2) + lambda (d_c N_a)^2).
template <typename TA>
__device__ __forceinline__ void dirichlet_diag(const MfGrid& g, int64_t i, int64_t j, int tx, int ty,
                                               const Patch<TA>& P, TA dg[2]) {
    const TA mu = TA(g.mu), lam = TA(g.lam), kap = TA(g.kappa), omk = TA(1.0 - g.kappa);
    dg[0] = dg[1] = TA(0);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int ex = e & 1, ey = e >> 1;       // cell to the lower-left (0) ... upper-right (3)
        const int64_t ci = i - 1 + ex, cj = j - 1 + ey;
        if (ci < 0 || cj < 0 || ci >= g.nx || cj >= g.ny) continue;
        const int a = (1 - ex) + 2 * (1 - ey);  // the node's vertex in that cell
        const int cx = tx + ex, cy = ty + ey;    // the cell's patch position
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            TA ph = TA(0);
#pragma unroll
            for (int b = 0; b < 4; ++b) ph += TA(nq(q, b)) * P.p[cy + (b >> 1)][cx + (b & 1)];
            const TA gg = omk * ph * ph + kap;
            const TA ga0 = TA(gq(q, a, 0)), ga1 = TA(gq(q, a, 1));
            const TA nn = ga0 * ga0 + ga1 * ga1;
            dg[0] += gg * (mu * (nn + ga0 * ga0) + lam * ga0 * ga0);
            dg[1] += gg * (mu * (nn + ga1 * ga1) + lam * ga1 * ga1);
        }
    }
}

// The masked M_uu row of the tile node at (tx, ty) (tx < kTX, ty < kTY) from the cells' LDS
// contributions: vertex 0 of the cell at (tx+1, ty+1), 1 of (tx, ty+1), 2 of (tx+1, ty), 3 of
// (tx, ty).  A Dirichlet row is its diagonal entry times x_r.
template <typename TA, typename TX>
__device__ __forceinline__ void node_row(const MfGrid& g, int64_t i, int64_t j, int64_t r, int tx, int ty,
                                         const Patch<TA>& P, const TX* __restrict__ x, TA y[2]) {
    const bool dir = i == 0 || j == 0 || i == g.nx || j == g.ny;
    if (dir) {
        TA dg[2];
        dirichlet_diag<TA>(g, i, j, tx, ty, P, dg);
        y[0] = dg[0] * TA(x[2 * r]);
        y[1] = dg[1] * TA(x[2 * r + 1]);
        return;
    }
#pragma unroll
    for (int c = 0; c < 2; ++c)
        y[c] = ((P.c[0][c][ty + 1][tx + 1] + P.c[1][c][ty + 1][tx]) + P.c[2][c][ty][tx + 1]) + P.c[3][c][ty][tx];
}

// Tile origin of this workgroup and the node of this thread (valid: inside the tile and mesh).
struct TileNode {
    int64_t i0, j0, i, j, r;
    int tx, ty;
    bool valid;
};

__device__ __forceinline__ TileNode tile_node(const MfGrid& g) {
    TileNode t;
    t.i0 = int64_t(blockIdx.x) * kTX;
    t.j0 = int64_t(blockIdx.y) * kTY;
    t.tx = threadIdx.x % kCX;
    t.ty = threadIdx.x / kCX;
    t.i = t.i0 + t.tx;
    t.j = t.j0 + t.ty;
    t.valid = t.tx < kTX && t.ty < kTY && t.i <= g.nx && t.j <= g.ny;
    t.r = t.i + t.j * g.n1;
    return t;
}

// Chebyshev step of the fine displacement level: r = b - M_uu x_old; d = alpha d + beta D^-1 r;
// x_new = x_old + d (the assembled kernel's update, same order of the update terms).
template <typename T>
__global__ void __launch_bounds__(256) k_mf_cheb(MfGrid g, const T* __restrict__ pt, const T* __restrict__ invd,
                                                 const T* __restrict__ x_old, const T* __restrict__ b,
                                                 T* __restrict__ d, T* __restrict__ x_new, T alpha, T beta) {
    __shared__ Patch<T> P;
    const TileNode t = tile_node(g);
    T bv[2], dv[2], iv[2], xo[2];
    if (t.valid) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            bv[c] = b[2 * t.r + c];
            dv[c] = alpha != T(0) ? d[2 * t.r + c] : T(0);
            iv[c] = invd[2 * t.r + c];
            xo[c] = x_old[2 * t.r + c];
        }
    }
    load_patch<T, T, T>(g, pt, x_old, t.i0, t.j0, P);
    __syncthreads();
    cell_contrib<T>(g, t.i0, t.j0, P);
    __syncthreads();
    if (!t.valid) return;
    T y[2];
    node_row<T, T>(g, t.i, t.j, t.r, t.tx, t.ty, P, x_old, y);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const T res = bv[c] - y[c];
        const T dn = (alpha != T(0) ? alpha * dv[c] : T(0)) + beta * iv[c] * res;
        d[2 * t.r + c] = dn;
        x_new[2 * t.r + c] = xo[c] + dn;
    }
}

// y = b - M_uu x on the fine displacement level
template <typename T>
__global__ void __launch_bounds__(256) k_mf_residual(MfGrid g, const T* __restrict__ pt, const T* __restrict__ x,
                                                     const T* __restrict__ b, T* __restrict__ y) {
    __shared__ Patch<T> P;
    const TileNode t = tile_node(g);
    T bv[2];
    if (t.valid) {
        bv[0] = b[2 * t.r];
        bv[1] = b[2 * t.r + 1];
    }
    load_patch<T, T, T>(g, pt, x, t.i0, t.j0, P);
    __syncthreads();
    cell_contrib<T>(g, t.i0, t.j0, P);
    __syncthreads();
    if (!t.valid) return;
    T acc[2];
    node_row<T, T>(g, t.i, t.j, t.r, t.tx, t.ty, P, x, acc);
    y[2 * t.r] = bv[0] - acc[0];
    y[2 * t.r + 1] = bv[1] - acc[1];
}

// y = J x over the coupled system with the displacement rows matrix-free (FP64 arithmetic; x
// FP64 or FP32 widened exactly) and the phase-field rows M_phiu x_u + M_phiphi x_phi from the
// stored blocks; xcopy (optional) receives the row's own entries of x at the Krylov slot *jp.
template <typename TX, typename CI>
__global__ void __launch_bounds__(256) k_jspmv_mf(MfGrid g, const double* __restrict__ pt, int C,
                                                  const int32_t* __restrict__ slice_ptr, const CI* __restrict__ col,
                                                  const double* __restrict__ pu, const double* __restrict__ pp,
                                                  const TX* __restrict__ x, double* __restrict__ y,
                                                  TX* __restrict__ xcopy, const int* __restrict__ jp,
                                                  int64_t xstride) {
    __shared__ Patch<double> P;
    const TileNode t = tile_node(g);
    const int64_t nf = g.n_nodes;
    const TX* xp = x + 2 * nf;
    double ap = 0.0;
    if (t.valid) {
        const int64_t r = t.r;
        const int64_t s = r / C;
        const int lane = int(r - s * C);
        const int32_t p0 = slice_ptr[s];
        const int w = (slice_ptr[s + 1] - p0) / C;
        int64_t slot = int64_t(p0) + lane;
        for (int k = 0; k < w; ++k, slot += C) {
            const int64_t c = sizeof(CI) == 2 ? r + int64_t(col[slot]) : int64_t(col[slot]);
            const double xu0 = double(x[2 * c]), xu1 = double(x[2 * c + 1]);
            const double xph = double(xp[c]);
            const double* vp = pu + slot * 2;
            ap += vp[0] * xu0;
            ap += vp[1] * xu1;
            ap += pp[slot] * xph;
        }
    }
    load_patch<double, TX, double>(g, pt, x, t.i0, t.j0, P);
    __syncthreads();
    cell_contrib<double>(g, t.i0, t.j0, P);
    __syncthreads();
    if (!t.valid) return;
    const int64_t r = t.r;
    double yu[2];
    node_row<double, TX>(g, t.i, t.j, r, t.tx, t.ty, P, x, yu);
    y[2 * r] = yu[0];
    y[2 * r + 1] = yu[1];
    y[2 * nf + r] = ap;
    if (xcopy) {
        TX* xc = jp ? xcopy + int64_t(*jp) * xstride : xcopy;
        xc[2 * r] = x[2 * r];
        xc[2 * r + 1] = x[2 * r + 1];
        xc[2 * nf + r] = xp[r];
    }
}

__global__ void k_to_f32(const double* __restrict__ a, float* __restrict__ b, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) b[i] = float(a[i]);
}

int grid_for(int64_t n) { return int((n + 255) / 256); }

dim3 tiles(const MfGrid& g) { return dim3(unsigned((g.n1 + kTX - 1) / kTX), unsigned((g.ny + 1 + kTY - 1) / kTY)); }

}  // namespace

bool mf_eligible(const DevMesh& m) {
    return m.on_device && m.dim == 2 && m.n_inst == 1 && !m.hanging && m.host.levels == 0 && m.host.n_hanging == 0;
}

void mf_prepare(DevSystem& sys, const double* pt, hipStream_t s) {
    DevMesh& m = *sys.mesh;
    sys.mf.valid = false;
    if (!mf_eligible(m)) return;
    MfGrid& g = sys.mf.grid;
    g.nx = m.host.desc.base[0];
    g.ny = m.host.desc.base[1];
    g.n1 = g.nx + 1;
    g.n_nodes = m.n_nodes;
    g.mu = sys.prm.mu;
    g.lam = sys.prm.lam;
    g.kappa = sys.prm.kappa;
    if (g.n1 * (g.ny + 1) != m.n_nodes || m.n_free != m.n_nodes) return;
    if ((g.n1 + kTX - 1) / kTX > 65535 || (g.ny + kTY) / kTY > 65535) return;   // tile grid limits
    sys.mf.pt.reserve(size_t(m.n_nodes), s);
    sys.mf.pt32.reserve(size_t(m.n_nodes), s);
    FR_HIP(hipMemcpyAsync(sys.mf.pt.p, pt, size_t(m.n_nodes) * sizeof(double), hipMemcpyDeviceToDevice, s));
    k_to_f32<<<grid_for(m.n_nodes), 256, 0, s>>>(sys.mf.pt.p, sys.mf.pt32.p, m.n_nodes);
    FR_LAUNCH_CHECK();
    sys.mf.valid = true;
}

template <typename T>
static const T* mf_pt(const MfState& mf);
template <>
const double* mf_pt<double>(const MfState& mf) { return mf.pt.p; }
template <>
const float* mf_pt<float>(const MfState& mf) { return mf.pt32.p; }

template <typename T>
void mf_cheb_step(const MfState& mf, const T* invd, const T* x_old, const T* b, T* d, T* x_new, T alpha, T beta,
                  hipStream_t s) {
    const MfGrid& g = mf.grid;
    // x gathered from three node rows (cached), phi_tilde, b, d, D^-1, x_old read; d, x_new written
    const double bytes = double(g.n_nodes) * (sizeof(T) * (2 * 6) + sizeof(T));
    ProfScope ps(sizeof(T) == 8 ? "mf_cheb_f64" : "mf_cheb_f32", s, bytes);
    k_mf_cheb<T><<<tiles(g), 256, 0, s>>>(g, mf_pt<T>(mf), invd, x_old, b, d, x_new, alpha, beta);
    FR_LAUNCH_CHECK();
}

template <typename T>
void mf_residual(const MfState& mf, const T* x, const T* b, T* y, hipStream_t s) {
    const MfGrid& g = mf.grid;
    const double bytes = double(g.n_nodes) * (sizeof(T) * (2 * 3) + sizeof(T));
    ProfScope ps(sizeof(T) == 8 ? "mf_resid_f64" : "mf_resid_f32", s, bytes);
    k_mf_residual<T><<<tiles(g), 256, 0, s>>>(g, mf_pt<T>(mf), x, b, y);
    FR_LAUNCH_CHECK();
}

template <typename TX>
void mf_jspmv(const DevSystem& sys, const TX* x, double* y, TX* xcopy, const int* jp, int64_t xstride,
              hipStream_t s) {
    const MfState& mf = sys.mf;
    const SellStruct& S = *sys.Juu.S;
    const double ib = S.col16 ? 2.0 : 4.0;
    const double bytes = double(S.nnz) * (3 * 8 + ib) + double(S.n_rows) * (3 * (sizeof(TX) + 8) + 8) +
                         (xcopy ? double(S.n_rows) * 3 * sizeof(TX) : 0.0);
    ProfScope ps(sizeof(TX) == 8 ? "jspmv_mf_d2" : "jspmv_mf_d2_x32", s, bytes);
    const dim3 gr = tiles(mf.grid);
    if (S.col16)
        k_jspmv_mf<TX, int16_t><<<gr, 256, 0, s>>>(mf.grid, mf.pt.p, S.C, S.slice_ptr, S.col16, sys.Jpu.val,
                                                   sys.Jpp.val, x, y, xcopy, jp, xstride);
    else
        k_jspmv_mf<TX, int32_t><<<gr, 256, 0, s>>>(mf.grid, mf.pt.p, S.C, S.slice_ptr, S.col, sys.Jpu.val,
                                                   sys.Jpp.val, x, y, xcopy, jp, xstride);
    FR_LAUNCH_CHECK();
}

template void mf_cheb_step<double>(const MfState&, const double*, const double*, const double*, double*, double*,
                                   double, double, hipStream_t);
template void mf_cheb_step<float>(const MfState&, const float*, const float*, const float*, float*, float*, float,
                                  float, hipStream_t);
template void mf_residual<double>(const MfState&, const double*, const double*, double*, hipStream_t);
template void mf_residual<float>(const MfState&, const float*, const float*, float*, hipStream_t);
template void mf_jspmv<double>(const DevSystem&, const double*, double*, double*, const int*, int64_t, hipStream_t);
template void mf_jspmv<float>(const DevSystem&, const float*, double*, float*, const int*, int64_t, hipStream_t);

}  // namespace fr
