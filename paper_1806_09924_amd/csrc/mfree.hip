// Matrix-free application of the fine-level Jacobian blocks of Section 3 ("Linear iterative
// solution") on uniform 2d meshes: M_uu (the block of equation E22ATW in the displacement),
// M_phiphi and M_phiu (the blocks of equation E33ATW in the phase field and the displacement).
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
// FP64 vector rate.  The phase-field rows are applied the same way from the assembly's u and
// phi and its active set (below).
//
// A workgroup works on a 31 x 7 tile of nodes (lexicographic numbering, x fastest): it reads the
// tile's patch of x and of the state once into LDS, computes each of the 32 x 8 cells around the
// tile once (one thread per cell: the Gauss-point quantities and the contributions to the cell's
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

// ---- phase-field rows ------------------------------------------------------------------------
// The phase-field rows of the masked Jacobian at the assembly's state (u_s, phi_s).  Per Gauss
// point q of a cell, with the reference gradients G of u_s and H of x_u, the stress in reference
// units sigma^ = 2 mu sym G + lambda tr G I, and w|J| = h^2 / 4 (the h factors of the physical
// gradients leave or become explicit):
//   M_phiphi x_phi:  x_phi(q) ((1 - kappa) sigma^ : sym G + h p tr G + (h^2 / 4) G_c / eps) N_a(q)
//                    + G_c eps grad^ x_phi(q) . grad^ N_a(q),
//   M_phiu x_u:      phi_s(q) (2 (1 - kappa) sigma^ : H + h p tr H) N_a(q),
// with x_phi zero at active nodes (their columns are eliminated), x_u zero at Dirichlet nodes,
// and an active row replaced by its diagonal entry times x_phi.  The gradient term is the Q1
// stiffness matrix of the reference square (2/3 on the diagonal, -1/6 along an edge, -1/3
// across), which the 2-point rule integrates exactly.
template <typename TA>
struct PPatch {
    TA u[2][kPY][kPX];                           // u_s (every node of the mesh, zero outside)
    TA x[kPY][kPX];                              // x_phi (zero at active nodes and outside)
    TA c[4][kCY][kCX];                           // cell contributions to vertex a
};

template <typename TA, typename TX, typename TU>
__device__ __forceinline__ void load_ppatch(const MfGrid& g, const TU* __restrict__ us, const uint8_t* __restrict__ act,
                                            const TX* __restrict__ xp, int64_t i0, int64_t j0, PPatch<TA>& F) {
    for (int t = threadIdx.x; t < kPX * kPY; t += blockDim.x) {
        const int px = t % kPX, py = t / kPX;
        const int64_t bi = i0 - 1 + px, bj = j0 - 1 + py;
        const bool in = bi >= 0 && bj >= 0 && bi <= g.nx && bj <= g.ny;
        const int64_t nb = bi + bj * g.n1;
        F.u[0][py][px] = in ? TA(us[2 * nb]) : TA(0);
        F.u[1][py][px] = in ? TA(us[2 * nb + 1]) : TA(0);
        F.x[py][px] = (in && act[nb] == 0) ? TA(xp[nb]) : TA(0);
    }
}

// Thread t's cell: its contributions to the phase-field rows of its four vertices (M_phiphi
// x_phi, plus M_phiu x_u when JPU, from the x_u patch xu and the phi_s patch ps).
template <typename TA, bool JPU>
__device__ __forceinline__ void phi_cell(const MfGrid& g, int64_t i0, int64_t j0, PPatch<TA>& F,
                                         const TA (*xu)[kPY][kPX], const TA (*ps)[kPX]) {
    const int cx = threadIdx.x % kCX, cy = threadIdx.x / kCX;
    const int64_t ci = i0 - 1 + cx, cj = j0 - 1 + cy;
    TA out[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) out[a] = TA(0);
    if (ci >= 0 && cj >= 0 && ci < g.nx && cj < g.ny) {
        const TA mu = TA(g.mu), lam = TA(g.lam), omk = TA(1.0 - g.kappa);
        const TA hp = TA(g.h * g.p), gh = TA(0.25 * g.h * g.h * g.Gc / g.eps), ge = TA(g.Gc * g.eps);
        const TA fP = TA(kP), fM = TA(kM), half = TA(0.5);
        TA uv[2][4], xv[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            uv[0][b] = F.u[0][cy + (b >> 1)][cx + (b & 1)];
            uv[1][b] = F.u[1][cy + (b >> 1)][cx + (b & 1)];
            xv[b] = F.x[cy + (b >> 1)][cx + (b & 1)];
        }
        // reference gradients of u_s: Gx[comp][q_y] = d/dxi, Gy[comp][q_x] = d/deta
        TA Gx[2][2], Gy[2][2];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const TA dx0 = uv[c][1] - uv[c][0], dx1 = uv[c][3] - uv[c][2];
            const TA dy0 = uv[c][2] - uv[c][0], dy1 = uv[c][3] - uv[c][1];
            Gx[c][0] = half * (fP * dx0 + fM * dx1);
            Gx[c][1] = half * (fM * dx0 + fP * dx1);
            Gy[c][0] = half * (fP * dy0 + fM * dy1);
            Gy[c][1] = half * (fM * dy0 + fP * dy1);
        }
        // x_phi along x in both vertex rows (then along y per Gauss point)
        TA xr[2][2];
#pragma unroll
        for (int by = 0; by < 2; ++by) {
            xr[by][0] = fP * xv[2 * by] + fM * xv[2 * by + 1];
            xr[by][1] = fM * xv[2 * by] + fP * xv[2 * by + 1];
        }
        TA Hx[2][2], Hy[2][2], pr[2][2];
        if constexpr (JPU) {
            TA wv[2][4], pv[4];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                wv[0][b] = xu[0][cy + (b >> 1)][cx + (b & 1)];
                wv[1][b] = xu[1][cy + (b >> 1)][cx + (b & 1)];
                pv[b] = ps[cy + (b >> 1)][cx + (b & 1)];
            }
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const TA dx0 = wv[c][1] - wv[c][0], dx1 = wv[c][3] - wv[c][2];
                const TA dy0 = wv[c][2] - wv[c][0], dy1 = wv[c][3] - wv[c][1];
                Hx[c][0] = half * (fP * dx0 + fM * dx1);
                Hx[c][1] = half * (fM * dx0 + fP * dx1);
                Hy[c][0] = half * (fP * dy0 + fM * dy1);
                Hy[c][1] = half * (fM * dy0 + fP * dy1);
            }
#pragma unroll
            for (int by = 0; by < 2; ++by) {
                pr[by][0] = fP * pv[2 * by] + fM * pv[2 * by + 1];
                pr[by][1] = fM * pv[2 * by] + fP * pv[2 * by + 1];
            }
        }
        TA v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int qx = q & 1, qy = q >> 1;
            const TA X = qy ? fM * xr[0][qx] + fP * xr[1][qx] : fP * xr[0][qx] + fM * xr[1][qx];
            const TA g00 = Gx[0][qy], g11 = Gy[1][qx], g01 = Gy[0][qx] + Gx[1][qy];   // g01: twice sym G[0][1]
            const TA tr = g00 + g11;
            const TA s00 = TA(2) * mu * g00 + lam * tr, s11 = TA(2) * mu * g11 + lam * tr, s01 = mu * g01;
            const TA se = s00 * g00 + s11 * g11 + s01 * g01;                          // sigma^ : sym G
            TA vq = (omk * se + hp * tr + gh) * X;
            if constexpr (JPU) {
                const TA ph = qy ? fM * pr[0][qx] + fP * pr[1][qx] : fP * pr[0][qx] + fM * pr[1][qx];
                const TA h00 = Hx[0][qy], h11 = Hy[1][qx], h01 = Hy[0][qx] + Hx[1][qy];
                const TA sh = s00 * h00 + s11 * h11 + s01 * h01;                      // sigma^ : H
                vq += ph * (TA(2) * omk * sh + hp * (h00 + h11));
            }
            v[q] = vq;
        }
        // sum over q of N_a(q) v_q, N_a(q) = f(a_x, q_x) f(a_y, q_y): along x, then along y
        TA V[2][2];
#pragma unroll
        for (int qy = 0; qy < 2; ++qy) {
            V[qy][0] = fP * v[2 * qy] + fM * v[2 * qy + 1];
            V[qy][1] = fM * v[2 * qy] + fP * v[2 * qy + 1];
        }
        const TA k0 = TA(2.0 / 3.0), k1 = TA(1.0 / 6.0), k3 = TA(1.0 / 3.0);
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const int ax = a & 1, ay = a >> 1;
            const TA m = ay ? fM * V[0][ax] + fP * V[1][ax] : fP * V[0][ax] + fM * V[1][ax];
            out[a] = m + ge * (k0 * xv[a] - k1 * (xv[a ^ 1] + xv[a ^ 2]) - k3 * xv[a ^ 3]);
        }
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) F.c[a][cy][cx] = out[a];
}

// The phase-field row of the tile node at (tx, ty) from its four cells' contributions.
template <typename TA>
__device__ __forceinline__ TA phi_row(const PPatch<TA>& F, int tx, int ty) {
    return ((F.c[0][ty + 1][tx + 1] + F.c[1][ty + 1][tx]) + F.c[2][ty][tx + 1]) + F.c[3][ty][tx];
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

// Chebyshev step of the fine phase-field level (M_phiphi, masked), as k_mf_cheb.
template <typename T>
__global__ void __launch_bounds__(256) k_mf_pcheb(MfGrid g, const T* __restrict__ us, const uint8_t* __restrict__ act,
                                                  const T* __restrict__ dpp, const T* __restrict__ invd,
                                                  const T* __restrict__ x_old, const T* __restrict__ b,
                                                  T* __restrict__ d, T* __restrict__ x_new, T alpha, T beta) {
    __shared__ PPatch<T> F;
    const TileNode t = tile_node(g);
    T bv = T(0), dv = T(0), iv = T(0), xo = T(0);
    bool on = false;
    if (t.valid) {
        bv = b[t.r];
        dv = alpha != T(0) ? d[t.r] : T(0);
        iv = invd[t.r];
        xo = x_old[t.r];
        on = act[t.r] != 0;
    }
    load_ppatch<T, T, T>(g, us, act, x_old, t.i0, t.j0, F);
    __syncthreads();
    phi_cell<T, false>(g, t.i0, t.j0, F, nullptr, nullptr);
    __syncthreads();
    if (!t.valid) return;
    const T y = on ? dpp[t.r] * xo : phi_row<T>(F, t.tx, t.ty);
    const T res = bv - y;
    const T dn = (alpha != T(0) ? alpha * dv : T(0)) + beta * iv * res;
    d[t.r] = dn;
    x_new[t.r] = xo + dn;
}

// y = b - M_phiphi x on the fine phase-field level
template <typename T>
__global__ void __launch_bounds__(256) k_mf_presidual(MfGrid g, const T* __restrict__ us,
                                                      const uint8_t* __restrict__ act, const T* __restrict__ dpp,
                                                      const T* __restrict__ x, const T* __restrict__ b,
                                                      T* __restrict__ y) {
    __shared__ PPatch<T> F;
    const TileNode t = tile_node(g);
    T bv = T(0), xo = T(0);
    bool on = false;
    if (t.valid) {
        bv = b[t.r];
        xo = x[t.r];
        on = act[t.r] != 0;
    }
    load_ppatch<T, T, T>(g, us, act, x, t.i0, t.j0, F);
    __syncthreads();
    phi_cell<T, false>(g, t.i0, t.j0, F, nullptr, nullptr);
    __syncthreads();
    if (!t.valid) return;
    y[t.r] = bv - (on ? dpp[t.r] * xo : phi_row<T>(F, t.tx, t.ty));
}

// y = J x with every row matrix-free: the displacement rows as in k_jspmv_mf, the phase-field
// rows M_phiu x_u + M_phiphi x_phi from u_s, phi_s and the active set (FP64 arithmetic, x FP64
// or FP32 widened exactly); xcopy (optional) receives the row's own entries of x at *jp.
template <typename TX>
__global__ void __launch_bounds__(256) k_jspmv_mf_all(MfGrid g, const double* __restrict__ pt,
                                                      const double* __restrict__ us, const double* __restrict__ ps,
                                                      const uint8_t* __restrict__ act, const double* __restrict__ dpp,
                                                      const TX* __restrict__ x, double* __restrict__ y,
                                                      TX* __restrict__ xcopy, const int* __restrict__ jp,
                                                      int64_t xstride) {
    __shared__ Patch<double> P;
    __shared__ PPatch<double> F;
    __shared__ double S[kPY][kPX];
    const TileNode t = tile_node(g);
    const int64_t nf = g.n_nodes;
    const TX* xp = x + 2 * nf;
    for (int k = threadIdx.x; k < kPX * kPY; k += blockDim.x) {
        const int px = k % kPX, py = k / kPX;
        const int64_t bi = t.i0 - 1 + px, bj = t.j0 - 1 + py;
        const bool in = bi >= 0 && bj >= 0 && bi <= g.nx && bj <= g.ny;
        const bool interior = bi > 0 && bj > 0 && bi < g.nx && bj < g.ny;
        const int64_t nb = bi + bj * g.n1;
        P.p[py][px] = in ? pt[nb] : 0.0;
        P.x[0][py][px] = interior ? double(x[2 * nb]) : 0.0;
        P.x[1][py][px] = interior ? double(x[2 * nb + 1]) : 0.0;
        F.u[0][py][px] = in ? us[2 * nb] : 0.0;
        F.u[1][py][px] = in ? us[2 * nb + 1] : 0.0;
        F.x[py][px] = (in && act[nb] == 0) ? double(xp[nb]) : 0.0;
        S[py][px] = in ? ps[nb] : 0.0;
    }
    __syncthreads();
    cell_contrib<double>(g, t.i0, t.j0, P);
    phi_cell<double, true>(g, t.i0, t.j0, F, P.x, S);
    __syncthreads();
    if (!t.valid) return;
    const int64_t r = t.r;
    double yu[2];
    node_row<double, TX>(g, t.i, t.j, r, t.tx, t.ty, P, x, yu);
    y[2 * r] = yu[0];
    y[2 * r + 1] = yu[1];
    y[2 * nf + r] = act[r] != 0 ? dpp[r] * double(xp[r]) : phi_row<double>(F, t.tx, t.ty);
    if (xcopy) {
        TX* xc = jp ? xcopy + int64_t(*jp) * xstride : xcopy;
        xc[2 * r] = x[2 * r];
        xc[2 * r + 1] = x[2 * r + 1];
        xc[2 * nf + r] = xp[r];
    }
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

// Diagonal of the stored (masked) M_phiphi: the row's entry in its own column (the first such
// slot among the row's entries; padding slots follow them), in FP64 and FP32.
template <typename CI>
__global__ void k_diag_pp(int64_t n, int C, const int32_t* __restrict__ sp, const int32_t* __restrict__ len,
                          const CI* __restrict__ col, const double* __restrict__ pp, double* __restrict__ d,
                          float* __restrict__ d32) {
    const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int64_t s0 = r / C;
    const int lane = int(r - s0 * C);
    int64_t slot = int64_t(sp[s0]) + lane;
    double v = 0.0;
    for (int k = 0; k < len[r]; ++k, slot += C) {
        const int64_t c = sizeof(CI) == 2 ? r + int64_t(col[slot]) : int64_t(col[slot]);
        if (c == r) {
            v = pp[slot];
            break;
        }
    }
    d[r] = v;
    d32[r] = float(v);
}

int grid_for(int64_t n) { return int((n + 255) / 256); }

dim3 tiles(const MfGrid& g) { return dim3(unsigned((g.n1 + kTX - 1) / kTX), unsigned((g.ny + 1 + kTY - 1) / kTY)); }

}  // namespace

bool mf_eligible(const DevMesh& m) {
    return m.on_device && m.dim == 2 && m.n_inst == 1 && !m.hanging && m.host.levels == 0 && m.host.n_hanging == 0;
}

void mf_prepare(DevSystem& sys, const double* u, const double* phi, const double* pt, hipStream_t s) {
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
    g.h = m.host.h_min;
    g.p = sys.prm.p;
    g.Gc = sys.prm.Gc;
    g.eps = sys.prm.eps;
    if (g.n1 * (g.ny + 1) != m.n_nodes || m.n_free != m.n_nodes) return;
    if ((g.n1 + kTX - 1) / kTX > 65535 || (g.ny + kTY) / kTY > 65535) return;   // tile grid limits
    const int64_t n = m.n_nodes;
    MfState& f = sys.mf;
    f.pt.reserve(size_t(n), s);
    f.pt32.reserve(size_t(n), s);
    f.us.reserve(size_t(2 * n), s);
    f.us32.reserve(size_t(2 * n), s);
    f.ps.reserve(size_t(n), s);
    f.act.reserve(size_t(n), s);
    f.dpp.reserve(size_t(n), s);
    f.dpp32.reserve(size_t(n), s);
    FR_HIP(hipMemcpyAsync(f.pt.p, pt, size_t(n) * sizeof(double), hipMemcpyDeviceToDevice, s));
    FR_HIP(hipMemcpyAsync(f.us.p, u, size_t(2 * n) * sizeof(double), hipMemcpyDeviceToDevice, s));
    FR_HIP(hipMemcpyAsync(f.ps.p, phi, size_t(n) * sizeof(double), hipMemcpyDeviceToDevice, s));
    FR_HIP(hipMemcpyAsync(f.act.p, sys.active.p, size_t(n), hipMemcpyDeviceToDevice, s));
    k_to_f32<<<grid_for(n), 256, 0, s>>>(f.pt.p, f.pt32.p, n);
    k_to_f32<<<grid_for(2 * n), 256, 0, s>>>(f.us.p, f.us32.p, 2 * n);
    const SellStruct& S = *sys.Jpp.S;
    if (S.col16)
        k_diag_pp<int16_t><<<grid_for(n), 256, 0, s>>>(n, S.C, S.slice_ptr, S.row_len, S.col16, sys.Jpp.val, f.dpp.p,
                                                        f.dpp32.p);
    else
        k_diag_pp<int32_t><<<grid_for(n), 256, 0, s>>>(n, S.C, S.slice_ptr, S.row_len, S.col, sys.Jpp.val, f.dpp.p,
                                                        f.dpp32.p);
    FR_LAUNCH_CHECK();
    f.valid = true;
}

template <typename T>
static const T* mf_pt(const MfState& mf);
template <>
const double* mf_pt<double>(const MfState& mf) { return mf.pt.p; }
template <>
const float* mf_pt<float>(const MfState& mf) { return mf.pt32.p; }
template <typename T>
static const T* mf_us(const MfState& mf);
template <>
const double* mf_us<double>(const MfState& mf) { return mf.us.p; }
template <>
const float* mf_us<float>(const MfState& mf) { return mf.us32.p; }
template <typename T>
static const T* mf_dpp(const MfState& mf);
template <>
const double* mf_dpp<double>(const MfState& mf) { return mf.dpp.p; }
template <>
const float* mf_dpp<float>(const MfState& mf) { return mf.dpp32.p; }

template <typename T>
void mf_cheb_step(const MfState& mf, int blk, const T* invd, const T* x_old, const T* b, T* d, T* x_new, T alpha,
                  T beta, hipStream_t s) {
    const MfGrid& g = mf.grid;
    const bool f64 = sizeof(T) == 8;
    if (blk == 0) {
        // x gathered from three node rows (cached), phi_tilde, b, d, D^-1, x_old read; d, x_new written
        const double bytes = double(g.n_nodes) * (sizeof(T) * (2 * 6) + sizeof(T));
        ProfScope ps(f64 ? "mf_cheb_f64" : "mf_cheb_f32", s, bytes);
        k_mf_cheb<T><<<tiles(g), 256, 0, s>>>(g, mf_pt<T>(mf), invd, x_old, b, d, x_new, alpha, beta);
    } else {
        // u_s (two words), the active flag, x_old, b, d, D^-1 read; d, x_new written
        const double bytes = double(g.n_nodes) * (sizeof(T) * 8 + 1);
        ProfScope ps(f64 ? "mf_pcheb_f64" : "mf_pcheb_f32", s, bytes);
        k_mf_pcheb<T><<<tiles(g), 256, 0, s>>>(g, mf_us<T>(mf), mf.act.p, mf_dpp<T>(mf), invd, x_old, b, d, x_new,
                                               alpha, beta);
    }
    FR_LAUNCH_CHECK();
}

template <typename T>
void mf_residual(const MfState& mf, int blk, const T* x, const T* b, T* y, hipStream_t s) {
    const MfGrid& g = mf.grid;
    const bool f64 = sizeof(T) == 8;
    if (blk == 0) {
        const double bytes = double(g.n_nodes) * (sizeof(T) * (2 * 3) + sizeof(T));
        ProfScope ps(f64 ? "mf_resid_f64" : "mf_resid_f32", s, bytes);
        k_mf_residual<T><<<tiles(g), 256, 0, s>>>(g, mf_pt<T>(mf), x, b, y);
    } else {
        const double bytes = double(g.n_nodes) * (sizeof(T) * 5 + 1);
        ProfScope ps(f64 ? "mf_presid_f64" : "mf_presid_f32", s, bytes);
        k_mf_presidual<T><<<tiles(g), 256, 0, s>>>(g, mf_us<T>(mf), mf.act.p, mf_dpp<T>(mf), x, b, y);
    }
    FR_LAUNCH_CHECK();
}

template <typename TX>
void mf_jspmv(const DevSystem& sys, bool phi_rows, const TX* x, double* y, TX* xcopy, const int* jp, int64_t xstride,
              hipStream_t s) {
    const MfState& mf = sys.mf;
    const dim3 gr = tiles(mf.grid);
    const bool x64 = sizeof(TX) == 8;
    const double nn = double(mf.grid.n_nodes);
    if (phi_rows) {
        // phi_tilde, u_s, phi_s, the active flag and x read, y (and the copy of x) written
        const double bytes = nn * (8 + 16 + 8 + 1 + 3 * sizeof(TX) + 24) + (xcopy ? nn * 3 * sizeof(TX) : 0.0);
        ProfScope ps(x64 ? "jspmv_mf_all_d2" : "jspmv_mf_all_d2_x32", s, bytes);
        k_jspmv_mf_all<TX><<<gr, 256, 0, s>>>(mf.grid, mf.pt.p, mf.us.p, mf.ps.p, mf.act.p, mf.dpp.p, x, y, xcopy, jp,
                                               xstride);
        FR_LAUNCH_CHECK();
        return;
    }
    const SellStruct& S = *sys.Juu.S;
    const double ib = S.col16 ? 2.0 : 4.0;
    const double bytes = double(S.nnz) * (3 * 8 + ib) + double(S.n_rows) * (3 * (sizeof(TX) + 8) + 8) +
                         (xcopy ? double(S.n_rows) * 3 * sizeof(TX) : 0.0);
    ProfScope ps(x64 ? "jspmv_mf_d2" : "jspmv_mf_d2_x32", s, bytes);
    if (S.col16)
        k_jspmv_mf<TX, int16_t><<<gr, 256, 0, s>>>(mf.grid, mf.pt.p, S.C, S.slice_ptr, S.col16, sys.Jpu.val,
                                                   sys.Jpp.val, x, y, xcopy, jp, xstride);
    else
        k_jspmv_mf<TX, int32_t><<<gr, 256, 0, s>>>(mf.grid, mf.pt.p, S.C, S.slice_ptr, S.col, sys.Jpu.val,
                                                   sys.Jpp.val, x, y, xcopy, jp, xstride);
    FR_LAUNCH_CHECK();
}

template void mf_cheb_step<double>(const MfState&, int, const double*, const double*, const double*, double*, double*,
                                   double, double, hipStream_t);
template void mf_cheb_step<float>(const MfState&, int, const float*, const float*, const float*, float*, float*,
                                  float, float, hipStream_t);
template void mf_residual<double>(const MfState&, int, const double*, const double*, double*, hipStream_t);
template void mf_residual<float>(const MfState&, int, const float*, const float*, float*, hipStream_t);
template void mf_jspmv<double>(const DevSystem&, bool, const double*, double*, double*, const int*, int64_t,
                               hipStream_t);
template void mf_jspmv<float>(const DevSystem&, bool, const float*, double*, float*, const int*, int64_t, hipStream_t);

}  // namespace fr
