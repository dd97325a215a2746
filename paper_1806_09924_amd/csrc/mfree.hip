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
// Each wave streams up a strip of node columns (lexicographic numbering, x fastest): one lane per
// node column, one node row after the other.  A lane reads its node of the row (coalesced across
// the wave), takes its right neighbour's values by a lane shuffle, computes the cell above-right
// of its node (the Gauss-point quantities and the contributions to the cell's four vertices), and
// sums its node's row from its own cell, the left lane's cell (shuffled) and the two cells of the
// row below (kept from the previous step).  No LDS and no barrier: the next row's loads are
// issued before the current row's arithmetic, so they are in flight while it runs.
#include "profile.h"
#include "system.h"

namespace fr {
namespace {

// 1d Q1 factors at the 2-point Gauss abscissae: (1 +- 1/sqrt(3)) / 2
constexpr double kP = 0.78867513459481288225;
constexpr double kM = 0.21132486540518711775;

// dN_b / dxi_k at Gauss point q on the reference square [-1, 1]^2 (bit k of b / q: upper side
// along axis k)
__device__ __forceinline__ constexpr double gq(int q, int b, int k) {
    const int o = 1 - k;   // the other axis
    return (((b >> k) & 1) ? 0.5 : -0.5) * (((b >> o) & 1) == ((q >> o) & 1) ? kP : kM);
}

// ---- cells ------------------------------------------------------------------------------------
// Vertex values in registers, vertex b = 0 (lower left), 1 (lower right), 2 (upper left), 3 (upper
// right).  The tensor-product structure of Q1 with 2 x 2 Gauss points is used: with f(b, q) = kP
// when the vertex and the Gauss point lie on the same side of the axis (else kM),
//   d/dxi of x at Gauss point q  = (f(0, q_y) (x_1 - x_0) + f(1, q_y) (x_3 - x_2)) / 2,
//   d/deta                       = (f(0, q_x) (x_2 - x_0) + f(1, q_x) (x_3 - x_1)) / 2,
// and a sum over q of N_a(q) v_q or of grad N_a(q) . s_q factors along the two axes.

// Reference gradients of a vertex field: Hx[comp][q_y] = d/dxi, Hy[comp][q_x] = d/deta.
template <typename TA>
__device__ __forceinline__ void ref_grad(const TA (&v)[2][4], TA (&Hx)[2][2], TA (&Hy)[2][2]) {
    const TA fP = TA(kP), fM = TA(kM), half = TA(0.5);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const TA dx0 = v[c][1] - v[c][0], dx1 = v[c][3] - v[c][2];
        const TA dy0 = v[c][2] - v[c][0], dy1 = v[c][3] - v[c][1];
        Hx[c][0] = half * (fP * dx0 + fM * dx1);
        Hx[c][1] = half * (fM * dx0 + fP * dx1);
        Hy[c][0] = half * (fP * dy0 + fM * dy1);
        Hy[c][1] = half * (fM * dy0 + fP * dy1);
    }
}

// A vertex scalar along x in both vertex rows: r[b_y][q_x] (then along y per Gauss point).
template <typename TA>
__device__ __forceinline__ void along_x(const TA (&v)[4], TA (&r)[2][2]) {
    const TA fP = TA(kP), fM = TA(kM);
#pragma unroll
    for (int by = 0; by < 2; ++by) {
        r[by][0] = fP * v[2 * by] + fM * v[2 * by + 1];
        r[by][1] = fM * v[2 * by] + fP * v[2 * by + 1];
    }
}
template <typename TA>
__device__ __forceinline__ TA at_q(const TA (&r)[2][2], int qx, int qy) {
    const TA fP = TA(kP), fM = TA(kM);
    return qy ? fM * r[0][qx] + fP * r[1][qx] : fP * r[0][qx] + fM * r[1][qx];
}

// Displacement block: a cell's contributions to its vertices' rows of M_uu x (Hx, Hy: the
// reference gradients of x, zero at the Dirichlet nodes), sum over the Gauss points of
// g_q sigma_q(x) grad N_a(q), and the Gauss-point degradations g_q = (1 - kappa) phi_tilde_q^2 + kappa.  The vertex contributions need only the
// stresses summed along one axis: c_(a, comp) = s_x(a) X_comp[a_y] + s_y(a) Y_comp[a_x],
// X_comp[a_y] = (f(a_y, 0) Sx_comp[0] + f(a_y, 1) Sx_comp[1]) / 2, Sx_comp[q_y] = sum over q_x of
// sigma[comp][0], and Y the same along the other axis with sigma[comp][1].
template <typename TA>
__device__ __forceinline__ void cell_u(const MfGrid& g, const TA (&Hx)[2][2], const TA (&Hy)[2][2], const TA (&pv)[4],
                                       TA (&out)[4][2], TA (&gg)[4]) {
    const TA mu = TA(g.mu), lam = TA(g.lam), kap = TA(g.kappa), omk = TA(1.0 - g.kappa);
    const TA fP = TA(kP), fM = TA(kM), half = TA(0.5);
    TA pr[2][2];
    along_x<TA>(pv, pr);
    TA Sx[2][2] = {{TA(0), TA(0)}, {TA(0), TA(0)}}, Sy[2][2] = {{TA(0), TA(0)}, {TA(0), TA(0)}};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int qx = q & 1, qy = q >> 1;
        const TA ph = at_q<TA>(pr, qx, qy);
        gg[q] = omk * ph * ph + kap;
        const TA h00 = Hx[0][qy], h01 = Hy[0][qx], h10 = Hx[1][qy], h11 = Hy[1][qx];
        const TA tr = h00 + h11;
        const TA s00 = gg[q] * (TA(2) * mu * h00 + lam * tr);
        const TA s11 = gg[q] * (TA(2) * mu * h11 + lam * tr);
        const TA s01 = gg[q] * (mu * (h01 + h10));
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

// A cell's part of the original diagonal entries of its vertices' two rows (what a Dirichlet row
// keeps): sum over q of g_q (mu (|grad N_a|^2 + (d_c N_a)^2) + lambda (d_c N_a)^2).
template <typename TA>
__device__ __forceinline__ void cell_u_diag(const MfGrid& g, const TA (&gg)[4], TA (&dg)[4][2]) {
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        dg[a][0] = dg[a][1] = TA(0);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double ga0 = gq(q, a, 0), ga1 = gq(q, a, 1), nn = ga0 * ga0 + ga1 * ga1;
            dg[a][0] += gg[q] * TA(g.mu * (nn + ga0 * ga0) + g.lam * ga0 * ga0);
            dg[a][1] += gg[q] * TA(g.mu * (nn + ga1 * ga1) + g.lam * ga1 * ga1);
        }
    }
}

// Phase-field rows of the masked Jacobian at the assembly's state (u_s, phi_s).  Per Gauss point
// q, with the reference gradients G of u_s and H of x_u, the stress in reference units
// sigma^ = 2 mu sym G + lambda tr G I, and w|J| = h^2 / 4 (the h factors of the physical
// gradients leave or become explicit):
//   M_phiphi x_phi:  x_phi(q) ((1 - kappa) sigma^ : sym G + h p tr G + (h^2 / 4) G_c / eps) N_a(q)
//                    + G_c eps grad^ x_phi(q) . grad^ N_a(q),
//   M_phiu x_u:      phi_s(q) (2 (1 - kappa) sigma^ : H + h p tr H) N_a(q),
// with x_phi zero at active nodes (their columns are eliminated), x_u zero at Dirichlet nodes,
// and an active row replaced by its diagonal entry times x_phi.  The gradient term is the Q1
// stiffness matrix of the reference square (2/3 on the diagonal, -1/6 along an edge, -1/3
// across), which the 2-point rule integrates exactly.  JPU adds the M_phiu part (Hx, Hy: the
// reference gradients of x_u; pv: phi_s).
template <typename TA, bool JPU>
__device__ __forceinline__ void cell_phi(const MfGrid& g, const TA (&uv)[2][4], const TA (&xv)[4], const TA (&Hx)[2][2],
                                         const TA (&Hy)[2][2], const TA (&pv)[4], TA (&out)[4]) {
    const TA mu = TA(g.mu), lam = TA(g.lam), omk = TA(1.0 - g.kappa);
    const TA hp = TA(g.h * g.p), gh = TA(0.25 * g.h * g.h * g.Gc / g.eps), ge = TA(g.Gc * g.eps);
    const TA fP = TA(kP), fM = TA(kM);
    TA Gx[2][2], Gy[2][2], xr[2][2];
    ref_grad<TA>(uv, Gx, Gy);
    along_x<TA>(xv, xr);
    TA pr[2][2];
    if constexpr (JPU) along_x<TA>(pv, pr);
    TA v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int qx = q & 1, qy = q >> 1;
        const TA X = at_q<TA>(xr, qx, qy);
        const TA g00 = Gx[0][qy], g11 = Gy[1][qx], g01 = Gy[0][qx] + Gx[1][qy];   // g01: twice sym G[0][1]
        const TA tr = g00 + g11;
        const TA s00 = TA(2) * mu * g00 + lam * tr, s11 = TA(2) * mu * g11 + lam * tr, s01 = mu * g01;
        const TA se = s00 * g00 + s11 * g11 + s01 * g01;                          // sigma^ : sym G
        TA vq = (omk * se + hp * tr + gh) * X;
        if constexpr (JPU) {
            const TA ph = at_q<TA>(pr, qx, qy);
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

// ---- wave strips ------------------------------------------------------------------------------
// A wave's lanes take the node columns s*kSW - 1 .. s*kSW + 62 of strip s; lane l computes the cell
// whose lower-left vertex is its node (lanes 0..62) and writes its node's rows (lanes 1..kSW), for
// the node rows of band b, [b*kBand, (b+1)*kBand).  Lane 0's cell feeds lane 1, lane 63's node
// is the right vertex of lane 62's cell.
constexpr int kWaveLanes = 64;
constexpr int kSW = kWaveLanes - 2;              // node columns a wave writes
constexpr int kBand = 16;                        // node rows a wave writes

struct WaveStrip {
    int64_t col, j0, j1;                         // the lane's node column; node rows written [j0, j1)
    int lane;
    bool valid, writer;
    bool col_in, col_int;                        // column inside the mesh / not on its left or right edge
};

__device__ __forceinline__ int64_t n_strips(const MfGrid& g) { return (g.n1 + kSW - 1) / kSW; }
__device__ __forceinline__ int64_t n_bands(const MfGrid& g) { return (g.ny + kBand) / kBand; }

__device__ __forceinline__ WaveStrip wave_strip(const MfGrid& g) {
    WaveStrip w;
    w.lane = int(threadIdx.x % kWaveLanes);
    const int64_t wv = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / kWaveLanes;
    const int64_t ns = n_strips(g);
    w.valid = wv < ns * n_bands(g);
    const int64_t s = wv % ns, b = wv / ns;
    w.col = s * kSW - 1 + w.lane;
    w.j0 = b * kBand;
    w.j1 = w.j0 + kBand < g.ny + 1 ? w.j0 + kBand : g.ny + 1;
    w.col_in = w.col >= 0 && w.col <= g.nx;
    w.col_int = w.col > 0 && w.col < g.nx;
    w.writer = w.valid && w.lane >= 1 && w.lane <= kSW && w.col <= g.nx;
    return w;
}

// the value of the lane to the right / left (the wave's last / first lane gets its own)
template <typename TA>
__device__ __forceinline__ TA from_right(TA v) { return __shfl_down(v, 1, kWaveLanes); }
template <typename TA>
__device__ __forceinline__ TA from_left(TA v) { return __shfl_up(v, 1, kWaveLanes); }

__device__ __forceinline__ bool cell_at(const MfGrid& g, const WaveStrip& w, int64_t j) {
    return w.lane < kWaveLanes - 1 && w.col >= 0 && w.col < g.nx && j >= 0 && j < g.ny;
}
__device__ __forceinline__ bool row_in(const MfGrid& g, int64_t j) { return j >= 0 && j <= g.ny; }
__device__ __forceinline__ bool dirichlet(const MfGrid& g, int64_t i, int64_t j) {
    return i == 0 || j == 0 || i == g.nx || j == g.ny;
}

// The displacement rows of a cell row: each lane's cell (Hx, Hy from masked_grad; the Dirichlet
// vertices' contributions replaced by their diagonal parts), then this lane's node of
// the bottom row: ((own cell + left cell) + own cell below + left cell below), the last two
// carried in c2 / c3 from the previous row.  Returns, for the Dirichlet node, the sum of the
// diagonal parts (the caller multiplies by x).
// Reference gradients over this lane's cell of x_u masked at the Dirichlet nodes (rows j, j + 1).
template <typename TA>
__device__ __forceinline__ void masked_grad(const MfGrid& g, const WaveStrip& w, int64_t j, const TA (&xB)[2],
                                            const TA (&xT)[2], TA (&Hx)[2][2], TA (&Hy)[2][2]) {
    const bool iB = w.col_int && j > 0 && j < g.ny, iT = w.col_int && j + 1 > 0 && j + 1 < g.ny;
    TA xv[2][4];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        xv[c][0] = iB ? xB[c] : TA(0);
        xv[c][2] = iT ? xT[c] : TA(0);
        xv[c][1] = from_right(xv[c][0]);
        xv[c][3] = from_right(xv[c][2]);
    }
    ref_grad<TA>(xv, Hx, Hy);
}

template <typename TA>
__device__ __forceinline__ void u_rows(const MfGrid& g, const WaveStrip& w, int64_t j, const TA (&Hx)[2][2],
                                       const TA (&Hy)[2][2], TA pB, TA pT, TA (&c2)[2], TA (&c3)[2], TA (&y)[2]) {
    TA pv[4];
    pv[0] = pB;
    pv[2] = pT;
    pv[1] = from_right(pB);
    pv[3] = from_right(pT);
    TA out[4][2];
#pragma unroll
    for (int a = 0; a < 4; ++a) out[a][0] = out[a][1] = TA(0);
    if (cell_at(g, w, j)) {
        TA gg[4];
        cell_u<TA>(g, Hx, Hy, pv, out, gg);
        if (w.col == 0 || w.col == g.nx - 1 || j == 0 || j == g.ny - 1) {
            TA dg[4][2];
            cell_u_diag<TA>(g, gg, dg);
#pragma unroll
            for (int a = 0; a < 4; ++a)
                if (dirichlet(g, w.col + (a & 1), j + (a >> 1))) {
                    out[a][0] = dg[a][0];
                    out[a][1] = dg[a][1];
                }
        }
    }
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const TA c1 = from_left(out[1][c]), c3n = from_left(out[3][c]);
        y[c] = ((out[0][c] + c1) + c2[c]) + c3[c];
        c2[c] = out[2][c];
        c3[c] = c3n;
    }
}

// The phase-field rows of a cell row, as u_rows (JPU: with M_phiu x_u from the gradients Hx, Hy
// of masked_grad and phi_s).
template <typename TA, bool JPU>
__device__ __forceinline__ TA phi_rows(const MfGrid& g, const WaveStrip& w, int64_t j, const TA (&uB)[2],
                                       const TA (&uT)[2], TA xB, TA xT, const TA (&Hx)[2][2], const TA (&Hy)[2][2],
                                       TA psB, TA psT, TA& c2, TA& c3) {
    TA uv[2][4], xv[4], pv[4];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        uv[c][0] = uB[c];
        uv[c][2] = uT[c];
        uv[c][1] = from_right(uB[c]);
        uv[c][3] = from_right(uT[c]);
    }
    xv[0] = xB;
    xv[2] = xT;
    xv[1] = from_right(xB);
    xv[3] = from_right(xT);
    if constexpr (JPU) {
        pv[0] = psB;
        pv[2] = psT;
        pv[1] = from_right(psB);
        pv[3] = from_right(psT);
    }
    TA out[4] = {TA(0), TA(0), TA(0), TA(0)};
    if (cell_at(g, w, j)) cell_phi<TA, JPU>(g, uv, xv, Hx, Hy, pv, out);
    const TA c1 = from_left(out[1]), c3n = from_left(out[3]);
    const TA y = ((out[0] + c1) + c2) + c3;
    c2 = out[2];
    c3 = c3n;
    return y;
}

// Chebyshev step of the fine displacement level: r = b - M_uu x_old; d = alpha d + beta D^-1 r;
// x_new = x_old + d (the assembled kernel's update, same order of the update terms).  MODE 1: a
// power step of the smoother bounds instead, d = D^-1 M_uu x_old (b and x_new untouched).
// MODE 2: the first two steps from x = 0 in one pass: x_old = d = beta0 D^-1 b (the first step,
// formed per node from b and D^-1 exactly as the separate first-step kernel forms it), then the
// step above (x_old is not read).
template <typename T, int MODE = 0>
__global__ void __launch_bounds__(256) k_mf_cheb(MfGrid g, const T* __restrict__ pt, const T* __restrict__ invd,
                                                 const T* __restrict__ x_old, const T* __restrict__ b,
                                                 T* __restrict__ d, T* __restrict__ x_new, T alpha, T beta,
                                                 T beta0 = T(0)) {
    constexpr bool POW = MODE == 1;
    const WaveStrip w = wave_strip(g);
    if (!w.valid) return;
    // MODE 2 keeps each row's b and D^-1 from its load (the row is written two steps later)
    auto ld = [&](int64_t j, T& p, T (&x)[2], T (&bb)[2], T (&ii)[2]) {
        const bool in = w.col_in && row_in(g, j);
        const int64_t r = w.col + j * g.n1;
        p = in ? pt[r] : T(0);
        if (MODE == 2) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                bb[c] = in ? b[2 * r + c] : T(0);
                ii[c] = in ? invd[2 * r + c] : T(0);
                x[c] = beta0 * ii[c] * bb[c];
            }
        } else {
            x[0] = in ? x_old[2 * r] : T(0);
            x[1] = in ? x_old[2 * r + 1] : T(0);
        }
    };
    T pB, pT, xB[2], xT[2], c2[2] = {T(0), T(0)}, c3[2] = {T(0), T(0)};
    T bB[2], bT[2], iB[2], iT[2];
    ld(w.j0 - 1, pB, xB, bB, iB);
    ld(w.j0, pT, xT, bT, iT);
    for (int64_t j = w.j0 - 1; j < w.j1; ++j) {
        T pN, xN[2], bN[2], iN[2];
        ld(j + 2, pN, xN, bN, iN);
        const bool wr = w.writer && j >= w.j0;
        const int64_t r = w.col + j * g.n1;
        T bv[2] = {T(0), T(0)}, dv[2] = {T(0), T(0)}, iv[2] = {T(0), T(0)};
        if (MODE == 2) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                bv[c] = bB[c];
                dv[c] = xB[c];
                iv[c] = iB[c];
            }
        } else if (wr) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                if (!POW) {
                    bv[c] = b[2 * r + c];
                    dv[c] = alpha != T(0) ? d[2 * r + c] : T(0);
                }
                iv[c] = invd[2 * r + c];
            }
        }
        T y[2], Hx[2][2], Hy[2][2];
        masked_grad<T>(g, w, j, xB, xT, Hx, Hy);
        u_rows<T>(g, w, j, Hx, Hy, pB, pT, c2, c3, y);
        if (wr) {
            const bool dir = dirichlet(g, w.col, j);
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const T yc = dir ? y[c] * xB[c] : y[c];
                if (POW) {
                    d[2 * r + c] = iv[c] * yc;
                } else {
                    const T res = bv[c] - yc;
                    const T dn = (alpha != T(0) ? alpha * dv[c] : T(0)) + beta * iv[c] * res;
                    d[2 * r + c] = dn;
                    x_new[2 * r + c] = xB[c] + dn;
                }
            }
        }
        pB = pT;
        pT = pN;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            xB[c] = xT[c];
            xT[c] = xN[c];
            if (MODE == 2) {
                bB[c] = bT[c];
                bT[c] = bN[c];
                iB[c] = iT[c];
                iT[c] = iN[c];
            }
        }
    }
}

// y = b - M_uu x on the fine displacement level
template <typename T>
__global__ void __launch_bounds__(256) k_mf_residual(MfGrid g, const T* __restrict__ pt, const T* __restrict__ x,
                                                     const T* __restrict__ b, T* __restrict__ y) {
    const WaveStrip w = wave_strip(g);
    if (!w.valid) return;
    auto ld = [&](int64_t j, T& p, T (&v)[2]) {
        const bool in = w.col_in && row_in(g, j);
        const int64_t r = w.col + j * g.n1;
        p = in ? pt[r] : T(0);
        v[0] = in ? x[2 * r] : T(0);
        v[1] = in ? x[2 * r + 1] : T(0);
    };
    T pB, pT, xB[2], xT[2], c2[2] = {T(0), T(0)}, c3[2] = {T(0), T(0)};
    ld(w.j0 - 1, pB, xB);
    ld(w.j0, pT, xT);
    for (int64_t j = w.j0 - 1; j < w.j1; ++j) {
        T pN, xN[2];
        ld(j + 2, pN, xN);
        const bool wr = w.writer && j >= w.j0;
        const int64_t r = w.col + j * g.n1;
        T bv[2];
        if (wr) {
            bv[0] = b[2 * r];
            bv[1] = b[2 * r + 1];
        }
        T acc[2], Hx[2][2], Hy[2][2];
        masked_grad<T>(g, w, j, xB, xT, Hx, Hy);
        u_rows<T>(g, w, j, Hx, Hy, pB, pT, c2, c3, acc);
        if (wr) {
            const bool dir = dirichlet(g, w.col, j);
            y[2 * r] = bv[0] - (dir ? acc[0] * xB[0] : acc[0]);
            y[2 * r + 1] = bv[1] - (dir ? acc[1] * xB[1] : acc[1]);
        }
        pB = pT;
        pT = pN;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            xB[c] = xT[c];
            xT[c] = xN[c];
        }
    }
}

// Chebyshev step of the fine phase-field level (M_phiphi, masked), as k_mf_cheb (MODE 1: a power
// step, d = D^-1 M_phiphi x_old; MODE 2: the first two steps from x = 0 in one pass).
template <typename T, int MODE = 0>
__global__ void __launch_bounds__(256) k_mf_pcheb(MfGrid g, const T* __restrict__ us, const uint8_t* __restrict__ act,
                                                  const T* __restrict__ dpp, const T* __restrict__ invd,
                                                  const T* __restrict__ x_old, const T* __restrict__ b,
                                                  T* __restrict__ d, T* __restrict__ x_new, T alpha, T beta,
                                                  T beta0 = T(0)) {
    constexpr bool POW = MODE == 1;
    const WaveStrip w = wave_strip(g);
    if (!w.valid) return;
    // u_s, x (raw), and x masked at active nodes
    // MODE 2 keeps each row's b and D^-1 from its load (the row is written two steps later)
    auto ld = [&](int64_t j, T (&u)[2], T& x, T& xm, T& bb, T& ii) {
        const bool in = w.col_in && row_in(g, j);
        const int64_t r = w.col + j * g.n1;
        u[0] = in ? us[2 * r] : T(0);
        u[1] = in ? us[2 * r + 1] : T(0);
        if (MODE == 2) {
            bb = in ? b[r] : T(0);
            ii = in ? invd[r] : T(0);
            x = beta0 * ii * bb;
        } else {
            x = in ? x_old[r] : T(0);
        }
        xm = (in && act[r] == 0) ? x : T(0);
    };
    T uB[2], uT[2], xB, xT, mB, mT, c2 = T(0), c3 = T(0);
    T bB = T(0), bT = T(0), iB = T(0), iT = T(0);
    ld(w.j0 - 1, uB, xB, mB, bB, iB);
    ld(w.j0, uT, xT, mT, bT, iT);
    const T none[2][2] = {{T(0), T(0)}, {T(0), T(0)}};
    for (int64_t j = w.j0 - 1; j < w.j1; ++j) {
        T uN[2], xN, mN, bN = T(0), iN = T(0);
        ld(j + 2, uN, xN, mN, bN, iN);
        const bool wr = w.writer && j >= w.j0;
        const int64_t r = w.col + j * g.n1;
        T bv = T(0), dv = T(0), iv = T(0), dg = T(0);
        bool on = false;
        if (wr) {
            if (MODE == 2) {
                bv = bB;
                dv = xB;
                iv = iB;
            } else {
                if (!POW) {
                    bv = b[r];
                    dv = alpha != T(0) ? d[r] : T(0);
                }
                iv = invd[r];
            }
            on = act[r] != 0;
            if (on) dg = dpp[r];
        }
        const T y = phi_rows<T, false>(g, w, j, uB, uT, mB, mT, none, none, T(0), T(0), c2, c3);
        if (wr) {
            const T ay = on ? dg * xB : y;
            if (POW) {
                d[r] = iv * ay;
            } else {
                const T res = bv - ay;
                const T dn = (alpha != T(0) ? alpha * dv : T(0)) + beta * iv * res;
                d[r] = dn;
                x_new[r] = xB + dn;
            }
        }
        uB[0] = uT[0];
        uB[1] = uT[1];
        uT[0] = uN[0];
        uT[1] = uN[1];
        xB = xT;
        xT = xN;
        mB = mT;
        mT = mN;
        bB = bT;
        bT = bN;
        iB = iT;
        iT = iN;
    }
}

// y = b - M_phiphi x on the fine phase-field level
template <typename T>
__global__ void __launch_bounds__(256) k_mf_presidual(MfGrid g, const T* __restrict__ us,
                                                      const uint8_t* __restrict__ act, const T* __restrict__ dpp,
                                                      const T* __restrict__ x, const T* __restrict__ b,
                                                      T* __restrict__ y) {
    const WaveStrip w = wave_strip(g);
    if (!w.valid) return;
    auto ld = [&](int64_t j, T (&u)[2], T& v, T& vm) {
        const bool in = w.col_in && row_in(g, j);
        const int64_t r = w.col + j * g.n1;
        u[0] = in ? us[2 * r] : T(0);
        u[1] = in ? us[2 * r + 1] : T(0);
        v = in ? x[r] : T(0);
        vm = (in && act[r] == 0) ? v : T(0);
    };
    T uB[2], uT[2], xB, xT, mB, mT, c2 = T(0), c3 = T(0);
    ld(w.j0 - 1, uB, xB, mB);
    ld(w.j0, uT, xT, mT);
    const T none[2][2] = {{T(0), T(0)}, {T(0), T(0)}};
    for (int64_t j = w.j0 - 1; j < w.j1; ++j) {
        T uN[2], xN, mN;
        ld(j + 2, uN, xN, mN);
        const bool wr = w.writer && j >= w.j0;
        const int64_t r = w.col + j * g.n1;
        T bv = T(0), dg = T(0);
        bool on = false;
        if (wr) {
            bv = b[r];
            on = act[r] != 0;
            if (on) dg = dpp[r];
        }
        const T acc = phi_rows<T, false>(g, w, j, uB, uT, mB, mT, none, none, T(0), T(0), c2, c3);
        if (wr) y[r] = bv - (on ? dg * xB : acc);
        uB[0] = uT[0];
        uB[1] = uT[1];
        uT[0] = uN[0];
        uT[1] = uN[1];
        xB = xT;
        xT = xN;
        mB = mT;
        mT = mN;
    }
}

// y = J x over the coupled system, by rows (FP64 arithmetic; x FP64 or FP32 widened exactly).
// PART 0: the displacement rows matrix-free and the phase-field rows from the stored blocks (SELL
// slots of the node graph); 1: the displacement rows matrix-free; 2: the phase-field rows
// M_phiu x_u + M_phiphi x_phi matrix-free (from u_s, phi_s and the active set).  Parts 1 and 2
// together make the whole product in two launches, each with half the live registers of one.
// xcopy (optional) receives the written rows' own entries of x at the Krylov slot *jp.
template <typename TX, int PART, typename CI>
__global__ void __launch_bounds__(256) k_jspmv_mf(MfGrid g, const double* __restrict__ pt,
                                                  const double* __restrict__ us, const double* __restrict__ ps,
                                                  const uint8_t* __restrict__ act, const double* __restrict__ dpp,
                                                  int C, const int32_t* __restrict__ slice_ptr,
                                                  const CI* __restrict__ col, const double* __restrict__ pu,
                                                  const double* __restrict__ pp, const TX* __restrict__ x,
                                                  double* __restrict__ y, TX* __restrict__ xcopy,
                                                  const int* __restrict__ jp, int64_t xstride) {
    constexpr bool U = PART != 2, PH = PART == 2;
    const WaveStrip w = wave_strip(g);
    if (!w.valid) return;
    const int64_t nf = g.n_nodes;
    const TX* xp = x + 2 * nf;
    struct Row {
        double p, x[2], xm, u[2], s;             // phi_tilde, x_u (raw), x_phi (masked), u_s, phi_s
    };
    auto ld = [&](int64_t j, Row& v) {
        const bool in = w.col_in && row_in(g, j);
        const int64_t r = w.col + j * g.n1;
        v.x[0] = in ? double(x[2 * r]) : 0.0;
        v.x[1] = in ? double(x[2 * r + 1]) : 0.0;
        if constexpr (U) v.p = in ? pt[r] : 0.0;
        if constexpr (PH) {
            v.xm = (in && act[r] == 0) ? double(xp[r]) : 0.0;
            v.u[0] = in ? us[2 * r] : 0.0;
            v.u[1] = in ? us[2 * r + 1] : 0.0;
            v.s = in ? ps[r] : 0.0;
        }
    };
    Row B, T;
    ld(w.j0 - 1, B);
    ld(w.j0, T);
    double c2[2] = {0.0, 0.0}, c3[2] = {0.0, 0.0};
    for (int64_t j = w.j0 - 1; j < w.j1; ++j) {
        Row N;
        ld(j + 2, N);
        const bool wr = w.writer && j >= w.j0;
        const int64_t r = w.col + j * g.n1;
        TX xo = TX(0);
        if (wr && PH) xo = xp[r];
        double Hx[2][2], Hy[2][2];
        masked_grad<double>(g, w, j, B.x, T.x, Hx, Hy);
        if constexpr (U) {
            double yu[2];
            u_rows<double>(g, w, j, Hx, Hy, B.p, T.p, c2, c3, yu);
            if (wr) {
                const bool dir = dirichlet(g, w.col, j);
                y[2 * r] = dir ? yu[0] * B.x[0] : yu[0];
                y[2 * r + 1] = dir ? yu[1] * B.x[1] : yu[1];
                if (xcopy) {
                    TX* xc = jp ? xcopy + int64_t(*jp) * xstride : xcopy;
                    xc[2 * r] = x[2 * r];
                    xc[2 * r + 1] = x[2 * r + 1];
                }
            }
        }
        if constexpr (PART == 0) {
            if (wr) {
                const int64_t sl = r / C;
                const int lane = int(r - sl * C);
                const int32_t p0 = slice_ptr[sl];
                const int wd = (slice_ptr[sl + 1] - p0) / C;
                int64_t slot = int64_t(p0) + lane;
                double ap = 0.0;
                for (int k = 0; k < wd; ++k, slot += C) {
                    const int64_t c = sizeof(CI) == 2 ? r + int64_t(col[slot]) : int64_t(col[slot]);
                    ap += pu[slot * 2] * double(x[2 * c]);
                    ap += pu[slot * 2 + 1] * double(x[2 * c + 1]);
                    ap += pp[slot] * double(xp[c]);
                }
                y[2 * nf + r] = ap;
                if (xcopy) (jp ? xcopy + int64_t(*jp) * xstride : xcopy)[2 * nf + r] = xp[r];
            }
        }
        if constexpr (PH) {
            const double yp = phi_rows<double, true>(g, w, j, B.u, T.u, B.xm, T.xm, Hx, Hy, B.s, T.s, c2[0], c3[0]);
            if (wr) {
                y[2 * nf + r] = act[r] != 0 ? dpp[r] * double(xo) : yp;
                if (xcopy) (jp ? xcopy + int64_t(*jp) * xstride : xcopy)[2 * nf + r] = xo;
            }
        }
        B = T;
        T = N;
    }
}

// ---- matrix-free transfers of the finest displacement level ------------------------------------
// P = (I - omega D^-1 M_uu) P_t with P_t's row of node i, aggregate a: B_i R_a^-1, B_i = [[1, 0,
// -(y_i - yc_a)], [0, 1, x_i - xc_a]] (the rigid-body modes about the aggregate's centroid).  So
// P_t x_c at node i is B_i w_a with w_a = R_a^-1 x_c,a, and P^T r = P_t^T (r - omega M_uu D^-1 r)
// (M_uu symmetric) sums B_i^T s_i over the aggregate's nodes and multiplies by R_a^-T.  The node
// coordinates are the mesh's (x0 + i h, y0 + j h).

// w_a = R_a^-1 x_c,a
template <typename T>
__global__ void k_agg_w(int64_t na, const T* __restrict__ info, const T* __restrict__ xc, T* __restrict__ w) {
    const int64_t a = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (a >= na) return;
    const T* R = info + a * kAggInfo;
    const T x0 = xc[3 * a], x1 = xc[3 * a + 1], x2 = xc[3 * a + 2];
#pragma unroll
    for (int k = 0; k < 3; ++k) w[3 * a + k] = (R[3 * k] * x0 + R[3 * k + 1] * x1) + R[3 * k + 2] * x2;
}

// P_t x_c at node (i, j) of aggregate a (negative: none): B_i w_a
template <typename T>
__device__ __forceinline__ void tent_value(const MfGrid& g, int32_t a, const T* __restrict__ info,
                                           const T* __restrict__ w, int64_t i, int64_t j, T (&z)[2]) {
    if (a < 0) {
        z[0] = z[1] = T(0);
        return;
    }
    const T dx = T(g.x0 + double(i) * g.h) - info[int64_t(a) * kAggInfo + 9];
    const T dy = T(g.y0 + double(j) * g.h) - info[int64_t(a) * kAggInfo + 10];
    const T w2 = w[3 * int64_t(a) + 2];
    z[0] = w[3 * int64_t(a)] - dy * w2;
    z[1] = w[3 * int64_t(a) + 1] + dx * w2;
}

// x += z - omega D^-1 M_uu z with z = P_t x_c (computed per node from the aggregate's w)
template <typename T>
__global__ void __launch_bounds__(256) k_mf_prolong(MfGrid g, const T* __restrict__ pt, const T* __restrict__ invd,
                                                    const int32_t* __restrict__ agg, const T* __restrict__ info,
                                                    const T* __restrict__ w, T omega, T* __restrict__ x) {
    const WaveStrip ws = wave_strip(g);
    if (!ws.valid) return;
    // two-stage row loads: a row's aggregate indices one step ahead of its gathers
    auto ld_agg = [&](int64_t j) -> int32_t {
        return (ws.col_in && row_in(g, j)) ? agg[ws.col + j * g.n1] : -1;
    };
    auto ld = [&](int64_t j, int32_t a, T& p, T (&z)[2]) {
        const bool in = ws.col_in && row_in(g, j);
        p = in ? pt[ws.col + j * g.n1] : T(0);
        tent_value<T>(g, in ? a : -1, info, w, ws.col, j, z);
    };
    T pB, pT, zB[2], zT[2], c2[2] = {T(0), T(0)}, c3[2] = {T(0), T(0)};
    ld(ws.j0 - 1, ld_agg(ws.j0 - 1), pB, zB);
    ld(ws.j0, ld_agg(ws.j0), pT, zT);
    int32_t aN = ld_agg(ws.j0 + 1);
    for (int64_t j = ws.j0 - 1; j < ws.j1; ++j) {
        const int32_t aNN = ld_agg(j + 3);
        T pN, zN[2];
        ld(j + 2, aN, pN, zN);
        aN = aNN;
        const bool wr = ws.writer && j >= ws.j0;
        const int64_t r = ws.col + j * g.n1;
        T xo[2] = {T(0), T(0)}, iv[2] = {T(0), T(0)};
        if (wr) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                xo[c] = x[2 * r + c];
                iv[c] = invd[2 * r + c];
            }
        }
        T y[2], Hx[2][2], Hy[2][2];
        masked_grad<T>(g, ws, j, zB, zT, Hx, Hy);
        u_rows<T>(g, ws, j, Hx, Hy, pB, pT, c2, c3, y);
        if (wr) {
            const bool dir = dirichlet(g, ws.col, j);
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const T az = dir ? y[c] * zB[c] : y[c];
                x[2 * r + c] = xo[c] + (zB[c] - omega * iv[c] * az);
            }
        }
        pB = pT;
        pT = pN;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            zB[c] = zT[c];
            zT[c] = zN[c];
        }
    }
}

// s = r - omega M_uu D^-1 r
template <typename T>
__global__ void __launch_bounds__(256) k_mf_restrict(MfGrid g, const T* __restrict__ pt, const T* __restrict__ invd,
                                                     const T* __restrict__ r_in, T omega, T* __restrict__ s_out) {
    const WaveStrip ws = wave_strip(g);
    if (!ws.valid) return;
    // per row: phi_tilde, r and D^-1 r (r is kept for the row's output, not loaded again)
    auto ld = [&](int64_t j, T& p, T (&rr)[2], T (&v)[2]) {
        const bool in = ws.col_in && row_in(g, j);
        const int64_t r = ws.col + j * g.n1;
        p = in ? pt[r] : T(0);
        rr[0] = in ? r_in[2 * r] : T(0);
        rr[1] = in ? r_in[2 * r + 1] : T(0);
        v[0] = in ? invd[2 * r] * rr[0] : T(0);
        v[1] = in ? invd[2 * r + 1] * rr[1] : T(0);
    };
    T pB, pT, rB[2], rT[2], vB[2], vT[2], c2[2] = {T(0), T(0)}, c3[2] = {T(0), T(0)};
    ld(ws.j0 - 1, pB, rB, vB);
    ld(ws.j0, pT, rT, vT);
    for (int64_t j = ws.j0 - 1; j < ws.j1; ++j) {
        T pN, rN[2], vN[2];
        ld(j + 2, pN, rN, vN);
        const bool wr = ws.writer && j >= ws.j0;
        const int64_t r = ws.col + j * g.n1;
        const T ro[2] = {rB[0], rB[1]};
        T y[2], Hx[2][2], Hy[2][2];
        masked_grad<T>(g, ws, j, vB, vT, Hx, Hy);
        u_rows<T>(g, ws, j, Hx, Hy, pB, pT, c2, c3, y);
        if (wr) {
            const bool dir = dirichlet(g, ws.col, j);
#pragma unroll
            for (int c = 0; c < 2; ++c) s_out[2 * r + c] = ro[c] - omega * (dir ? y[c] * vB[c] : y[c]);
        }
        pB = pT;
        pT = pN;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            rB[c] = rT[c];
            rT[c] = rN[c];
            vB[c] = vT[c];
            vT[c] = vN[c];
        }
    }
}

// b_c,a = R_a^-T sum over the aggregate's nodes of B_i^T s_i: 16 lanes per aggregate, lane g
// takes members g, g + 16, ... (in increasing node order), the group sums by an xor butterfly
constexpr int kAggLanes = 16;
template <typename T>
__global__ void __launch_bounds__(256) k_agg_restrict(MfGrid g, int64_t na, const int32_t* __restrict__ aptr,
                                                      const int32_t* __restrict__ anodes, const T* __restrict__ info,
                                                      const T* __restrict__ s, T* __restrict__ bc) {
    const int64_t a = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / kAggLanes;
    const int lg = int(threadIdx.x % kAggLanes);
    if (a >= na) return;   // whole groups leave together
    const T* R = info + a * kAggInfo;
    const T xc = R[9], yc = R[10];
    T t0 = T(0), t1 = T(0), t2 = T(0);
    for (int32_t m = aptr[a] + lg; m < aptr[a + 1]; m += kAggLanes) {
        const int32_t node = anodes[m];
        const int32_t j = node / int32_t(g.n1), i = node - j * int32_t(g.n1);
        const T dx = T(g.x0 + double(i) * g.h) - xc, dy = T(g.y0 + double(j) * g.h) - yc;
        const T s0 = s[2 * int64_t(node)], s1 = s[2 * int64_t(node) + 1];
        t0 += s0;
        t1 += s1;
        t2 += -dy * s0 + dx * s1;
    }
#pragma unroll
    for (int o = kAggLanes / 2; o > 0; o >>= 1) {
        t0 += __shfl_xor(t0, o, kAggLanes);
        t1 += __shfl_xor(t1, o, kAggLanes);
        t2 += __shfl_xor(t2, o, kAggLanes);
    }
    if (lg < 3) bc[3 * a + lg] = (R[lg] * t0 + R[3 + lg] * t1) + R[6 + lg] * t2;
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

// workgroups of four waves over the strips x bands of the mesh
int64_t strip_waves(const MfGrid& g) { return ((g.n1 + kSW - 1) / kSW) * ((g.ny + kBand) / kBand); }
dim3 tiles(const MfGrid& g) { return dim3(unsigned((strip_waves(g) + 3) / 4)); }

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
    g.x0 = m.host.desc.lo[0];
    g.y0 = m.host.desc.lo[1];
    if (g.n1 * (g.ny + 1) != m.n_nodes || m.n_free != m.n_nodes) return;
    if ((strip_waves(g) + 3) / 4 >= (int64_t(1) << 31)) return;   // grid limit
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
void mf_cheb_first2(const MfState& mf, int blk, const T* invd, const T* b, T* d, T* x_new, T beta0, T alpha, T beta,
                    hipStream_t s) {
    const MfGrid& g = mf.grid;
    const bool f64 = sizeof(T) == 8;
    if (blk == 0) {
        // b, D^-1 (two words each) and phi_tilde read, d and x_new written
        const double bytes = double(g.n_nodes) * sizeof(T) * (2 * 2 + 1 + 2 * 2);
        ProfScope ps(f64 ? "mf_cheb2_f64" : "mf_cheb2_f32", s, bytes);
        k_mf_cheb<T, 2><<<tiles(g), 256, 0, s>>>(g, mf_pt<T>(mf), invd, nullptr, b, d, x_new, alpha, beta, beta0);
    } else {
        // u_s (two words), b, D^-1, the active flag read, d and x_new written
        const double bytes = double(g.n_nodes) * (sizeof(T) * (2 + 2 + 2) + 1);
        ProfScope ps(f64 ? "mf_pcheb2_f64" : "mf_pcheb2_f32", s, bytes);
        k_mf_pcheb<T, 2><<<tiles(g), 256, 0, s>>>(g, mf_us<T>(mf), mf.act.p, mf_dpp<T>(mf), invd, nullptr, b, d, x_new,
                                                  alpha, beta, beta0);
    }
    FR_LAUNCH_CHECK();
}

void mf_power_step(const MfState& mf, int blk, const double* invd, const double* x, double* y, hipStream_t s) {
    const MfGrid& g = mf.grid;
    if (blk == 0)
        k_mf_cheb<double, 1><<<tiles(g), 256, 0, s>>>(g, mf.pt.p, invd, x, nullptr, y, nullptr, 0.0, 0.0);
    else
        k_mf_pcheb<double, 1><<<tiles(g), 256, 0, s>>>(g, mf.us.p, mf.act.p, mf.dpp.p, invd, x, nullptr, y,
                                                          nullptr, 0.0, 0.0);
    FR_LAUNCH_CHECK();
}

template <typename T>
static const T* agg_info(const AggTransfer& t);
template <>
const double* agg_info<double>(const AggTransfer& t) { return t.info.p; }
template <>
const float* agg_info<float>(const AggTransfer& t) { return t.info32.p; }
template <typename T>
static T* agg_w(const AggTransfer& t);
template <>
double* agg_w<double>(const AggTransfer& t) { return t.w.p; }
template <>
float* agg_w<float>(const AggTransfer& t) { return t.w32.p; }

template <typename T>
void mf_prolong(const MfState& mf, const AggTransfer& t, const T* invd, const T* xc, T* x, hipStream_t st) {
    const MfGrid& g = mf.grid;
    const bool f64 = sizeof(T) == 8;
    // w: the coarse vector and the aggregates' factors read, w written; then per node the
    // aggregate index, phi_tilde, D^-1 and x (read and written), w and the factors gathered (cached)
    const double bytes = double(t.n_agg) * sizeof(T) * (3 + kAggInfo + 3) +
                         double(g.n_nodes) * (4 + sizeof(T) * (1 + 2 + 4));
    ProfScope ps(f64 ? "mf_prolong_f64" : "mf_prolong_f32", st, bytes);
    if (t.n_agg) k_agg_w<T><<<grid_for(t.n_agg), 256, 0, st>>>(t.n_agg, agg_info<T>(t), xc, agg_w<T>(t));
    k_mf_prolong<T><<<tiles(g), 256, 0, st>>>(g, mf_pt<T>(mf), invd, t.agg.p, agg_info<T>(t), agg_w<T>(t),
                                               T(t.omega), x);
    FR_LAUNCH_CHECK();
}

template <typename T>
void mf_restrict(const MfState& mf, const AggTransfer& t, const T* invd, const T* r, T* s, T* bc, hipStream_t st) {
    const MfGrid& g = mf.grid;
    const bool f64 = sizeof(T) == 8;
    // per node phi_tilde, D^-1, r read, s written; then s, the member list read and the
    // aggregates' factors read, b_c written
    const double bytes = double(g.n_nodes) * (sizeof(T) * (1 + 2 + 2 + 2) + sizeof(T) * 2 + 4) +
                         double(t.n_agg) * (sizeof(T) * (kAggInfo + 3) + 4);
    ProfScope ps(f64 ? "mf_restrict_f64" : "mf_restrict_f32", st, bytes);
    k_mf_restrict<T><<<tiles(g), 256, 0, st>>>(g, mf_pt<T>(mf), invd, r, T(t.omega), s);
    if (t.n_agg)
        k_agg_restrict<T><<<grid_for(t.n_agg * kAggLanes), 256, 0, st>>>(g, t.n_agg, t.aptr.p, t.anodes.p,
                                                                         agg_info<T>(t), s, bc);
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
    const SellStruct& S = *sys.Juu.S;
    if (phi_rows) {
        // displacement rows: phi_tilde, x_u read, y_u (and the copy of x_u) written; phase-field
        // rows: u_s, phi_s, the active flag, x_u, x_phi read, y_phi (and the copy) written
        const double bu = nn * (8 + 2 * sizeof(TX) + 16) + (xcopy ? nn * 2 * sizeof(TX) : 0.0);
        const double bp = nn * (16 + 8 + 1 + 3 * sizeof(TX) + 8) + (xcopy ? nn * sizeof(TX) : 0.0);
        {
            ProfScope ps(x64 ? "jspmv_mf_u_d2" : "jspmv_mf_u_d2_x32", s, bu);
            k_jspmv_mf<TX, 1, int32_t><<<gr, 256, 0, s>>>(mf.grid, mf.pt.p, nullptr, nullptr, nullptr, nullptr, S.C,
                                                          S.slice_ptr, S.col, nullptr, nullptr, x, y, xcopy, jp,
                                                          xstride);
            FR_LAUNCH_CHECK();
        }
        ProfScope ps(x64 ? "jspmv_mf_phi_d2" : "jspmv_mf_phi_d2_x32", s, bp);
        k_jspmv_mf<TX, 2, int32_t><<<gr, 256, 0, s>>>(mf.grid, nullptr, mf.us.p, mf.ps.p, mf.act.p, mf.dpp.p, S.C,
                                                      S.slice_ptr, S.col, nullptr, nullptr, x, y, xcopy, jp, xstride);
        FR_LAUNCH_CHECK();
        return;
    }
    const double ib = S.col16 ? 2.0 : 4.0;
    const double bytes = double(S.nnz) * (3 * 8 + ib) + double(S.n_rows) * (3 * (sizeof(TX) + 8) + 8) +
                         (xcopy ? double(S.n_rows) * 3 * sizeof(TX) : 0.0);
    ProfScope ps(x64 ? "jspmv_mf_d2" : "jspmv_mf_d2_x32", s, bytes);
    if (S.col16)
        k_jspmv_mf<TX, 0, int16_t><<<gr, 256, 0, s>>>(mf.grid, mf.pt.p, nullptr, nullptr, nullptr, nullptr, S.C,
                                                          S.slice_ptr, S.col16, sys.Jpu.val, sys.Jpp.val, x, y, xcopy,
                                                          jp, xstride);
    else
        k_jspmv_mf<TX, 0, int32_t><<<gr, 256, 0, s>>>(mf.grid, mf.pt.p, nullptr, nullptr, nullptr, nullptr, S.C,
                                                          S.slice_ptr, S.col, sys.Jpu.val, sys.Jpp.val, x, y, xcopy,
                                                          jp, xstride);
    FR_LAUNCH_CHECK();
}

template void mf_cheb_step<double>(const MfState&, int, const double*, const double*, const double*, double*, double*,
                                   double, double, hipStream_t);
template void mf_cheb_step<float>(const MfState&, int, const float*, const float*, const float*, float*, float*,
                                  float, float, hipStream_t);
template void mf_residual<double>(const MfState&, int, const double*, const double*, double*, hipStream_t);
template void mf_cheb_first2<double>(const MfState&, int, const double*, const double*, double*, double*, double,
                                     double, double, hipStream_t);
template void mf_cheb_first2<float>(const MfState&, int, const float*, const float*, float*, float*, float, float,
                                    float, hipStream_t);
template void mf_prolong<double>(const MfState&, const AggTransfer&, const double*, const double*, double*, hipStream_t);
template void mf_prolong<float>(const MfState&, const AggTransfer&, const float*, const float*, float*, hipStream_t);
template void mf_restrict<double>(const MfState&, const AggTransfer&, const double*, const double*, double*, double*,
                                  hipStream_t);
template void mf_restrict<float>(const MfState&, const AggTransfer&, const float*, const float*, float*, float*,
                                 hipStream_t);
template void mf_residual<float>(const MfState&, int, const float*, const float*, float*, hipStream_t);
template void mf_jspmv<double>(const DevSystem&, bool, const double*, double*, double*, const int*, int64_t,
                               hipStream_t);
template void mf_jspmv<float>(const DevSystem&, bool, const float*, double*, float*, const int*, int64_t, hipStream_t);

}  // namespace fr
