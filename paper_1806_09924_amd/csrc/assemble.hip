// Element-parallel Q1 assembly of Formulation 1 (Section 2) on gfx950: residual of
// E22ATW / E33ATW, lumped phi mass, primal-dual active set, the Jacobian blocks
// M_uu, M_phiu, M_phiphi of Section 3 with the elimination of Dirichlet and active rows,
// the Newton update and the TCV / COD functionals of Section 4.
//
// Assembly is node-centric: one thread owns one free node (one block row of every matrix
// and the matching residual entries), walks the cells that carry its basis function and
// accumulates in a fixed order.  No atomics: results are bitwise reproducible.
#include <atomic>
#include <cmath>
#include <mutex>

#include "system.h"

namespace fr {

Params make_params(const fr_params& p) {
    Params q{};
    q.E = p.E; q.nu = p.nu; q.Gc = p.Gc; q.kappa = p.kappa; q.eps = p.eps; q.p = p.p;
    q.c_pdas = p.c_pdas;
    q.tau = p.tau_pdas > 0 ? p.tau_pdas : 1e-10 * p.Gc / p.eps;
    q.mu = p.E / (2.0 * (1.0 + p.nu));
    q.lam = p.E * p.nu / ((1.0 + p.nu) * (1.0 - 2.0 * p.nu));
    return q;
}

namespace {

// 1d Q1 factors at the 2-point Gauss abscissae: (1 +- 1/sqrt(3)) / 2
constexpr double kGP = 0.78867513459481288225;
constexpr double kGM = 0.21132486540518711775;

template <int D>
__device__ __forceinline__ double shp(int q, int a) {
    double v = 1.0;
#pragma unroll
    for (int k = 0; k < D; ++k) v *= (((a >> k) & 1) == ((q >> k) & 1)) ? kGP : kGM;
    return v;
}

// d N_a / d x_k at Gauss point q of a cell with edge h (ih = 1/h)
template <int D>
__device__ __forceinline__ double dshp(int q, int a, int k, double ih) {
    double v = ((a >> k) & 1) ? ih : -ih;
#pragma unroll
    for (int m = 0; m < D; ++m)
        if (m != k) v *= (((a >> m) & 1) == ((q >> m) & 1)) ? kGP : kGM;
    return v;
}

struct MeshView {
    const int32_t* cells;
    const double* cell_h;
    const double* cell_lo;
    const int32_t* node_of_free;
    const int32_t* free_of_node;
    const int32_t* con_ptr;
    const int32_t* con_master;
    const double* con_w;
    const uint8_t* dir;
    const int32_t* slice_ptr;
    const int32_t* row_len;
    const int32_t* col;
    const int32_t* ent_ptr;
    const int32_t* ent_cell;
    const uint8_t* ent_a;
    const uint8_t* ent_k;
    const double* ent_w;
    const int32_t* hang_ptr;       // masters' row positions for hanging vertices (hanging meshes)
    const uint8_t* hang_k;
    // Rows with more than 2^d entries (masters of hanging nodes: their dependents' cells too)
    // run in a second launch over this list, so that they do not hold up the waves of
    // ordinary rows; pass 0 skips them, pass 1 takes them.
    const int32_t* heavy;
    int64_t n_heavy;
    int pass;
    int C;
    int64_t n_free;
    const int32_t* inst_of_free;   // nullptr for one instance
    const int32_t* inst_of_cell;
    const Params* prm_arr;         // per-instance constants, nullptr for one instance
};

MeshView view(const DevMesh& m) {
    MeshView v;
    v.cells = m.cells.p; v.cell_h = m.cell_h.p; v.cell_lo = m.cell_lo.p;
    v.node_of_free = m.node_of_free.p; v.free_of_node = m.free_of_node.p;
    v.con_ptr = m.con_ptr.p; v.con_master = m.con_master.p; v.con_w = m.con_w.p;
    v.dir = m.dir_free.p;
    v.slice_ptr = m.graph->slice_ptr; v.row_len = m.graph->row_len; v.col = m.graph->col;
    v.ent_ptr = m.ent_ptr.p; v.ent_cell = m.ent_cell.p; v.ent_a = m.ent_a.p; v.ent_k = m.ent_k.p;
    v.ent_w = m.ent_w.p;
    v.hang_ptr = m.hang_ptr.p; v.hang_k = m.hang_k.p;
    v.heavy = m.n_heavy > 0 ? m.heavy_rows.p : nullptr;
    v.n_heavy = m.n_heavy;
    v.pass = 0;
    v.C = m.graph->C;
    v.n_free = m.n_free;
    v.inst_of_free = m.n_inst > 1 ? m.inst_of_free.p : nullptr;
    v.inst_of_cell = m.n_inst > 1 ? m.inst_of_cell.p : nullptr;
    v.prm_arr = nullptr;
    return v;
}

MeshView view(const DevSystem& sys) {
    MeshView v = view(*sys.mesh);
    v.prm_arr = sys.mesh->n_inst > 1 ? sys.prm_d.p : nullptr;
    return v;
}

// Row of this thread in the current pass, or -1.
template <int NV>
__device__ __forceinline__ int64_t pass_row(const MeshView& mv) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (mv.pass == 1) return t < mv.n_heavy ? int64_t(mv.heavy[t]) : -1;
    if (t >= mv.n_free) return -1;
    if (mv.heavy && mv.ent_ptr[t + 1] - mv.ent_ptr[t] > NV) return -1;
    return t;
}

__device__ __forceinline__ Params row_params(const MeshView& mv, const Params& prm0, int64_t f) {
    return mv.prm_arr ? mv.prm_arr[mv.inst_of_free[f]] : prm0;
}

// Nodal values at a cell vertex; with hanging nodes the value is interpolated from the
// free masters (the user arrays are only read at free nodes).
template <int D, bool HANG>
__device__ __forceinline__ void gather_node(const MeshView& mv, int32_t n, const double* u, const double* phi,
                                            const double* pt, double* un, double& pn, double& ptn) {
    if (!HANG) {
#pragma unroll
        for (int c = 0; c < D; ++c) un[c] = u[int64_t(n) * D + c];
        pn = phi[n];
        ptn = pt ? pt[n] : 0.0;
    } else {
#pragma unroll
        for (int c = 0; c < D; ++c) un[c] = 0.0;
        pn = 0.0;
        ptn = 0.0;
        for (int32_t j = mv.con_ptr[n]; j < mv.con_ptr[n + 1]; ++j) {
            const int32_t src = mv.node_of_free[mv.con_master[j]];
            const double w = mv.con_w[j];
#pragma unroll
            for (int c = 0; c < D; ++c) un[c] += w * u[int64_t(src) * D + c];
            pn += w * phi[src];
            if (pt) ptn += w * pt[src];
        }
    }
}

template <int D>
__device__ __forceinline__ void strain_stress(const double (&gu)[D][D], double mu, double lam, double (&sig)[D][D],
                                              double& s, double& tr) {
    tr = 0.0;
#pragma unroll
    for (int c = 0; c < D; ++c) tr += gu[c][c];
    s = 0.0;
#pragma unroll
    for (int c = 0; c < D; ++c)
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const double e = 0.5 * (gu[c][k] + gu[k][c]);
            sig[c][k] = 2.0 * mu * e + (c == k ? lam * tr : 0.0);
            s += sig[c][k] * e;
        }
}

// ---- residual + lumped mass -------------------------------------------------------------
template <int D>
__global__ void __launch_bounds__(256) k_residual(MeshView mv, Params prm0, const double* __restrict__ u,
                                                  const double* __restrict__ phi, const double* __restrict__ pt,
                                                  double* __restrict__ R, double* __restrict__ B) {
    constexpr int NV = 1 << D;
    const int64_t f = pass_row<NV>(mv);
    if (f < 0) return;
    const Params prm = row_params(mv, prm0, f);
    double ru[D];
#pragma unroll
    for (int c = 0; c < D; ++c) ru[c] = 0.0;
    double rp = 0.0, bm = 0.0;
    for (int32_t e = mv.ent_ptr[f]; e < mv.ent_ptr[f + 1]; ++e) {
        const int32_t cell = mv.ent_cell[e];
        const int a = mv.ent_a[e];
        const double w = mv.ent_w[e];
        const double h = mv.cell_h[cell];
        const double ih = 1.0 / h;
        double W = 1.0;
#pragma unroll
        for (int k = 0; k < D; ++k) W *= 0.5 * h;
        W *= w;
        double ue[NV][D], pe[NV], pte[NV];
#pragma unroll
        for (int b = 0; b < NV; ++b) gather_node<D, false>(mv, mv.cells[int64_t(cell) * NV + b], u, phi, pt, ue[b], pe[b], pte[b]);
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            double gu[D][D], gp[D];
            double ph = 0.0, pq = 0.0;
#pragma unroll
            for (int c = 0; c < D; ++c) {
                gp[c] = 0.0;
#pragma unroll
                for (int k = 0; k < D; ++k) gu[c][k] = 0.0;
            }
#pragma unroll
            for (int b = 0; b < NV; ++b) {
                const double nb = shp<D>(q, b);
                ph += nb * pe[b];
                pq += nb * pte[b];
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    const double db = dshp<D>(q, b, k, ih);
                    gp[k] += db * pe[b];
#pragma unroll
                    for (int c = 0; c < D; ++c) gu[c][k] += db * ue[b][c];
                }
            }
            double sig[D][D], s, tr;
            strain_stress<D>(gu, prm.mu, prm.lam, sig, s, tr);
            const double g = (1.0 - prm.kappa) * pq * pq + prm.kappa;
            const double na = shp<D>(q, a);
            double dna[D];
#pragma unroll
            for (int k = 0; k < D; ++k) dna[k] = dshp<D>(q, a, k, ih);
            const double pres = pq * pq * prm.p;
#pragma unroll
            for (int c = 0; c < D; ++c) {
                double t = 0.0;
#pragma unroll
                for (int k = 0; k < D; ++k) t += sig[c][k] * dna[k];
                ru[c] += W * (g * t + pres * dna[c]);
            }
            const double react = (1.0 - prm.kappa) * ph * s + 2.0 * prm.p * ph * tr - (prm.Gc / prm.eps) * (1.0 - ph);
            double lap = 0.0;
#pragma unroll
            for (int k = 0; k < D; ++k) lap += gp[k] * dna[k];
            rp += W * (react * na + prm.Gc * prm.eps * lap);
            bm += W * na;
        }
    }
#pragma unroll
    for (int c = 0; c < D; ++c) R[f * D + c] = ru[c];
    R[D * mv.n_free + f] = rp;
    B[f] = bm;
}

// ---- active set -------------------------------------------------------------------------
// lambda = -R_phi / B; A = { lambda + c (phi - phi_old) > tau }; optional cycle freeze.
__global__ void __launch_bounds__(256) k_active(int64_t nf, int D, Params prm0, const Params* __restrict__ prm_arr,
                                                const int32_t* __restrict__ inst_of_free,
                                                const int32_t* __restrict__ node_of_free,
                                                const double* __restrict__ R, const double* __restrict__ B,
                                                const double* __restrict__ phi, const double* __restrict__ phi_old,
                                                uint8_t* __restrict__ active, uint8_t* __restrict__ prev,
                                                uint8_t* __restrict__ frozen, int use_freeze,
                                                int32_t* __restrict__ part_cnt, double* __restrict__ part_min) {
    __shared__ double shm[16];
    __shared__ int shi[16];
    const int64_t f = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    int changed = 0;
    double mm = INFINITY;
    if (f < nf) {
        const int32_t n = node_of_free[f];
        const Params prm = prm_arr ? prm_arr[inst_of_free[f]] : prm0;
        const double lam = -R[D * nf + f] / B[f];
        const double margin = lam + prm.c_pdas * (phi[n] - phi_old[n]) - prm.tau;
        mm = fabs(margin);
        uint8_t a_new = margin > 0.0 ? 1 : 0;
        const uint8_t a_cur = active[f];
        if (use_freeze) {
            const uint8_t a_prev = prev[f];
            if (a_prev != a_cur && a_cur != a_new) frozen[f] = 1;
        }
        if (frozen[f]) a_new = 1;
        prev[f] = a_cur;
        active[f] = a_new;
        changed = a_new != a_cur;
    }
    int c = wave_sum_int(changed);
    double m = wave_min(mm);
    const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
    if (l == 0) { shi[w] = c; shm[w] = m; }
    __syncthreads();
    if (threadIdx.x == 0) {
        int tc = 0;
        double tm = INFINITY;
        for (int i = 0; i < int(blockDim.x / kWave); ++i) { tc += shi[i]; tm = fmin(tm, shm[i]); }
        part_cnt[blockIdx.x] = tc;
        part_min[blockIdx.x] = tm;
    }
}

// ---- Jacobian + elimination ---------------------------------------------------------------
template <int D>
__device__ __forceinline__ int64_t slot_of(const MeshView& mv, int64_t f, int k) {
    return int64_t(mv.slice_ptr[f / mv.C]) + int64_t(k) * mv.C + (f % mv.C);
}

// One thread per free row.  u, phi, pt hold every vertex's value (hanging ones filled); with
// HANG the columns of hanging vertices are distributed to their masters, whose row positions
// come from the pattern's hang_k table.
template <int D, bool HANG>
__global__ void __launch_bounds__(128) k_jacobian(MeshView mv, Params prm0, const double* __restrict__ u,
                                                  const double* __restrict__ phi, const double* __restrict__ phi_old,
                                                  const double* __restrict__ pt, const double* __restrict__ R,
                                                  const uint8_t* __restrict__ active, double* __restrict__ Juu,
                                                  double* __restrict__ Jpu, double* __restrict__ Jpp,
                                                  double* __restrict__ F) {
    constexpr int NV = 1 << D;
    constexpr int DD = D * D;
    const int64_t f = pass_row<NV>(mv);
    if (f < 0) return;
    const Params prm = row_params(mv, prm0, f);
    const int64_t sl = f / mv.C;
    const int width = (mv.slice_ptr[sl + 1] - mv.slice_ptr[sl]) / mv.C;
    int32_t hc = HANG ? mv.hang_ptr[f] : 0;   // next master position of a hanging vertex
    // Rows of up to 128 slots record which slots they have written: a slot's first
    // contribution is stored, later ones added, and the slots never written (padding) are
    // zeroed at the end, so no slot is zeroed and then read back.  Longer rows zero first.
    const bool track = width <= 128;
    uint64_t touched[2] = {0u, 0u};
    if (!track) {
        for (int k = 0; k < width; ++k) {
            const int64_t s = slot_of<D>(mv, f, k);
#pragma unroll
            for (int i = 0; i < DD; ++i) Juu[s * DD + i] = 0.0;
#pragma unroll
            for (int i = 0; i < D; ++i) Jpu[s * D + i] = 0.0;
            Jpp[s] = 0.0;
        }
    }
    // slot k += w * (kuu, kpu, kpp), or = on its first write
    auto add_slot = [&](int k, double w, const double (&ku)[D][D], const double (&kp)[D], double kq) {
        const int64_t s = slot_of<D>(mv, f, k);
        const uint64_t bit = uint64_t(1) << (k & 63);
        const bool first = track && !(touched[k >> 6] & bit);
        if (track) touched[k >> 6] |= bit;
        if (first) {
#pragma unroll
            for (int c = 0; c < D; ++c)
#pragma unroll
                for (int d = 0; d < D; ++d) Juu[s * DD + c * D + d] = w * ku[c][d];
#pragma unroll
            for (int d = 0; d < D; ++d) Jpu[s * D + d] = w * kp[d];
            Jpp[s] = w * kq;
        } else {
#pragma unroll
            for (int c = 0; c < D; ++c)
#pragma unroll
                for (int d = 0; d < D; ++d) Juu[s * DD + c * D + d] += w * ku[c][d];
#pragma unroll
            for (int d = 0; d < D; ++d) Jpu[s * D + d] += w * kp[d];
            Jpp[s] += w * kq;
        }
    };
    for (int32_t e = mv.ent_ptr[f]; e < mv.ent_ptr[f + 1]; ++e) {
        const int32_t cell = mv.ent_cell[e];
        const int a = mv.ent_a[e];
        const double w = mv.ent_w[e];
        const double h = mv.cell_h[cell];
        const double ih = 1.0 / h;
        double W = 1.0;
#pragma unroll
        for (int k = 0; k < D; ++k) W *= 0.5 * h;
        W *= w;
        double ue[NV][D], pe[NV], pte[NV];
#pragma unroll
        for (int b = 0; b < NV; ++b) gather_node<D, false>(mv, mv.cells[int64_t(cell) * NV + b], u, phi, pt, ue[b], pe[b], pte[b]);
        // Gauss-point fields folded with the row's vertex a, which is fixed for the entry:
        //   Ga[q][k] = g_q dN_a/dx_k,  Sa[q] = N_a (cp_q sigma_q + pp_q I) (symmetric, packed),
        //   ra[q] = N_a re_q.
        // A column b then needs T[k][l] = sum_q Ga[q][k] dN_b/dx_l (which gives the u-u block),
        // sum_q Sa[q] grad N_b (the phi-u row) and sum_q ra[q] N_b (the phi-phi reaction term).
        constexpr int NS = D * (D + 1) / 2;
        double Ga[NV][D], Sa[NV][NS], ra[NV];
        double va[2][D], sa[D];
#pragma unroll
        for (int m = 0; m < D; ++m) {
            const bool am = (a >> m) & 1;
            va[0][m] = am ? kGM : kGP;   // 1d factor of N_a at the abscissa of bit 0 / bit 1
            va[1][m] = am ? kGP : kGM;
            sa[m] = am ? ih : -ih;
        }
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            double gu[D][D];
            double ph = 0.0, pq = 0.0;
#pragma unroll
            for (int c = 0; c < D; ++c)
#pragma unroll
                for (int k = 0; k < D; ++k) gu[c][k] = 0.0;
#pragma unroll
            for (int b2 = 0; b2 < NV; ++b2) {
                const double nb = shp<D>(q, b2);
                ph += nb * pe[b2];
                pq += nb * pte[b2];
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    const double db = dshp<D>(q, b2, k, ih);
#pragma unroll
                    for (int c = 0; c < D; ++c) gu[c][k] += db * ue[b2][c];
                }
            }
            double sg[D][D], s_, tr;
            strain_stress<D>(gu, prm.mu, prm.lam, sg, s_, tr);
            const double g = (1.0 - prm.kappa) * pq * pq + prm.kappa;
            const double cp = 2.0 * (1.0 - prm.kappa) * ph;
            const double pp = 2.0 * prm.p * ph;
            const double re = (1.0 - prm.kappa) * s_ + 2.0 * prm.p * tr + prm.Gc / prm.eps;
            double na = 1.0;
#pragma unroll
            for (int m = 0; m < D; ++m) na *= va[(q >> m) & 1][m];
#pragma unroll
            for (int k = 0; k < D; ++k) {
                double dk = sa[k];
#pragma unroll
                for (int m = 0; m < D; ++m)
                    if (m != k) dk *= va[(q >> m) & 1][m];
                Ga[q][k] = g * dk;
            }
            int i = 0;
#pragma unroll
            for (int c = 0; c < D; ++c)
#pragma unroll
                for (int k = c; k < D; ++k) Sa[q][i++] = na * (cp * sg[c][k] + (c == k ? pp : 0.0));
            ra[q] = na * re;
        }
#pragma unroll(D == 2 ? NV : 1)
        for (int b = 0; b < NV; ++b) {
            double vb[2][D], sb[D];
#pragma unroll
            for (int m = 0; m < D; ++m) {
                const bool bm = (b >> m) & 1;
                vb[0][m] = bm ? kGM : kGP;
                vb[1][m] = bm ? kGP : kGM;
                sb[m] = bm ? ih : -ih;
            }
            double T[D][D], kpu[D], kpp = 0.0;
#pragma unroll
            for (int c = 0; c < D; ++c) {
                kpu[c] = 0.0;
#pragma unroll
                for (int d = 0; d < D; ++d) T[c][d] = 0.0;
            }
#pragma unroll
            for (int q = 0; q < NV; ++q) {
                double nb = 1.0, dnb[D];
#pragma unroll
                for (int m = 0; m < D; ++m) nb *= vb[(q >> m) & 1][m];
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    double dk = sb[k];
#pragma unroll
                    for (int m = 0; m < D; ++m)
                        if (m != k) dk *= vb[(q >> m) & 1][m];
                    dnb[k] = dk;
                }
#pragma unroll
                for (int k = 0; k < D; ++k)
#pragma unroll
                    for (int l = 0; l < D; ++l) T[k][l] += Ga[q][k] * dnb[l];
#pragma unroll
                for (int d = 0; d < D; ++d) {
#pragma unroll
                    for (int k = 0; k < D; ++k) {
                        const int lo = d < k ? d : k, hi = d < k ? k : d;
                        kpu[d] += Sa[q][lo * D - lo * (lo - 1) / 2 + (hi - lo)] * dnb[k];
                    }
                }
                kpp += ra[q] * nb;
            }
            // Laplacian term: the 2-point rule is exact for Q1 gradient products, so
            // sum_q grad N_a . grad N_b = ih^2 sum_k s_k 2 prod_{m != k} (2/3 or 1/3)
            double lap = 0.0;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                double t = (((a ^ b) >> k) & 1) ? -2.0 : 2.0;
#pragma unroll
                for (int m = 0; m < D; ++m)
                    if (m != k) t *= (((a ^ b) >> m) & 1) ? (1.0 / 3.0) : (2.0 / 3.0);
                lap += t;
            }
            kpp += prm.Gc * prm.eps * lap * ih * ih;
            double trT = 0.0;
#pragma unroll
            for (int k = 0; k < D; ++k) trT += T[k][k];
            double kuu[D][D];
#pragma unroll
            for (int c = 0; c < D; ++c)
#pragma unroll
                for (int d = 0; d < D; ++d) kuu[c][d] = prm.mu * ((c == d ? trT : 0.0) + T[d][c]) + prm.lam * T[c][d];
            const int kk = mv.ent_k[int64_t(e) * NV + b];
            if (kk != 255) {
                add_slot(kk, W, kuu, kpu, kpp);
            } else if (HANG) {
                const int32_t n = mv.cells[int64_t(cell) * NV + b];
                for (int32_t j = mv.con_ptr[n]; j < mv.con_ptr[n + 1]; ++j) {
                    const int k2 = mv.hang_k[hc++];
                    add_slot(k2, W * mv.con_w[j], kuu, kpu, kpp);
                }
            }
        }
    }
    if (track) {
        for (int k = 0; k < width; ++k) {
            if (touched[k >> 6] & (uint64_t(1) << (k & 63))) continue;
            const int64_t s = slot_of<D>(mv, f, k);
#pragma unroll
            for (int i = 0; i < DD; ++i) Juu[s * DD + i] = 0.0;
#pragma unroll
            for (int i = 0; i < D; ++i) Jpu[s * D + i] = 0.0;
            Jpp[s] = 0.0;
        }
    }
    // elimination of Dirichlet u DoFs (target u = 0) and active phi DoFs (target phi_old)
    const int64_t nf = mv.n_free;
    const bool dir_f = mv.dir[f] != 0;
    const bool act_f = active[f] != 0;
    const int32_t nodef = mv.node_of_free[f];
    double fu[D], fp;
#pragma unroll
    for (int c = 0; c < D; ++c) fu[c] = -R[f * D + c];
    fp = -R[D * nf + f];
    const int len = mv.row_len[f];
    double diag_u[D], diag_p = 0.0;
#pragma unroll
    for (int c = 0; c < D; ++c) diag_u[c] = 0.0;
    for (int k = 0; k < len; ++k) {
        const int64_t s = slot_of<D>(mv, f, k);
        const int32_t g = mv.col[s];
        const int32_t nodeg = mv.node_of_free[g];
        if (g == f) {
#pragma unroll
            for (int c = 0; c < D; ++c) diag_u[c] = Juu[s * DD + c * D + c];
            diag_p = Jpp[s];
        }
        const bool dir_g = mv.dir[g] != 0;
        const bool act_g = active[g] != 0;
        // u columns of Dirichlet nodes
        if (dir_g && g != f) {
            double tg[D];
#pragma unroll
            for (int d = 0; d < D; ++d) tg[d] = -u[int64_t(nodeg) * D + d];
#pragma unroll
            for (int c = 0; c < D; ++c) {
                double t = 0.0;
#pragma unroll
                for (int d = 0; d < D; ++d) t += Juu[s * DD + c * D + d] * tg[d];
                fu[c] -= t;
            }
            double t = 0.0;
#pragma unroll
            for (int d = 0; d < D; ++d) t += Jpu[s * D + d] * tg[d];
            fp -= t;
#pragma unroll
            for (int i = 0; i < DD; ++i) Juu[s * DD + i] = 0.0;
#pragma unroll
            for (int i = 0; i < D; ++i) Jpu[s * D + i] = 0.0;
        } else if (dir_g && g == f) {
            // both row and column Dirichlet: keep only the diagonal of the block
#pragma unroll
            for (int c = 0; c < D; ++c)
#pragma unroll
                for (int d = 0; d < D; ++d)
                    if (c != d) Juu[s * DD + c * D + d] = 0.0;
            double tg[D];
#pragma unroll
            for (int d = 0; d < D; ++d) tg[d] = -u[int64_t(nodeg) * D + d];
            double t = 0.0;
#pragma unroll
            for (int d = 0; d < D; ++d) t += Jpu[s * D + d] * tg[d];
            fp -= t;
#pragma unroll
            for (int i = 0; i < D; ++i) Jpu[s * D + i] = 0.0;
        }
        if (dir_f && g != f) {
#pragma unroll
            for (int i = 0; i < DD; ++i) Juu[s * DD + i] = 0.0;
        }
        // phi columns of active nodes
        if (act_g && g != f) {
            const int32_t ng = nodeg;
            fp -= Jpp[s] * (phi_old[ng] - phi[ng]);
            Jpp[s] = 0.0;
        }
    }
    if (act_f) {
        for (int k = 0; k < len; ++k) {
            const int64_t s = slot_of<D>(mv, f, k);
#pragma unroll
            for (int i = 0; i < D; ++i) Jpu[s * D + i] = 0.0;
            if (mv.col[s] != f) Jpp[s] = 0.0;
        }
        fp = diag_p * (phi_old[nodef] - phi[nodef]);
    }
    if (dir_f) {
#pragma unroll
        for (int c = 0; c < D; ++c) fu[c] = diag_u[c] * (-u[int64_t(nodef) * D + c]);
    }
#pragma unroll
    for (int c = 0; c < D; ++c) F[f * D + c] = fu[c];
    F[D * nf + f] = fp;
}

// ---- masked residual norm and rhs norm (block partials) ---------------------------------
__global__ void __launch_bounds__(256) k_norm_parts(int64_t nf, int D, const double* __restrict__ R,
                                                    const double* __restrict__ F, const uint8_t* __restrict__ dir,
                                                    const uint8_t* __restrict__ active, double* __restrict__ part) {
    __shared__ double sh[16];
    const int64_t f = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    double r2 = 0.0, f2 = 0.0, na = 0.0;
    if (f < nf) {
        if (!dir[f])
            for (int c = 0; c < D; ++c) r2 += R[f * D + c] * R[f * D + c];
        if (!active[f]) r2 += R[D * nf + f] * R[D * nf + f];
        else na = 1.0;
        if (F) {
            for (int c = 0; c < D; ++c) f2 += F[f * D + c] * F[f * D + c];
            f2 += F[D * nf + f] * F[D * nf + f];
        }
    }
    const double a = block_sum(r2, sh);
    const double b = block_sum(f2, sh);
    const double c = block_sum(na, sh);
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x + 0] = a;
        part[3 * blockIdx.x + 1] = b;
        part[3 * blockIdx.x + 2] = c;
    }
}

// Per instance of a batch (one workgroup each, rows in a fixed order): ||R~||^2 (Dirichlet
// u rows and active phi rows left out), active phi rows, and rows whose active flag changed
// in the last active-set update.
__global__ void __launch_bounds__(256) k_inst_norms(int D, int64_t nf, const int64_t* __restrict__ off,
                                                    const double* __restrict__ R, const uint8_t* __restrict__ dir,
                                                    const uint8_t* __restrict__ active, const uint8_t* __restrict__ prev,
                                                    double* __restrict__ out) {
    __shared__ double sh[16];
    const int i = blockIdx.x;
    double r2 = 0.0, na = 0.0, nc = 0.0;
    for (int64_t f = off[i] + threadIdx.x; f < off[i + 1]; f += blockDim.x) {
        if (!dir[f])
            for (int c = 0; c < D; ++c) r2 += R[f * D + c] * R[f * D + c];
        if (!active[f]) r2 += R[D * nf + f] * R[D * nf + f];
        else na += 1.0;
        if (active[f] != prev[f]) nc += 1.0;
    }
    const double a = block_sum(r2, sh);
    const double b = block_sum(na, sh);
    const double c = block_sum(nc, sh);
    if (threadIdx.x == 0) {
        out[3 * i + 0] = a;
        out[3 * i + 1] = b;
        out[3 * i + 2] = c;
    }
}

// u += omega_i du, phi += omega_i dphi at the free nodes of instance i
// ---- update -----------------------------------------------------------------------------
// u += w du, phi += w du on free node f; with `fix` (the Newton loop) the DoFs that the
// elimination fixes take their constraint values instead: Dirichlet u DoFs 0, active phi DoFs
// phi_old, so that a damped step cannot leave an active DoF off phi_old.
struct FixedDofs {
    const uint8_t* dir;        // per free node, nullptr: no projection
    const uint8_t* active;     // per free node
    const double* phi_old;     // per node
};

__device__ __forceinline__ void update_node(int64_t f, int64_t nf, int D, int64_t n, const double* __restrict__ du,
                                            double w, const FixedDofs& fix, double* __restrict__ u,
                                            double* __restrict__ phi) {
    const bool ud = fix.dir && fix.dir[f];
    for (int c = 0; c < D; ++c) u[n * D + c] = ud ? 0.0 : u[n * D + c] + w * du[f * D + c];
    phi[n] = (fix.dir && fix.active[f]) ? fix.phi_old[n] : phi[n] + w * du[D * nf + f];
}

__global__ void k_update_free_inst(int64_t nf, int D, const int32_t* __restrict__ node_of_free,
                                   const int32_t* __restrict__ inst_of_free, const double* __restrict__ du,
                                   const double* __restrict__ omega, FixedDofs fix, double* __restrict__ u,
                                   double* __restrict__ phi) {
    const int64_t f = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (f >= nf) return;
    const double w = omega[inst_of_free[f]];
    if (w == 0.0) return;   // finished or failed instance: left exactly as it is
    update_node(f, nf, D, node_of_free[f], du, w, fix, u, phi);
}

__global__ void k_update_free(int64_t nf, int D, const int32_t* __restrict__ node_of_free,
                              const double* __restrict__ du, double omega, FixedDofs fix, double* __restrict__ u,
                              double* __restrict__ phi) {
    const int64_t f = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (f >= nf) return;
    update_node(f, nf, D, node_of_free[f], du, omega, fix, u, phi);
}

__global__ void k_fill_hanging(int64_t nn, int D, const int32_t* __restrict__ free_of_node,
                               const int32_t* __restrict__ node_of_free, const int32_t* __restrict__ con_ptr,
                               const int32_t* __restrict__ con_master, const double* __restrict__ con_w,
                               double* __restrict__ u, double* __restrict__ phi) {
    const int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (n >= nn || free_of_node[n] >= 0) return;
    double uu[3] = {0, 0, 0}, pp = 0.0;
    for (int32_t j = con_ptr[n]; j < con_ptr[n + 1]; ++j) {
        const int64_t src = node_of_free[con_master[j]];
        for (int c = 0; c < D; ++c) uu[c] += con_w[j] * u[src * D + c];
        pp += con_w[j] * phi[src];
    }
    for (int c = 0; c < D; ++c) u[n * D + c] = uu[c];
    phi[n] = pp;
}

// Nodal u, phi, phi~ with the hanging values interpolated from the free masters, so that the
// element kernels gather every vertex directly (the user arrays are only read at free nodes).
template <int D>
__global__ void __launch_bounds__(256) k_nodal_fill(int64_t nn, const int32_t* __restrict__ free_of_node,
                                                    const int32_t* __restrict__ node_of_free,
                                                    const int32_t* __restrict__ con_ptr,
                                                    const int32_t* __restrict__ con_master,
                                                    const double* __restrict__ con_w, const double* __restrict__ u,
                                                    const double* __restrict__ phi, const double* __restrict__ pt,
                                                    double* __restrict__ uo, double* __restrict__ po,
                                                    double* __restrict__ pto) {
    const int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (n >= nn) return;
    double uu[D], pp = 0.0, tt = 0.0;
#pragma unroll
    for (int c = 0; c < D; ++c) uu[c] = 0.0;
    for (int32_t j = con_ptr[n]; j < con_ptr[n + 1]; ++j) {
        const int64_t src = node_of_free[con_master[j]];
        const double w = con_w[j];
#pragma unroll
        for (int c = 0; c < D; ++c) uu[c] += w * u[src * D + c];
        pp += w * phi[src];
        if (pt) tt += w * pt[src];
    }
#pragma unroll
    for (int c = 0; c < D; ++c) uo[n * D + c] = uu[c];
    po[n] = pp;
    if (pt) pto[n] = tt;
}

// ---- functionals --------------------------------------------------------------------------
template <int D, bool HANG>
__global__ void __launch_bounds__(256) k_tcv(int64_t c0, int64_t nc, MeshView mv, const double* __restrict__ u,
                                             const double* __restrict__ phi, double* __restrict__ part) {
    __shared__ double sh[16];
    constexpr int NV = 1 << D;
    const int64_t c = c0 + int64_t(blockIdx.x) * blockDim.x + threadIdx.x;   // cells [c0, nc)
    double acc = 0.0;
    if (c < nc) {
        const double h = mv.cell_h[c], ih = 1.0 / h;
        double W = 1.0;
        for (int k = 0; k < D; ++k) W *= 0.5 * h;
        double ue[NV][D], pe[NV], dummy;
#pragma unroll
        for (int b = 0; b < NV; ++b) gather_node<D, HANG>(mv, mv.cells[c * NV + b], u, phi, nullptr, ue[b], pe[b], dummy);
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            double uq[D], gp[D];
#pragma unroll
            for (int k = 0; k < D; ++k) { uq[k] = 0.0; gp[k] = 0.0; }
#pragma unroll
            for (int b = 0; b < NV; ++b) {
                const double nb = shp<D>(q, b);
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    uq[k] += nb * ue[b][k];
                    gp[k] += dshp<D>(q, b, k, ih) * pe[b];
                }
            }
            double t = 0.0;
#pragma unroll
            for (int k = 0; k < D; ++k) t += uq[k] * gp[k];
            acc += W * t;
        }
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// COD: 1/2 of the line integral of u . grad phi along the last axis at x0 (1d 2-point Gauss)
template <int D, bool HANG>
__global__ void __launch_bounds__(256) k_cod(int64_t c0, int64_t nc, MeshView mv, const double* __restrict__ u,
                                             const double* __restrict__ phi, const double* __restrict__ xs,
                                             double* __restrict__ part) {
    __shared__ double sh[16];
    constexpr int NV = 1 << D;
    const int64_t c = c0 + int64_t(blockIdx.x) * blockDim.x + threadIdx.x;   // cells [c0, nc)
    const int sample = blockIdx.y;
    double acc = 0.0;
    if (c < nc) {
        const double h = mv.cell_h[c], ih = 1.0 / h;
        bool hit = true;
        double xi[D];
        for (int k = 0; k < D - 1; ++k) {
            const double lo = mv.cell_lo[c * D + k];
            const double x0 = xs[sample * (D - 1) + k];
            hit = hit && (lo <= x0) && (x0 < lo + h);
            xi[k] = 2.0 * (x0 - lo) / h - 1.0;
        }
        if (hit) {
            double ue[NV][D], pe[NV], dummy;
#pragma unroll
            for (int b = 0; b < NV; ++b) gather_node<D, HANG>(mv, mv.cells[c * NV + b], u, phi, nullptr, ue[b], pe[b], dummy);
            const double g1 = 0.57735026918962576451;   // 1/sqrt(3)
            for (int q = 0; q < 2; ++q) {
                xi[D - 1] = q ? g1 : -g1;
                double uq[D], gp[D];
                for (int k = 0; k < D; ++k) { uq[k] = 0.0; gp[k] = 0.0; }
                for (int b = 0; b < NV; ++b) {
                    double nb = 1.0;
                    double dn[D];
                    for (int k = 0; k < D; ++k) dn[k] = 1.0;
                    for (int m = 0; m < D; ++m) {
                        const double sgn = ((b >> m) & 1) ? 1.0 : -1.0;
                        const double fac = 0.5 * (1.0 + sgn * xi[m]);
                        nb *= fac;
                        for (int k = 0; k < D; ++k) dn[k] *= (k == m) ? sgn * ih : fac;
                    }
                    for (int k = 0; k < D; ++k) {
                        uq[k] += nb * ue[b][k];
                        gp[k] += dn[k] * pe[b];
                    }
                }
                double t = 0.0;
                for (int k = 0; k < D; ++k) t += uq[k] * gp[k];
                acc += 0.5 * h * t;
            }
        }
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) part[int64_t(sample) * gridDim.x + blockIdx.x] = 0.5 * s;
}

__global__ void k_sum_rows(const double* __restrict__ part, int64_t n_part, int n_rows, int stride_row,
                           int stride_elem, double* __restrict__ out) {
    // one block per output row, fixed-order sum
    __shared__ double sh[16];
    const int r = blockIdx.x;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n_part; i += blockDim.x) acc += part[int64_t(r) * stride_row + i * stride_elem];
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) out[r] = s;
}

// ---- failed instances of a batch, flag counts, finiteness -----------------------------------
// Rows of the instances flagged in `bad` become identity rows with a zero right-hand side (and
// residual), so that their non-finite values stay out of the preconditioner and the solve of
// the other instances (which never couple to them); their increment is then zero.
template <int D>
__global__ void __launch_bounds__(256) k_neutralize(int64_t nf, const int32_t* __restrict__ inst_of_free,
                                                    const int* __restrict__ bad, const int32_t* __restrict__ slice_ptr,
                                                    const int32_t* __restrict__ row_len, const int32_t* __restrict__ col,
                                                    int C, double* __restrict__ Juu, double* __restrict__ Jpu,
                                                    double* __restrict__ Jpp, double* __restrict__ F,
                                                    double* __restrict__ R) {
    const int64_t f = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (f >= nf || !bad[inst_of_free[f]]) return;
    const int64_t base = int64_t(slice_ptr[f / C]) + (f % C);
    const int len = row_len[f];
    for (int k = 0; k < len; ++k) {
        const int64_t slot = base + int64_t(k) * C;
        const double one = col[slot] == f ? 1.0 : 0.0;
#pragma unroll
        for (int a = 0; a < D; ++a) {
#pragma unroll
            for (int b = 0; b < D; ++b) Juu[slot * D * D + a * D + b] = a == b ? one : 0.0;
            Jpu[slot * D + a] = 0.0;
        }
        Jpp[slot] = one;
    }
#pragma unroll
    for (int c = 0; c < D; ++c) {
        F[f * D + c] = 0.0;
        R[f * D + c] = 0.0;
    }
    F[D * nf + f] = 0.0;
    R[D * nf + f] = 0.0;
}

// cnt[instance] += number of nonzero flags (cnt zeroed by the caller)
__global__ void __launch_bounds__(256) k_count_flags(int64_t nf, const int32_t* __restrict__ inst_of_free,
                                                     const uint8_t* __restrict__ flags,
                                                     unsigned long long* __restrict__ cnt) {
    const int64_t f = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (f < nf && flags[f]) atomicAdd(&cnt[inst_of_free ? inst_of_free[f] : 0], 1ull);
}

// *flag = 1 when any of x[0..n) is not finite (flag zeroed by the caller)
__global__ void __launch_bounds__(256) k_nonfinite(const double* __restrict__ x, int64_t n, int* __restrict__ flag) {
    bool bad = false;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        bad = bad || !isfinite(x[i]);
    if (bad) atomicOr(flag, 1);
}

}  // namespace

// ---- host side --------------------------------------------------------------------------

std::unique_ptr<DevMesh> mesh_create(const fr_mesh_desc* d, int n_inst, hipStream_t s, bool upload) {
    return mesh_from_host(build_mesh_batch(d, n_inst), s, upload);
}

std::unique_ptr<DevMesh> mesh_from_host(HostMesh&& host, hipStream_t s, bool upload) {
    static std::atomic<uint64_t> next_serial{1};
    auto m = std::make_unique<DevMesh>();
    m->serial = next_serial.fetch_add(1);
    const int n_inst = host.n_inst;
    m->host = std::move(host);
    m->n_inst = n_inst;
    m->pat = build_pattern(m->host, 64);
    const HostMesh& h = m->host;
    const Pattern& p = m->pat;
    m->stream = s;
    m->dim = h.dim;
    m->nv = h.nv;
    m->n_nodes = h.n_nodes;
    m->n_cells = h.n_cells;
    m->n_free = h.n_free;
    m->hanging = h.n_hanging > 0;
    m->on_device = upload;
    if (!upload) return m;
    if (n_inst > 1) {
        std::vector<int32_t> iof(size_t(h.n_free)), ioc(size_t(h.n_cells));
        for (int i = 0; i < n_inst; ++i) {
            for (int64_t f = h.free_off[size_t(i)]; f < h.free_off[size_t(i) + 1]; ++f) iof[size_t(f)] = i;
            for (int64_t c = h.cell_off[size_t(i)]; c < h.cell_off[size_t(i) + 1]; ++c) ioc[size_t(c)] = i;
        }
        m->inst_of_free.upload(iof, s);
        m->inst_of_cell.upload(ioc, s);
    }
    m->cells.upload(h.cells, s);
    m->cell_h.upload(h.cell_h, s);
    m->cell_lo.upload(h.cell_lo, s);
    m->node_of_free.upload(h.node_of_free, s);
    m->free_of_node.upload(h.free_of_node, s);
    m->con_ptr.upload(h.con_ptr, s);
    m->con_master.upload(h.con_master, s);
    m->con_w.upload(h.con_w, s);
    std::vector<uint8_t> dirf(size_t(h.n_free));
    std::vector<double> cf(size_t(h.n_free) * h.dim);
    for (int64_t f = 0; f < h.n_free; ++f) {
        const int64_t n = h.node_of_free[size_t(f)];
        dirf[size_t(f)] = h.dirichlet[size_t(n)];
        for (int c = 0; c < h.dim; ++c) cf[size_t(f) * h.dim + c] = h.coords[size_t(n) * h.dim + c];
    }
    m->dir_free.upload(dirf, s);
    m->coords_free.upload(cf, s);
    auto g = std::make_shared<SellStruct>();
    g->C = p.C;
    g->n_rows = p.n_rows;
    g->n_cols = p.n_rows;
    g->n_slices = p.n_slices;
    g->n_slots = p.n_slots;
    g->nnz = p.nnz;
    g->max_len = p.max_row;
    g->own_slice.upload(p.slice_ptr, s);
    g->own_len.upload(p.row_len, s);
    g->own_col.upload(p.col, s);
    g->slice_ptr = g->own_slice.p;
    g->row_len = g->own_len.p;
    g->col = g->own_col.p;
    make_col16(*g, s);
    m->graph = g;
    m->ent_ptr.upload(p.ent_ptr, s);
    m->ent_cell.upload(p.ent_cell, s);
    m->ent_a.upload(p.ent_a, s);
    m->ent_k.upload(p.ent_k, s);
    m->ent_w.upload(p.ent_w, s);
    if (!p.hang_k.empty()) {
        m->hang_ptr.upload(p.hang_ptr, s);
        m->hang_k.upload(p.hang_k, s);
    }
    {
        // rows with more entries than a cell has vertices (hanging-node masters)
        std::vector<int32_t>& heavy = m->heavy_host;   // stays alive past the asynchronous upload
        heavy.clear();
        const int nv = 1 << h.dim;
        for (int64_t f = 0; f < p.n_rows; ++f)
            if (p.ent_ptr[size_t(f) + 1] - p.ent_ptr[size_t(f)] > nv) heavy.push_back(int32_t(f));
        m->n_heavy = int64_t(heavy.size());
        if (!heavy.empty()) m->heavy_rows.upload(heavy, s);
    }
    FR_HIP(hipStreamSynchronize(s));   // host vectors of the pattern stay alive in m
    return m;
}

static int blocks_for(int64_t n, int t) { return int(ceil_div(n, t)); }

// Hanging meshes: fills sys.nodal and redirects u, phi, pt (pt stays null when null) to it.
static void nodal_fill(DevSystem& sys, const double*& u, const double*& phi, const double*& pt) {
    DevMesh& m = *sys.mesh;
    const hipStream_t s = sys.stream;
    const int64_t nn = m.n_nodes;
    sys.nodal.reserve(size_t(nn) * size_t(m.dim + 2), s);
    double* uo = sys.nodal.p;
    double* po = uo + nn * m.dim;
    double* pto = po + nn;
    const int nb = blocks_for(nn, 256);
    if (m.dim == 2)
        k_nodal_fill<2><<<nb, 256, 0, s>>>(nn, m.free_of_node.p, m.node_of_free.p, m.con_ptr.p, m.con_master.p,
                                           m.con_w.p, u, phi, pt, uo, po, pto);
    else
        k_nodal_fill<3><<<nb, 256, 0, s>>>(nn, m.free_of_node.p, m.node_of_free.p, m.con_ptr.p, m.con_master.p,
                                           m.con_w.p, u, phi, pt, uo, po, pto);
    FR_LAUNCH_CHECK();
    u = uo;
    phi = po;
    if (pt) pt = pto;
}

void assemble_residual(DevSystem& sys, const double* u, const double* phi, const double* pt) {
    DevMesh& m = *sys.mesh;
    MeshView mv = view(sys);
    const hipStream_t s = sys.stream;
    const int nb = blocks_for(m.n_free, 256);
    if (m.hanging) nodal_fill(sys, u, phi, pt);
    for (int pass = 0; pass < (m.n_heavy > 0 ? 2 : 1); ++pass) {
        mv.pass = pass;
        const int g = pass == 0 ? nb : blocks_for(m.n_heavy, 256);
        if (m.dim == 2) k_residual<2><<<g, 256, 0, s>>>(mv, sys.prm, u, phi, pt, sys.R.p, sys.B.p);
        else k_residual<3><<<g, 256, 0, s>>>(mv, sys.prm, u, phi, pt, sys.R.p, sys.B.p);
    }
    FR_LAUNCH_CHECK();
    sys.have_residual = true;
}

void assemble_active_impl(DevSystem& sys, const double* phi, const double* phi_old, int use_freeze) {
    DevMesh& m = *sys.mesh;
    const hipStream_t s = sys.stream;
    const int nb = blocks_for(m.n_free, 256);
    sys.red.reserve(size_t(nb) + 16, s);
    sys.ired.reserve(size_t(nb) + 16, s);
    k_active<<<nb, 256, 0, s>>>(m.n_free, m.dim, sys.prm, m.n_inst > 1 ? sys.prm_d.p : nullptr,
                                m.n_inst > 1 ? m.inst_of_free.p : nullptr, m.node_of_free.p, sys.R.p, sys.B.p, phi, phi_old,
                                sys.active.p, sys.active_prev.p, sys.frozen.p, use_freeze, sys.ired.p, sys.red.p);
    FR_LAUNCH_CHECK();
    auto cnt = download(sys.ired.p, size_t(nb), s);
    auto mm = download(sys.red.p, size_t(nb), s);
    int64_t ch = 0;
    double mn = INFINITY;
    for (int32_t c : cnt) ch += c;
    for (double v : mm) mn = std::fmin(mn, v);
    sys.last_changes = ch;
    sys.last_min_margin = mn;
    sys.have_active = true;
}

void assemble_active(DevSystem& sys, const double* phi, const double* phi_old) {
    assemble_active_impl(sys, phi, phi_old, 0);
}

void assemble_active_freeze(DevSystem& sys, const double* phi, const double* phi_old) {
    assemble_active_impl(sys, phi, phi_old, 1);
}

void assemble_jacobian(DevSystem& sys, const double* u, const double* phi, const double* phi_old, const double* pt) {
    DevMesh& m = *sys.mesh;
    MeshView mv = view(sys);
    const hipStream_t s = sys.stream;
    if (m.hanging) nodal_fill(sys, u, phi, pt);
    for (int pass = 0; pass < (m.n_heavy > 0 ? 2 : 1); ++pass) {
        mv.pass = pass;
        const int nb = blocks_for(pass == 0 ? m.n_free : m.n_heavy, 128);
#define FR_JAC(D_, H_)                                                                                  \
    k_jacobian<D_, H_><<<nb, 128, 0, s>>>(mv, sys.prm, u, phi, phi_old, pt, sys.R.p, sys.active.p, sys.Juu.val, \
                                          sys.Jpu.val, sys.Jpp.val, sys.F.p);
        if (m.dim == 2) {
            if (m.hanging) { FR_JAC(2, true) }
            else { FR_JAC(2, false) }
        } else {
            if (m.hanging) { FR_JAC(3, true) }
            else { FR_JAC(3, false) }
        }
#undef FR_JAC
    }
    FR_LAUNCH_CHECK();
    sys.have_jacobian = true;
    sys.version++;
    mf_prepare(sys, u, phi, pt, s);
}

void system_norms(DevSystem& sys, const double* phi, const double* phi_old, double* norms, int64_t* n_active,
                  double* min_margin) {
    (void)phi;
    (void)phi_old;
    DevMesh& m = *sys.mesh;
    const hipStream_t s = sys.stream;
    const int nb = blocks_for(m.n_free, 256);
    sys.red.reserve(size_t(3 * nb) + 16, s);
    k_norm_parts<<<nb, 256, 0, s>>>(m.n_free, m.dim, sys.R.p, sys.have_jacobian ? sys.F.p : nullptr, m.dir_free.p,
                                    sys.active.p, sys.red.p);
    FR_LAUNCH_CHECK();
    auto part = download(sys.red.p, size_t(3 * nb), s);
    double a = 0, b = 0, c = 0;
    for (int i = 0; i < nb; ++i) { a += part[size_t(3 * i)]; b += part[size_t(3 * i + 1)]; c += part[size_t(3 * i + 2)]; }
    if (norms) { norms[0] = std::sqrt(a); norms[1] = std::sqrt(b); }
    if (n_active) *n_active = int64_t(c + 0.5);
    if (min_margin) *min_margin = sys.last_min_margin;
}

void system_norms_inst(DevSystem& sys, std::vector<double>& rnorm, std::vector<int64_t>& n_active,
                       std::vector<int64_t>& changes) {
    DevMesh& m = *sys.mesh;
    const hipStream_t s = sys.stream;
    const int ni = m.n_inst;
    if (sys.inst_off.p == nullptr) sys.inst_off.upload(m.host.free_off, s);
    sys.red.reserve(size_t(3 * ni) + 16, s);
    k_inst_norms<<<ni, 256, 0, s>>>(m.dim, m.n_free, sys.inst_off.p, sys.R.p, m.dir_free.p, sys.active.p,
                                    sys.active_prev.p, sys.red.p);
    FR_LAUNCH_CHECK();
    auto part = download(sys.red.p, size_t(3 * ni), s);
    rnorm.resize(size_t(ni));
    n_active.resize(size_t(ni));
    changes.resize(size_t(ni));
    for (int i = 0; i < ni; ++i) {
        rnorm[size_t(i)] = std::sqrt(part[size_t(3 * i)]);
        n_active[size_t(i)] = int64_t(part[size_t(3 * i + 1)] + 0.5);
        changes[size_t(i)] = int64_t(part[size_t(3 * i + 2)] + 0.5);
    }
}

void system_neutralize(DevSystem& sys, const int* bad_dev) {
    DevMesh& m = *sys.mesh;
    if (m.n_inst < 2) fail(FR_EINTERNAL, "system_neutralize: batched meshes only");
    const SellStruct& S = *m.graph;
    const int nb = blocks_for(m.n_free, 256);
    const hipStream_t s = sys.stream;
    if (m.dim == 2)
        k_neutralize<2><<<nb, 256, 0, s>>>(m.n_free, m.inst_of_free.p, bad_dev, S.slice_ptr, S.row_len, S.col, S.C,
                                           sys.Juu.val, sys.Jpu.val, sys.Jpp.val, sys.F.p, sys.R.p);
    else
        k_neutralize<3><<<nb, 256, 0, s>>>(m.n_free, m.inst_of_free.p, bad_dev, S.slice_ptr, S.row_len, S.col, S.C,
                                           sys.Juu.val, sys.Jpu.val, sys.Jpp.val, sys.F.p, sys.R.p);
    FR_LAUNCH_CHECK();
}

std::vector<int64_t> count_flags_inst(DevSystem& sys, const uint8_t* flags) {
    DevMesh& m = *sys.mesh;
    const hipStream_t s = sys.stream;
    DBuf<unsigned long long> cnt;
    cnt.alloc(size_t(m.n_inst), s);
    cnt.zero(s);
    k_count_flags<<<blocks_for(std::max<int64_t>(1, m.n_free), 256), 256, 0, s>>>(
        m.n_free, m.n_inst > 1 ? m.inst_of_free.p : nullptr, flags, cnt.p);
    FR_LAUNCH_CHECK();
    auto h = download(cnt.p, size_t(m.n_inst), s);
    return std::vector<int64_t>(h.begin(), h.end());
}

bool system_all_finite(const DevSystem& sys, hipStream_t s) {
    DBuf<int> flag;
    flag.alloc(1, s);
    flag.zero(s);
    const int64_t slots = sys.mesh->graph->n_slots;
    const int D = sys.mesh->dim;
    const struct { const double* p; int64_t n; } arrays[] = {
        {sys.Juu.val, slots * D * D}, {sys.Jpu.val, slots * D}, {sys.Jpp.val, slots}, {sys.F.p, sys.n_solve}};
    for (const auto& a : arrays) {
        const int g = int(std::min<int64_t>(4096, std::max<int64_t>(1, blocks_for(a.n, 256))));
        k_nonfinite<<<g, 256, 0, s>>>(a.p, a.n, flag.p);
        FR_LAUNCH_CHECK();
    }
    return download1(flag.p, s) == 0;
}

void mesh_update_inst(DevMesh& m, const double* du, const double* omega, double* u, double* phi, hipStream_t s,
                      const uint8_t* active, const double* phi_old) {
    const FixedDofs fix{active ? m.dir_free.p : nullptr, active, phi_old};
    k_update_free_inst<<<blocks_for(m.n_free, 256), 256, 0, s>>>(m.n_free, m.dim, m.node_of_free.p, m.inst_of_free.p,
                                                                 du, omega, fix, u, phi);
    FR_LAUNCH_CHECK();
    if (m.hanging) {
        k_fill_hanging<<<blocks_for(m.n_nodes, 256), 256, 0, s>>>(m.n_nodes, m.dim, m.free_of_node.p, m.node_of_free.p,
                                                                   m.con_ptr.p, m.con_master.p, m.con_w.p, u, phi);
        FR_LAUNCH_CHECK();
    }
}

// Linear extrapolation in time of the phase field (Formulation 1's phi_tilde):
// clip(phi1 + w (phi1 - phi2), 0, 1) at every free node; a hanging node takes the
// interpolation of its masters' extrapolated values, since the discrete field is fixed by its
// free values and clipping does not commute with the interpolation.  No contraction into an
// FMA, so the value is the plain product-then-sum.  A NaN input stays NaN.
__device__ inline double extrap_clip(double a, double b, double w) {
#pragma clang fp contract(off)
    const double v = a + w * (a - b);
    return v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v);
}

__global__ void __launch_bounds__(256) k_extrapolate(int64_t nn, const int32_t* __restrict__ free_of_node,
                                                     const int32_t* __restrict__ node_of_free,
                                                     const int32_t* __restrict__ con_ptr,
                                                     const int32_t* __restrict__ con_master,
                                                     const double* __restrict__ con_w,
                                                     const double* __restrict__ p1, const double* __restrict__ p2,
                                                     double w, double* __restrict__ out) {
    const int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (n >= nn) return;
    if (free_of_node == nullptr || free_of_node[n] >= 0) {
        out[n] = extrap_clip(p1[n], p2[n], w);
        return;
    }
    double v = 0.0;
    for (int32_t j = con_ptr[n]; j < con_ptr[n + 1]; ++j) {
        const int64_t src = node_of_free[con_master[j]];
        v += con_w[j] * extrap_clip(p1[src], p2[src], w);
    }
    out[n] = v;
}

void extrapolate(DevMesh& m, const double* p1, const double* p2, double w, double* out, hipStream_t s) {
    if (m.n_nodes == 0) return;
    const bool h = m.hanging;
    k_extrapolate<<<blocks_for(m.n_nodes, 256), 256, 0, s>>>(m.n_nodes, h ? m.free_of_node.p : nullptr,
                                                             m.node_of_free.p, m.con_ptr.p, m.con_master.p,
                                                             m.con_w.p, p1, p2, w, out);
    FR_LAUNCH_CHECK();
}

// Nodal value of `src` at vertex n of the source mesh: the node's own value, or for a
// hanging node the weighted values of its free masters.
__device__ __forceinline__ double src_value(int32_t n, int c, int ncomp, const int32_t* __restrict__ con_ptr,
                                            const int32_t* __restrict__ con_master,
                                            const double* __restrict__ con_w,
                                            const int32_t* __restrict__ node_of_free,
                                            const double* __restrict__ src) {
    if (con_ptr == nullptr) return src[int64_t(n) * ncomp + c];
    double v = 0.0;
    for (int32_t j = con_ptr[n]; j < con_ptr[n + 1]; ++j)
        v += con_w[j] * src[int64_t(node_of_free[con_master[j]]) * ncomp + c];
    return v;
}

// One thread per node of the refined mesh: the Q1 interpolant of the source cell that holds
// the node, at the node's local coordinates (exact for a refinement: the spaces are nested).
template <int D>
__global__ void __launch_bounds__(256) k_transfer(int64_t nn, int ncomp, const int32_t* __restrict__ loc_cell,
                                                  const double* __restrict__ loc_xi,
                                                  const int32_t* __restrict__ cells,
                                                  const int32_t* __restrict__ con_ptr,
                                                  const int32_t* __restrict__ con_master,
                                                  const double* __restrict__ con_w,
                                                  const int32_t* __restrict__ node_of_free,
                                                  const double* __restrict__ src, double* __restrict__ dst) {
    constexpr int NV = 1 << D;
    const int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (n >= nn) return;
    const int64_t cell = loc_cell[n];
    double xi[D];
#pragma unroll
    for (int k = 0; k < D; ++k) xi[k] = loc_xi[n * D + k];
    for (int c = 0; c < ncomp; ++c) {
        double v = 0.0;
#pragma unroll
        for (int a = 0; a < NV; ++a) {
            double w = 1.0;
#pragma unroll
            for (int k = 0; k < D; ++k) w *= ((a >> k) & 1) ? xi[k] : 1.0 - xi[k];
            v += w * src_value(cells[cell * NV + a], c, ncomp, con_ptr, con_master, con_w, node_of_free, src);
        }
        dst[n * ncomp + c] = v;
    }
}

void mesh_transfer(const DevMesh& from, const DevMesh& to, const double* src, int ncomp, double* dst,
                   hipStream_t s) {
    if (to.n_nodes == 0) return;
    const bool h = from.hanging;
    const int nb = blocks_for(to.n_nodes, 256);
#define FR_TRANSFER(D_)                                                                                    \
    k_transfer<D_><<<nb, 256, 0, s>>>(to.n_nodes, ncomp, to.parent_cell.p, to.parent_xi.p, from.cells.p,  \
                                      h ? from.con_ptr.p : nullptr, from.con_master.p, from.con_w.p,      \
                                      from.node_of_free.p, src, dst)
    if (from.dim == 2) FR_TRANSFER(2);
    else FR_TRANSFER(3);
#undef FR_TRANSFER
    FR_LAUNCH_CHECK();
}

// d u_comp / d x_k at local coordinates xi of a cell of edge h with nodal values un[a][comp].
template <int D>
__device__ __forceinline__ double cell_grad(const double (&un)[1 << D][D], int comp, int k, const double* xi,
                                            double h) {
    double g = 0.0;
#pragma unroll
    for (int a = 0; a < (1 << D); ++a) {
        double w = ((a >> k) & 1) ? 1.0 : -1.0;
#pragma unroll
        for (int t = 0; t < D; ++t)
            if (t != k) w *= ((a >> t) & 1) ? xi[t] : 1.0 - xi[t];
        g += w * un[a][comp];
    }
    return g / h;
}

template <int D>
__device__ __forceinline__ void cell_values(int64_t c, const int32_t* __restrict__ cells,
                                            const int32_t* __restrict__ con_ptr,
                                            const int32_t* __restrict__ con_master,
                                            const double* __restrict__ con_w,
                                            const int32_t* __restrict__ node_of_free, const double* __restrict__ u,
                                            double (&un)[1 << D][D]) {
#pragma unroll
    for (int a = 0; a < (1 << D); ++a)
#pragma unroll
        for (int comp = 0; comp < D; ++comp)
            un[a][comp] = src_value(cells[c * (1 << D) + a], comp, D, con_ptr, con_master, con_w, node_of_free, u);
}

// One thread per cell: the gradient-jump indicator (Kelly-type) of the displacement.
template <int D>
__global__ void __launch_bounds__(256) k_kelly(int64_t nc, const int32_t* __restrict__ cells,
                                               const double* __restrict__ cell_lo, const double* __restrict__ cell_h,
                                               const int32_t* __restrict__ fptr, const int32_t* __restrict__ fnbr,
                                               const int32_t* __restrict__ con_ptr,
                                               const int32_t* __restrict__ con_master,
                                               const double* __restrict__ con_w,
                                               const int32_t* __restrict__ node_of_free,
                                               const double* __restrict__ u, double* __restrict__ eta2) {
    constexpr int NV = 1 << D;
    const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    double uo[NV][D], un[NV][D];
    cell_values<D>(c, cells, con_ptr, con_master, con_w, node_of_free, u, uo);
    const double h = cell_h[c];
    double lo[D];
#pragma unroll
    for (int k = 0; k < D; ++k) lo[k] = cell_lo[c * D + k];
    double acc = 0.0;
    for (int j = 0; j < 2 * D; ++j) {
        const int k = j >> 1, side = j & 1;
        const double xk = lo[k] + side * h;
        for (int32_t e = fptr[c * 2 * D + j]; e < fptr[c * 2 * D + j + 1]; ++e) {
            const int64_t n = fnbr[e];
            cell_values<D>(n, cells, con_ptr, con_master, con_w, node_of_free, u, un);
            const double hn = cell_h[n];
            double lon[D];
#pragma unroll
            for (int t = 0; t < D; ++t) lon[t] = cell_lo[n * D + t];
            // integrate over the smaller of the two faces
            const bool finer = hn < h;
            const double rh = finer ? hn : h;
            double wq = 1.0;
#pragma unroll
            for (int t = 0; t < D - 1; ++t) wq *= 0.5 * rh;
            for (int g = 0; g < (1 << (D - 1)); ++g) {
                double x[D];
                int b = 0;
#pragma unroll
                for (int t = 0; t < D; ++t) {
                    if (t == k) {
                        x[t] = xk;
                        continue;
                    }
                    x[t] = (finer ? lon[t] : lo[t]) + rh * (((g >> b) & 1) ? kGP : kGM);
                    ++b;
                }
                double xi_o[D], xi_n[D];
#pragma unroll
                for (int t = 0; t < D; ++t) {
                    xi_o[t] = (x[t] - lo[t]) / h;
                    xi_n[t] = (x[t] - lon[t]) / hn;
                }
                double jj = 0.0;
#pragma unroll
                for (int comp = 0; comp < D; ++comp) {
                    const double d = cell_grad<D>(uo, comp, k, xi_o, h) - cell_grad<D>(un, comp, k, xi_n, hn);
                    jj += d * d;
                }
                acc += wq * jj;
            }
        }
    }
    eta2[c] = h / 24.0 * acc;
}

void mesh_kelly(DevMesh& m, const double* u, double* eta2, hipStream_t s) {
    if (m.n_cells == 0) return;
    if (m.face_ptr.p == nullptr) {
        std::vector<int32_t> ptr, nbr;
        face_neighbors(m.host, ptr, nbr);
        m.face_ptr.upload(ptr, s);
        m.face_nbr.upload(nbr.empty() ? std::vector<int32_t>{0} : nbr, s);
        FR_HIP(hipStreamSynchronize(s));          // the host tables go out of scope
    }
    const bool h = m.hanging;
    const int nb = blocks_for(m.n_cells, 256);
#define FR_KELLY(D_)                                                                                       \
    k_kelly<D_><<<nb, 256, 0, s>>>(m.n_cells, m.cells.p, m.cell_lo.p, m.cell_h.p, m.face_ptr.p, m.face_nbr.p, \
                                   h ? m.con_ptr.p : nullptr, m.con_master.p, m.con_w.p, m.node_of_free.p, u, \
                                   eta2)
    if (m.dim == 2) FR_KELLY(2);
    else FR_KELLY(3);
#undef FR_KELLY
    FR_LAUNCH_CHECK();
}

// One thread per cell: the crack-region mark.
template <int D>
__global__ void __launch_bounds__(256) k_mark_crack(int64_t nc, const int32_t* __restrict__ cells,
                                                    const double* __restrict__ cell_h,
                                                    const int32_t* __restrict__ con_ptr,
                                                    const int32_t* __restrict__ con_master,
                                                    const double* __restrict__ con_w,
                                                    const int32_t* __restrict__ node_of_free,
                                                    const double* __restrict__ phi, double phi_max,
                                                    double h_target, uint8_t* __restrict__ flags) {
    constexpr int NV = 1 << D;
    const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    uint8_t f = 0;
    if (cell_h[c] > h_target) {
#pragma unroll
        for (int a = 0; a < NV; ++a)
            if (src_value(cells[c * NV + a], 0, 1, con_ptr, con_master, con_w, node_of_free, phi) < phi_max) f = 1;
    }
    flags[c] = f;
}

void mesh_mark_crack(const DevMesh& m, const double* phi, double phi_max, double h_target, uint8_t* flags_dev,
                     hipStream_t s) {
    if (m.n_cells == 0) return;
    const bool h = m.hanging;
    const int nb = blocks_for(m.n_cells, 256);
#define FR_MARK(D_)                                                                                        \
    k_mark_crack<D_><<<nb, 256, 0, s>>>(m.n_cells, m.cells.p, m.cell_h.p, h ? m.con_ptr.p : nullptr,       \
                                        m.con_master.p, m.con_w.p, m.node_of_free.p, phi, phi_max,         \
                                        h_target, flags_dev)
    if (m.dim == 2) FR_MARK(2);
    else FR_MARK(3);
#undef FR_MARK
    FR_LAUNCH_CHECK();
}

void mesh_update(DevMesh& m, const double* du, double omega, double* u, double* phi, hipStream_t s,
                 const uint8_t* active, const double* phi_old) {
    const FixedDofs fix{active ? m.dir_free.p : nullptr, active, phi_old};
    k_update_free<<<blocks_for(m.n_free, 256), 256, 0, s>>>(m.n_free, m.dim, m.node_of_free.p, du, omega, fix, u,
                                                            phi);
    FR_LAUNCH_CHECK();
    if (m.hanging) {
        k_fill_hanging<<<blocks_for(m.n_nodes, 256), 256, 0, s>>>(m.n_nodes, m.dim, m.free_of_node.p, m.node_of_free.p,
                                                                   m.con_ptr.p, m.con_master.p, m.con_w.p, u, phi);
        FR_LAUNCH_CHECK();
    }
}

// TCV and COD of every instance with the caller's device buffers: xs (the sample abscissae,
// already on the device), part (at least blocks x max(1, n_cod) doubles for the largest
// instance) and out (max(1, n_cod) doubles).  Results go straight into the host arrays.
static void functionals_into(DevMesh& m, const double* u, const double* phi, const double* xs, int n_cod,
                             double* cod, double* tcv, double* part, double* out, hipStream_t s) {
    MeshView mv = view(m);
    const HostMesh& hm = m.host;
    const int D1 = m.dim - 1;
    // one reduction per instance over its cell range (instances never share cells)
    for (int i = 0; i < m.n_inst; ++i) {
        const int64_t c0 = hm.cell_off[size_t(i)], c1 = hm.cell_off[size_t(i) + 1];
        const int nb = blocks_for(std::max<int64_t>(1, c1 - c0), 256);
        if (tcv) {
            if (m.dim == 2) {
                if (m.hanging) k_tcv<2, true><<<nb, 256, 0, s>>>(c0, c1, mv, u, phi, part);
                else k_tcv<2, false><<<nb, 256, 0, s>>>(c0, c1, mv, u, phi, part);
            } else {
                if (m.hanging) k_tcv<3, true><<<nb, 256, 0, s>>>(c0, c1, mv, u, phi, part);
                else k_tcv<3, false><<<nb, 256, 0, s>>>(c0, c1, mv, u, phi, part);
            }
            FR_LAUNCH_CHECK();
            k_sum_rows<<<1, 256, 0, s>>>(part, nb, 1, 0, 1, out);
            FR_LAUNCH_CHECK();
            FR_HIP(hipMemcpyAsync(tcv + i, out, sizeof(double), hipMemcpyDeviceToHost, s));
            FR_HIP(hipStreamSynchronize(s));
        }
        if (cod && n_cod > 0) {
            dim3 grid(nb, n_cod);
            const double* xi = xs + size_t(i) * n_cod * D1;
            if (m.dim == 2) {
                if (m.hanging) k_cod<2, true><<<grid, 256, 0, s>>>(c0, c1, mv, u, phi, xi, part);
                else k_cod<2, false><<<grid, 256, 0, s>>>(c0, c1, mv, u, phi, xi, part);
            } else {
                if (m.hanging) k_cod<3, true><<<grid, 256, 0, s>>>(c0, c1, mv, u, phi, xi, part);
                else k_cod<3, false><<<grid, 256, 0, s>>>(c0, c1, mv, u, phi, xi, part);
            }
            FR_LAUNCH_CHECK();
            k_sum_rows<<<n_cod, 256, 0, s>>>(part, nb, n_cod, nb, 1, out);
            FR_LAUNCH_CHECK();
            FR_HIP(hipMemcpyAsync(cod + size_t(i) * n_cod, out, size_t(n_cod) * sizeof(double),
                                  hipMemcpyDeviceToHost, s));
            FR_HIP(hipStreamSynchronize(s));
        }
    }
    FR_HIP(hipStreamSynchronize(s));
}

// Partial-sum blocks of the largest instance (the reductions of every instance reuse them).
static int64_t functionals_blocks(const DevMesh& m) {
    int64_t nb = 1;
    for (int i = 0; i < m.n_inst; ++i) {
        const int64_t nc = m.host.cell_off[size_t(i) + 1] - m.host.cell_off[size_t(i)];
        nb = std::max<int64_t>(nb, blocks_for(std::max<int64_t>(1, nc), 256));
    }
    return nb;
}

void mesh_functionals(DevMesh& m, const double* u, const double* phi, const double* cod_x, int n_cod, double* cod,
                      double* tcv, hipStream_t s) {
    const int D1 = m.dim - 1;
    DBuf<double> part, out, xs;
    part.alloc(size_t(functionals_blocks(m)) * size_t(std::max(1, n_cod)), s);
    out.alloc(size_t(std::max(1, n_cod)), s);
    if (n_cod > 0) {
        xs.alloc(size_t(m.n_inst) * n_cod * D1, s);
        xs.upload(cod_x, size_t(m.n_inst) * n_cod * D1, s);
    }
    functionals_into(m, u, phi, xs.p, n_cod, cod, tcv, part.p, out.p, s);
}

}  // namespace fr

// ---- functionals without allocation -------------------------------------------------------
// Device memory of fracture_functionals_noalloc: the sample abscissae, the per-block partial
// sums and the reduced values live in this fixed array (each device holds its own copy for the
// life of the process).  Host code reaches it only through the address hipGetSymbolAddress
// returns for the current device.
static __device__ __align__(256) double scratch[fr::kFunctionalsScratchDoubles];

namespace fr {

int64_t functionals_scratch_need(const DevMesh& m, int n_cod) {
    const int64_t nc = std::max(1, n_cod);
    return int64_t(m.n_inst) * n_cod * (m.dim - 1) + nc + functionals_blocks(m) * nc;
}

// The current device's address of `scratch`, looked up once per device (with it current).
static double* functionals_scratch() {
    static std::mutex mu;
    static void* addr[kMaxScratchDevices] = {};
    int dev = 0;
    FR_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxScratchDevices) fail(FR_EDEVICE, "functionals_noalloc: device ordinal out of range");
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr) {
            (void)hipGetLastError();
            fail(FR_EDEVICE, std::string("functionals_noalloc: hipGetSymbolAddress failed: ") + hipGetErrorString(e));
        }
        addr[dev] = p;
    }
    return static_cast<double*>(addr[dev]);
}

void mesh_functionals_noalloc(DevMesh& m, const double* u, const double* phi, const double* cod_x, int n_cod,
                              double* cod, double* tcv, hipStream_t s) {
    if (functionals_scratch_need(m, n_cod) > int64_t(kFunctionalsScratchDoubles))
        fail(FR_EINVAL, "functionals_noalloc: mesh and n_cod need more than the fixed scratch");
    double* base = functionals_scratch();
    const int64_t nx = int64_t(m.n_inst) * n_cod * (m.dim - 1);
    double* xs = base;
    double* out = base + nx;
    double* part = out + std::max(1, n_cod);
    if (nx > 0) FR_HIP(hipMemcpyAsync(xs, cod_x, size_t(nx) * sizeof(double), hipMemcpyHostToDevice, s));
    functionals_into(m, u, phi, xs, n_cod, cod, tcv, part, out, s);
}

}  // namespace fr
