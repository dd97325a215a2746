// Flexible GMRES (right preconditioned, restarted) for the masked Newton system of Section 3,
// FP64, for one instance or many independent instances solved in lockstep.
//
// The solve vector of a batch is the disjoint union of the instances (u block, then phi
// block, each instance-major), so SpMV and the V-cycles run on the union unchanged.  Every
// reduction is segmented: vector kernels run over a table of blocks that never straddle an
// instance, partial sums are combined per instance in a fixed order (deterministic).
// Arnoldi uses classical Gram-Schmidt with one re-orthogonalisation pass (CGS2): one
// multi-vector dot sweep, one fused update + dot sweep, one update + norm sweep.  Givens
// rotations, the convergence test and the back substitution run on the device, one thread
// per instance; the host reads one flag word per instance per iteration to stop.
//
// The Krylov index j of the current cycle lives on the device (State::j): every kernel of an
// Arnoldi step reads it there (basis pointers, vector counts, the Givens column), and the step's
// last kernel advances it.  An Arnoldi step is therefore the same launch sequence for every j,
// and with use_graphs it is captured once per preconditioner setup (both V-cycles, J z,
// Gram-Schmidt, rotations, summary) as one HIP graph that the host replays once per iteration.
#include <algorithm>
#include <cmath>
#include <vector>

#include "profile.h"
#include "system.h"

namespace fr {
namespace {

constexpr int kE = 4;                 // elements per thread in the vector sweeps
// the second Gram-Schmidt pass runs where the first cut |w| by more than this factor
// (the orthogonality left is then at least 2^-10 u-level: about 1e-13)
constexpr double kReorthEta = 1.0 / 1024.0;
// the host waits for an iteration's convergence flags once some instance's residual estimate
// is within this factor of its target
constexpr double kSpecRatio = 64.0;
constexpr int kChunk = 256 * kE;      // elements per block
constexpr int kMaxM = 120;            // largest restart length

struct Seg {
    const int64_t* start;   // [nb] first element of the block
    const int32_t* len;     // [nb] elements in the block (<= kChunk)
    const int32_t* inst;    // [nb] instance of the block
};

// part[v * nb + g] = sum over segment g of V_v[i] w[i] (v < nv), and with `self` also
// part[nv * nb + g] = sum of w[i]^2.  Segments of an instance whose flag in `need` is 0 are
// skipped (need may be null); the grid may be smaller than the segment count.
__global__ void __launch_bounds__(256) k_seg_dots(const double* __restrict__ V, int64_t n, const int* __restrict__ jp,
                                                  const double* __restrict__ w, Seg sg, int nb,
                                                  double* __restrict__ part, const int* __restrict__ need, int self) {
    __shared__ double sh[kMaxM + 8][4];
    const int nv = *jp + 1;   // V_0 .. V_j
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int rows = nv + (self ? 1 : 0);
    for (int g = blockIdx.x; g < nb; g += gridDim.x) {
        if (need && !need[sg.inst[g]]) continue;
        const int64_t s0 = sg.start[g];
        const int len = sg.len[g];
        double wv[kE];
#pragma unroll
        for (int e = 0; e < kE; ++e) {
            const int o = threadIdx.x + 256 * e;
            wv[e] = o < len ? w[s0 + o] : 0.0;
        }
        for (int v = 0; v < nv; ++v) {
            const double* Vv = V + int64_t(v) * n + s0;
            double acc = 0.0;
#pragma unroll
            for (int e = 0; e < kE; ++e) {
                const int o = threadIdx.x + 256 * e;
                if (o < len) acc += Vv[o] * wv[e];
            }
            acc = wave_sum(acc);
            if (lane == 0) sh[v][wave] = acc;
        }
        if (self) {
            double acc = 0.0;
#pragma unroll
            for (int e = 0; e < kE; ++e) acc += wv[e] * wv[e];   // wv is 0 past len
            acc = wave_sum(acc);
            if (lane == 0) sh[nv][wave] = acc;
        }
        __syncthreads();
        for (int v = threadIdx.x; v < rows; v += blockDim.x)
            part[int64_t(v) * nb + g] = sh[v][0] + sh[v][1] + sh[v][2] + sh[v][3];
        __syncthreads();
    }
}

// w -= sum_k c_inst[k] V_k; part[g] = sum of the new w^2 over segment g.  Segments of an
// instance whose flag in `need` is 0 are skipped (need may be null); the grid may be
// smaller than the segment count.
__global__ void __launch_bounds__(256) k_seg_update_norm(const double* __restrict__ V, int64_t n,
                                                         const int* __restrict__ jp, const double* __restrict__ c,
                                                         int cstride, double* __restrict__ w, Seg sg, int nb,
                                                         double* __restrict__ part, const int* __restrict__ need) {
    __shared__ double sh[16];
    __shared__ double cs[kMaxM + 8];
    const int nv = *jp + 1;
    for (int g = blockIdx.x; g < nb; g += gridDim.x) {
        if (need && !need[sg.inst[g]]) continue;
        const int64_t s0 = sg.start[g];
        const int len = sg.len[g];
        const double* ci = c + int64_t(sg.inst[g]) * cstride;
        for (int k = threadIdx.x; k < nv; k += blockDim.x) cs[k] = ci[k];
        __syncthreads();
        double acc = 0.0;
#pragma unroll
        for (int e = 0; e < kE; ++e) {
            const int o = threadIdx.x + 256 * e;
            if (o < len) {
                double t = w[s0 + o];
                for (int k = 0; k < nv; ++k) t -= cs[k] * V[int64_t(k) * n + s0 + o];
                w[s0 + o] = t;
                acc += t * t;
            }
        }
        const double sum = block_sum(acc, sh);
        if (threadIdx.x == 0) part[g] = sum;
        __syncthreads();
    }
}

// r = F - r (r holds J x on entry, or nothing when from_zero: r = F); part[b] = sum r^2
__global__ void __launch_bounds__(256) k_seg_resid(const double* __restrict__ F, double* __restrict__ r, int from_zero,
                                                   Seg sg, double* __restrict__ part) {
    __shared__ double sh[16];
    const int64_t s0 = sg.start[blockIdx.x];
    const int len = sg.len[blockIdx.x];
    double acc = 0.0;
#pragma unroll
    for (int e = 0; e < kE; ++e) {
        const int o = threadIdx.x + 256 * e;
        if (o < len) {
            const double t = from_zero ? F[s0 + o] : F[s0 + o] - r[s0 + o];
            r[s0 + o] = t;
            acc += t * t;
        }
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// dst = src * scale[inst] (with jp: dst + (*jp + 1) n, the next basis vector); also the
// preconditioner's input when it is staged: the same values in FP32 (u part, solve index < n_u,
// to f_u; phi part to f_p) or in FP64 (d_copy).
__global__ void __launch_bounds__(256) k_seg_scale(const double* __restrict__ src, double* __restrict__ dst,
                                                   const int* __restrict__ jp, int64_t n,
                                                   const double* __restrict__ scale, Seg sg, float* __restrict__ f_u,
                                                   float* __restrict__ f_p, int64_t n_u, double* __restrict__ d_copy) {
    if (jp) dst += int64_t(*jp + 1) * n;
    const int64_t s0 = sg.start[blockIdx.x];
    const int len = sg.len[blockIdx.x];
    const double a = scale[sg.inst[blockIdx.x]];
#pragma unroll
    for (int e = 0; e < kE; ++e) {
        const int o = threadIdx.x + 256 * e;
        if (o < len) {
            const int64_t i = s0 + o;
            const double v = a * src[i];
            dst[i] = v;
            if (d_copy) d_copy[i] = v;
            if (f_u) {
                if (i < n_u) f_u[i] = float(v);
                else f_p[i - n_u] = float(v);
            }
        }
    }
}

// x += sum_k y_inst[k] Z_k (Z FP64, or FP32 widened exactly)
template <typename TZ>
__global__ void __launch_bounds__(256) k_seg_combine(const TZ* __restrict__ Z, int64_t n, int nz,
                                                     const double* __restrict__ y, int ystride,
                                                     double* __restrict__ x, Seg sg) {
    __shared__ double ys[kMaxM + 8];
    const int64_t s0 = sg.start[blockIdx.x];
    const int len = sg.len[blockIdx.x];
    const double* yi = y + int64_t(sg.inst[blockIdx.x]) * ystride;
    for (int k = threadIdx.x; k < nz; k += blockDim.x) ys[k] = yi[k];
    __syncthreads();
#pragma unroll
    for (int e = 0; e < kE; ++e) {
        const int o = threadIdx.x + 256 * e;
        if (o < len) {
            double t = x[s0 + o];
            for (int k = 0; k < nz; ++k) t += ys[k] * double(Z[int64_t(k) * n + s0 + o]);
            x[s0 + o] = t;
        }
    }
}

// out[inst * stride + v] = sum of part[v * nb + b] over the blocks of the instance (only
// for instances whose flag in `only` is set, when given; with jp only for v < *jp + 1 + extra,
// the grid covering the largest count).  Four independent partial sums per thread keep several
// loads in flight; the order is fixed.
constexpr int kReduceT = 512;
__global__ void __launch_bounds__(kReduceT) k_seg_reduce(const double* __restrict__ part, int nb,
                                                         const int32_t* __restrict__ bptr, double* __restrict__ out,
                                                         int stride, const int* __restrict__ only = nullptr,
                                                         const int* __restrict__ jp = nullptr, int extra = 0) {
    __shared__ double sh[16];
    const int v = blockIdx.x, inst = blockIdx.y;
    if (only && !only[inst]) return;
    if (jp && v >= *jp + 1 + extra) return;
    const double* p = part + int64_t(v) * nb;
    const int b1 = bptr[inst + 1];
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    int b = bptr[inst] + threadIdx.x;
    for (; b + 3 * kReduceT < b1; b += 4 * kReduceT) {
#pragma unroll
        for (int q = 0; q < 4; ++q) a[q] += p[b + q * kReduceT];
    }
    for (; b < b1; b += kReduceT) a[0] += p[b];
    const double s = block_sum((a[0] + a[1]) + (a[2] + a[3]), sh);
    if (threadIdx.x == 0) out[int64_t(inst) * stride + v] = s;
}

// Per-instance solver state (device).
struct State {
    double* h1;      // [ni][m+2] pass-1 coefficients (then the Hessenberg column)
    double* h2;      // [ni][m+2] pass-2 coefficients
    double* nrm2;    // [ni] ||w||^2 after orthogonalisation
    double* H;       // [ni][(m+1) m] upper triangle after rotations, column-major
    double* cs;      // [ni][m]
    double* sn;      // [ni][m]
    double* g;       // [ni][m+1]
    double* y;       // [ni][m]
    double* target;  // [ni] rtol ||F_i||
    double* scale;   // [ni] 1/||w|| for the next basis vector (0 once done)
    double* beta2;   // [ni] squared residual norm
    int* done;       // [ni] converged (or stopped) in this cycle
    int* jused;      // [ni] Krylov columns used by the instance in this cycle
    int* bad;        // [ni] non-finite residual (the right-hand side or the iterate)
    int* need;       // [ni] the second Gram-Schmidt pass is applied in this iteration
    int* brk;        // [ni] breakdown: non-finite Arnoldi quantities, or a zero Arnoldi norm
                     //      whose cycle left the true residual above the target
    int* zhit;       // [ni] the last cycle ended on a zero Arnoldi norm
    int* j;          // [1] Krylov index of the next Arnoldi step in the current cycle
};

// Classical Gram-Schmidt with the second pass only where it is needed: after one pass the
// part of w left in the span of the basis is of the order of the unit roundoff times
// |w_before| / |w_after|, so the pass is repeated where the norm dropped below eta times its
// value before (h1[nv] holds |w_before|^2, nrm2 |w_after|^2).  h2 is cleared everywhere;
// the second pass fills it where it runs.
__global__ void k_reorth_decide(int ni, int m, State st, double eta2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ni) return;
    const int nv = *st.j + 1;
    double* h2 = st.h2 + int64_t(i) * (m + 2);
    for (int k = 0; k <= nv; ++k) h2[k] = 0.0;
    const double before = st.h1[int64_t(i) * (m + 2) + nv];
    const double after = st.nrm2[i];
    st.need[i] = (!st.done[i] && !(after >= eta2 * before)) ? 1 : 0;   // NaN -> second pass
}

// new cycle: g = (beta, 0, ...), scale = 1/beta, done when beta <= target.  A previous cycle
// that ended on a zero Arnoldi norm (an invariant Krylov space) without reaching the target is a
// breakdown: the next cycle would rebuild the same space.
__global__ void k_cycle_start(int ni, int m, State st) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ni) return;
    const double beta = sqrt(st.beta2[i]);
    for (int k = 0; k <= m; ++k) st.g[int64_t(i) * (m + 1) + k] = 0.0;
    st.g[int64_t(i) * (m + 1)] = beta;
    const bool fin = isfinite(beta);
    if (!fin) st.bad[i] = 1;
    if (fin && st.zhit[i] && !(beta <= st.target[i])) st.brk[i] = 1;
    st.zhit[i] = 0;
    const bool dn = !fin || st.brk[i] || beta <= st.target[i];
    st.done[i] = dn ? 1 : 0;
    st.jused[i] = 0;
    st.scale[i] = (!dn && beta > 0.0) ? 1.0 / beta : 0.0;
}

// Hessenberg column j: combine the two passes, apply the previous rotations, make the new
// one, update g, test convergence.  Instances already done are left untouched.
__global__ void k_givens(int ni, int m, State st) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ni) return;
    const int j = *st.j;
    if (st.done[i]) {
        st.scale[i] = 0.0;
        return;
    }
    double* h = st.h1 + int64_t(i) * (m + 2);
    const double* h2 = st.h2 + int64_t(i) * (m + 2);
    double* cs = st.cs + int64_t(i) * m;
    double* sn = st.sn + int64_t(i) * m;
    double* g = st.g + int64_t(i) * (m + 1);
    double* H = st.H + int64_t(i) * (m + 1) * m;
    for (int k = 0; k <= j; ++k) h[k] += h2[k];
    const double nw = sqrt(st.nrm2[i]);
    bool fin_col = isfinite(nw);
    for (int k = 0; k <= j; ++k) fin_col = fin_col && isfinite(h[k]);
    if (!fin_col) {
        // breakdown with finite inputs (e.g. a preconditioner that overflowed): the column is
        // dropped, so the update uses the j finite columns before it
        st.brk[i] = 1;
        st.done[i] = 1;
        st.jused[i] = j;
        st.scale[i] = 0.0;
        return;
    }
    h[j + 1] = nw;
    for (int k = 0; k < j; ++k) {
        const double a = h[k], b = h[k + 1];
        h[k] = cs[k] * a + sn[k] * b;
        h[k + 1] = -sn[k] * a + cs[k] * b;
    }
    const double a = h[j], b = h[j + 1];
    const double r = hypot(a, b);
    cs[j] = r > 0.0 ? a / r : 1.0;
    sn[j] = r > 0.0 ? b / r : 0.0;
    h[j] = r;
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
    for (int k = 0; k <= j; ++k) H[int64_t(j) * (m + 1) + k] = h[k];
    st.jused[i] = j + 1;
    const bool fin = isfinite(g[j + 1]);
    if (!fin) st.brk[i] = 1;
    const bool conv = fabs(g[j + 1]) <= st.target[i];
    const bool inv = !(nw > 0.0);      // invariant subspace: the solution is in the basis
    if (inv) st.zhit[i] = 1;           // unless the true residual says otherwise (next cycle)
    if (!fin || conv || inv || j + 1 == m) st.done[i] = 1;
    st.scale[i] = (st.done[i] || !(nw > 0.0)) ? 0.0 : 1.0 / nw;
}

// The host's view of iteration j: whether every instance is done, and how far the running
// ones still are from their targets, written to out[j & 1] (the host reads the two slots
// alternately); then the step's Krylov index advances.
__global__ void k_summary(int ni, int m, State st, IterSummary* out) {
    __shared__ int all;
    __shared__ double worst;
    const int j = *st.j;
    if (threadIdx.x == 0) { all = 1; worst = 0.0; }
    __syncthreads();
    for (int i = threadIdx.x; i < ni; i += blockDim.x) {
        if (st.done[i]) continue;
        atomicAnd(&all, 0);
        const double r = fabs(st.g[int64_t(i) * (m + 1) + j + 1]) / st.target[i];
        // doubles compare as their bit patterns when non-negative (NaN: stays large)
        atomicMax(reinterpret_cast<unsigned long long*>(&worst), __double_as_longlong(isfinite(r) ? r : 1e300));
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        IterSummary& o = out[j & 1];
        o.all_done = all;
        o.pad = 0;
        o.ratio = worst;
        *st.j = j + 1;
    }
}

__global__ void k_set_int(int* p, int v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// y = H^-1 g on the jused x jused upper triangle
__global__ void k_backsolve(int ni, int m, State st) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ni) return;
    const int ju = st.jused[i];
    const double* H = st.H + int64_t(i) * (m + 1) * m;
    const double* g = st.g + int64_t(i) * (m + 1);
    double* y = st.y + int64_t(i) * m;
    for (int k = 0; k < m; ++k) y[k] = 0.0;
    for (int r = ju - 1; r >= 0; --r) {
        double t = g[r];
        for (int k = r + 1; k < ju; ++k) t -= H[int64_t(k) * (m + 1) + r] * y[k];
        const double d = H[int64_t(r) * (m + 1) + r];
        y[r] = d != 0.0 ? t / d : 0.0;
    }
}

}  // namespace

// Block table of the segmented sweeps (built once per system / restart length).
static void build_table(DevSystem& sys, DevKrylov& ws, hipStream_t s) {
    const HostMesh& hm = sys.mesh->host;
    const int D = sys.mesh->dim;
    const int64_t nf = hm.n_free;
    std::vector<int64_t> st;
    std::vector<int32_t> ln, in, bp;
    for (int i = 0; i < hm.n_inst; ++i) {
        bp.push_back(int32_t(st.size()));
        const int64_t f0 = hm.free_off[size_t(i)], f1 = hm.free_off[size_t(i) + 1];
        const int64_t ranges[2][2] = {{D * f0, D * f1}, {D * nf + f0, D * nf + f1}};
        for (auto& r : ranges)
            for (int64_t a = r[0]; a < r[1]; a += kChunk) {
                st.push_back(a);
                ln.push_back(int32_t(std::min<int64_t>(kChunk, r[1] - a)));
                in.push_back(i);
            }
    }
    bp.push_back(int32_t(st.size()));
    ws.seg_start.upload(st, s);
    ws.seg_len.upload(ln, s);
    ws.seg_inst.upload(in, s);
    ws.seg_bptr.upload(bp, s);
    ws.nb = int(st.size());
    ws.n_inst = hm.n_inst;
}

// Doubles the basis capacity (up to the restart length), keeping V_0..V_j and Z_0..Z_{j-1}
// (Z in the precision it is kept in).
template <typename T>
static void grow_keep(DBuf<T>& b, size_t keep, size_t count, hipStream_t s) {
    if (!b.p) return;
    DBuf<T> nb;
    nb.alloc(count, s);
    if (keep) FR_HIP(hipMemcpyAsync(nb.p, b.p, keep * sizeof(T), hipMemcpyDeviceToDevice, s));
    b = std::move(nb);
}

static void grow_basis(DevKrylov& ws, int j, hipStream_t s) {
    const int cap = std::min(ws.m, std::max(j + 1, 2 * ws.cap));
    const size_t n = size_t(ws.n);
    grow_keep(ws.V, size_t(j + 1) * n, size_t(cap + 1) * n, s);
    grow_keep(ws.Z, size_t(j) * n, size_t(cap) * n, s);
    grow_keep(ws.Z32, size_t(j) * n, size_t(cap) * n, s);
    ws.cap = cap;
    ws.layout = next_epoch();
}

// Everything one Arnoldi step needs; the step itself reads the Krylov index from the device.
struct StepCtx {
    DevSystem* sys;
    DevAmg* amg;
    DevKrylov* ws;
    State st;
    Seg sg;
    int ni, M;
    int64_t n;
    bool z32, staged;          // staged: the preconditioner runs from / to the fixed staged buffers
    float* f_u;
    float* f_p;
    double* d_copy;            // staging targets of k_seg_scale (null: none)
    void* vout;                // staged preconditioner output
    bool mf;                   // J x with the displacement rows matrix-free
    bool mf_phi;               // and the phase-field rows too
};

// y = J x, x also copied to xcopy + (*jp) n when xcopy is given; the displacement rows
// matrix-free where the preconditioner's fine displacement level is (uniform 2d meshes), the
// phase-field rows too where its fine phase-field level is as well, else from the stored blocks.
template <typename TX>
static void jmul(const StepCtx& c, const TX* x, double* y, TX* xcopy, const int* jp, hipStream_t s) {
    if (c.mf) mf_jspmv<TX>(*c.sys, c.mf_phi, x, y, xcopy, jp, c.n, s);
    else if (xcopy) jspmv_copy(*c.sys, x, y, xcopy, jp, c.n, s);
    else jspmv(*c.sys, x, y, s);
}

// One Arnoldi step at the device's Krylov index j: z = M^-1 v_j (kept as Z_j), w = J z, CGS2
// against V_0..V_j, the Hessenberg column and its rotations, v_{j+1} = w / |w| (and the next
// staged preconditioner input), the summary of the step, j + 1.  j_host is used only for the
// unstaged preconditioner call (direct launches); a staged step is the same launch sequence for
// every j, so it can be captured.
static void arnoldi_step(const StepCtx& c, int j_host, hipStream_t s) {
    DevSystem& sys = *c.sys;
    DevKrylov& ws = *c.ws;
    const State& st = c.st;
    const int64_t n = c.n;
    const int nb = ws.nb;
    const int ni = c.ni;
    const int gi = int(ceil_div(ni, 64));
    if (c.staged) {
        // both V-cycles from the staged input; the product J z copies z into Z_j as it reads it
        amg_precondition_staged(*c.amg, s);
        if (c.z32) jmul(c, static_cast<const float*>(c.vout), ws.w.p, ws.Z32.p, st.j, s);
        else jmul(c, static_cast<const double*>(c.vout), ws.w.p, ws.Z.p, st.j, s);
    } else if (c.z32) {
        float* Zj = ws.Z32.p + int64_t(j_host) * n;
        amg_precondition32(*c.amg, nullptr, Zj, s);   // input staged by k_seg_scale
        jmul<float>(c, Zj, ws.w.p, nullptr, nullptr, s);
    } else {
        double* Zj = ws.Z.p + int64_t(j_host) * n;
        amg_precondition(*c.amg, ws.V.p + int64_t(j_host) * n, Zj, s);
        jmul<double>(c, Zj, ws.w.p, nullptr, nullptr, s);
    }
    // Gram-Schmidt reductions cover the largest vector count of the current basis; rows past
    // the step's own count return at once
    const int rows = ws.cap + 2;
    const int nv_h = j_host + 1;   // for the profile's byte counts only
    const double md_bytes = double(nv_h + 1) * double(n) * 8.0;
    const double up_bytes = double(nv_h + 2) * double(n) * 8.0;
    const int gc = std::min(nb, 1024);   // grid of the conditional second pass
    double* part = ws.part.p;
    const int M = c.M;
    {
        ProfScope ps("gs_multidot", s, md_bytes);
        k_seg_dots<<<nb, 256, 0, s>>>(ws.V.p, n, st.j, ws.w.p, c.sg, nb, part, nullptr, 1);
        FR_LAUNCH_CHECK();
    }
    k_seg_reduce<<<dim3(rows, ni), kReduceT, 0, s>>>(part, nb, ws.seg_bptr.p, st.h1, M + 2, nullptr, st.j, 1);
    FR_LAUNCH_CHECK();
    {
        ProfScope ps("gs_update", s, up_bytes);
        k_seg_update_norm<<<nb, 256, 0, s>>>(ws.V.p, n, st.j, st.h1, M + 2, ws.w.p, c.sg, nb, part, nullptr);
        FR_LAUNCH_CHECK();
    }
    k_seg_reduce<<<dim3(1, ni), kReduceT, 0, s>>>(part, nb, ws.seg_bptr.p, st.nrm2, 1);
    FR_LAUNCH_CHECK();
    k_reorth_decide<<<gi, 64, 0, s>>>(ni, M, st, kReorthEta * kReorthEta);
    FR_LAUNCH_CHECK();
    {
        // the bytes depend on how many instances need the pass (a device decision)
        ProfScope ps("gs_second_pass", s, 0.0);
        k_seg_dots<<<gc, 256, 0, s>>>(ws.V.p, n, st.j, ws.w.p, c.sg, nb, part, st.need, 0);
        FR_LAUNCH_CHECK();
        k_seg_reduce<<<dim3(rows, ni), kReduceT, 0, s>>>(part, nb, ws.seg_bptr.p, st.h2, M + 2, st.need, st.j, 0);
        FR_LAUNCH_CHECK();
        k_seg_update_norm<<<gc, 256, 0, s>>>(ws.V.p, n, st.j, st.h2, M + 2, ws.w.p, c.sg, nb, part, st.need);
        FR_LAUNCH_CHECK();
        k_seg_reduce<<<dim3(1, ni), kReduceT, 0, s>>>(part, nb, ws.seg_bptr.p, st.nrm2, 1, st.need);
        FR_LAUNCH_CHECK();
    }
    k_givens<<<gi, 64, 0, s>>>(ni, M, st);
    FR_LAUNCH_CHECK();
    k_seg_scale<<<nb, 256, 0, s>>>(ws.w.p, ws.V.p, st.j, n, st.scale, c.sg, c.f_u, c.f_p, sys.n_u, c.d_copy);
    FR_LAUNCH_CHECK();
    k_summary<<<1, 64, 0, s>>>(ni, M, st, ws.dsum.p);
    FR_LAUNCH_CHECK();
    FR_HIP(hipMemcpyAsync(ws.hsum, ws.dsum.p, 2 * sizeof(IterSummary), hipMemcpyDeviceToHost, s));
}

// The captured Arnoldi step of the current preconditioner, basis capacity and workspace
// (captured again when any of them changed).  The capture runs on a stream of the workspace (the
// caller's may be the legacy default stream, which cannot be captured) after s has drained, so
// that every buffer it records exists.
static hipGraphExec_t step_graph(const StepCtx& c, hipStream_t s) {
    DevKrylov& ws = *c.ws;
    const IterKey key{c.sys, c.sys->version, c.amg->epoch, ws.layout};
    if (ws.step_exec && ws.step_key == key) return ws.step_exec;
    FR_HIP(hipStreamSynchronize(s));
    ws.drop_step();
    if (!ws.cstream) FR_HIP(hipStreamCreateWithFlags(&ws.cstream, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    FR_HIP(hipStreamBeginCapture(ws.cstream, hipStreamCaptureModeThreadLocal));
    try {
        arnoldi_step(c, 0, ws.cstream);
    } catch (...) {
        (void)hipStreamEndCapture(ws.cstream, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
    }
    FR_HIP(hipStreamEndCapture(ws.cstream, &g));
    hipGraphExec_t ex = nullptr;
    const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    FR_HIP(e);
    ws.step_exec = ex;
    ws.step_key = key;
    ++ws.captures;
    return ex;
}

fr_status fgmres(DevSystem& sys, DevAmg& amg, const fr_solve_opts& o, double* du, fr_solve_stats* stats,
                 DevKrylov& ws, hipStream_t s) {
    const int64_t n = sys.n_solve;
    const int ni = sys.mesh->n_inst;
    const int m = std::max(1, std::min(o.restart, kMaxM));
    const bool z32 = amg.opts.precision == 32;
    if (!ws.hsum) {
        FR_HIP(hipHostMalloc(reinterpret_cast<void**>(&ws.hsum), 2 * sizeof(IterSummary), hipHostMallocDefault));
        for (auto& e : ws.ev_sum) FR_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        ws.dsum.alloc(2, s);
    }
    if (ws.n != n || ws.m != m || ws.n_inst != ni || ws.z32 != z32) {
        ws.n = n;
        ws.m = m;
        ws.z32 = z32;
        // the bases start at kInitBasis vectors and grow with the iterations a cycle takes;
        // Z is kept in the preconditioner's precision
        ws.cap = std::min(m, kInitBasis);
        ws.V.alloc(size_t(ws.cap + 1) * size_t(n), s);
        if (z32) {
            ws.Z.release();
            ws.Z32.alloc(size_t(ws.cap) * size_t(n), s);
        } else {
            ws.Z32.release();
            ws.Z.alloc(size_t(ws.cap) * size_t(n), s);
        }
        ws.w.alloc(size_t(n), s);
        build_table(sys, ws, s);
        ws.part.alloc(size_t(ws.nb) * (kMaxM + 2) + 64, s);
        const size_t per = size_t(2 * (m + 2) + 1 + (m + 1) * m + 2 * m + (m + 1) + m + 3);
        ws.state.alloc(per * size_t(ni), s);
        ws.istate.alloc(size_t(6 * ni) + 1, s);
        ws.layout = next_epoch();
    }
    const int M = ws.m;
    State st;
    {
        double* p = ws.state.p;
        auto take = [&](size_t k) { double* q = p; p += k * size_t(ni); return q; };
        st.h1 = take(M + 2);
        st.h2 = take(M + 2);
        st.nrm2 = take(1);
        st.H = take(size_t(M + 1) * M);
        st.cs = take(M);
        st.sn = take(M);
        st.g = take(M + 1);
        st.y = take(M);
        st.target = take(1);
        st.scale = take(1);
        st.beta2 = take(1);
        st.done = ws.istate.p;
        st.jused = ws.istate.p + ni;
        st.bad = ws.istate.p + 2 * ni;
        st.need = ws.istate.p + 3 * ni;
        st.brk = ws.istate.p + 4 * ni;
        st.zhit = ws.istate.p + 5 * ni;
        st.j = ws.istate.p + 6 * ni;
    }
    const Seg sg{ws.seg_start.p, ws.seg_len.p, ws.seg_inst.p};
    // The preconditioner's argument is staged while the basis vector is written: with graphs
    // into the fixed staged input (FP32 or FP64); without graphs, with the FP32 hierarchy,
    // straight into its level-0 right-hand sides.
    const bool graphs = o.use_graphs != 0 && !prof_enabled();
    StepCtx c{&sys, &amg, &ws, st, sg, ni, M, n, z32, graphs, nullptr, nullptr, nullptr, nullptr,
              amg.h[0].mf != nullptr, amg.h[0].mf != nullptr && amg.h[1].mf != nullptr};
    if (graphs && z32) {
        c.f_u = static_cast<float*>(amg_graph_input(amg));
        c.f_p = c.f_u + sys.n_u;
    } else if (graphs) {
        c.d_copy = static_cast<double*>(amg_graph_input(amg));
    } else if (z32) {
        c.f_u = amg_input32(amg, 0);
        c.f_p = amg_input32(amg, 1);
    }
    if (graphs) c.vout = amg_graph_output(amg);
    const int nb = ws.nb;
    const int gi = int(ceil_div(ni, 64));
    double* part = ws.part.p;
    FR_HIP(hipMemsetAsync(ws.istate.p, 0, (size_t(6 * ni) + 1) * sizeof(int), s));

    // ||F_i||, targets
    k_seg_resid<<<nb, 256, 0, s>>>(sys.F.p, ws.w.p, 1, sg, part);
    FR_LAUNCH_CHECK();
    k_seg_reduce<<<dim3(1, ni), kReduceT, 0, s>>>(part, nb, ws.seg_bptr.p, st.beta2, 1);
    FR_LAUNCH_CHECK();
    std::vector<double> bn2 = download(st.beta2, size_t(ni), s);
    const size_t nis = static_cast<size_t>(ni);
    std::vector<double> bnorm(nis, 0.0), target(nis, 0.0);
    for (int i = 0; i < ni; ++i) {
        bnorm[size_t(i)] = std::sqrt(bn2[size_t(i)]);
        target[size_t(i)] = o.rtol * bnorm[size_t(i)];
    }
    FR_HIP(hipMemcpyAsync(st.target, target.data(), size_t(ni) * 8, hipMemcpyHostToDevice, s));
    FR_HIP(hipMemsetAsync(du, 0, size_t(n) * sizeof(double), s));

    std::vector<int> iters(size_t(ni), 0), conv(size_t(ni), 0);
    std::vector<double> relres(size_t(ni), 0.0);
    int total = 0;
    bool first = true;
    while (true) {
        // r = F - J x per instance, its norm, the new cycle
        if (!first) jmul<double>(c, du, ws.w.p, nullptr, nullptr, s);
        k_seg_resid<<<nb, 256, 0, s>>>(sys.F.p, ws.w.p, first ? 1 : 0, sg, part);
        FR_LAUNCH_CHECK();
        k_seg_reduce<<<dim3(1, ni), kReduceT, 0, s>>>(part, nb, ws.seg_bptr.p, st.beta2, 1);
        FR_LAUNCH_CHECK();
        first = false;
        k_cycle_start<<<gi, 64, 0, s>>>(ni, M, st);
        FR_LAUNCH_CHECK();
        std::vector<double> b2 = download(st.beta2, size_t(ni), s);
        std::vector<int> dn = download(st.done, size_t(ni), s);
        bool all_done = true;
        for (int i = 0; i < ni; ++i) {
            relres[size_t(i)] = bnorm[size_t(i)] > 0 ? std::sqrt(b2[size_t(i)]) / bnorm[size_t(i)] : 0.0;
            conv[size_t(i)] = dn[size_t(i)];
            all_done = all_done && dn[size_t(i)];
        }
        if (all_done || total >= o.maxit) break;
        k_seg_scale<<<nb, 256, 0, s>>>(ws.w.p, ws.V.p, nullptr, n, st.scale, sg, c.f_u, c.f_p, sys.n_u, c.d_copy);
        FR_LAUNCH_CHECK();
        k_set_int<<<1, 64, 0, s>>>(st.j, 0);
        FR_LAUNCH_CHECK();
        int j = 0;
        for (; j < M && total < o.maxit; ++j) {
            if (j + 1 > ws.cap) grow_basis(ws, j, s);
            if (graphs) FR_HIP(hipGraphLaunch(step_graph(c, s), s));
            else arnoldi_step(c, j, s);
            // convergence readback without a round trip per iteration: the summary of step j
            // lands in slot j & 1 of a pinned ring; the host waits for it only when the
            // previous step's summary (already on the host) leaves an instance within
            // kSpecRatio of its target, and otherwise enqueues the next step at once.  A step
            // run after every instance has finished changes nothing (finished instances are
            // frozen).
            const int slot = j & 1;
            FR_HIP(hipEventRecord(ws.ev_sum[slot], s));
            ++total;
            bool wait = true;
            if (j > 0) {
                const hipError_t q = hipEventQuery(ws.ev_sum[slot ^ 1]);
                if (q == hipSuccess) {
                    const IterSummary& prev = ws.hsum[slot ^ 1];
                    wait = prev.all_done || !(prev.ratio > kSpecRatio);
                } else {
                    (void)hipGetLastError();   // not ready: not an error
                }
            }
            if (wait) {
                FR_HIP(hipEventSynchronize(ws.ev_sum[slot]));
                if (ws.hsum[slot].all_done) { ++j; break; }
            }
        }
        k_backsolve<<<gi, 64, 0, s>>>(ni, M, st);
        FR_LAUNCH_CHECK();
        std::vector<int> ju = download(st.jused, size_t(ni), s);
        int jmax = 0;
        for (int i = 0; i < ni; ++i) {
            iters[size_t(i)] += ju[size_t(i)];
            jmax = std::max(jmax, ju[size_t(i)]);
        }
        if (jmax > 0) {
            if (z32) k_seg_combine<float><<<nb, 256, 0, s>>>(ws.Z32.p, n, jmax, st.y, M, du, sg);
            else k_seg_combine<double><<<nb, 256, 0, s>>>(ws.Z.p, n, jmax, st.y, M, du, sg);
            FR_LAUNCH_CHECK();
        }
        // instances with a non-finite residual or a breakdown are marked done by the next
        // cycle start; the others go on
    }
    ws.last_iters = total;
    std::vector<int> bad = download(st.bad, size_t(ni), s);
    std::vector<int> brk = download(st.brk, size_t(ni), s);
    fr_status worst = FR_OK;
    for (int i = 0; i < ni; ++i) {
        fr_status si = FR_OK;
        if (bad[size_t(i)]) si = FR_ENAN;
        else if (brk[size_t(i)]) si = FR_EBREAKDOWN;
        else if (!(relres[size_t(i)] <= o.rtol)) si = FR_ENOCONV;
        if (stats) {
            stats[i].iters = iters[size_t(i)];
            stats[i].relres = relres[size_t(i)];
            stats[i].status = si;
        }
        worst = worse_status(worst, si);
    }
    return worst;
}

}  // namespace fr
