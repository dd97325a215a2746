// Device-resident objects behind the C handles: mesh, assembled system, sparse matrices
// in block SELL-C layout, AMG hierarchies and the Krylov workspace.
#pragma once
#include <memory>
#include <vector>

#include "common.h"
#include "mesh.h"

namespace fr {

// Material and method constants as the kernels see them.
struct Params {
    double E, nu, Gc, kappa, eps, p, c_pdas, tau;
    double mu, lam;
};

Params make_params(const fr_params& p);

// ---- sparse storage ---------------------------------------------------------------------
// Block SELL-C: rows are grouped in slices of C consecutive block rows; inside a slice the
// k-th entry of the row at lane l sits at slot slice_ptr[s] + k*C + l (lanes read
// consecutive slots: coalesced).  A slot holds a column index and a br x bc block stored
// row-major.  Padding slots repeat a valid column of the row with a zero block.
struct SellStruct {
    int C = 64;
    int64_t n_rows = 0, n_cols = 0, n_slices = 0, n_slots = 0, nnz = 0;
    int max_len = 0;                // longest row (entries)
    int G = 0;                      // lanes per row chosen by the launch-shape tuner (0: by row length)
    int32_t* slice_ptr = nullptr;   // [n_slices+1]
    int32_t* row_len = nullptr;     // [n_rows]
    int32_t* col = nullptr;         // [n_slots]
    // [n_slots] or null: the columns as int16 offsets from the row (slot's column - row), when
    // all fit; the one-lane-per-row SpMV, Chebyshev and J-SpMV kernels then read these
    int16_t* col16 = nullptr;
    DBuf<int32_t> own_slice, own_len, own_col;
    DBuf<int16_t> own_col16;
};

template <typename T>
struct BMat {
    int br = 1, bc = 1;
    std::shared_ptr<SellStruct> S;
    T* val = nullptr;               // [n_slots * br * bc]
    DBuf<T> own_val;
    int64_t rows() const { return S ? S->n_rows : 0; }
    int64_t cols() const { return S ? S->n_cols : 0; }
};

// ---- mesh -------------------------------------------------------------------------------
struct DevMesh {
    HostMesh host;
    Pattern pat;
    hipStream_t stream = nullptr;
    int dim = 2, nv = 4;
    int64_t n_nodes = 0, n_cells = 0, n_free = 0;
    bool hanging = false;
    bool on_device = false;                      // false: host-only mesh (inspection)
    int n_inst = 1;                              // independent instances (disjoint union)
    DBuf<int32_t> inst_of_free, inst_of_cell;    // only when n_inst > 1
    DBuf<int32_t> cells, node_of_free, free_of_node, con_ptr, con_master;
    DBuf<double> cell_h, cell_lo, con_w, coords_free;
    DBuf<uint8_t> dir_free;                      // Dirichlet flag per free node
    std::shared_ptr<SellStruct> graph;           // node graph (free x free)
    DBuf<int32_t> ent_ptr, ent_cell;
    DBuf<uint8_t> ent_a, ent_k, hang_k;
    DBuf<int32_t> hang_ptr;
    DBuf<int32_t> heavy_rows;                    // rows with more than 2^dim assembly entries
    std::vector<int32_t> heavy_host;
    int64_t n_heavy = 0;
    DBuf<double> ent_w;
    uint64_t serial = 0;                         // unique per mesh in the process
    // A mesh made by refine_mesh: where its nodes lie in the mesh it was made from.
    uint64_t parent_serial = 0;                  // that mesh's serial (0: none)
    int64_t parent_nodes = 0;
    DBuf<int32_t> parent_cell;                   // [n_nodes]
    DBuf<double> parent_xi;                      // [n_nodes][dim]
    // Face neighbours (built on first use by mesh_kelly)
    DBuf<int32_t> face_ptr, face_nbr;
};

std::unique_ptr<DevMesh> mesh_create(const fr_mesh_desc* d, int n_inst, hipStream_t s, bool upload);
std::unique_ptr<DevMesh> mesh_from_host(HostMesh&& host, hipStream_t s, bool upload);
// Nodal fields of `from` interpolated at the nodes of `to` (made from `from` by refine_mesh):
// dst[n][c] = sum_a N_a(xi_n) src[vertex a of cell_n][c], hanging vertices of `from` taken from
// their constraints.
void mesh_transfer(const DevMesh& from, const DevMesh& to, const double* src, int ncomp, double* dst, hipStream_t s);
// Gradient-jump indicator of u: eta2[c] = h_c / 24 * sum over the faces of cell c of the
// integral of |jump of du/dn|^2 (all components), 2-point Gauss per face axis on the smaller
// of the two faces; boundary faces contribute nothing.
void mesh_kelly(DevMesh& m, const double* u, double* eta2, hipStream_t s);
// Crack-region marks: flag[c] = 1 when the cell's edge exceeds h_target and phi (hanging
// vertices from their constraints) is below phi_max at one of its vertices.
void mesh_mark_crack(const DevMesh& m, const double* phi, double phi_max, double h_target, uint8_t* flags_dev,
                     hipStream_t s);

struct AggTransfer;

// ---- matrix-free fine-level operators on uniform 2d meshes (mfree.hip) --------------------
struct MfGrid {
    int64_t nx = 0, ny = 0, n1 = 0, n_nodes = 0;   // cells per axis, nodes per row, nodes
    double mu = 0, lam = 0, kappa = 0;
    double h = 0, p = 0, Gc = 0, eps = 0;          // cell edge, pressure, G_c, epsilon
    double x0 = 0, y0 = 0;                         // lower-left corner (node (i, j) at x0 + i h, y0 + j h)
};
struct MfState {
    bool valid = false;                          // the system's mesh allows it and the state is copied
    MfGrid grid;
    DBuf<double> pt;                             // phi_tilde of the last Jacobian assembly, all nodes
    DBuf<float> pt32;                            // the same in FP32 (the FP32 hierarchy's smoother)
    DBuf<double> us, ps;                         // u (node-major) and phi of that assembly
    DBuf<float> us32;
    DBuf<uint8_t> act;                           // its active set (per node)
    DBuf<double> dpp;                            // diagonal of M_phiphi (kept for active rows)
    DBuf<float> dpp32;
};

// ---- assembled system -------------------------------------------------------------------
struct DevSystem {
    DevMesh* mesh = nullptr;
    Params prm{};                                // instance 0
    std::vector<Params> prm_h;                   // per instance
    DBuf<Params> prm_d;                          // per instance (device), when n_inst > 1
    hipStream_t stream = nullptr;
    int64_t n_solve = 0, n_u = 0;
    BMat<double> Juu, Jpu, Jpp;                  // share the node-graph structure
    DBuf<double> R, F, B;                        // residual, masked rhs, lumped mass
    DBuf<uint8_t> active, active_prev, frozen;   // per free node
    DBuf<double> red;                            // reduction scratch
    DBuf<int32_t> ired;
    DBuf<double> nodal;                          // hanging meshes: u, phi, phi~ with hanging values filled
    DBuf<int64_t> inst_off;                      // batches: first free row of every instance
    bool have_residual = false, have_active = false, have_jacobian = false;
    int64_t last_changes = 0;
    double last_min_margin = 0.0;
    uint64_t version = 0;                        // bumped at every Jacobian assembly
    MfState mf;                                  // matrix-free fine-level blocks (uniform 2d meshes)
};

// Matrix-free fine-level blocks (Section 3's M_uu and M_phiphi, and the phase-field rows
// M_phiu, M_phiphi of the J-SpMV) on uniform 2d single-instance meshes: the masked operators
// the assembly stores, applied from the assembly's state (phi_tilde, u, phi, active set) and
// the vector alone.  blk 0: M_uu, 1: M_phiphi.
bool mf_eligible(const DevMesh& m);
// Copies the state for the matrix-free operators; sys.mf.valid tells whether they apply.
void mf_prepare(DevSystem& sys, const double* u, const double* phi, const double* pt, hipStream_t s);
template <typename T>
void mf_cheb_step(const MfState& mf, int blk, const T* invd, const T* x_old, const T* b, T* d, T* x_new, T alpha,
                  T beta, hipStream_t s);
template <typename T>
void mf_residual(const MfState& mf, int blk, const T* x, const T* b, T* y, hipStream_t s);
// The first two Chebyshev steps from x = 0 in one pass (x_1 = beta0 D^-1 b formed per node;
// then the step with alpha, beta into d and x_new): the two separate launches' values.
template <typename T>
void mf_cheb_first2(const MfState& mf, int blk, const T* invd, const T* b, T* d, T* x_new, T beta0, T alpha, T beta,
                    hipStream_t s);
// y = D^-1 A x with the block's fine operator matrix-free (a power step of the smoother bounds)
void mf_power_step(const MfState& mf, int blk, const double* invd, const double* x, double* y, hipStream_t s);
// The finest displacement level's transfers matrix-free, P = (I - omega D^-1 M_uu) P_t:
// x += P x_c (xc on the aggregates), and b_c = P^T r = P_t^T (r - omega M_uu D^-1 r) (s: a
// scratch vector of the fine level's size).
template <typename T>
void mf_prolong(const MfState& mf, const AggTransfer& t, const T* invd, const T* xc, T* x, hipStream_t st);
template <typename T>
void mf_restrict(const MfState& mf, const AggTransfer& t, const T* invd, const T* r, T* s, T* bc, hipStream_t st);
// y = J x with the displacement rows matrix-free, and the phase-field rows too when `phi_rows`
// (x FP64 or FP32), xcopy as for jspmv_copy
template <typename TX>
void mf_jspmv(const DevSystem& sys, bool phi_rows, const TX* x, double* y, TX* xcopy, const int* jp, int64_t xstride,
              hipStream_t s);

void assemble_residual(DevSystem& sys, const double* u, const double* phi, const double* pt);
void assemble_active(DevSystem& sys, const double* phi, const double* phi_old);
void assemble_active_freeze(DevSystem& sys, const double* phi, const double* phi_old);
void assemble_jacobian(DevSystem& sys, const double* u, const double* phi, const double* phi_old,
                       const double* pt);
// norms: [0] ||R~||, [1] ||F||; also n_active, min |margin|
void system_norms(DevSystem& sys, const double* phi, const double* phi_old, double* norms,
                  int64_t* n_active, double* min_margin);
void system_matvec(DevSystem& sys, const double* x, double* y);
// u += omega du, phi += omega du on the free nodes (hanging nodes refilled).  With `active`
// (per free node) the fixed DoFs take their constraint values instead: Dirichlet u 0, active
// phi phi_old.
void mesh_update(DevMesh& m, const double* du, double omega, double* u, double* phi, hipStream_t s,
                 const uint8_t* active = nullptr, const double* phi_old = nullptr);
// out = clip(p1 + w (p1 - p2), 0, 1) on the free nodes, hanging nodes interpolated from them.
void extrapolate(DevMesh& m, const double* p1, const double* p2, double w, double* out, hipStream_t s);
// Batches: per-instance ||R~||, active phi rows and active-flag changes of the last update.
void system_norms_inst(DevSystem& sys, std::vector<double>& rnorm, std::vector<int64_t>& n_active,
                       std::vector<int64_t>& changes);
// Batches: the rows of every instance i with bad_dev[i] != 0 (device, one int per instance)
// become identity rows with zero right-hand side and residual (their increments are then 0
// and their non-finite values stay out of the other instances' preconditioner and solve).
void system_neutralize(DevSystem& sys, const int* bad_dev);
// Per-instance count of nonzero entries of a per-free-node flag array (synchronises).
std::vector<int64_t> count_flags_inst(DevSystem& sys, const uint8_t* flags);
// Whether every value of the three Jacobian blocks and of F is finite (synchronises s).
bool system_all_finite(const DevSystem& sys, hipStream_t s);
// Batches: u += omega[i] du on instance i (omega: device, one per instance); instances with
// omega[i] == 0 are not touched.
void mesh_update_inst(DevMesh& m, const double* du, const double* omega, double* u, double* phi, hipStream_t s,
                      const uint8_t* active = nullptr, const double* phi_old = nullptr);
void mesh_functionals(DevMesh& m, const double* u, const double* phi, const double* cod_x, int n_cod,
                      double* cod, double* tcv, hipStream_t s);
// The same results with no allocation: every device buffer is a slice of a fixed per-device
// array of kFunctionalsScratchDoubles doubles (FR_EINVAL when the call needs more, see
// functionals_scratch_need).  Calls that overlap on one device share that array and race.
constexpr size_t kFunctionalsScratchDoubles = size_t(1) << 19;   // 4 MiB per device
constexpr int kMaxScratchDevices = 64;
int64_t functionals_scratch_need(const DevMesh& m, int n_cod);
void mesh_functionals_noalloc(DevMesh& m, const double* u, const double* phi, const double* cod_x, int n_cod,
                              double* cod, double* tcv, hipStream_t s);

// ---- generic device primitives (sparse.hip) ---------------------------------------------
// out[0..n] exclusive scan of in[0..n-1]; returns the total (synchronises).
int64_t scan_exclusive(const int32_t* in, int32_t* out, int64_t n, hipStream_t s);
// sum of squares / dot in a fixed order; result written to *dres (device).
void dev_dot(const double* x, const double* y, int64_t n, double* dres, DBuf<double>& scratch, hipStream_t s);
double host_norm2(const double* x, int64_t n, DBuf<double>& scratch, hipStream_t s);
void cast_f64_f32(const double* x, float* y, int64_t n, hipStream_t s);
void cast_f32_f64(const float* x, double* y, int64_t n, hipStream_t s);
void vec_copy(const double* x, double* y, int64_t n, hipStream_t s);
void vec_fill(double* y, double v, int64_t n, hipStream_t s);
// row_len set -> slice_ptr, n_slots, nnz, max_len (one host round trip; flag, when given,
// is read in the same trip into *flag_out)
void layout_from_lengths(SellStruct& S, hipStream_t s, const int* flag = nullptr, int* flag_out = nullptr);
void scan_exclusive_async(const int32_t* in, int32_t* out, int64_t n, hipStream_t s);

template <typename T>
void spmv(const BMat<T>& A, const T* x, T* y, hipStream_t s, int level = -1);   // y = A x
template <typename T>
void spmv_residual(const BMat<T>& A, const T* x, const T* b, T* y, hipStream_t s, int level = -1);  // y = b - A x
template <typename T>
void spmv_add(const BMat<T>& A, const T* x, T* y, hipStream_t s, int level = -1);   // y += A x
template <typename T>
void cheb_step(const BMat<T>& A, const T* invd, const T* x_old, const T* b, T* d, T* x_new,
               T alpha, T beta, hipStream_t s, int level = -1);
template <typename T>
void cheb_first(const T* invd, const T* b, T* d, T* x, T beta, int64_t n, hipStream_t s, int level = -1);
// fused J-SpMV over the three blocks: y = J x (solve order); x may be FP32 (exactly widened)
// y = D^-1 A x (the power iteration of the smoother bounds; its own kernel, k_power_step).
void diag_scaled_matvec(const BMat<double>& A, const double* invd, const double* x, double* y, hipStream_t s);
// Sets S.col16 (columns as int16 row offsets) when every offset fits.
void make_col16(SellStruct& S, hipStream_t s);
// Launch shape: lanes per row of the SpMV / Chebyshev kernels for a matrix.
int launch_lanes(const SellStruct& S);
// Same matrix in slice height C.
BMat<double> relayout(const BMat<double>& A, int C, hipStream_t s);

// Picks slice height and lanes per row for M by timing (op 0: smoother, 1: y = M x,
// 2: y += M x) in FP32 or FP64; replaces M by its relayout when another slice height wins.
// Process-wide cache.
void tune_layout(BMat<double>& M, int op, bool f32, hipStream_t s);
void tune_clear();
int tune_entries();
std::string tune_export();
void tune_import(const char* text);
void jspmv(const DevSystem& sys, const double* x, double* y, hipStream_t s);
void jspmv(const DevSystem& sys, const float* x, double* y, hipStream_t s);
// the same, also copying x to xcopy + (*jp) xstride (the Krylov basis slot of the device's index)
void jspmv_copy(const DevSystem& sys, const double* x, double* y, double* xcopy, const int* jp, int64_t xstride,
                hipStream_t s);
void jspmv_copy(const DevSystem& sys, const float* x, double* y, float* xcopy, const int* jp, int64_t xstride,
                hipStream_t s);

// ---- AMG (amg.hip) ----------------------------------------------------------------------
// The finest displacement level's aggregation, kept so that the V-cycle can apply its
// transfers matrix-free (uniform 2d meshes): per node its aggregate, per aggregate its member
// nodes and the factors of the tentative prolongator (rows B_i R_a^-1, B_i the rigid-body modes
// of node i about the aggregate's centroid): R_a^-1 (3 x 3, row-major) and the centroid (2).
constexpr int kAggInfo = 11;
struct AggTransfer {
    int64_t n_agg = 0;
    double omega = 0;                            // the prolongator smoothing weight 4 / (3 lambda_max)
    DBuf<int32_t> agg, aptr, anodes;
    DBuf<double> info;                           // n_agg x kAggInfo
    DBuf<float> info32;
    DBuf<double> w;                              // n_agg x 3 scratch (R_a^-1 x_c)
    DBuf<float> w32;
};

struct AmgLevel {
    BMat<double> A, P, R;
    std::unique_ptr<AggTransfer> mt;             // level 0 of the u hierarchy on uniform 2d meshes
    BMat<double> Pt, AP;                         // kept for a numeric-only refresh
    BMat<float> A32, P32, R32;
    DBuf<double> invd;
    DBuf<float> invd32;
    double lmax = 0;
    double omega = 0;                            // prolongator smoothing weight of the build, 4/(3 lmax)
    int ns = 1;                                  // near-nullspace size (block size of the next level)
    // V-cycle work vectors (scalar length n = rows * br)
    DBuf<double> vb, vx0, vx1, vd, vr;
    DBuf<float> fb, fx0, fx1, fd, fr;
};

struct Hierarchy {
    std::vector<std::unique_ptr<AmgLevel>> lv;
    DBuf<double> dense_inv;                      // coarsest A^-1, row-major
    int64_t n_coarse = 0;
    bool refreshable = false;                    // Pt and AP kept on every level but the last
    const MfState* mf = nullptr;                 // level 0 applied matrix-free (uniform 2d meshes)
    int blk = 0;                                 // 0: the u block's hierarchy, 1: the phi block's
};

struct DevAmg {
    DevSystem* sys = nullptr;
    fr_amg_opts opts{};
    hipStream_t stream = nullptr;
    Hierarchy h[2];                              // 0: u block, 1: phi block
    uint64_t sys_version = 0;
    // the phi V-cycle runs on a second stream (default priority) beside the u V-cycle
    hipStream_t side = nullptr;
    hipStream_t aux[2] = {nullptr, nullptr};     // setup: power iterations of the u / phi hierarchy
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    DBuf<float> z32;                             // FP32 result staging of amg_precondition
    // Staged preconditioner input and output (solve order, [u | phi], in the hierarchy's
    // precision) of amg_precondition_staged, the form a captured FGMRES iteration uses.  epoch
    // is renewed (process-wide unique, next_epoch) at every setup and buffer change after which
    // such a capture is stale: a preconditioner made at the address of a destroyed one never
    // matches the old one's captures.
    DBuf<double> vin64, vout64;
    DBuf<float> vin32, vout32;
    uint64_t epoch = 0;
    ~DevAmg() {
        for (auto a : aux)
            if (a) (void)hipStreamSynchronize(a);
        if (side) (void)hipStreamSynchronize(side);
        if (stream) (void)hipStreamSynchronize(stream);
        // the phase-field hierarchy's buffers are freed on the side stream: before it goes
        for (auto& H : h) {
            H.lv.clear();
            H.dense_inv.release();
        }
        if (side) forget_stream(side);   // synchronises the side stream
        for (auto a : aux)
            if (a) forget_stream(a);
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        if (ev_join) (void)hipEventDestroy(ev_join);
        if (side) (void)hipStreamDestroy(side);
        for (auto a : aux)
            if (a) (void)hipStreamDestroy(a);
    }
};

void amg_build(DevAmg& amg, DevSystem& sys, const fr_amg_opts& o, hipStream_t s);
void amg_precondition(DevAmg& amg, const double* r, double* z, hipStream_t s);
// FP32 hierarchy only: z (FP32) = M^-1 r.  r == nullptr: the input is already in the
// level-0 right-hand sides, amg_input32(amg, 0) (u part) and amg_input32(amg, 1) (phi part).
void amg_precondition32(DevAmg& amg, const double* r, float* z, hipStream_t s);
float* amg_input32(DevAmg& amg, int blk);
// The two V-cycles (u on s, phi on the side stream) from the staged input amg_graph_input
// (the caller stages M^-1's argument there, in the hierarchy's precision, solve order) to the
// staged output amg_graph_output; fixed buffers, so the launches can be captured in a graph.
void amg_precondition_staged(DevAmg& amg, hipStream_t s);
void* amg_graph_input(DevAmg& amg);
void* amg_graph_output(DevAmg& amg);
void amg_level_export(DevAmg& amg, int blk, int level, int which, int64_t& n_rows, int64_t& n_cols,
                      std::vector<int64_t>& rp, std::vector<int32_t>& ci, std::vector<double>& vv, hipStream_t s);
void amg_info(DevAmg& amg, int blk, int level, int& n_levels, int64_t& rows, int& bsize, int64_t& nnzb,
              double& lmax, hipStream_t s);
void amg_level_shape(DevAmg& amg, int blk, int level, int which, int& C, int& G);

// ---- Krylov (krylov.hip) ----------------------------------------------------------------
constexpr int kInitBasis = 24;                   // initial Krylov basis capacity (vectors)

// Per-iteration convergence summary read back asynchronously (pinned host ring).
struct IterSummary {
    int all_done;      // every instance converged or stopped
    int pad;
    double ratio;      // largest |residual estimate| / target over the running instances
};

// Process-wide unique serial numbers (never 0) for the epochs of captured work.
uint64_t next_epoch();

// What a captured Arnoldi step depends on: the system and its Jacobian assembly, the
// preconditioner's setup epoch and the workspace layout (renewed whenever the Krylov buffers are
// reallocated or grown).
struct IterKey {
    const void* sys = nullptr;
    uint64_t sys_version = 0;                    // the Jacobian assembly (parameters captured by value)
    uint64_t amg_epoch = 0;
    uint64_t layout = 0;
    bool operator==(const IterKey& o) const {
        return sys == o.sys && sys_version == o.sys_version && amg_epoch == o.amg_epoch && layout == o.layout;
    }
};

struct DevKrylov {
    int64_t n = 0;
    int m = 0, n_inst = 0, nb = 0;
    DBuf<IterSummary> dsum;                      // [2] device summaries (slot j & 1)
    IterSummary* hsum = nullptr;                 // [2] pinned host ring
    hipEvent_t ev_sum[2] = {nullptr, nullptr};
    // the captured Arnoldi step (use_graphs) and the stream it is captured on
    hipGraphExec_t step_exec = nullptr;
    IterKey step_key;
    hipStream_t cstream = nullptr;
    int64_t captures = 0;                        // captures made (one per preconditioner setup)
    uint64_t layout = 0;                         // renewed (next_epoch) whenever V, Z, w, part, state move
    int last_iters = 0;                          // Arnoldi steps of the last solve
    void drop_step() {
        if (step_exec) { (void)hipGraphExecDestroy(step_exec); step_exec = nullptr; }
    }
    DevKrylov() = default;
    DevKrylov(const DevKrylov&) = delete;
    DevKrylov& operator=(const DevKrylov&) = delete;
    ~DevKrylov() {
        for (auto& e : ev_sum)
            if (e) { (void)hipEventSynchronize(e); (void)hipEventDestroy(e); }
        if (hsum) (void)hipHostFree(hsum);
        drop_step();
        if (cstream) (void)hipStreamDestroy(cstream);
    }
    int cap = 0;                                 // vectors held in Z (V holds cap + 1)
    bool z32 = false;                            // Z kept in FP32 (FP32 preconditioner)
    DBuf<double> V, Z, w, part, state;
    DBuf<float> Z32;                             // the Z basis when the preconditioner is FP32
    DBuf<int> istate;
    DBuf<int64_t> seg_start;                     // segmented-sweep block table
    DBuf<int32_t> seg_len, seg_inst, seg_bptr;
};

// stats: host, one per instance (nullable). Returns the worst instance status.
fr_status fgmres(DevSystem& sys, DevAmg& amg, const fr_solve_opts& o, double* du, fr_solve_stats* stats,
                 DevKrylov& ws, hipStream_t s);

}  // namespace fr
