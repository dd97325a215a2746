/*
 * fracture.h -- C ABI of the MI355X (gfx950) Newton-step linear solve for pressurized
 * phase-field fracture (Heister & Wick 2018).
 *
 * The library computes, on one GPU, the Newton step of Formulation 1 (Section 2):
 * Q1 assembly of the residual of equations E22ATW / E33ATW and of the Jacobian blocks
 * M_uu, M_phiu, M_phiphi (Section 3, "Linear iterative solution"; M_uphi = 0), the
 * primal-dual active set of the irreversibility constraint phi <= phi_old with the
 * elimination of active rows and columns (Section 3, commented algorithm, steps 2-4),
 * an FGMRES solve preconditioned by block-diagonal smoothed-aggregation AMG (one V-cycle
 * per diagonal block, Section 3), the Newton / active-set loop with line search
 * (steps 1-6) and the TCV / COD functionals (Section 4).
 *
 * Conventions shared by every call:
 *  - Every array argument is a DEVICE pointer unless its comment says "host".
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream). Work is
 *    enqueued on it; calls that return host scalars synchronise it (said per call).
 *  - User vectors cover all mesh nodes: u is [n_nodes][dim] (node-major, AoS), phi,
 *    phi_old, phi_tilde are [n_nodes]. Hanging-node values are overwritten by the
 *    library from the constraints (edge midpoints 1/2 + 1/2, face centres 1/4 each).
 *  - Solve-order vectors (du, residual, right-hand side) have n_solve = (dim+1) n_free
 *    entries: the u block node-major over free nodes (index f*dim + c), then the phi
 *    block (index dim*n_free + f), the block basis of Section 3. Dirichlet u DoFs and
 *    active phi DoFs stay in the system as rows with their original diagonal.
 *  - Handles are owned by the library and released by the matching *_destroy. The caller
 *    owns every array argument and keeps it alive until the stream has reached the call.
 *  - Arguments are validated before any device work (FR_EINVAL). Errors never throw
 *    across the ABI; fracture_last_error() returns a message for the calling thread.
 */
#ifndef FRACTURE_H
#define FRACTURE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FR_OK = 0,
    FR_EINVAL = 1,      /* bad argument (checked before any device work)            */
    FR_ENOMEM = 2,      /* device or host allocation failed                          */
    FR_EDEVICE = 3,     /* HIP runtime error, or no usable gfx950 device             */
    FR_ENOCONV = 4,     /* iteration limit reached; outputs hold the last iterate     */
    FR_EBREAKDOWN = 5,  /* Krylov breakdown (zero or non-finite Arnoldi norm)         */
    FR_ENAN = 6,        /* non-finite value in the residual, Jacobian or solution    */
    FR_ECYCLE = 7,      /* active set still changing after the cycle freeze          */
    FR_EINTERNAL = 8    /* internal capacity exceeded (message names the limit)      */
} fr_status;

typedef struct fr_mesh_s* fr_mesh;
typedef struct fr_system_s* fr_system;
typedef struct fr_amg_s* fr_amg;

/* Mesh of B = [lo, hi] (Section 2: homogeneous Dirichlet u on the outer boundary,
 * no condition on phi). Cells are cubes: (hi[k]-lo[k])/base[k] must agree on all axes.
 * levels = 0: uniform mesh of base[0] x ... cells. levels > 0: every cell whose box comes
 * within refine_radius of the crack (2d: segment |x - c_x| <= crack_half_len on the line
 * y = c_y; 3d: disk of radius crack_half_len in the plane z = c_z) is split, `levels`
 * times, followed by 2:1 balancing: cells that share a point (a vertex, edge or face) differ by
 * at most one level (Section 3 adaptive meshes). */
typedef struct {
    int dim;                 /* 2 or 3 */
    double lo[3], hi[3];
    int base[3];
    int levels;
    double refine_radius;
    double crack_center[3];
    double crack_half_len;
} fr_mesh_desc;

/* Material and method constants (Section 2, Formulation 1; Section 4). The active set is
 * A = { i : -R_phi,i / B_ii + c_pdas (phi_i - phi_old,i) > tau_pdas }, B the lumped phi
 * mass; tau_pdas <= 0 selects 1e-10 Gc / eps. */
typedef struct {
    double E, nu, Gc, kappa, eps, p, c_pdas, tau_pdas;
} fr_params;

/* Smoothed-aggregation AMG options (one hierarchy per diagonal block). */
typedef struct {
    int precision;       /* 64: FP64 hierarchy and V-cycle; 32: FP32 storage and arithmetic */
    double theta;        /* strength threshold, |A_ij| >= theta sqrt(|A_ii| |A_jj|) (block Frobenius norms);
                            negative (the default): 0.08 in 2d, 0.02 in 3d, the fastest measured
                            for the Sneddon workloads (2d iterations fall from 30 to 23 between
                            0.02 and 0.08 and rise steeply above 0.1; 3d prefers 0.01-0.02) */
    int cheb_degree;     /* Chebyshev smoother degree (>= 1) */
    double cheb_ratio;   /* smoothing interval [1.1 lambda_max / ratio, 1.1 lambda_max] of D^-1 A
                            (default 8: 3d needs less than half the iterations of ratio 12) */
    int coarse_max;      /* coarsest level solved densely once it has <= coarse_max rows */
    int max_levels;      /* cap on the number of levels (>= 1) */
    int reuse_u_block;   /* nonzero: amg_setup keeps an existing displacement-block hierarchy.
                            M_uu depends only on phi_tilde and the Dirichlet set, so within one
                            loading step it does not change between Newton iterations;
                            fracture_newton rebuilds it once per call when this is set. */
    int refresh_phi;     /* amg_setup on a system whose phase-field hierarchy exists (fracture_newton
                            from its second Newton iteration on): 0 builds it anew; 1 (the default)
                            keeps its aggregates and sparsity and recomputes every level's values
                            (the Jacobian pattern never changes; masked entries stay as zeros; the
                            prolongators are smoothed with the build's weights 4/(3 lambda_max),
                            while each level's new lambda_max bounds its smoother); 2
                            recomputes only the finest level's diagonal and lambda_max and keeps
                            the coarse levels and transfers of the build (a lagged preconditioner,
                            as the displacement hierarchy under reuse_u_block; the finest level's
                            operator is the current one either way).  2 saves the refresh (4.7 ms
                            per Newton step on 2048^2, with the same iterations there) but can
                            cost iterations where the active set moves between steps. */
    int autotune;        /* nonzero: the launch shape of every coarse-level smoother and transfer
                            product (SELL slice height 64 or 1, lanes per row 1/4/16/64) is
                            picked by timing the candidates on the level's matrix, in the
                            V-cycle's precision, during the setup; choices are cached per process
                            by (operation, block shape, log2 rows, mean row length, precision)
                            and reused by later setups.  Different
                            lane counts sum a row in a different order, so results are
                            reproducible for a given cache (amg_level_shape reports the choice). */
    int fine_matrix_free; /* bit mask, on a uniform 2d mesh (one instance); other meshes use the
                            stored blocks either way.  Bit 0 (1): the finest displacement level's
                            smoother and residual, and the displacement rows of the J-SpMV in
                            fracture_solve, apply M_uu matrix-free from phi_tilde.  Bit 1 (2): the
                            finest phase-field level's smoother and residual apply the masked
                            M_phiphi from the assembly's u and active set, and (with bit 0) the
                            phase-field rows of the J-SpMV apply M_phiu and M_phiphi from its u,
                            phi and active set.  Bit 2 (4, with bit 0): the finest displacement
                            level's prolongation and restriction apply P = (I - omega D^-1 M_uu) P_t
                            and P^T = P_t^T (I - omega M_uu D^-1) from the aggregation (per node its
                            aggregate, per aggregate the tentative prolongator's R^-1 and centroid)
                            instead of the stored P and R.  The same operators as the stored
                            blocks, summed in another order: equal up to rounding.  Default 7. */
} fr_amg_opts;

/* FGMRES options (right preconditioned, x0 = 0). */
typedef struct {
    double rtol;         /* stop when ||F - J du||_2 <= rtol ||F||_2 (true residual, FP64) */
    int restart;         /* Krylov basis size before a restart */
    int maxit;           /* total iteration cap */
    int use_graphs;      /* nonzero: the two V-cycles are captured once per amg_setup as HIP graphs
                            and replayed every iteration (one launch each instead of one per
                            kernel); ignored while fracture_profile records */
} fr_solve_opts;

typedef struct {
    int iters;           /* FGMRES iterations */
    double relres;       /* true relative residual ||F - J du|| / ||F|| at exit */
    int status;          /* fr_status of this solve */
} fr_solve_stats;

typedef struct {
    double tol;          /* stop when the active set is unchanged and ||R~|| <= max(tol ||R~(U0)||, atol) */
    int max_it;          /* Newton iteration cap */
    int ls_max;          /* line search tries omega = 1, 1/2, ..., 2^-ls_max */
    double atol;         /* absolute floor of the stop test (>= 0; the algorithm of Section 3 states
                            an absolute TOL): a loading step that starts at equilibrium has
                            ||R~(U0)|| at rounding level, which the relative part cannot undercut */
    int no_cycle_freeze; /* nonzero leaves out the cycle rule (a diagnostic: Section 3 detects and
                            constrains alternating active-set indices; with this set a loop whose
                            active set alternates runs to max_it and returns FR_ECYCLE) */
} fr_newton_opts;

typedef struct {
    int iterations;      /* Newton iterations taken */
    int linear_iters;    /* sum of FGMRES iterations */
    double res0, res;    /* ||R~(U0)|| and ||R~|| at exit */
    int64_t n_active;    /* active phi DoFs at exit */
    int status;          /* fr_status of this instance (see fracture_newton) */
    double t_assemble, t_setup, t_solve, t_other;  /* seconds, HIP-event timed */
    int64_t n_frozen;    /* phi DoFs frozen active by the cycle rule */
    int linear_noconv;   /* Newton iterations whose FGMRES solve stopped at maxit above rtol */
    int linear_status;   /* worst fr_solve_stats.status of the instance's FGMRES solves */
} fr_newton_stats;

/* Flags of fracture_assemble. */
#define FR_RESIDUAL   1u   /* residual R (unmasked) and lumped mass B              */
#define FR_ACTIVE_SET 2u   /* active set from R, B, phi, phi_old (needs R)          */
#define FR_JACOBIAN   4u   /* masked Jacobian and right-hand side F (needs the set) */

/* ---- mesh ------------------------------------------------------------------------- */

/* Builds the mesh, its node numbering, Dirichlet flags, hanging-node constraints, the
 * node-graph sparsity (SELL-C layout) and the assembly tables, and uploads them on
 * `stream`. desc: host, one descriptor. */
fr_status fracture_mesh_create(const fr_mesh_desc* desc, fr_mesh* out, void* stream);

/* Host outputs (any may be NULL). n_all = (dim+1) n_nodes (the DoF count of Table 1). */
fr_status fracture_mesh_info(fr_mesh mesh, int64_t* n_nodes, int64_t* n_cells, int64_t* n_free,
                             int64_t* n_all, int64_t* n_solve, int64_t* n_hanging,
                             double* h_min, int64_t* nnz_node_graph);

/* The nodes of the Q1 space of Section 3 (cell vertices of the uniform or adaptive mesh; the
 * initial crack of Section 4 and every nodal field are given at them). Host outputs:
 * xyz[n_nodes*dim] node coordinates; lattice (nullable) integer coordinates
 * in units of the finest cell edge; dirichlet (nullable) 1 for boundary nodes (u = 0 on the
 * outer boundary, Section 2); free_index (nullable) solve-order node index or -1 for hanging
 * nodes. */
fr_status fracture_mesh_nodes(fr_mesh mesh, double* xyz, int64_t* lattice, uint8_t* dirichlet,
                              int32_t* free_index);

/* Builds the same mesh on the host only (no device memory, no device needed), for
 * inspection with fracture_mesh_info / _nodes / _cells / _constraints. Every call that
 * needs the device rejects such a mesh with FR_EINVAL. */
fr_status fracture_mesh_create_host(const fr_mesh_desc* desc, fr_mesh* out);

/* Host outputs (nullable): cells[n_cells][2^dim] vertex node ids (vertex a at the lower
 * corner plus bit k of a along axis k), cell_lo[n_cells][dim] lower corners, cell_h[n_cells]
 * edge lengths. */
fr_status fracture_mesh_cells(fr_mesh mesh, int32_t* cells, double* cell_lo, double* cell_h);

/* Face neighbours, host CSR over (cell, face) for inspection (the table fracture_kelly uses):
 * the cells across face j = 2k + side (axis k; side 0 low, 1 high) of cell c are
 * nbr[ptr[2 dim c + j] .. ptr[2 dim c + j + 1]): none on the boundary, one of the same or the
 * next coarser level, or the 2^(dim-1) cells of the next finer level. *n_entries is always
 * set; ptr (2 dim n_cells + 1 entries) and nbr are nullable. Works on host-only meshes. */
fr_status fracture_mesh_faces(fr_mesh mesh, int64_t* n_entries, int32_t* ptr, int32_t* nbr);

/* Hanging-node conformity map, host CSR over nodes: value(node n) =
 * sum_j con_w[j] value(free node con_master[j]) for j in [con_ptr[n], con_ptr[n+1]);
 * a free node lists itself with weight 1. *n_entries is always set; arrays are nullable
 * (con_ptr has n_nodes+1 entries). */
fr_status fracture_mesh_constraints(fr_mesh mesh, int64_t* n_entries, int32_t* con_ptr,
                                    int32_t* con_master, double* con_w);

/* Batch of n_inst independent meshes (desc: host, n_inst descriptors of one dim) stored as
 * their disjoint union: nodes, cells and free nodes are numbered instance by instance, and
 * every other call treats the batch as one system whose instances never couple (the
 * batched studies over domain size and eps of Section 4). fracture_assemble then takes
 * n_inst parameter sets, fracture_solve fills n_inst stats and tests convergence per
 * instance, fracture_functionals reports per instance. fracture_newton needs n_inst = 1. */
fr_status fracture_mesh_create_batch(const fr_mesh_desc* desc, int n_inst, fr_mesh* out, void* stream);

/* Host outputs (nullable) for instance inst of a (batched) mesh: offsets and counts of its
 * nodes, free nodes and cells in the union, and its finest cell edge. */
fr_status fracture_mesh_instance(fr_mesh mesh, int inst, int64_t* node_offset, int64_t* n_nodes,
                                 int64_t* free_offset, int64_t* n_free, int64_t* cell_offset,
                                 int64_t* n_cells, double* h_min);

/* Refinement between loading steps: the mesh obtained from `mesh` (one instance) by splitting
 * every cell c with flags[c] != 0 into 2^dim children, then splitting further until cells that
 * share a point differ by at most one level (2:1 balance, as for fracture_mesh_create). The
 * result has one more level than `mesh` when a cell of its finest level is flagged. It records
 * where each of its nodes lies in `mesh`, for fracture_transfer. flags: host [n_cells] (e.g.
 * from fracture_mark_crack). The new mesh is on the device when `mesh` is; it is independent
 * of `mesh` except that fracture_transfer from `mesh` needs `mesh` alive. Synchronises. */
fr_status fracture_mesh_refine(fr_mesh mesh, const uint8_t* flags, fr_mesh* out, void* stream);

/* Interpolates nodal fields of `from` at the nodes of `to`, a mesh made from `from` by
 * fracture_mesh_refine: dst[n][c] = value at node n of the Q1 function of `from` whose nodal
 * values are src[.][c] (hanging vertices of `from` taken from their constraints). The spaces are
 * nested, so the function is reproduced exactly (the solution transfer between loading steps).
 * src: device [n_nodes(from)][ncomp], dst: device [n_nodes(to)][ncomp], 1 <= ncomp <= 16, no
 * aliasing. Enqueued on `stream`. */
fr_status fracture_transfer(fr_mesh from, fr_mesh to, const double* src, int ncomp, double* dst,
                            void* stream);

/* Gradient-jump indicator of the displacement (the estimator Section 3 adds to the crack-region
 * refinement): eta2[c] = h_c / 24 * sum over the faces F of cell c of the integral over F of
 * |jump of du/dn|^2 (all components; h_c the cell edge), integrated exactly by 2-point Gauss per
 * face axis on the smaller of the two faces at a level change; boundary faces contribute
 * nothing. u: device [n_nodes][dim] (hanging values from their constraints); eta2: device
 * [n_cells] (one instance or a batch). The face-neighbour table is built on the first call and
 * kept with the mesh, so concurrent first calls on one mesh race. Enqueued on `stream` (the
 * first call synchronises it). */
fr_status fracture_kelly(fr_mesh mesh, const double* u, double* eta2, void* stream);

/* Crack-region marks (the refinement that keeps eps = 2h in the crack region, Section 3):
 * flags[c] = 1 when cell c's edge exceeds h_target and phi is below phi_max at one of its
 * vertices (hanging vertices from their constraints), else 0. phi: device [n_nodes]; flags:
 * host [n_cells]; n_marked: host, optional. Synchronises `stream`. */
fr_status fracture_mark_crack(fr_mesh mesh, const double* phi, double phi_max, double h_target,
                              uint8_t* flags, int64_t* n_marked, void* stream);

void fracture_mesh_destroy(fr_mesh mesh);

/* ---- assembly --------------------------------------------------------------------- */

/* Assembles at the state (u, phi) with the constraint phi <= phi_old and the
 * extrapolation phi_tilde (Formulation 1). *sys == NULL creates the system object (its
 * matrices follow the mesh pattern); otherwise it is reused. flags selects the stages.
 * The active set of the FR_JACOBIAN stage is the one computed by the last FR_ACTIVE_SET
 * stage (callers may also install one with fracture_set_active). u and phi are read on
 * all nodes; only their values at free nodes enter (hanging values are interpolated).
 * prm: host, one parameter set per instance (one for an ordinary mesh). */
fr_status fracture_assemble(fr_mesh mesh, const fr_params* prm /*host*/, const double* u,
                            const double* phi, const double* phi_old, const double* phi_tilde,
                            unsigned flags, fr_system* sys, void* stream);

/* The quantities of the stop test of the Section 3 algorithm (active set unchanged and the
 * residual below TOL). Host outputs: norms[0] = ||R~||_2 (R with Dirichlet u rows and active
 * phi rows zeroed), norms[1] = ||F||_2 (masked right-hand side, if assembled);
 * n_active = |A|; active_changes = entries that changed in the last FR_ACTIVE_SET;
 * min_margin = min_i |lambda_i + c(phi_i - phi_old,i) - tau| (distance of the closest
 * decision to the threshold). Synchronises `stream`. Any pointer may be NULL. Returns
 * FR_ENAN (outputs still written) when a norm is not finite. */
fr_status fracture_residual_norms(fr_system sys, double* norms, int64_t* n_active,
                                  int64_t* active_changes, double* min_margin, void* stream);

/* Device copies of the system vectors (any pointer may be NULL): R[n_solve] residual,
 * F[n_solve] masked right-hand side, B[n_free] lumped phi mass, active[n_free] (0/1). */
fr_status fracture_system_vectors(fr_system sys, double* R, double* F, double* B, uint8_t* active,
                                  void* stream);

/* Installs an active set (device, n_free bytes of 0/1) for the next FR_JACOBIAN stage. */
fr_status fracture_set_active(fr_system sys, const uint8_t* active, void* stream);

/* y = J x with the masked Jacobian (device vectors of n_solve entries). */
fr_status fracture_matvec(fr_system sys, const double* x, double* y, void* stream);

/* y = J x as fracture_solve applies it on a uniform 2d mesh (one instance): the same masked
 * Jacobian (Section 3: the blocks of equations E22ATW and E33ATW, active phase-field rows and
 * columns and Dirichlet displacement rows and columns eliminated, diagonals kept) computed
 * cell by cell from the last assembly's state instead of read from the stored blocks, equal to
 * fracture_matvec up to rounding.  rows = 1: the displacement rows matrix-free, the phase-field
 * rows from the stored blocks; rows = 3: every row matrix-free.  FR_EINVAL on other meshes
 * (see fine_matrix_free) or another `rows`. */
fr_status fracture_matvec_free(fr_system sys, int rows, const double* x, double* y, void* stream);

/* Masked Jacobian as scalar CSR in solve order, host arrays: row_ptr[n_solve+1],
 * col[nnz], val[nnz] with nnz from a first call with col == NULL (it sets *nnz).
 * Explicit zeros of masked entries are kept. Synchronises `stream`. */
fr_status fracture_system_csr(fr_system sys, int64_t* nnz, int64_t* row_ptr, int32_t* col,
                              double* val, void* stream);

void fracture_system_destroy(fr_system sys);

/* ---- AMG and solve ---------------------------------------------------------------- */

/* Builds the block-diagonal preconditioner P^-1 = diag(M_uu~^-1, M_phiphi~^-1) of
 * Section 3: one smoothed-aggregation hierarchy per diagonal block of the masked
 * Jacobian (strength graph, MIS-2 aggregation, tentative prolongator from the rigid-body
 * modes (u) or constants (phi), damped-Jacobi prolongator smoothing, Galerkin R A P),
 * Chebyshev smoothers and a dense coarsest-level inverse. *amg == NULL creates it,
 * otherwise it is rebuilt in place. The host synchronises `stream` between levels.
 * FR_ENAN (nothing built) when the Jacobian or F holds a non-finite value. */
fr_status amg_setup(fr_system sys, const fr_amg_opts* opts /*host*/, fr_amg* amg, void* stream);

/* Host outputs for hierarchy `block` (0 = u, 1 = phi): number of levels, and for level
 * `level`: rows, block size, nnz blocks of A, lambda_max estimate. */
fr_status amg_level_info(fr_amg amg, int block, int level, int* n_levels, int64_t* rows,
                         int* bsize, int64_t* nnz_blocks, double* lambda_max);

/* Launch shape of level operator `which` (0 = A, 1 = P, 2 = R) of hierarchy `block`: SELL
 * slice height and lanes per block row of its SpMV / Chebyshev kernels (host outputs,
 * nullable). FR_EINVAL for a level out of range or an operator the level does not have. */
fr_status amg_level_shape(fr_amg amg, int block, int level, int which, int* slice_height, int* lanes);

/* Forgets the launch shapes the tuner has cached in this process (the next setups time
 * their candidates again). */
fr_status fracture_tune_clear(void);

/* The tuner's cached launch shapes as text, one line per entry, eight integers: operation
 * (0 Chebyshev step, 1 restriction, 2 prolongation), block rows, block columns, floor(log2
 * rows), mean stored blocks per row, FP32 flag, then the chosen slice height (1 or 64) and
 * lanes per row (1, 4, 16, 64).  Two-call protocol: *len receives the text's length without
 * its terminating NUL; with buf non-NULL the text and the NUL are copied when cap > *len, and
 * FR_EINVAL is returned (nothing copied) otherwise.  A table saved from one process and
 * imported into another before its setups makes that process use the same shapes without
 * timing them (deterministic kernels across runs, no tuning cost). */
fr_status fracture_tune_export(char* buf, size_t cap, size_t* len);

/* Adds the entries of a table in the format above to this process's cache (an entry replaces
 * a cached choice with the same key; blank lines are skipped).  The whole text is checked
 * first: FR_EINVAL, with the cache unchanged, for a line that is not eight integers or holds
 * a value out of range. */
fr_status fracture_tune_import(const char* text);

/* Level operator `which` (0 = A, 1 = P, 2 = R) of hierarchy `block` as scalar CSR, host
 * arrays, two-call protocol as fracture_system_csr. FP64 values. */
fr_status amg_level_csr(fr_amg amg, int block, int level, int which, int64_t* n_rows,
                        int64_t* n_cols, int64_t* nnz, int64_t* row_ptr, int32_t* col,
                        double* val, void* stream);

/* z = P^-1 r: one V-cycle per diagonal block (device vectors of n_solve entries). */
fr_status amg_apply(fr_amg amg, const double* r, double* z, void* stream);

void amg_destroy(fr_amg amg);

/* Solves J du = F (masked system): the linear solve of Section 3 ("Linear iterative
 * solution": GMRES preconditioned by the block-diagonal P^-1, one AMG V-cycle per block) as
 * right-preconditioned restarted FGMRES from du = 0, to the true FP64 relative residual
 * ||F - J du|| <= rtol ||F|| (1e-8, the tolerance of the solver study of Table 1). du: device,
 * n_solve. stats: host, one per instance (nullable); each instance stops on its own
 * relative residual, the return value is the worst instance status. Synchronises `stream`
 * once per iteration (one flag per instance). Statuses: FR_ENOCONV with du and stats filled
 * (the last iterate) when maxit is reached; FR_ENAN when F (or the iterate) is not finite;
 * FR_EBREAKDOWN when the Arnoldi process yields a non-finite value from finite inputs (e.g. an
 * FP32 hierarchy whose values overflow), or a zero Arnoldi norm while the true residual is
 * still above the target: the instance stops and du keeps the update of the finite columns. */
fr_status fracture_solve(fr_system sys, fr_amg amg, const fr_solve_opts* opts /*host*/,
                         double* du, fr_solve_stats* stats, void* stream);

/* u[free] += omega du_u, phi[free] += omega du_phi, then hanging values interpolated. */
fr_status fracture_update(fr_mesh mesh, const double* du, double omega, double* u, double* phi,
                          void* stream);

/* The Newton / active-set loop of one loading step (Section 3 algorithm): assemble,
 * active set, masked Jacobian, AMG setup, FGMRES, line search, stop test (active set unchanged
 * and ||R~|| <= max(tol ||R~(U0)||, atol)), with the cycle rule of Section 3 (detect and
 * constrain alternating active-set indices): from the third iterate on, a phi DoF whose
 * membership flipped twice over three consecutive iterates (in-out-in or out-in-out) is frozen
 * active for the rest of the call. The line search scales the update of the DoFs that
 * are not fixed; the fixed ones take their constraint values (Dirichlet u 0, active phi
 * phi_old), so that the loop never stops with an active DoF off phi_old. u and phi are updated in place (device).
 * amg_opts / solve_opts / newton_opts / stats: host. prm and stats hold one entry per
 * instance: on a batched mesh all instances iterate together (one assembly, setup and solve
 * per iteration), each with its own line search and stop test; a finished instance takes no
 * further update, and the loop ends when every instance has finished or failed, or max_it is
 * reached. Status per instance (stats[i].status; the return value is the worst of them, in
 * the order FR_OK < FR_ENOCONV < FR_ECYCLE < FR_EBREAKDOWN < FR_ENAN):
 *   FR_OK        the stop test was met and every FGMRES solve reached rtol;
 *   FR_ENOCONV   max_it reached with ||R~|| above the stop test, or the stop test met while
 *                some FGMRES solve stopped at maxit above rtol (stats.linear_noconv counts
 *                them; each such step was still taken, guarded by the line search);
 *   FR_ECYCLE    max_it reached with the residual part of the stop test met and only the
 *                active set still changing (the cycle rule did not settle it);
 *   FR_EBREAKDOWN an FGMRES breakdown; the instance stops with the state before that step;
 *   FR_ENAN      a non-finite residual (e.g. non-finite input); no Jacobian, preconditioner or
 *                solve is built from it. On a batch only that instance stops (its u and phi
 *                are left as they are); its rows are set to identity rows with zero right-hand
 *                side, so the other instances go on unaffected.
 * Outputs (u, phi, stats) always hold the last iterate. Timings are for the whole call.
 * The working storage (system, preconditioner, Krylov bases) stays with the mesh for the
 * next call, which recomputes all of it; calls on one mesh run one at a time. It is freed
 * by fracture_mesh_destroy, or by a call on another stream (the first stream must stay
 * valid until then). Synchronises `stream`. */
fr_status fracture_newton(fr_mesh mesh, const fr_params* prm, double* u, double* phi,
                          const double* phi_old, const double* phi_tilde,
                          const fr_amg_opts* amg_opts, const fr_solve_opts* solve_opts,
                          const fr_newton_opts* newton_opts, fr_newton_stats* stats,
                          void* stream);

/* Device copies of the active set and of the DoFs frozen by the cycle rule at the end of the
 * last fracture_newton (or fracture_loading step) on this mesh: active, frozen: device
 * [n_free] bytes of 0/1 (either may be NULL). FR_EINVAL before any Newton loop ran on the
 * mesh. Enqueued on `stream` (the loop's stream or one ordered after it). */
fr_status fracture_newton_masks(fr_mesh mesh, uint8_t* active, uint8_t* frozen, void* stream);

/* ---- loading steps (Formulation 1, steps n = 1, 2, 3, ...) ------------------------ */

/* phi_tilde = clip(phi1 + w (phi1 - phi2), 0, 1): the linear extrapolation in time of the
 * phase field that convexifies Formulation 1 (Section 2), with phi1 = phi^{n-1}, phi2 =
 * phi^{n-2} and w = (t_n - t_{n-1}) / (t_{n-1} - t_{n-2}); w = 0 copies phi1. Computed at the
 * free nodes; a hanging node gets the interpolation of its masters' values (clipping and
 * interpolation do not commute; the discrete field is fixed by its free values). The sum is
 * product-then-add, without a fused multiply-add. phi1, phi2, phi_tilde: device [n_nodes];
 * phi_tilde may alias neither input. Enqueued on `stream`; does not synchronise. */
fr_status fracture_extrapolate(fr_mesh mesh, const double* phi1, const double* phi2, double w,
                               double* phi_tilde, void* stream);

/* Quasi-static loading steps n = 1 .. n_steps (Formulation 1 per step). Before step n:
 * phi_old = phi^{n-1} (phi as it enters the step) and phi_tilde = fracture_extrapolate of
 * (phi^{n-1}, phi^{n-2}) to t[n]; at the first step phi^{n-2} is phi_prev at t_prev when
 * phi_prev is given, else phi_tilde = phi^0 (only one state is known). Then the Newton loop of
 * fracture_newton with the parameters prm[(n-1) * n_inst + i] of instance i (the load
 * schedule: p, and any other constant, may change per step), starting from the previous
 * step's (u, phi). t: host [n_steps + 1], strictly increasing, t[0] the time of the state
 * passed in. u, phi: device, updated in place (the state after the last step run). phi_prev:
 * device [n_nodes] or NULL; t_prev < t[0]. stats: host [n_steps * n_inst] or NULL; tcv: host
 * [n_steps * n_inst] or NULL, the TCV of every instance after every step (Section 4). The
 * first step whose Newton loop fails ends the call with its status (its stats and tcv are
 * written, later entries are not). Synchronises `stream`. */
fr_status fracture_loading(fr_mesh mesh, const fr_params* prm, int n_steps, const double* t,
                           double* u, double* phi, const double* phi_prev, double t_prev,
                           const fr_amg_opts* amg_opts, const fr_solve_opts* solve_opts,
                           const fr_newton_opts* newton_opts, fr_newton_stats* stats, double* tcv,
                           void* stream);

/* ---- functionals (Section 4) ------------------------------------------------------ */

/* Per instance i (n_inst of them; 1 for an ordinary mesh): tcv[i] (host) = integral over
 * B_i of u . grad phi; cod[i*n_cod + k] (host) = 1/2 integral of u . grad phi along the
 * line through cod_x[(i*n_cod + k)*(dim-1) ..] parallel to the last axis (cod_x: host, in
 * the instance's coordinates). Either output may be NULL. Synchronises `stream`. */
fr_status fracture_functionals(fr_mesh mesh, const double* u, const double* phi,
                               const double* cod_x, int n_cod, double* cod, double* tcv,
                               void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc): the same results as fracture_functionals, bit for bit (same
 * kernels, same summation order), with no allocation of any kind. Its device buffers (the
 * sample abscissae, per-block partial sums and reduced values) are slices of one fixed array of
 * 524288 doubles (4 MiB) that every device the library runs on holds for the life of the
 * process. Limit: n_inst * n_cod * (dim - 1) + (1 + ceil(c / 256)) * max(1, n_cod) <= 524288,
 * c the cell count of the largest instance (a 2048 x 2048 mesh allows n_cod <= 31); larger calls
 * return FR_EINVAL before any device work. Calls that overlap on one device share the array and
 * race: issue them one at a time per device. Same arguments and synchronisation as
 * fracture_functionals. */
fr_status fracture_functionals_noalloc(fr_mesh mesh, const double* u, const double* phi,
                                       const double* cod_x, int n_cod, double* cod, double* tcv,
                                       void* stream);

/* ---- kernel timing ---------------------------------------------------------------- */

/* enable != 0 starts recording a HIP event pair on the launch stream around every launch
 * of the sparse, smoother, coupled-Jacobian and Gram-Schmidt kernels (and one pair around
 * each block's V-cycle and each AMG setup phase, names "setup_*", which include any host
 * round trips), together with the algorithmic bytes each launch must move; 0 stops.
 * Either call discards what was recorded. */
fr_status fracture_profile(int enable);

/* Entry i of the recording (host outputs): kernel name (valid until the next
 * fracture_profile call), launches, summed event time in ms, summed algorithmic bytes.
 * FR_EINVAL once i is past the last entry. Synchronises the recorded events. */
fr_status fracture_profile_read(int i, const char** name, int64_t* launches, double* ms, double* bytes);

/* ---- misc ------------------------------------------------------------------------- */

/* Device memory from the caller's allocator (e.g. a PyTorch caching allocator): every device
 * allocation the library makes after this call goes through alloc(bytes, device, stream, ctx),
 * which returns a device pointer of at least `bytes` bytes usable in stream order on `stream`
 * (NULL: the call fails with FR_ENOMEM), and the block goes back through
 * dealloc(ptr, bytes, device, stream, ctx) when the library frees it, with the stream its last
 * use was ordered on (the stream it was allocated on). Blocks from the caller's allocator are not
 * cached by the library. Both NULL restores the library's own pool. Blocks remember the allocator
 * that made them, so objects created before a change stay valid; the functions and ctx must stay
 * callable until every block they made is freed. Both must be thread safe (the library may
 * allocate from two host threads during a setup). FR_EINVAL if exactly one is NULL. */
typedef void* (*fr_alloc_fn)(size_t bytes, int device, void* stream, void* ctx);
typedef void (*fr_free_fn)(void* ptr, size_t bytes, int device, void* stream, void* ctx);
fr_status fracture_set_allocator(fr_alloc_fn alloc, fr_free_fn dealloc, void* ctx);

/* Device memory of every object comes from a stream-ordered pool per device, and memory an
 * object gives up is cached for later allocations on the same stream (repeated calls of
 * one size then make no allocation calls). This hands the current device's cached and
 * unused pool memory back to the driver; it synchronises the device. Objects that are
 * alive keep their memory. */
fr_status fracture_trim_pool(void);

const char* fracture_last_error(void);
/* Checks that a gfx950 device is current; FR_EDEVICE otherwise. */
fr_status fracture_device_check(void);
const char* fracture_version(void);

#ifdef __cplusplus
}
#endif
#endif /* FRACTURE_H */
