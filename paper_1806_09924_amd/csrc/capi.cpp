// C ABI of the fracture library: argument validation, handle lifetimes, error reporting and
// the native Newton / active-set driver (Section 3 algorithm) over the device kernels.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>

#include "profile.h"
#include "system.h"

namespace fr {
void assemble_active_freeze(DevSystem& sys, const double* phi, const double* phi_old);
}

struct fr_system_s {
    fr::DevSystem sys;
    fr::DevKrylov kry;
};

struct fr_amg_s {
    fr::DevAmg amg;
};

// Working storage of fracture_newton, kept with the mesh between calls: the assembled
// system, the preconditioner, the Krylov bases and the line-search copies.  Everything in
// it is recomputed by every call; only the allocations are reused.
struct NewtonWork {
    hipStream_t stream = nullptr;
    fr_system_s S;
    fr_amg_s A;
    fr::DBuf<double> du, u_save, p_save;
    bool ran = false;                            // a loop has run: S holds its final active set
};

struct fr_mesh_s {
    std::unique_ptr<fr::DevMesh> m;
    std::mutex newton_mu;                        // fracture_newton calls on one mesh run one at a time
    std::unique_ptr<NewtonWork> nw;              // released before the mesh
};

namespace {

thread_local std::string g_err;

fr_status set_err(fr_status s, const std::string& m) {
    g_err = m;
    return s;
}

template <typename F>
fr_status guard(F&& f) {
    try {
        return f();
    } catch (const fr::Error& e) {
        return set_err(e.status, e.what());
    } catch (const std::bad_alloc&) {
        return set_err(FR_ENOMEM, "host allocation failed");
    } catch (const std::exception& e) {
        return set_err(FR_EINTERNAL, e.what());
    }
}

#define FR_REQUIRE(cond, msg)                     \
    do {                                          \
        if (!(cond)) return set_err(FR_EINVAL, msg); \
    } while (0)

fr_status check_device() {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return set_err(FR_EDEVICE, "no HIP device available");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return set_err(FR_EDEVICE, "hipGetDevice failed");
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) return set_err(FR_EDEVICE, "hipGetDeviceProperties failed");
    if (std::strncmp(p.gcnArchName, "gfx950", 6) != 0)
        return set_err(FR_EDEVICE, std::string("device is ") + p.gcnArchName + ", the library is built for gfx950");
    return FR_OK;
}

fr_status check_params(const fr_params* p) {
    FR_REQUIRE(p != nullptr, "params: NULL");
    FR_REQUIRE(p->E > 0 && std::isfinite(p->E), "params: E must be > 0");
    FR_REQUIRE(p->nu > -1.0 && p->nu < 0.5, "params: nu must be in (-1, 0.5)");
    FR_REQUIRE(p->Gc > 0 && std::isfinite(p->Gc), "params: Gc must be > 0");
    FR_REQUIRE(p->eps > 0 && std::isfinite(p->eps), "params: eps must be > 0");
    FR_REQUIRE(p->kappa > 0 && p->kappa < 1, "params: kappa must be in (0, 1)");
    FR_REQUIRE(std::isfinite(p->p), "params: p must be finite");
    FR_REQUIRE(std::isfinite(p->c_pdas) && p->c_pdas > 0, "params: c_pdas must be > 0");
    return FR_OK;
}

fr_amg_opts default_amg() {
    fr_amg_opts o;
    o.precision = 64;
    o.theta = -1.0;
    o.cheb_degree = 2;
    o.cheb_ratio = 8.0;
    o.coarse_max = 96;
    o.max_levels = 10;
    o.reuse_u_block = 1;
    o.refresh_phi = 1;
    o.autotune = 1;
    o.fine_matrix_free = 7;
    return o;
}

fr_status check_amg(const fr_amg_opts& o) {
    FR_REQUIRE(o.precision == 32 || o.precision == 64, "amg: precision must be 32 or 64");
    FR_REQUIRE(o.theta < 1, "amg: theta must be below 1 (negative: the default of the dimension)");
    FR_REQUIRE(o.cheb_degree >= 1 && o.cheb_degree <= 16, "amg: cheb_degree must be in [1, 16]");
    FR_REQUIRE(o.cheb_ratio > 1, "amg: cheb_ratio must be > 1");
    FR_REQUIRE(o.coarse_max >= 1 && o.coarse_max <= 4096, "amg: coarse_max must be in [1, 4096]");
    FR_REQUIRE(o.max_levels >= 1 && o.max_levels <= 30, "amg: max_levels must be in [1, 30]");
    FR_REQUIRE(o.fine_matrix_free >= 0 && o.fine_matrix_free <= 7, "amg: fine_matrix_free must be in [0, 7]");
    FR_REQUIRE(o.refresh_phi >= 0 && o.refresh_phi <= 2, "amg: refresh_phi must be 0, 1 or 2");
    return FR_OK;
}

fr_status check_solve(const fr_solve_opts& o) {
    FR_REQUIRE(o.rtol > 0 && o.rtol < 1, "solve: rtol must be in (0, 1)");
    FR_REQUIRE(o.restart >= 1 && o.restart <= 120, "solve: restart must be in [1, 120]");
    FR_REQUIRE(o.maxit >= 1, "solve: maxit must be >= 1");
    return FR_OK;
}

// Allocates the system's arrays (kept when the system already belongs to this mesh) and
// resets its state as for a new system.
void system_init(fr_system_s& S, fr::DevMesh& m, hipStream_t s) {
    fr::DevSystem& sys = S.sys;
    const bool fresh = sys.mesh != &m || sys.R.p == nullptr;
    sys.mesh = &m;
    sys.stream = s;
    sys.n_u = m.n_free * m.dim;
    sys.n_solve = m.n_free * (m.dim + 1);
    sys.have_residual = sys.have_active = sys.have_jacobian = false;
    sys.last_changes = 0;
    sys.last_min_margin = 0.0;
    const int64_t slots = m.graph->n_slots;
    auto mk = [&](fr::BMat<double>& b, int br, int bc) {
        b.br = br;
        b.bc = bc;
        b.S = m.graph;
        if (fresh) b.own_val.alloc(size_t(std::max<int64_t>(1, slots)) * br * bc, s);
        b.val = b.own_val.p;
        b.own_val.zero(s);
    };
    mk(sys.Juu, m.dim, m.dim);
    mk(sys.Jpu, 1, m.dim);
    mk(sys.Jpp, 1, 1);
    if (fresh) {
        sys.R.alloc(size_t(sys.n_solve), s);
        sys.F.alloc(size_t(sys.n_solve), s);
        sys.B.alloc(size_t(m.n_free), s);
        sys.active.alloc(size_t(m.n_free), s);
        sys.active_prev.alloc(size_t(m.n_free), s);
        sys.frozen.alloc(size_t(m.n_free), s);
    }
    sys.active.zero(s);
    sys.active_prev.zero(s);
    sys.frozen.zero(s);
    sys.R.zero(s);
    sys.F.zero(s);
}

struct EventTimer {
    hipEvent_t a = nullptr, b = nullptr;
    hipStream_t s;
    explicit EventTimer(hipStream_t st) : s(st) {
        FR_HIP(hipEventCreate(&a));
        FR_HIP(hipEventCreate(&b));
        FR_HIP(hipEventRecord(a, s));
    }
    double stop() {
        FR_HIP(hipEventRecord(b, s));
        FR_HIP(hipEventSynchronize(b));
        float ms = 0;
        FR_HIP(hipEventElapsedTime(&ms, a, b));
        return double(ms) * 1e-3;
    }
    ~EventTimer() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

}  // namespace

extern "C" {

const char* fracture_last_error(void) { return g_err.c_str(); }

fr_status fracture_profile(int enable) {
    return guard([&]() {
        fr::prof_enable(enable != 0);
        return FR_OK;
    });
}

fr_status fracture_profile_read(int i, const char** name, int64_t* launches, double* ms, double* bytes) {
    return guard([&]() {
        if (!fr::prof_read(i, name, launches, ms, bytes)) return set_err(FR_EINVAL, "profile_read: no such entry");
        return FR_OK;
    });
}

const char* fracture_version(void) { return "fracture-gfx950 0.1"; }

fr_status fracture_set_allocator(fr_alloc_fn alloc, fr_free_fn dealloc, void* ctx) {
    FR_REQUIRE((alloc == nullptr) == (dealloc == nullptr), "set_allocator: give both functions or neither");
    return guard([&]() {
        fr::set_allocator(alloc, dealloc, ctx);
        return FR_OK;
    });
}

fr_status fracture_trim_pool(void) {
    return guard([&]() {
        fr::trim_pool();
        return FR_OK;
    });
}

fr_status fracture_device_check(void) {
    return guard([&]() { return check_device(); });
}

fr_status fracture_mesh_create(const fr_mesh_desc* desc, fr_mesh* out, void* stream) {
    FR_REQUIRE(desc != nullptr && out != nullptr, "mesh_create: NULL argument");
    FR_REQUIRE(desc->dim == 2 || desc->dim == 3, "mesh_create: dim must be 2 or 3");
    FR_REQUIRE(desc->levels >= 0 && desc->levels <= 12, "mesh_create: levels must be in [0, 12]");
    for (int k = 0; k < desc->dim; ++k) {
        FR_REQUIRE(desc->base[k] >= 1, "mesh_create: base must be >= 1");
        FR_REQUIRE(desc->hi[k] > desc->lo[k], "mesh_create: need hi > lo");
    }
    return guard([&]() {
        fr_status st = check_device();
        if (st != FR_OK) return st;
        auto h = std::make_unique<fr_mesh_s>();
        h->m = fr::mesh_create(desc, 1, fr::as_stream(stream), true);
        *out = h.release();
        return FR_OK;
    });
}

fr_status fracture_mesh_create_batch(const fr_mesh_desc* desc, int n_inst, fr_mesh* out, void* stream) {
    FR_REQUIRE(desc != nullptr && out != nullptr, "mesh_create_batch: NULL argument");
    FR_REQUIRE(n_inst >= 1 && n_inst <= 65535, "mesh_create_batch: n_inst must be in [1, 65535]");
    for (int i = 0; i < n_inst; ++i) {
        FR_REQUIRE(desc[i].dim == desc[0].dim, "mesh_create_batch: instances must share dim");
        FR_REQUIRE(desc[i].dim == 2 || desc[i].dim == 3, "mesh_create_batch: dim must be 2 or 3");
        FR_REQUIRE(desc[i].levels >= 0 && desc[i].levels <= 12, "mesh_create_batch: levels must be in [0, 12]");
        for (int k = 0; k < desc[i].dim; ++k) {
            FR_REQUIRE(desc[i].base[k] >= 1, "mesh_create_batch: base must be >= 1");
            FR_REQUIRE(desc[i].hi[k] > desc[i].lo[k], "mesh_create_batch: need hi > lo");
        }
    }
    return guard([&]() {
        fr_status st = check_device();
        if (st != FR_OK) return st;
        auto h = std::make_unique<fr_mesh_s>();
        h->m = fr::mesh_create(desc, n_inst, fr::as_stream(stream), true);
        *out = h.release();
        return FR_OK;
    });
}

fr_status fracture_mesh_refine(fr_mesh mesh, const uint8_t* flags, fr_mesh* out, void* stream) {
    FR_REQUIRE(mesh != nullptr && mesh->m && flags != nullptr && out != nullptr, "mesh_refine: NULL argument");
    FR_REQUIRE(mesh->m->n_inst == 1, "mesh_refine: batched meshes are not supported");
    return guard([&]() {
        const fr::DevMesh& old = *mesh->m;
        if (old.on_device) {
            const fr_status st = check_device();
            if (st != FR_OK) return st;
        }
        hipStream_t s = fr::as_stream(stream);
        std::vector<int32_t> loc_cell;
        std::vector<double> loc_xi;
        fr::HostMesh hm = fr::refine_mesh(old.host, flags, loc_cell, loc_xi);
        auto h = std::make_unique<fr_mesh_s>();
        h->m = fr::mesh_from_host(std::move(hm), s, old.on_device);
        h->m->parent_serial = old.serial;
        h->m->parent_nodes = old.n_nodes;
        if (old.on_device) {
            h->m->parent_cell.upload(loc_cell, s);
            h->m->parent_xi.upload(loc_xi, s);
            FR_HIP(hipStreamSynchronize(s));        // the host tables above go out of scope
        }
        *out = h.release();
        return FR_OK;
    });
}

fr_status fracture_transfer(fr_mesh from, fr_mesh to, const double* src, int ncomp, double* dst, void* stream) {
    FR_REQUIRE(from != nullptr && from->m && to != nullptr && to->m, "transfer: NULL mesh");
    FR_REQUIRE(ncomp >= 1 && ncomp <= 16, "transfer: ncomp must be in [1, 16]");
    FR_REQUIRE(to->m->parent_serial == from->m->serial && to->m->parent_nodes == from->m->n_nodes,
               "transfer: `to` was not made from `from` by fracture_mesh_refine");
    FR_REQUIRE(from->m->on_device && to->m->on_device, "transfer: host-only mesh");
    FR_REQUIRE(src != nullptr && dst != nullptr && src != dst, "transfer: NULL or aliased arrays");
    return guard([&]() {
        fr::mesh_transfer(*from->m, *to->m, src, ncomp, dst, fr::as_stream(stream));
        return FR_OK;
    });
}

fr_status fracture_kelly(fr_mesh mesh, const double* u, double* eta2, void* stream) {
    FR_REQUIRE(mesh != nullptr && mesh->m, "kelly: NULL mesh");
    FR_REQUIRE(mesh->m->on_device, "kelly: host-only mesh");
    FR_REQUIRE(u != nullptr && eta2 != nullptr, "kelly: NULL array");
    return guard([&]() {
        fr::mesh_kelly(*mesh->m, u, eta2, fr::as_stream(stream));
        return FR_OK;
    });
}

fr_status fracture_mark_crack(fr_mesh mesh, const double* phi, double phi_max, double h_target, uint8_t* flags,
                              int64_t* n_marked, void* stream) {
    FR_REQUIRE(mesh != nullptr && mesh->m, "mark_crack: NULL mesh");
    FR_REQUIRE(std::isfinite(phi_max) && std::isfinite(h_target) && h_target > 0, "mark_crack: bad thresholds");
    FR_REQUIRE(mesh->m->on_device, "mark_crack: host-only mesh");
    FR_REQUIRE(phi != nullptr && flags != nullptr, "mark_crack: NULL array");
    return guard([&]() {
        hipStream_t s = fr::as_stream(stream);
        const fr::DevMesh& m = *mesh->m;
        fr::DBuf<uint8_t> fd;
        fd.alloc(size_t(m.n_cells), s);
        fr::mesh_mark_crack(m, phi, phi_max, h_target, fd.p, s);
        FR_HIP(hipMemcpyAsync(flags, fd.p, size_t(m.n_cells), hipMemcpyDeviceToHost, s));
        FR_HIP(hipStreamSynchronize(s));
        if (n_marked) {
            int64_t k = 0;
            for (int64_t c = 0; c < m.n_cells; ++c) k += flags[c] ? 1 : 0;
            *n_marked = k;
        }
        return FR_OK;
    });
}

fr_status fracture_mesh_instance(fr_mesh mesh, int inst, int64_t* node_offset, int64_t* n_nodes,
                                 int64_t* free_offset, int64_t* n_free, int64_t* cell_offset, int64_t* n_cells,
                                 double* h_min) {
    FR_REQUIRE(mesh != nullptr && mesh->m, "mesh_instance: NULL mesh");
    const fr::HostMesh& h = mesh->m->host;
    FR_REQUIRE(inst >= 0 && inst < h.n_inst, "mesh_instance: instance out of range");
    const size_t i = size_t(inst);
    if (node_offset) *node_offset = h.node_off[i];
    if (n_nodes) *n_nodes = h.node_off[i + 1] - h.node_off[i];
    if (free_offset) *free_offset = h.free_off[i];
    if (n_free) *n_free = h.free_off[i + 1] - h.free_off[i];
    if (cell_offset) *cell_offset = h.cell_off[i];
    if (n_cells) *n_cells = h.cell_off[i + 1] - h.cell_off[i];
    if (h_min) *h_min = h.inst_h_min[i];
    return FR_OK;
}

fr_status fracture_mesh_create_host(const fr_mesh_desc* desc, fr_mesh* out) {
    FR_REQUIRE(desc != nullptr && out != nullptr, "mesh_create_host: NULL argument");
    FR_REQUIRE(desc->dim == 2 || desc->dim == 3, "mesh_create_host: dim must be 2 or 3");
    return guard([&]() {
        auto h = std::make_unique<fr_mesh_s>();
        h->m = fr::mesh_create(desc, 1, nullptr, false);
        *out = h.release();
        return FR_OK;
    });
}

fr_status fracture_mesh_cells(fr_mesh mesh, int32_t* cells, double* cell_lo, double* cell_h) {
    FR_REQUIRE(mesh != nullptr && mesh->m, "mesh_cells: NULL mesh");
    const fr::HostMesh& h = mesh->m->host;
    if (cells) std::memcpy(cells, h.cells.data(), h.cells.size() * sizeof(int32_t));
    if (cell_lo) std::memcpy(cell_lo, h.cell_lo.data(), h.cell_lo.size() * sizeof(double));
    if (cell_h) std::memcpy(cell_h, h.cell_h.data(), h.cell_h.size() * sizeof(double));
    return FR_OK;
}

fr_status fracture_mesh_constraints(fr_mesh mesh, int64_t* n_entries, int32_t* con_ptr, int32_t* con_master,
                                    double* con_w) {
    FR_REQUIRE(mesh != nullptr && mesh->m && n_entries, "mesh_constraints: NULL argument");
    const fr::HostMesh& h = mesh->m->host;
    *n_entries = int64_t(h.con_master.size());
    if (con_ptr) std::memcpy(con_ptr, h.con_ptr.data(), h.con_ptr.size() * sizeof(int32_t));
    if (con_master) std::memcpy(con_master, h.con_master.data(), h.con_master.size() * sizeof(int32_t));
    if (con_w) std::memcpy(con_w, h.con_w.data(), h.con_w.size() * sizeof(double));
    return FR_OK;
}

fr_status fracture_mesh_faces(fr_mesh mesh, int64_t* n_entries, int32_t* ptr, int32_t* nbr) {
    FR_REQUIRE(mesh != nullptr && mesh->m && n_entries, "mesh_faces: NULL argument");
    return guard([&]() {
        std::vector<int32_t> p, n;
        fr::face_neighbors(mesh->m->host, p, n);
        *n_entries = int64_t(n.size());
        if (ptr) std::memcpy(ptr, p.data(), p.size() * sizeof(int32_t));
        if (nbr) std::memcpy(nbr, n.data(), n.size() * sizeof(int32_t));
        return FR_OK;
    });
}

fr_status fracture_mesh_info(fr_mesh mesh, int64_t* n_nodes, int64_t* n_cells, int64_t* n_free, int64_t* n_all,
                             int64_t* n_solve, int64_t* n_hanging, double* h_min, int64_t* nnz_node_graph) {
    FR_REQUIRE(mesh != nullptr && mesh->m, "mesh_info: NULL mesh");
    const fr::HostMesh& h = mesh->m->host;
    if (n_nodes) *n_nodes = h.n_nodes;
    if (n_cells) *n_cells = h.n_cells;
    if (n_free) *n_free = h.n_free;
    if (n_all) *n_all = (h.dim + 1) * h.n_nodes;
    if (n_solve) *n_solve = (h.dim + 1) * h.n_free;
    if (n_hanging) *n_hanging = h.n_hanging;
    if (h_min) *h_min = h.h_min;
    if (nnz_node_graph) *nnz_node_graph = mesh->m->pat.nnz;
    return FR_OK;
}

fr_status fracture_mesh_nodes(fr_mesh mesh, double* xyz, int64_t* lattice, uint8_t* dirichlet, int32_t* free_index) {
    FR_REQUIRE(mesh != nullptr && mesh->m, "mesh_nodes: NULL mesh");
    const fr::HostMesh& h = mesh->m->host;
    const size_t nd = size_t(h.n_nodes) * h.dim;
    if (xyz) std::memcpy(xyz, h.coords.data(), nd * sizeof(double));
    if (lattice) std::memcpy(lattice, h.lattice.data(), nd * sizeof(int64_t));
    if (dirichlet) std::memcpy(dirichlet, h.dirichlet.data(), size_t(h.n_nodes));
    if (free_index) std::memcpy(free_index, h.free_of_node.data(), size_t(h.n_nodes) * sizeof(int32_t));
    return FR_OK;
}

void fracture_mesh_destroy(fr_mesh mesh) {
    if (!mesh) return;
    if (mesh->nw) (void)hipStreamSynchronize(mesh->nw->stream);
    if (mesh->m) (void)hipStreamSynchronize(mesh->m->stream);
    delete mesh;
}

fr_status fracture_assemble(fr_mesh mesh, const fr_params* prm, const double* u, const double* phi,
                            const double* phi_old, const double* phi_tilde, unsigned flags, fr_system* sys,
                            void* stream) {
    FR_REQUIRE(mesh != nullptr && mesh->m, "assemble: NULL mesh");
    FR_REQUIRE(mesh->m->on_device, "assemble: host-only mesh");
    FR_REQUIRE(sys != nullptr, "assemble: NULL system pointer");
    FR_REQUIRE((flags & ~7u) == 0 && flags != 0, "assemble: unknown or empty flags");
    FR_REQUIRE(prm != nullptr, "assemble: NULL params");
    for (int i = 0; i < mesh->m->n_inst; ++i) {
        fr_status ps = check_params(prm + i);
        if (ps != FR_OK) return ps;
    }
    if (flags & (FR_RESIDUAL | FR_JACOBIAN)) FR_REQUIRE(u && phi && phi_tilde, "assemble: u, phi, phi_tilde required");
    if (flags & (FR_ACTIVE_SET | FR_JACOBIAN)) FR_REQUIRE(phi && phi_old, "assemble: phi, phi_old required");
    if (*sys && (*sys)->sys.mesh != mesh->m.get()) return set_err(FR_EINVAL, "assemble: system belongs to another mesh");
    if (!*sys && (flags & (FR_ACTIVE_SET | FR_JACOBIAN)) && !(flags & FR_RESIDUAL))
        return set_err(FR_EINVAL, "assemble: a new system needs FR_RESIDUAL first");
    if (*sys && (flags & FR_ACTIVE_SET) && !(flags & FR_RESIDUAL) && !(*sys)->sys.have_residual)
        return set_err(FR_EINVAL, "assemble: FR_ACTIVE_SET needs a residual");
    return guard([&]() {
        hipStream_t s = fr::as_stream(stream);
        std::unique_ptr<fr_system_s> created;
        fr_system_s* S = *sys;
        if (!S) {
            created = std::make_unique<fr_system_s>();
            S = created.get();
            system_init(*S, *mesh->m, s);
        }
        S->sys.stream = s;
        S->sys.prm = fr::make_params(prm[0]);
        const int ni = mesh->m->n_inst;
        S->sys.prm_h.resize(size_t(ni));
        for (int i = 0; i < ni; ++i) S->sys.prm_h[size_t(i)] = fr::make_params(prm[i]);
        if (ni > 1) S->sys.prm_d.upload(S->sys.prm_h, s);
        if (flags & FR_RESIDUAL) fr::assemble_residual(S->sys, u, phi, phi_tilde);
        if (flags & FR_ACTIVE_SET) fr::assemble_active(S->sys, phi, phi_old);
        if (flags & FR_JACOBIAN) fr::assemble_jacobian(S->sys, u, phi, phi_old, phi_tilde);
        if (created) *sys = created.release();
        return FR_OK;
    });
}

fr_status fracture_residual_norms(fr_system sys, double* norms, int64_t* n_active, int64_t* active_changes,
                                  double* min_margin, void* stream) {
    FR_REQUIRE(sys != nullptr, "residual_norms: NULL system");
    FR_REQUIRE(sys->sys.have_residual, "residual_norms: nothing assembled");
    return guard([&]() {
        sys->sys.stream = fr::as_stream(stream);
        double nr[2] = {0, 0};
        fr::system_norms(sys->sys, nullptr, nullptr, nr, n_active, min_margin);
        if (norms) { norms[0] = nr[0]; norms[1] = nr[1]; }
        if (active_changes) *active_changes = sys->sys.last_changes;
        if (!std::isfinite(nr[0]) || !std::isfinite(nr[1]))
            return set_err(FR_ENAN, "residual_norms: non-finite residual or right-hand side");
        return FR_OK;
    });
}

fr_status fracture_system_vectors(fr_system sys, double* R, double* F, double* B, uint8_t* active, void* stream) {
    FR_REQUIRE(sys != nullptr, "system_vectors: NULL system");
    return guard([&]() {
        hipStream_t s = fr::as_stream(stream);
        const fr::DevSystem& S = sys->sys;
        const int64_t nf = S.mesh->n_free;
        if (R) FR_HIP(hipMemcpyAsync(R, S.R.p, size_t(S.n_solve) * 8, hipMemcpyDeviceToDevice, s));
        if (F) FR_HIP(hipMemcpyAsync(F, S.F.p, size_t(S.n_solve) * 8, hipMemcpyDeviceToDevice, s));
        if (B) FR_HIP(hipMemcpyAsync(B, S.B.p, size_t(nf) * 8, hipMemcpyDeviceToDevice, s));
        if (active) FR_HIP(hipMemcpyAsync(active, S.active.p, size_t(nf), hipMemcpyDeviceToDevice, s));
        return FR_OK;
    });
}

fr_status fracture_set_active(fr_system sys, const uint8_t* active, void* stream) {
    FR_REQUIRE(sys != nullptr && active != nullptr, "set_active: NULL argument");
    return guard([&]() {
        hipStream_t s = fr::as_stream(stream);
        fr::DevSystem& S = sys->sys;
        FR_HIP(hipMemcpyAsync(S.active.p, active, size_t(S.mesh->n_free), hipMemcpyDeviceToDevice, s));
        S.have_active = true;
        return FR_OK;
    });
}

fr_status fracture_matvec(fr_system sys, const double* x, double* y, void* stream) {
    FR_REQUIRE(sys != nullptr && x != nullptr && y != nullptr, "matvec: NULL argument");
    FR_REQUIRE(sys->sys.have_jacobian, "matvec: no Jacobian assembled");
    return guard([&]() {
        fr::jspmv(sys->sys, x, y, fr::as_stream(stream));
        return FR_OK;
    });
}

fr_status fracture_matvec_free(fr_system sys, int rows, const double* x, double* y, void* stream) {
    FR_REQUIRE(sys != nullptr && x != nullptr && y != nullptr, "matvec_free: NULL argument");
    FR_REQUIRE(rows == 1 || rows == 3, "matvec_free: rows must be 1 or 3");
    FR_REQUIRE(sys->sys.have_jacobian, "matvec_free: no Jacobian assembled");
    FR_REQUIRE(sys->sys.mf.valid, "matvec_free: the mesh is not a uniform 2d single-instance mesh");
    return guard([&]() {
        fr::mf_jspmv<double>(sys->sys, rows == 3, x, y, nullptr, nullptr, 0, fr::as_stream(stream));
        return FR_OK;
    });
}

fr_status fracture_system_csr(fr_system sys, int64_t* nnz, int64_t* row_ptr, int32_t* col, double* val, void* stream) {
    FR_REQUIRE(sys != nullptr && nnz != nullptr, "system_csr: NULL argument");
    FR_REQUIRE(sys->sys.have_jacobian, "system_csr: no Jacobian assembled");
    return guard([&]() {
        hipStream_t s = fr::as_stream(stream);
        fr::DevSystem& S = sys->sys;
        const fr::DevMesh& m = *S.mesh;
        const fr::Pattern& p = m.pat;
        const int D = m.dim;
        const int64_t nf = m.n_free;
        const int64_t total = p.nnz * int64_t(D * D + D + D + 1);
        if (!col) {
            *nnz = total;
            return FR_OK;
        }
        FR_REQUIRE(row_ptr && val && *nnz >= total, "system_csr: output arrays too small");
        auto uu = fr::download(S.Juu.val, size_t(p.n_slots) * D * D, s);
        auto pu = fr::download(S.Jpu.val, size_t(p.n_slots) * D, s);
        auto pp = fr::download(S.Jpp.val, size_t(p.n_slots), s);
        int64_t c = 0;
        auto slot = [&](int64_t f, int k) { return int64_t(p.slice_ptr[size_t(f / p.C)]) + int64_t(k) * p.C + f % p.C; };
        row_ptr[0] = 0;
        for (int64_t f = 0; f < nf; ++f)
            for (int r = 0; r < D; ++r) {
                for (int k = 0; k < p.row_len[size_t(f)]; ++k) {
                    const int64_t sl = slot(f, k);
                    const int64_t g = p.col[size_t(sl)];
                    for (int d = 0; d < D; ++d) {
                        col[c] = int32_t(g * D + d);
                        val[c++] = uu[size_t(sl * D * D + r * D + d)];
                    }
                }
                row_ptr[f * D + r + 1] = c;
            }
        for (int64_t f = 0; f < nf; ++f) {
            for (int k = 0; k < p.row_len[size_t(f)]; ++k) {
                const int64_t sl = slot(f, k);
                const int64_t g = p.col[size_t(sl)];
                for (int d = 0; d < D; ++d) {
                    col[c] = int32_t(g * D + d);
                    val[c++] = pu[size_t(sl * D + d)];
                }
            }
            for (int k = 0; k < p.row_len[size_t(f)]; ++k) {
                const int64_t sl = slot(f, k);
                col[c] = int32_t(D * nf + p.col[size_t(sl)]);
                val[c++] = pp[size_t(sl)];
            }
            row_ptr[D * nf + f + 1] = c;
        }
        *nnz = c;
        return FR_OK;
    });
}

void fracture_system_destroy(fr_system sys) {
    if (!sys) return;
    (void)hipStreamSynchronize(sys->sys.stream);
    delete sys;
}

fr_status amg_setup(fr_system sys, const fr_amg_opts* opts, fr_amg* amg, void* stream) {
    FR_REQUIRE(sys != nullptr && amg != nullptr, "amg_setup: NULL argument");
    FR_REQUIRE(sys->sys.have_jacobian, "amg_setup: no Jacobian assembled");
    fr_amg_opts o = opts ? *opts : default_amg();
    fr_status cs = check_amg(o);
    if (cs != FR_OK) return cs;
    if (*amg && (*amg)->amg.sys && (*amg)->amg.sys != &sys->sys) return set_err(FR_EINVAL, "amg_setup: preconditioner belongs to another system");
    return guard([&]() {
        hipStream_t s = fr::as_stream(stream);
        // a non-finite value would flow through the aggregation and the dense coarse inverse
        if (!fr::system_all_finite(sys->sys, s))
            return set_err(FR_ENAN, "amg_setup: the Jacobian or right-hand side holds a non-finite value");
        std::unique_ptr<fr_amg_s> created;
        fr_amg_s* A = *amg;
        if (!A) {
            created = std::make_unique<fr_amg_s>();
            A = created.get();
        }
        fr::amg_build(A->amg, sys->sys, o, s);
        if (created) *amg = created.release();
        return FR_OK;
    });
}

fr_status amg_level_info(fr_amg amg, int block, int level, int* n_levels, int64_t* rows, int* bsize,
                         int64_t* nnz_blocks, double* lambda_max) {
    FR_REQUIRE(amg != nullptr, "amg_level_info: NULL amg");
    FR_REQUIRE(block == 0 || block == 1, "amg_level_info: block must be 0 or 1");
    return guard([&]() {
        int nl = 0, bs = 0;
        int64_t r = 0, nz = 0;
        double lm = 0;
        fr::amg_info(amg->amg, block, level, nl, r, bs, nz, lm, amg->amg.stream);
        if (n_levels) *n_levels = nl;
        if (level < 0 || level >= nl) return set_err(FR_EINVAL, "amg_level_info: level out of range");
        if (rows) *rows = r;
        if (bsize) *bsize = bs;
        if (nnz_blocks) *nnz_blocks = nz;
        if (lambda_max) *lambda_max = lm;
        return FR_OK;
    });
}

fr_status amg_level_shape(fr_amg amg, int block, int level, int which, int* slice_height, int* lanes) {
    FR_REQUIRE(amg != nullptr, "amg_level_shape: NULL amg");
    FR_REQUIRE(block == 0 || block == 1, "amg_level_shape: block must be 0 or 1");
    FR_REQUIRE(which >= 0 && which <= 2, "amg_level_shape: which must be 0 (A), 1 (P) or 2 (R)");
    return guard([&]() {
        int C = 0, G = 0;
        fr::amg_level_shape(amg->amg, block, level, which, C, G);
        if (slice_height) *slice_height = C;
        if (lanes) *lanes = G;
        return FR_OK;
    });
}

fr_status fracture_tune_clear(void) {
    return guard([&]() {
        fr::tune_clear();
        return FR_OK;
    });
}

fr_status fracture_tune_export(char* buf, size_t cap, size_t* len) {
    FR_REQUIRE(len != nullptr, "fracture_tune_export: NULL len");
    return guard([&]() {
        const std::string t = fr::tune_export();
        *len = t.size();
        if (buf == nullptr) return FR_OK;
        FR_REQUIRE(cap > t.size(), "fracture_tune_export: buffer of " + std::to_string(cap) + " bytes, the table needs " +
                                       std::to_string(t.size() + 1));
        std::memcpy(buf, t.c_str(), t.size() + 1);
        return FR_OK;
    });
}

fr_status fracture_tune_import(const char* text) {
    FR_REQUIRE(text != nullptr, "fracture_tune_import: NULL text");
    return guard([&]() {
        fr::tune_import(text);
        return FR_OK;
    });
}

fr_status amg_level_csr(fr_amg amg, int block, int level, int which, int64_t* n_rows, int64_t* n_cols, int64_t* nnz,
                        int64_t* row_ptr, int32_t* col, double* val, void* stream) {
    FR_REQUIRE(amg != nullptr && nnz != nullptr, "amg_level_csr: NULL argument");
    FR_REQUIRE(block == 0 || block == 1, "amg_level_csr: block must be 0 or 1");
    FR_REQUIRE(which >= 0 && which <= 2, "amg_level_csr: which must be 0 (A), 1 (P) or 2 (R)");
    return guard([&]() {
        int64_t nr = 0, nc = 0;
        std::vector<int64_t> rp;
        std::vector<int32_t> ci;
        std::vector<double> vv;
        fr::amg_level_export(amg->amg, block, level, which, nr, nc, rp, ci, vv, fr::as_stream(stream));
        if (n_rows) *n_rows = nr;
        if (n_cols) *n_cols = nc;
        if (!col) {
            *nnz = int64_t(ci.size());
            return FR_OK;
        }
        if (*nnz < int64_t(ci.size()) || !row_ptr || !val) return set_err(FR_EINVAL, "amg_level_csr: output arrays too small");
        std::memcpy(row_ptr, rp.data(), rp.size() * sizeof(int64_t));
        std::memcpy(col, ci.data(), ci.size() * sizeof(int32_t));
        std::memcpy(val, vv.data(), vv.size() * sizeof(double));
        *nnz = int64_t(ci.size());
        return FR_OK;
    });
}

fr_status amg_apply(fr_amg amg, const double* r, double* z, void* stream) {
    FR_REQUIRE(amg != nullptr && r != nullptr && z != nullptr, "amg_apply: NULL argument");
    return guard([&]() {
        fr::amg_precondition(amg->amg, r, z, fr::as_stream(stream));
        return FR_OK;
    });
}

void amg_destroy(fr_amg amg) {
    if (!amg) return;
    if (amg->amg.stream) (void)hipStreamSynchronize(amg->amg.stream);
    delete amg;
}

fr_status fracture_solve(fr_system sys, fr_amg amg, const fr_solve_opts* opts, double* du, fr_solve_stats* stats,
                         void* stream) {
    FR_REQUIRE(sys != nullptr && amg != nullptr && opts != nullptr && du != nullptr, "solve: NULL argument");
    FR_REQUIRE(sys->sys.have_jacobian, "solve: no Jacobian assembled");
    FR_REQUIRE(amg->amg.sys == &sys->sys, "solve: preconditioner built for another system");
    fr_status cs = check_solve(*opts);
    if (cs != FR_OK) return cs;
    return guard([&]() {
        const fr_status r = fr::fgmres(sys->sys, amg->amg, *opts, du, stats, sys->kry, fr::as_stream(stream));
        if (r == FR_ENOCONV) set_err(r, "solve: iteration limit reached");
        if (r == FR_ENAN) set_err(r, "solve: non-finite right-hand side or iterate");
        if (r == FR_EBREAKDOWN) set_err(r, "solve: Krylov breakdown (non-finite or zero Arnoldi norm)");
        return r;
    });
}

fr_status fracture_update(fr_mesh mesh, const double* du, double omega, double* u, double* phi, void* stream) {
    FR_REQUIRE(mesh != nullptr && mesh->m && du && u && phi, "update: NULL argument");
    FR_REQUIRE(mesh->m->on_device, "update: host-only mesh");
    FR_REQUIRE(std::isfinite(omega), "update: omega must be finite");
    return guard([&]() {
        fr::mesh_update(*mesh->m, du, omega, u, phi, fr::as_stream(stream));
        return FR_OK;
    });
}

// Message of a failed Newton loop.
static std::string newton_message(fr_status st, const char* who) {
    const std::string w(who);
    switch (st) {
        case FR_ENOCONV: return "newton: " + w + " reached max_it above the stop test, or an FGMRES solve stopped at maxit";
        case FR_ECYCLE: return "newton: " + w + " reached max_it with a converged residual and a still changing active set";
        case FR_EBREAKDOWN: return "newton: FGMRES breakdown in " + w;
        case FR_ENAN: return "newton: non-finite residual in " + w;
        default: return "newton: failed";
    }
}

// Newton / active-set loop over a batch of independent instances (one disjoint-union system):
// every iteration assembles, sets up and solves all instances together; the line search
// halves each instance's step on its own (omega_i from its own residual norm), and an
// instance whose active set is unchanged and whose residual is below max(tol x its initial
// one, atol) is finished: its later updates get omega = 0.  An instance whose residual turns
// non-finite, or whose linear solve breaks down, has failed: it takes no further step and its
// rows are replaced by identity rows with zero right-hand side from then on, so that the
// others go on unaffected.  Runs until every instance has finished or failed, or max_it.
static fr_status newton_batch(NewtonWork& W, fr::DevMesh& m, const fr_params* prm, double* u, double* phi,
                              const double* phi_old, const double* phi_tilde, const fr_amg_opts& ao,
                              const fr_solve_opts& so, const fr_newton_opts& no, fr_newton_stats* stats,
                              hipStream_t s) {
    const int ni = m.n_inst;
    const size_t nis = static_cast<size_t>(ni);
    fr_system_s* S = &W.S;
    system_init(*S, m, s);
    fr::DevSystem& sys = S->sys;
    sys.prm_h.resize(nis);
    for (int i = 0; i < ni; ++i) sys.prm_h[size_t(i)] = fr::make_params(prm[i]);
    sys.prm = sys.prm_h[0];
    sys.prm_d.upload(sys.prm_h, s);
    fr_amg_s* A = &W.A;
    const int64_t nn = m.n_nodes;
    if (W.du.p == nullptr) W.du.alloc(size_t(sys.n_solve), s);
    if (W.u_save.p == nullptr) W.u_save.alloc(size_t(nn) * m.dim, s);
    if (W.p_save.p == nullptr) W.p_save.alloc(size_t(nn), s);
    fr::DBuf<double> om_d;
    om_d.alloc(nis, s);
    fr::DBuf<int> bad_d;
    std::vector<fr_newton_stats> ns(nis);
    std::vector<fr_solve_stats> st(nis);
    std::vector<double> r0, rk, nr;
    std::vector<int64_t> n_act, chg;
    std::vector<char> done(nis, 0), ok(nis, 0);
    std::vector<fr_status> failed(nis, FR_OK), lin_worst(nis, FR_OK);
    std::vector<int> lin_noconv(nis, 0);
    std::vector<double> om(nis, 0.0);
    auto live = [&](int i) { return !done[size_t(i)] && failed[size_t(i)] == FR_OK; };
    double t_asm = 0, t_setup = 0, t_solve = 0, t_other = 0;
    {
        EventTimer t(s);
        fr::assemble_residual(sys, u, phi, phi_tilde);
        fr::assemble_active(sys, phi, phi_old);
        t_asm += t.stop();
    }
    fr::system_norms_inst(sys, r0, n_act, chg);
    rk = r0;
    for (int i = 0; i < ni; ++i) {
        ns[size_t(i)].res0 = r0[size_t(i)];
        ns[size_t(i)].res = r0[size_t(i)];
        ns[size_t(i)].n_active = n_act[size_t(i)];
        if (!std::isfinite(r0[size_t(i)])) failed[size_t(i)] = FR_ENAN;
    }
    int it = 0;
    while (it < no.max_it) {
        bool any_live = false, any_failed = false;
        for (int i = 0; i < ni; ++i) {
            any_live = any_live || live(i);
            any_failed = any_failed || failed[size_t(i)] != FR_OK;
        }
        if (!any_live) break;
        {
            EventTimer t(s);
            fr::assemble_jacobian(sys, u, phi, phi_old, phi_tilde);
            if (any_failed) {
                std::vector<int> bad(nis);
                for (int i = 0; i < ni; ++i) bad[size_t(i)] = failed[size_t(i)] != FR_OK;
                bad_d.upload(bad, s);
                fr::system_neutralize(sys, bad_d.p);
            }
            t_asm += t.stop();
        }
        {
            EventTimer t(s);
            fr_amg_opts ao_it = ao;
            ao_it.reuse_u_block = (it > 0 && ao.reuse_u_block) ? 1 : 0;
            if (it == 0) A->amg.h[1].refreshable = false;
            fr::amg_build(A->amg, sys, ao_it, s);
            t_setup += t.stop();
        }
        {
            EventTimer t(s);
            (void)fr::fgmres(sys, A->amg, so, W.du.p, st.data(), S->kry, s);
            t_solve += t.stop();
        }
        for (int i = 0; i < ni; ++i) {
            if (!live(i)) continue;
            const fr_status si = fr_status(st[size_t(i)].status);
            ns[size_t(i)].linear_iters += st[size_t(i)].iters;
            lin_worst[size_t(i)] = fr::worse_status(lin_worst[size_t(i)], si);
            if (si == FR_ENAN || si == FR_EBREAKDOWN) failed[size_t(i)] = si;   // no step from this solve
            else if (si == FR_ENOCONV) ++lin_noconv[size_t(i)];
        }
        EventTimer t(s);
        FR_HIP(hipMemcpyAsync(W.u_save.p, u, size_t(nn) * m.dim * 8, hipMemcpyDeviceToDevice, s));
        FR_HIP(hipMemcpyAsync(W.p_save.p, phi, size_t(nn) * 8, hipMemcpyDeviceToDevice, s));
        std::vector<char> stepped(nis, 0);
        for (int i = 0; i < ni; ++i) {
            stepped[size_t(i)] = live(i);
            ok[size_t(i)] = !live(i);
            om[size_t(i)] = live(i) ? 1.0 : 0.0;
        }
        for (int mm = 0; mm <= no.ls_max; ++mm) {
            for (int i = 0; i < ni; ++i)
                if (!ok[size_t(i)]) om[size_t(i)] = std::ldexp(1.0, -mm);
            if (mm > 0) {
                FR_HIP(hipMemcpyAsync(u, W.u_save.p, size_t(nn) * m.dim * 8, hipMemcpyDeviceToDevice, s));
                FR_HIP(hipMemcpyAsync(phi, W.p_save.p, size_t(nn) * 8, hipMemcpyDeviceToDevice, s));
            }
            om_d.upload(om, s);
            fr::mesh_update_inst(m, W.du.p, om_d.p, u, phi, s, sys.active.p, phi_old);
            fr::assemble_residual(sys, u, phi, phi_tilde);
            fr::system_norms_inst(sys, nr, n_act, chg);
            bool all = true;
            for (int i = 0; i < ni; ++i) {
                if (!ok[size_t(i)] && nr[size_t(i)] < rk[size_t(i)]) ok[size_t(i)] = 1;
                all = all && ok[size_t(i)];
            }
            if (all) break;
        }
        ++it;
        if (it >= 2 && !no.no_cycle_freeze) fr::assemble_active_freeze(sys, phi, phi_old);
        else fr::assemble_active(sys, phi, phi_old);
        fr::system_norms_inst(sys, rk, n_act, chg);
        t_other += t.stop();
        for (int i = 0; i < ni; ++i) {
            fr_newton_stats& q = ns[size_t(i)];
            if (!stepped[size_t(i)]) continue;
            q.iterations = it;
            q.res = rk[size_t(i)];
            q.n_active = n_act[size_t(i)];
            if (!std::isfinite(rk[size_t(i)])) failed[size_t(i)] = FR_ENAN;
            else if (chg[size_t(i)] == 0 && rk[size_t(i)] <= std::max(no.tol * r0[size_t(i)], no.atol))
                done[size_t(i)] = 1;
        }
    }
    const std::vector<int64_t> nfz = it >= 2 ? fr::count_flags_inst(sys, sys.frozen.p) : std::vector<int64_t>(nis, 0);
    fr_status worst = FR_OK;
    for (int i = 0; i < ni; ++i) {
        fr_newton_stats& q = ns[size_t(i)];
        fr_status si;
        if (failed[size_t(i)] != FR_OK) si = failed[size_t(i)];
        else if (done[size_t(i)]) si = lin_noconv[size_t(i)] ? FR_ENOCONV : FR_OK;
        else si = q.res <= std::max(no.tol * r0[size_t(i)], no.atol) ? FR_ECYCLE : FR_ENOCONV;
        q.status = si;
        q.n_frozen = nfz[size_t(i)];
        q.linear_noconv = lin_noconv[size_t(i)];
        q.linear_status = lin_worst[size_t(i)];
        q.t_assemble = t_asm;
        q.t_setup = t_setup;
        q.t_solve = t_solve;
        q.t_other = t_other;
        worst = fr::worse_status(worst, si);
    }
    if (stats) std::copy(ns.begin(), ns.end(), stats);
    FR_HIP(hipStreamSynchronize(s));
    W.ran = true;
    if (worst != FR_OK) set_err(worst, newton_message(worst, "an instance"));
    return worst;
}

// Options of a Newton loop with the library defaults for NULL pointers, validated.
static fr_status newton_options(const fr_amg_opts* amg_opts, const fr_solve_opts* solve_opts,
                                const fr_newton_opts* newton_opts, fr_amg_opts& ao, fr_solve_opts& so,
                                fr_newton_opts& no) {
    ao = amg_opts ? *amg_opts : default_amg();
    if (check_amg(ao) != FR_OK) return FR_EINVAL;
    so = fr_solve_opts{1e-8, 100, 500, 1};
    if (solve_opts) so = *solve_opts;
    if (check_solve(so) != FR_OK) return FR_EINVAL;
    no = fr_newton_opts{1e-8, 30, 8, 0.0, 0};
    if (newton_opts) no = *newton_opts;
    FR_REQUIRE(no.tol > 0 && no.atol >= 0 && std::isfinite(no.atol) && no.max_it >= 1 && no.ls_max >= 0 &&
                   no.ls_max <= 60,
               "newton: bad options");
    return FR_OK;
}

// One Newton / active-set loop on a validated mesh and validated options (fracture_newton
// and every step of fracture_loading).  Throws on HIP errors; the callers wrap it in guard().
static fr_status newton_run(fr_mesh mesh, const fr_params* prm, double* u, double* phi, const double* phi_old,
                            const double* phi_tilde, const fr_amg_opts& ao, const fr_solve_opts& so,
                            const fr_newton_opts& no, fr_newton_stats* stats, hipStream_t s) {
    fr::DevMesh& m = *mesh->m;
    std::lock_guard<std::mutex> lk(mesh->newton_mu);
    if (mesh->nw && mesh->nw->stream != s) {
        // storage is freed on the stream it was allocated on
        FR_HIP(hipStreamSynchronize(mesh->nw->stream));
        mesh->nw.reset();
    }
    const bool fresh = !mesh->nw;
    if (fresh) {
        mesh->nw = std::make_unique<NewtonWork>();
        mesh->nw->stream = s;
    }
    NewtonWork& W = *mesh->nw;
    if (m.n_inst > 1) return newton_batch(W, m, prm, u, phi, phi_old, phi_tilde, ao, so, no, stats, s);
    fr_newton_stats ns{};
    fr_system_s* S = &W.S;
    system_init(*S, m, s);
    fr::DevSystem& sys = S->sys;
    sys.prm = fr::make_params(*prm);
    sys.prm_h = {sys.prm};
    fr_amg_s* A = &W.A;
    const int64_t nn = m.n_nodes;
    fr::DBuf<double>& du = W.du;
    fr::DBuf<double>& u_save = W.u_save;
    fr::DBuf<double>& p_save = W.p_save;
    if (du.p == nullptr) du.alloc(size_t(sys.n_solve), s);
    if (u_save.p == nullptr) u_save.alloc(size_t(nn) * m.dim, s);
    if (p_save.p == nullptr) p_save.alloc(size_t(nn), s);
    double t_asm = 0, t_setup = 0, t_solve = 0, t_other = 0;
    {
        EventTimer t(s);
        fr::assemble_residual(sys, u, phi, phi_tilde);
        fr::assemble_active(sys, phi, phi_old);
        t_asm += t.stop();
    }
    double nr[2];
    int64_t n_act = 0;
    fr::system_norms(sys, nullptr, nullptr, nr, &n_act, nullptr);
    const double r0 = nr[0];
    double rk = r0;
    ns.res0 = r0;
    ns.n_active = n_act;
    int it = 0, lin_noconv = 0;
    fr_status lin_worst = FR_OK;
    // FR_ENAN / FR_EBREAKDOWN end the loop; nothing is built from a non-finite residual
    fr_status failed = std::isfinite(r0) ? FR_OK : FR_ENAN;
    bool converged = false;
    while (failed == FR_OK && it < no.max_it) {
        {
            EventTimer t(s);
            fr::assemble_jacobian(sys, u, phi, phi_old, phi_tilde);
            t_asm += t.stop();
        }
        {
            EventTimer t(s);
            fr_amg_opts ao_it = ao;
            ao_it.reuse_u_block = (it > 0 && ao.reuse_u_block) ? 1 : 0;
            // the first iteration of every call builds both hierarchies from scratch (the
            // phase-field one keeps what a later refresh needs when refresh_phi is set)
            if (it == 0) A->amg.h[1].refreshable = false;
            fr::amg_build(A->amg, sys, ao_it, s);
            t_setup += t.stop();
        }
        fr_solve_stats st{};
        {
            EventTimer t(s);
            const fr_status r = fr::fgmres(sys, A->amg, so, du.p, &st, S->kry, s);
            t_solve += t.stop();
            ns.linear_iters += st.iters;
            lin_worst = fr::worse_status(lin_worst, r);
            if (r == FR_ENAN || r == FR_EBREAKDOWN) {   // no step from this solve
                failed = r;
                break;
            }
            if (r == FR_ENOCONV) ++lin_noconv;
        }
        EventTimer t(s);
        // line search on ||R~|| with the current active set; the fixed DoFs take their
        // constraint values at every trial (Dirichlet u 0, active phi phi_old)
        FR_HIP(hipMemcpyAsync(u_save.p, u, size_t(nn) * m.dim * 8, hipMemcpyDeviceToDevice, s));
        FR_HIP(hipMemcpyAsync(p_save.p, phi, size_t(nn) * 8, hipMemcpyDeviceToDevice, s));
        for (int mm = 0; mm <= no.ls_max; ++mm) {
            const double omega = std::ldexp(1.0, -mm);
            if (mm > 0) {
                FR_HIP(hipMemcpyAsync(u, u_save.p, size_t(nn) * m.dim * 8, hipMemcpyDeviceToDevice, s));
                FR_HIP(hipMemcpyAsync(phi, p_save.p, size_t(nn) * 8, hipMemcpyDeviceToDevice, s));
            }
            fr::mesh_update(m, du.p, omega, u, phi, s, sys.active.p, phi_old);
            fr::assemble_residual(sys, u, phi, phi_tilde);
            fr::system_norms(sys, nullptr, nullptr, nr, nullptr, nullptr);
            if (nr[0] < rk) break;
        }
        ++it;
        // the cycle rule: from the third iterate on, alternating phi DoFs are frozen active
        if (it >= 2 && !no.no_cycle_freeze) fr::assemble_active_freeze(sys, phi, phi_old);
        else fr::assemble_active(sys, phi, phi_old);
        fr::system_norms(sys, nullptr, nullptr, nr, &n_act, nullptr);
        rk = nr[0];
        ns.n_active = n_act;
        t_other += t.stop();
        if (!std::isfinite(rk)) {
            failed = FR_ENAN;
            break;
        }
        if (sys.last_changes == 0 && rk <= std::max(no.tol * r0, no.atol)) {
            converged = true;
            break;
        }
    }
    fr_status status;
    if (failed != FR_OK) status = failed;
    else if (converged) status = lin_noconv ? FR_ENOCONV : FR_OK;
    // the iteration cap: a loop held back only by a still-changing active set is a cycle the
    // rule did not settle, anything else is plain non-convergence
    else status = rk <= std::max(no.tol * r0, no.atol) ? FR_ECYCLE : FR_ENOCONV;
    ns.iterations = it;
    ns.res = rk;
    ns.status = status;
    ns.n_frozen = it >= 2 ? fr::count_flags_inst(sys, sys.frozen.p)[0] : 0;
    ns.linear_noconv = lin_noconv;
    ns.linear_status = lin_worst;
    ns.t_assemble = t_asm;
    ns.t_setup = t_setup;
    ns.t_solve = t_solve;
    ns.t_other = t_other;
    if (stats) *stats = ns;
    FR_HIP(hipStreamSynchronize(s));
    W.ran = true;
    if (status != FR_OK) set_err(status, newton_message(status, "the loop"));
    return status;
}

fr_status fracture_newton(fr_mesh mesh, const fr_params* prm, double* u, double* phi, const double* phi_old,
                          const double* phi_tilde, const fr_amg_opts* amg_opts, const fr_solve_opts* solve_opts,
                          const fr_newton_opts* newton_opts, fr_newton_stats* stats, void* stream) {
    FR_REQUIRE(mesh != nullptr && mesh->m, "newton: NULL mesh");
    FR_REQUIRE(mesh->m->on_device, "newton: host-only mesh");
    FR_REQUIRE(u && phi && phi_old && phi_tilde, "newton: NULL state array");
    FR_REQUIRE(prm != nullptr, "newton: NULL params");
    for (int i = 0; i < mesh->m->n_inst; ++i) {
        fr_status ps = check_params(prm + i);
        if (ps != FR_OK) return ps;
    }
    fr_amg_opts ao;
    fr_solve_opts so;
    fr_newton_opts no;
    const fr_status os = newton_options(amg_opts, solve_opts, newton_opts, ao, so, no);
    if (os != FR_OK) return os;
    return guard([&]() {
        return newton_run(mesh, prm, u, phi, phi_old, phi_tilde, ao, so, no, stats, fr::as_stream(stream));
    });
}

fr_status fracture_newton_masks(fr_mesh mesh, uint8_t* active, uint8_t* frozen, void* stream) {
    FR_REQUIRE(mesh != nullptr && mesh->m, "newton_masks: NULL mesh");
    FR_REQUIRE(mesh->m->on_device, "newton_masks: host-only mesh");
    std::lock_guard<std::mutex> lk(mesh->newton_mu);
    FR_REQUIRE(mesh->nw && mesh->nw->ran, "newton_masks: no Newton loop has run on this mesh");
    return guard([&]() {
        hipStream_t s = fr::as_stream(stream);
        const fr::DevSystem& S = mesh->nw->S.sys;
        const size_t nf = size_t(mesh->m->n_free);
        if (active) FR_HIP(hipMemcpyAsync(active, S.active.p, nf, hipMemcpyDeviceToDevice, s));
        if (frozen) FR_HIP(hipMemcpyAsync(frozen, S.frozen.p, nf, hipMemcpyDeviceToDevice, s));
        return FR_OK;
    });
}

fr_status fracture_extrapolate(fr_mesh mesh, const double* phi1, const double* phi2, double w, double* phi_tilde,
                               void* stream) {
    FR_REQUIRE(mesh != nullptr && mesh->m, "extrapolate: NULL mesh");
    FR_REQUIRE(mesh->m->on_device, "extrapolate: host-only mesh");
    FR_REQUIRE(phi1 && phi2 && phi_tilde, "extrapolate: NULL array");
    FR_REQUIRE(std::isfinite(w), "extrapolate: w must be finite");
    return guard([&]() {
        fr::extrapolate(*mesh->m, phi1, phi2, w, phi_tilde, fr::as_stream(stream));
        return FR_OK;
    });
}

fr_status fracture_loading(fr_mesh mesh, const fr_params* prm, int n_steps, const double* t, double* u, double* phi,
                           const double* phi_prev, double t_prev, const fr_amg_opts* amg_opts,
                           const fr_solve_opts* solve_opts, const fr_newton_opts* newton_opts,
                           fr_newton_stats* stats, double* tcv, void* stream) {
    FR_REQUIRE(mesh != nullptr && mesh->m, "loading: NULL mesh");
    FR_REQUIRE(prm != nullptr && t != nullptr, "loading: NULL params or times");
    FR_REQUIRE(n_steps >= 1 && n_steps <= 100000, "loading: n_steps out of range");
    const int ni = mesh->m->n_inst;
    for (int k = 0; k < n_steps; ++k) {
        FR_REQUIRE(std::isfinite(t[k]) && std::isfinite(t[k + 1]) && t[k + 1] > t[k],
                   "loading: times must be finite and increasing");
        for (int i = 0; i < ni; ++i) {
            const fr_status ps = check_params(prm + size_t(k) * ni + i);
            if (ps != FR_OK) return ps;
        }
    }
    FR_REQUIRE(phi_prev == nullptr || (std::isfinite(t_prev) && t_prev < t[0]),
               "loading: t_prev must be finite and before t[0]");
    FR_REQUIRE(mesh->m->on_device, "loading: host-only mesh");
    FR_REQUIRE(u && phi, "loading: NULL state array");
    fr_amg_opts ao;
    fr_solve_opts so;
    fr_newton_opts no;
    const fr_status os = newton_options(amg_opts, solve_opts, newton_opts, ao, so, no);
    if (os != FR_OK) return os;
    return guard([&]() {
        hipStream_t s = fr::as_stream(stream);
        fr::DevMesh& m = *mesh->m;
        const size_t nn = size_t(m.n_nodes);
        // phi^{n-1} (phi_old of step n), phi^{n-2} and phi_tilde
        fr::DBuf<double> cur, before, pt;
        cur.alloc(nn, s);
        pt.alloc(nn, s);
        bool have_before = phi_prev != nullptr;
        double t_before = t_prev;
        if (have_before) {
            before.alloc(nn, s);
            FR_HIP(hipMemcpyAsync(before.p, phi_prev, nn * 8, hipMemcpyDeviceToDevice, s));
        }
        fr_status worst = FR_OK;
        for (int k = 0; k < n_steps; ++k) {
            FR_HIP(hipMemcpyAsync(cur.p, phi, nn * 8, hipMemcpyDeviceToDevice, s));
            const double w = have_before ? (t[k + 1] - t[k]) / (t[k] - t_before) : 0.0;
            // w = 0 reproduces phi^{n-1} on the free nodes (and interpolates the hanging ones)
            fr::extrapolate(m, cur.p, have_before ? before.p : cur.p, w, pt.p, s);
            fr_newton_stats* st = stats ? stats + size_t(k) * ni : nullptr;
            const fr_status r = newton_run(mesh, prm + size_t(k) * ni, u, phi, cur.p, pt.p, ao, so, no, st, s);
            if (tcv) fr::mesh_functionals(m, u, phi, nullptr, 0, nullptr, tcv + size_t(k) * ni, s);
            if (r != FR_OK) {
                worst = r;
                break;
            }
            if (!have_before) {
                before.alloc(nn, s);
                have_before = true;
            }
            std::swap(before, cur);
            t_before = t[k];
        }
        FR_HIP(hipStreamSynchronize(s));
        return worst;
    });
}

fr_status fracture_functionals(fr_mesh mesh, const double* u, const double* phi, const double* cod_x, int n_cod,
                               double* cod, double* tcv, void* stream) {
    FR_REQUIRE(mesh != nullptr && mesh->m && u && phi, "functionals: NULL argument");
    FR_REQUIRE(mesh->m->on_device, "functionals: host-only mesh");
    FR_REQUIRE(n_cod >= 0 && n_cod <= 65535, "functionals: n_cod out of range");
    FR_REQUIRE(n_cod == 0 || (cod_x && cod), "functionals: cod_x and cod required when n_cod > 0");
    return guard([&]() {
        fr::mesh_functionals(*mesh->m, u, phi, cod_x, n_cod, cod, tcv, fr::as_stream(stream));
        return FR_OK;
    });
}

fr_status fracture_functionals_noalloc(fr_mesh mesh, const double* u, const double* phi, const double* cod_x,
                                       int n_cod, double* cod, double* tcv, void* stream) {
    FR_REQUIRE(mesh != nullptr && mesh->m && u && phi, "functionals_noalloc: NULL argument");
    FR_REQUIRE(mesh->m->on_device, "functionals_noalloc: host-only mesh");
    FR_REQUIRE(n_cod >= 0 && n_cod <= 65535, "functionals_noalloc: n_cod out of range");
    FR_REQUIRE(n_cod == 0 || (cod_x && cod), "functionals_noalloc: cod_x and cod required when n_cod > 0");
    FR_REQUIRE(fr::functionals_scratch_need(*mesh->m, n_cod) <= int64_t(fr::kFunctionalsScratchDoubles),
               "functionals_noalloc: n_inst * n_cod * (dim - 1) + (1 + ceil(largest instance's cells / 256)) * "
               "max(1, n_cod) exceeds the 524288 doubles of the fixed scratch");
    return guard([&]() {
        fr::mesh_functionals_noalloc(*mesh->m, u, phi, cod_x, n_cod, cod, tcv, fr::as_stream(stream));
        return FR_OK;
    });
}

}  // extern "C"
