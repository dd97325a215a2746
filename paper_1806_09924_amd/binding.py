"""ctypes binding of libfracture.so (include/fracture.h).  Argument marshalling only: every
step of the computation runs in the library's HIP kernels.  Device arrays are torch
tensors on the current HIP device; calls are ordered on torch's current stream.

The library must have been built (python -m paper_1806_09924_amd.build); importing this
module without it raises, there is no fallback path.
"""
import ctypes
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfracture.so")

FR_OK, FR_EINVAL, FR_ENOMEM, FR_EDEVICE, FR_ENOCONV, FR_EBREAKDOWN, FR_ENAN, FR_ECYCLE, FR_EINTERNAL = range(9)
STATUS_NAMES = ["FR_OK", "FR_EINVAL", "FR_ENOMEM", "FR_EDEVICE", "FR_ENOCONV", "FR_EBREAKDOWN", "FR_ENAN",
                "FR_ECYCLE", "FR_EINTERNAL"]
FR_RESIDUAL, FR_ACTIVE_SET, FR_JACOBIAN = 1, 2, 4

c_double3 = ctypes.c_double * 3
c_int3 = ctypes.c_int * 3


class MeshDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("lo", c_double3), ("hi", c_double3), ("base", c_int3),
                ("levels", ctypes.c_int), ("refine_radius", ctypes.c_double),
                ("crack_center", c_double3), ("crack_half_len", ctypes.c_double)]


class Params(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("E", "nu", "Gc", "kappa", "eps", "p", "c_pdas", "tau_pdas")]


class AmgOpts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("theta", ctypes.c_double), ("cheb_degree", ctypes.c_int),
                ("cheb_ratio", ctypes.c_double), ("coarse_max", ctypes.c_int), ("max_levels", ctypes.c_int),
                ("reuse_u_block", ctypes.c_int), ("refresh_phi", ctypes.c_int), ("autotune", ctypes.c_int),
                ("fine_matrix_free", ctypes.c_int)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("restart", ctypes.c_int), ("maxit", ctypes.c_int),
                ("use_graphs", ctypes.c_int)]


class SolveStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("relres", ctypes.c_double), ("status", ctypes.c_int)]


class NewtonOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_it", ctypes.c_int), ("ls_max", ctypes.c_int),
                ("atol", ctypes.c_double), ("no_cycle_freeze", ctypes.c_int)]


class NewtonStats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("linear_iters", ctypes.c_int), ("res0", ctypes.c_double),
                ("res", ctypes.c_double), ("n_active", ctypes.c_int64), ("status", ctypes.c_int),
                ("t_assemble", ctypes.c_double), ("t_setup", ctypes.c_double), ("t_solve", ctypes.c_double),
                ("t_other", ctypes.c_double), ("n_frozen", ctypes.c_int64), ("linear_noconv", ctypes.c_int),
                ("linear_status", ctypes.c_int)]


class FractureError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES[status] if 0 <= status < 9 else status}: {msg}")
        self.status = status


_P = ctypes.c_void_p
_I64P = ctypes.POINTER(ctypes.c_int64)
_DP = ctypes.POINTER(ctypes.c_double)
_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p)

_SIGNATURES = {
    "fracture_mesh_create": [ctypes.POINTER(MeshDesc), ctypes.POINTER(_P), _P],
    "fracture_mesh_info": [_P, _I64P, _I64P, _I64P, _I64P, _I64P, _I64P, _DP, _I64P],
    "fracture_mesh_nodes": [_P, _P, _P, _P, _P],
    "fracture_mesh_create_host": [ctypes.POINTER(MeshDesc), ctypes.POINTER(_P)],
    "fracture_mesh_create_batch": [ctypes.POINTER(MeshDesc), ctypes.c_int, ctypes.POINTER(_P), _P],
    "fracture_mesh_instance": [_P, ctypes.c_int, _I64P, _I64P, _I64P, _I64P, _I64P, _I64P, _DP],
    "fracture_mesh_cells": [_P, _P, _P, _P],
    "fracture_mesh_constraints": [_P, _I64P, _P, _P, _P],
    "fracture_mesh_destroy": [_P],
    "fracture_assemble": [_P, ctypes.POINTER(Params), _P, _P, _P, _P, ctypes.c_uint, ctypes.POINTER(_P), _P],
    "fracture_residual_norms": [_P, _DP, _I64P, _I64P, _DP, _P],
    "fracture_system_vectors": [_P, _P, _P, _P, _P, _P],
    "fracture_set_active": [_P, _P, _P],
    "fracture_matvec": [_P, _P, _P, _P],
    "fracture_matvec_free": [_P, ctypes.c_int, _P, _P, _P],
    "fracture_system_csr": [_P, _I64P, _P, _P, _P, _P],
    "fracture_system_destroy": [_P],
    "amg_setup": [_P, ctypes.POINTER(AmgOpts), ctypes.POINTER(_P), _P],
    "amg_level_shape": [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                        ctypes.POINTER(ctypes.c_int)],
    "fracture_tune_clear": [],
    "fracture_tune_export": [ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)],
    "fracture_tune_import": [ctypes.c_char_p],
    "amg_level_info": [_P, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int), _I64P,
                       ctypes.POINTER(ctypes.c_int), _I64P, _DP],
    "amg_level_csr": [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, _I64P, _I64P, _I64P, _P, _P, _P, _P],
    "amg_apply": [_P, _P, _P, _P],
    "amg_destroy": [_P],
    "fracture_solve": [_P, _P, ctypes.POINTER(SolveOpts), _P, ctypes.POINTER(SolveStats), _P],
    "fracture_update": [_P, _P, ctypes.c_double, _P, _P, _P],
    "fracture_newton": [_P, ctypes.POINTER(Params), _P, _P, _P, _P, ctypes.POINTER(AmgOpts),
                        ctypes.POINTER(SolveOpts), ctypes.POINTER(NewtonOpts), ctypes.POINTER(NewtonStats), _P],
    "fracture_extrapolate": [_P, _P, _P, ctypes.c_double, _P, _P],
    "fracture_newton_masks": [_P, _P, _P, _P],
    "fracture_mesh_refine": [_P, _P, ctypes.POINTER(_P), _P],
    "fracture_transfer": [_P, _P, _P, ctypes.c_int, _P, _P],
    "fracture_mark_crack": [_P, _P, ctypes.c_double, ctypes.c_double, _P, _I64P, _P],
    "fracture_kelly": [_P, _P, _P, _P],
    "fracture_mesh_faces": [_P, _I64P, _P, _P],
    "fracture_loading": [_P, ctypes.POINTER(Params), ctypes.c_int, _DP, _P, _P, _P, ctypes.c_double,
                         ctypes.POINTER(AmgOpts), ctypes.POINTER(SolveOpts), ctypes.POINTER(NewtonOpts),
                         ctypes.POINTER(NewtonStats), _DP, _P],
    "fracture_functionals": [_P, _P, _P, _P, ctypes.c_int, _P, _P, _P],
    "fracture_functionals_noalloc": [_P, _P, _P, _P, ctypes.c_int, _P, _P, _P],
    "fracture_profile": [ctypes.c_int],
    "fracture_profile_read": [ctypes.c_int, ctypes.POINTER(ctypes.c_char_p), _I64P, _DP, _DP],
    "fracture_last_error": [],
    "fracture_device_check": [],
    "fracture_trim_pool": [],
    "fracture_set_allocator": [_ALLOC_FN, _FREE_FN, _P],
    "fracture_version": [],
}
_VOID = {"fracture_mesh_destroy", "fracture_system_destroy", "amg_destroy"}
_CHARP = {"fracture_last_error", "fracture_version"}

_lib = None


def load():
    """Loads the built library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1806_09924_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, args in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = None if name in _VOID else (ctypes.c_char_p if name in _CHARP else ctypes.c_int)
    _lib = lib
    return lib


def last_error():
    return load().fracture_last_error().decode()


def _check(status):
    if status != FR_OK:
        raise FractureError(status, last_error())
    return status


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, dtype=torch.float64):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"contiguous {dtype} tensor expected")
    return ctypes.c_void_p(t.data_ptr())


def params(E=1.0, nu=0.2, Gc=1.0, kappa=1e-10, eps=1.0 / 16, p=1e-3, c_pdas=1.0, tau_pdas=0.0):
    return Params(E, nu, Gc, kappa, eps, p, c_pdas, tau_pdas)


def amg_opts(precision=64, theta=-1.0, cheb_degree=2, cheb_ratio=8.0, coarse_max=96, max_levels=12,
             reuse_u_block=1, refresh_phi=1, autotune=1, fine_matrix_free=7):
    return AmgOpts(precision, theta, cheb_degree, cheb_ratio, coarse_max, max_levels, reuse_u_block, refresh_phi,
                   autotune, fine_matrix_free)


def solve_opts(rtol=1e-8, restart=100, maxit=500, use_graphs=1):
    return SolveOpts(rtol, restart, maxit, use_graphs)


def newton_opts(tol=1e-8, max_it=30, ls_max=8, atol=0.0, no_cycle_freeze=0):
    return NewtonOpts(tol, max_it, ls_max, atol, no_cycle_freeze)


# statuses of a solve or Newton loop that leave valid outputs (the last iterate) behind
SOLVER_STATUSES = (FR_ENOCONV, FR_ECYCLE, FR_EBREAKDOWN, FR_ENAN)


def mesh_desc(dim, lo, hi, base, levels=0, refine_radius=0.0, crack_center=(0.0, 0.0, 0.0), crack_half_len=0.0):
    d = MeshDesc()
    d.dim = dim
    for k in range(3):
        d.lo[k] = lo if k < dim else 0.0
        d.hi[k] = hi if k < dim else 1.0
        d.base[k] = base if k < dim else 1
        d.crack_center[k] = crack_center[k] if k < len(crack_center) else 0.0
    d.levels = levels
    d.refine_radius = refine_radius
    d.crack_half_len = crack_half_len
    return d


class Mesh:
    """A mesh, or a batch of independent meshes when `desc` is a list of descriptors."""

    def __init__(self, desc, host_only=False, _handle=None):
        lib = load()
        h = _P()
        self.n_inst = 1
        self.host_only = host_only
        if _handle is not None:
            h = _handle
        elif isinstance(desc, (list, tuple)):
            arr = (MeshDesc * len(desc))(*desc)
            self.n_inst = len(desc)
            _check(lib.fracture_mesh_create_batch(arr, len(desc), ctypes.byref(h), _stream()))
            desc = desc[0]
        elif host_only:
            _check(lib.fracture_mesh_create_host(ctypes.byref(desc), ctypes.byref(h)))
        else:
            _check(lib.fracture_mesh_create(ctypes.byref(desc), ctypes.byref(h), _stream()))
        self.h = h
        self.desc = desc
        vals = [ctypes.c_int64() for _ in range(6)]
        hmin = ctypes.c_double()
        nnz = ctypes.c_int64()
        _check(lib.fracture_mesh_info(h, *[ctypes.byref(v) for v in vals], ctypes.byref(hmin), ctypes.byref(nnz)))
        (self.n_nodes, self.n_cells, self.n_free, self.n_all, self.n_solve, self.n_hanging) = [v.value for v in vals]
        self.h_min = hmin.value
        self.nnz_graph = nnz.value
        self.dim = desc.dim

    def nodes(self):
        xyz = np.zeros((self.n_nodes, self.dim))
        lat = np.zeros((self.n_nodes, self.dim), dtype=np.int64)
        dirichlet = np.zeros(self.n_nodes, dtype=np.uint8)
        free = np.zeros(self.n_nodes, dtype=np.int32)
        _check(load().fracture_mesh_nodes(self.h, xyz.ctypes.data_as(_P), lat.ctypes.data_as(_P),
                                          dirichlet.ctypes.data_as(_P), free.ctypes.data_as(_P)))
        return xyz, lat, dirichlet, free

    def instance(self, i):
        v = [ctypes.c_int64() for _ in range(6)]
        hm = ctypes.c_double()
        _check(load().fracture_mesh_instance(self.h, i, *[ctypes.byref(x) for x in v], ctypes.byref(hm)))
        keys = ("node_offset", "n_nodes", "free_offset", "n_free", "cell_offset", "n_cells")
        out = {k: x.value for k, x in zip(keys, v)}
        out["h_min"] = hm.value
        return out

    def cells(self):
        nv = 1 << self.dim
        cells = np.zeros((self.n_cells, nv), dtype=np.int32)
        lo = np.zeros((self.n_cells, self.dim))
        h = np.zeros(self.n_cells)
        _check(load().fracture_mesh_cells(self.h, cells.ctypes.data_as(_P), lo.ctypes.data_as(_P),
                                          h.ctypes.data_as(_P)))
        return cells, lo, h

    def faces(self):
        """(ptr [2 dim n_cells + 1], nbr): the cells across every face of every cell."""
        lib = load()
        n = ctypes.c_int64()
        _check(lib.fracture_mesh_faces(self.h, ctypes.byref(n), None, None))
        ptr = np.zeros(2 * self.dim * self.n_cells + 1, dtype=np.int32)
        nbr = np.zeros(max(1, n.value), dtype=np.int32)
        _check(lib.fracture_mesh_faces(self.h, ctypes.byref(n), ptr.ctypes.data_as(_P), nbr.ctypes.data_as(_P)))
        return ptr, nbr[:n.value]

    def constraints(self):
        lib = load()
        n = ctypes.c_int64()
        _check(lib.fracture_mesh_constraints(self.h, ctypes.byref(n), None, None, None))
        ptr = np.zeros(self.n_nodes + 1, dtype=np.int32)
        mas = np.zeros(n.value, dtype=np.int32)
        w = np.zeros(n.value)
        _check(lib.fracture_mesh_constraints(self.h, ctypes.byref(n), ptr.ctypes.data_as(_P), mas.ctypes.data_as(_P),
                                             w.ctypes.data_as(_P)))
        return ptr, mas, w

    def refine(self, flags):
        """The mesh with the flagged cells split (2:1 balanced); keeps this mesh alive for
        transfers from it."""
        f = np.ascontiguousarray(np.asarray(flags, dtype=np.uint8))
        if f.shape != (self.n_cells,):
            raise ValueError(f"need {self.n_cells} flags, got {f.shape}")
        h = _P()
        _check(load().fracture_mesh_refine(self.h, f.ctypes.data_as(_P), ctypes.byref(h),
                                           None if self.host_only else _stream()))
        out = Mesh(self.desc, host_only=self.host_only, _handle=h)
        out.parent = self
        return out

    def __del__(self):
        if getattr(self, "h", None) is not None and _lib is not None:
            _lib.fracture_mesh_destroy(self.h)
            self.h = None


def transfer(src_mesh, dst_mesh, src, dst):
    """Interpolates nodal fields (torch [n_nodes] or [n_nodes, ncomp]) of src_mesh onto the
    nodes of dst_mesh, a refinement of it."""
    ncomp = 1 if src.dim() == 1 else src.shape[1]
    _check(load().fracture_transfer(src_mesh.h, dst_mesh.h, _ptr(src), ncomp, _ptr(dst), _stream()))


def kelly(mesh, u, eta2):
    """Gradient-jump indicator of u per cell into eta2 (torch [n_cells])."""
    _check(load().fracture_kelly(mesh.h, _ptr(u), _ptr(eta2), _stream()))


def mark_crack(mesh, phi, phi_max, h_target):
    """Crack-region marks: (flags uint8 [n_cells], count)."""
    flags = np.zeros(mesh.n_cells, dtype=np.uint8)
    n = ctypes.c_int64()
    _check(load().fracture_mark_crack(mesh.h, _ptr(phi), float(phi_max), float(h_target), flags.ctypes.data_as(_P),
                                      ctypes.byref(n), _stream()))
    return flags, n.value


class System:
    def __init__(self, mesh):
        self.mesh = mesh
        self.h = _P()

    def assemble(self, prm, u, phi, phi_old, phi_tilde, flags=FR_RESIDUAL | FR_ACTIVE_SET | FR_JACOBIAN):
        """prm: one Params, or a list of one per instance of a batched mesh."""
        plist = list(prm) if isinstance(prm, (list, tuple)) else [prm]
        if len(plist) != self.mesh.n_inst:
            raise ValueError(f"need {self.mesh.n_inst} parameter sets, got {len(plist)}")
        arr = (Params * len(plist))(*plist)
        _check(load().fracture_assemble(self.mesh.h, arr, _ptr(u), _ptr(phi), _ptr(phi_old),
                                        _ptr(phi_tilde), flags, ctypes.byref(self.h), _stream()))
        return self

    def norms(self):
        nr = (ctypes.c_double * 2)()
        na, ch = ctypes.c_int64(), ctypes.c_int64()
        mm = ctypes.c_double()
        _check(load().fracture_residual_norms(self.h, nr, ctypes.byref(na), ctypes.byref(ch), ctypes.byref(mm),
                                              _stream()))
        return dict(res=nr[0], rhs=nr[1], n_active=na.value, changes=ch.value, min_margin=mm.value)

    def vectors(self):
        m = self.mesh
        dev = torch.device("cuda")
        R = torch.empty(m.n_solve, dtype=torch.float64, device=dev)
        F = torch.empty_like(R)
        B = torch.empty(m.n_free, dtype=torch.float64, device=dev)
        act = torch.empty(m.n_free, dtype=torch.uint8, device=dev)
        _check(load().fracture_system_vectors(self.h, _ptr(R), _ptr(F), _ptr(B), _ptr(act, torch.uint8), _stream()))
        return R, F, B, act

    def set_active(self, active):
        _check(load().fracture_set_active(self.h, _ptr(active, torch.uint8), _stream()))

    def matvec(self, x, y):
        _check(load().fracture_matvec(self.h, _ptr(x), _ptr(y), _stream()))

    def matvec_free(self, x, y, rows=3):
        _check(load().fracture_matvec_free(self.h, rows, _ptr(x), _ptr(y), _stream()))

    def csr(self):
        lib = load()
        nnz = ctypes.c_int64()
        _check(lib.fracture_system_csr(self.h, ctypes.byref(nnz), None, None, None, _stream()))
        n = self.mesh.n_solve
        rp = np.zeros(n + 1, dtype=np.int64)
        ci = np.zeros(nnz.value, dtype=np.int32)
        vv = np.zeros(nnz.value)
        _check(lib.fracture_system_csr(self.h, ctypes.byref(nnz), rp.ctypes.data_as(_P), ci.ctypes.data_as(_P),
                                       vv.ctypes.data_as(_P), _stream()))
        return rp, ci[:nnz.value], vv[:nnz.value]

    def __del__(self):
        if getattr(self, "h", None) is not None and self.h.value and _lib is not None:
            _lib.fracture_system_destroy(self.h)
            self.h = None


class Amg:
    def __init__(self, system, opts=None):
        self.system = system
        self.h = _P()
        self.setup(opts)

    def setup(self, opts=None):
        o = opts if opts is not None else amg_opts()
        _check(load().amg_setup(self.system.h, ctypes.byref(o), ctypes.byref(self.h), _stream()))
        return self

    def level_info(self, block, level):
        nl, bs = ctypes.c_int(), ctypes.c_int()
        rows, nz = ctypes.c_int64(), ctypes.c_int64()
        lm = ctypes.c_double()
        _check(load().amg_level_info(self.h, block, level, ctypes.byref(nl), ctypes.byref(rows), ctypes.byref(bs),
                                     ctypes.byref(nz), ctypes.byref(lm)))
        return dict(n_levels=nl.value, rows=rows.value, bsize=bs.value, nnz_blocks=nz.value, lambda_max=lm.value)

    def level_shape(self, block, level, which):
        """(SELL slice height, lanes per row) of operator which (0 A, 1 P, 2 R) on a level."""
        c, g = ctypes.c_int(), ctypes.c_int()
        _check(load().amg_level_shape(self.h, block, level, which, ctypes.byref(c), ctypes.byref(g)))
        return c.value, g.value

    def n_levels(self, block):
        nl = ctypes.c_int()
        load().amg_level_info(self.h, block, 0, ctypes.byref(nl), None, None, None, None)
        return nl.value

    def level_csr(self, block, level, which):
        lib = load()
        nr, nc, nnz = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib.amg_level_csr(self.h, block, level, which, ctypes.byref(nr), ctypes.byref(nc), ctypes.byref(nnz),
                                 None, None, None, _stream()))
        rp = np.zeros(nr.value + 1, dtype=np.int64)
        ci = np.zeros(max(1, nnz.value), dtype=np.int32)
        vv = np.zeros(max(1, nnz.value))
        _check(lib.amg_level_csr(self.h, block, level, which, ctypes.byref(nr), ctypes.byref(nc), ctypes.byref(nnz),
                                 rp.ctypes.data_as(_P), ci.ctypes.data_as(_P), vv.ctypes.data_as(_P), _stream()))
        return (nr.value, nc.value), rp, ci[:nnz.value], vv[:nnz.value]

    def apply(self, r, z):
        _check(load().amg_apply(self.h, _ptr(r), _ptr(z), _stream()))

    def __del__(self):
        if getattr(self, "h", None) is not None and self.h.value and _lib is not None:
            _lib.amg_destroy(self.h)
            self.h = None


def solve(system, amg, du, opts=None, raise_on_noconv=True, raise_on_status=True):
    """FGMRES; returns the stats dict (a list of them for a batched mesh).  raise_on_status=False
    returns the stats (with their status) for every solver status instead of raising."""
    ni = system.mesh.n_inst
    st = (SolveStats * ni)()
    o = opts if opts is not None else solve_opts()
    status = load().fracture_solve(system.h, amg.h, ctypes.byref(o), _ptr(du), st, _stream())
    quiet = (not raise_on_status and status in SOLVER_STATUSES) or (not raise_on_noconv and status == FR_ENOCONV)
    if status != FR_OK and not quiet:
        raise FractureError(status, last_error())
    out = [dict(iters=s.iters, relres=s.relres, status=s.status) for s in st]
    return out[0] if ni == 1 else out


def update(mesh, du, omega, u, phi):
    _check(load().fracture_update(mesh.h, _ptr(du), float(omega), _ptr(u), _ptr(phi), _stream()))


def newton(mesh, prm, u, phi, phi_old, phi_tilde, amg=None, solve=None, newton=None, raise_on_noconv=True,
           raise_on_status=True):
    """Newton / active-set loop; prm: one Params, or a list of one per instance of a batched
    mesh.  Returns the stats dict (a list of them for a batched mesh).  raise_on_status=False
    returns the stats for every solver status (FR_ENOCONV, FR_ECYCLE, FR_EBREAKDOWN, FR_ENAN)."""
    ni = mesh.n_inst
    plist = list(prm) if isinstance(prm, (list, tuple)) else [prm]
    if len(plist) != ni:
        raise ValueError(f"need {ni} parameter sets, got {len(plist)}")
    arr = (Params * ni)(*plist)
    st = (NewtonStats * ni)()
    status = load().fracture_newton(mesh.h, arr, _ptr(u), _ptr(phi), _ptr(phi_old), _ptr(phi_tilde),
                                    ctypes.byref(amg if amg is not None else amg_opts()),
                                    ctypes.byref(solve if solve is not None else solve_opts()),
                                    ctypes.byref(newton if newton is not None else newton_opts()),
                                    st, _stream())
    quiet = (not raise_on_status and status in SOLVER_STATUSES) or (not raise_on_noconv and status == FR_ENOCONV)
    if status != FR_OK and not quiet:
        raise FractureError(status, last_error())
    out = [{f: getattr(x, f) for f, _ in NewtonStats._fields_} for x in st]
    return out[0] if ni == 1 else out


def newton_masks(mesh):
    """(active, frozen): uint8 device tensors [n_free] of the last Newton loop on the mesh."""
    act = torch.empty(mesh.n_free, dtype=torch.uint8, device="cuda")
    frz = torch.empty(mesh.n_free, dtype=torch.uint8, device="cuda")
    _check(load().fracture_newton_masks(mesh.h, _ptr(act, torch.uint8), _ptr(frz, torch.uint8), _stream()))
    return act, frz


def extrapolate(mesh, phi1, phi2, w, out):
    """out = clip(phi1 + w (phi1 - phi2), 0, 1) (device arrays of n_nodes)."""
    _check(load().fracture_extrapolate(mesh.h, _ptr(phi1), _ptr(phi2), float(w), _ptr(out), _stream()))


def loading(mesh, prm_steps, times, u, phi, phi_prev=None, t_prev=0.0, amg=None, solve=None, newton=None,
            raise_on_noconv=True):
    """Loading steps; prm_steps[n] is step n+1's Params (a list of one per instance on a batched
    mesh), times[0] the time of (u, phi).  Returns (stats, tcv): stats[n] is a dict (a list of
    them on a batched mesh), tcv an array [n_steps] ([n_steps, n_inst] batched)."""
    ni = mesh.n_inst
    ns = len(prm_steps)
    flat = []
    for p in prm_steps:
        row = list(p) if isinstance(p, (list, tuple)) else [p]
        if len(row) != ni:
            raise ValueError(f"need {ni} parameter sets per step, got {len(row)}")
        flat += row
    t = np.ascontiguousarray(np.asarray(times, dtype=np.float64))
    if t.shape != (ns + 1,):
        raise ValueError(f"need {ns + 1} times, got {t.shape}")
    arr = (Params * len(flat))(*flat)
    st = (NewtonStats * len(flat))()
    tcv = np.full(ns * ni, np.nan)
    status = load().fracture_loading(mesh.h, arr, ns, t.ctypes.data_as(_DP), _ptr(u), _ptr(phi),
                                     _ptr(phi_prev) if phi_prev is not None else None, float(t_prev),
                                     ctypes.byref(amg if amg is not None else amg_opts()),
                                     ctypes.byref(solve if solve is not None else solve_opts()),
                                     ctypes.byref(newton if newton is not None else newton_opts()),
                                     st, tcv.ctypes.data_as(_DP), _stream())
    if status != FR_OK and (raise_on_noconv or status != FR_ENOCONV):
        raise FractureError(status, last_error())
    out = [{f: getattr(x, f) for f, _ in NewtonStats._fields_} for x in st]
    if ni == 1:
        return out, tcv
    return [out[k * ni:(k + 1) * ni] for k in range(ns)], tcv.reshape(ns, ni)


def functionals(mesh, u, phi, cod_x=(), noalloc=False):
    """(cod, tcv). One mesh: cod_x [n_cod][dim-1] -> cod [n_cod], tcv float. Batched mesh:
    cod_x [n_inst][n_cod][dim-1] -> cod [n_inst][n_cod], tcv [n_inst].  noalloc: the entry
    point that allocates nothing (fixed per-device scratch)."""
    ni = mesh.n_inst
    cod_x = np.ascontiguousarray(np.asarray(cod_x, dtype=np.float64).reshape(ni, -1, mesh.dim - 1))
    n = cod_x.shape[1]
    cod = np.zeros(max(1, ni * n))
    tcv = np.zeros(ni)
    fn = load().fracture_functionals_noalloc if noalloc else load().fracture_functionals
    _check(fn(mesh.h, _ptr(u), _ptr(phi), cod_x.ctypes.data_as(_P) if n else None, n,
              cod.ctypes.data_as(_P) if n else None, tcv.ctypes.data_as(_P), _stream()))
    if ni == 1:
        return cod[:n], float(tcv[0])
    return cod[:ni * n].reshape(ni, n), tcv


def _torch_alloc(nbytes, device, stream, ctx):
    try:
        return torch.cuda.caching_allocator_alloc(int(nbytes), int(device), int(stream or 0))
    except Exception:   # out of memory: the library reports FR_ENOMEM
        return None


def _torch_free(ptr, nbytes, device, stream, ctx):
    torch.cuda.caching_allocator_delete(ptr)


# kept alive for the life of the process: blocks made through them may outlive any setting
_TORCH_HOOKS = (_ALLOC_FN(_torch_alloc), _FREE_FN(_torch_free))


def set_allocator(kind):
    """kind="torch": the library's device memory comes from PyTorch's caching allocator (on the
    stream of each allocation); kind=None: the library's own pool again."""
    if kind == "torch":
        _check(load().fracture_set_allocator(_TORCH_HOOKS[0], _TORCH_HOOKS[1], None))
    elif kind is None:
        _check(load().fracture_set_allocator(_ALLOC_FN(), _FREE_FN(), None))
    else:
        raise ValueError("kind must be 'torch' or None")


def trim_pool():
    _check(load().fracture_trim_pool())


def device_check():
    return load().fracture_device_check()


def tune_clear():
    """Forgets the launch shapes cached by the tuner in this process."""
    _check(load().fracture_tune_clear())


def tune_table():
    """The tuner's cached launch shapes as text (one line per entry: op, block rows, block
    columns, floor(log2 rows), mean blocks per row, FP32 flag, slice height, lanes per row)."""
    lib = load()
    n = ctypes.c_size_t(0)
    _check(lib.fracture_tune_export(None, 0, ctypes.byref(n)))
    buf = ctypes.create_string_buffer(n.value + 1)
    _check(lib.fracture_tune_export(buf, n.value + 1, ctypes.byref(n)))
    return buf.value.decode()


def tune_load(text):
    """Adds a table written by tune_table to this process's cache (same-key entries replaced)."""
    _check(load().fracture_tune_import(text.encode()))


def profile(enable):
    """Starts (True) or stops (False) per-kernel HIP-event timing inside the library."""
    _check(load().fracture_profile(1 if enable else 0))


def profile_read():
    """{kernel: dict(launches, ms, bytes)} of the current recording."""
    lib = load()
    out = {}
    i = 0
    while True:
        name = ctypes.c_char_p()
        n = ctypes.c_int64()
        ms, by = ctypes.c_double(), ctypes.c_double()
        if lib.fracture_profile_read(i, ctypes.byref(name), ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by)) != FR_OK:
            break
        out[name.value.decode()] = dict(launches=n.value, ms=ms.value, bytes=by.value)
        i += 1
    return out
