"""Sneddon pressurized-crack workloads (Section 4 of the paper) as synthetic inputs.

The benchmark has no dataset: a crack of half-length l0 in [-L, L]^d under constant
pressure p, homogeneous Dirichlet displacement on the boundary.  The initial crack is
described by the phase field (Section 4); the set-up details live in the authors' earlier
papers, so the recipe here is a reading:

    phi_0(node) = 0  iff  |x_0 - c_0| <= l0 (2d) or |(x_0,x_1) - (c_0,c_1)| <= l0 (3d)
                     and  |x_last - c_last| <= eps / 2,
    phi_0(node) = 1  otherwise,

which with eps = 2h marks three node layers across the crack.  For one loading step
u^0 = 0 and phi^0 = phi_old = phi_tilde = phi_0.
"""
from dataclasses import dataclass, field
import numpy as np


@dataclass
class Workload:
    name: str
    dim: int
    L: float                     # domain [-L, L]^d
    n: int                       # cells per axis of the (base) mesh
    l0: float = 0.25
    p: float = 1e-3
    E: float = 1.0
    nu: float = 0.2
    Gc: float = 1.0
    kappa: float = 1e-10
    eps_factor: float = 2.0      # eps = eps_factor * h_min
    center: tuple = (0.0, 0.0, 0.0)
    levels: int = 0              # adaptive refinement levels (0 = uniform)
    refine_radius: float = 0.0
    newton: str = "one_step"     # "one_step" or "loop"
    description: str = ""

    @property
    def h(self):
        return 2.0 * self.L / (self.n * (1 << self.levels))

    @property
    def eps(self):
        return self.eps_factor * self.h

    def params(self):
        return dict(E=self.E, nu=self.nu, Gc=self.Gc, kappa=self.kappa, eps=self.eps, p=self.p)


WORKLOADS = {
    "sneddon2d_128": Workload(
        "sneddon2d_128", 2, 2.0, 128, newton="one_step",
        description="2d Sneddon, [-2,2]^2, 128x128 Q1, h=1/32, eps=2h, l0=0.25, one Newton step"),
    "sneddon2d_2048": Workload(
        "sneddon2d_2048", 2, 10.0, 2048, newton="loop",
        description="2d Sneddon, [-10,10]^2, 2048x2048 Q1 (12,595,203 DoFs), eps=2h, l0=0.25, "
                    "full Newton / active-set loop"),
    "sneddon3d_64": Workload(
        "sneddon3d_64", 3, 2.0, 64, l0=0.5, newton="one_step",
        description="3d penny crack r=0.5 in [-2,2]^3, uniform 64^3 hexes, eps=2h"),
}


def crack_band_phi(coords, l0, eps, center=(0.0, 0.0, 0.0)):
    """Nodal phi_0 of the initial crack (see module docstring)."""
    coords = np.asarray(coords, dtype=np.float64)
    d = coords.shape[1]
    c = np.asarray(center[:d], dtype=np.float64)
    rel = coords - c[None, :]
    slack = 1e-9 * eps
    if d == 2:
        along = np.abs(rel[:, 0])
    else:
        along = np.sqrt(rel[:, 0] ** 2 + rel[:, 1] ** 2)
    across = np.abs(rel[:, d - 1])
    inside = (along <= l0 + slack) & (across <= 0.5 * eps + slack)
    return np.where(inside, 0.0, 1.0)


def random_state(n_nodes, dim, seed, u_scale=1e-3):
    """A generic state (u, phi, phi_old, phi_tilde) for derivative and parity checks."""
    rng = np.random.default_rng(seed)
    u = u_scale * rng.standard_normal((n_nodes, dim))
    phi = rng.uniform(0.0, 1.0, n_nodes)
    phi_old = np.minimum(1.0, phi + rng.uniform(0.0, 0.2, n_nodes))
    phi_tilde = rng.uniform(0.0, 1.0, n_nodes)
    return u, phi, phi_old, phi_tilde


def batched_instances(n_inst=48, seed=9924):
    """Independent 2d Sneddon instances of uneven size (domain-size / eps studies).

    Drawn in this order, one array each: L ~ U[1, 20]; eps factor in {2, 4};
    p ~ U[5e-4, 2e-3]; crack centre offsets x_c, y_c ~ U[-0.1, 0.1];
    N ~ U_int[max(81, ceil(32 L)), 706] cells per axis (h <= l0/4 keeps nodes in the band).
    """
    rng = np.random.default_rng(seed)
    L = rng.uniform(1.0, 20.0, n_inst)
    fac = rng.choice([2.0, 4.0], n_inst)
    p = rng.uniform(5e-4, 2e-3, n_inst)
    xc = rng.uniform(-0.1, 0.1, n_inst)
    yc = rng.uniform(-0.1, 0.1, n_inst)
    lo_n = np.maximum(81, np.ceil(32.0 * L)).astype(np.int64)
    N = np.array([rng.integers(lo, 707) for lo in lo_n])
    out = []
    for i in range(n_inst):
        out.append(Workload(f"batch{i}", 2, float(L[i]), int(N[i]), p=float(p[i]),
                            eps_factor=float(fac[i]), center=(float(xc[i]), float(yc[i]), 0.0),
                            newton="one_step"))
    return out


# Section 4.2: influence of the finite domain size in 2d (crack half-length l0 = 1 in
# [-L, L]^2 for domain sizes 10, 20, 40, 80).  The paper refines adaptively towards the crack;
# the reading here: base cells of edge 1 (2L per axis), `levels` refinements of every cell
# within `refine_radius` of the crack segment (2:1 balanced), eps = 2 h_min, p = 1e-3, and the
# value extrapolated in h from the finest levels.  Exact (infinite-domain) TCV:
# 2 pi p l0^2 (1 - nu^2) / E = 6.0319E-03.
DOMAIN_STUDY_HALF_WIDTHS = (5.0, 10.0, 20.0, 40.0)
DOMAIN_STUDY_LEVELS = (5, 6, 7)
DOMAIN_STUDY_RADIUS = 4.0


def domain_study(half_widths=DOMAIN_STUDY_HALF_WIDTHS, levels=DOMAIN_STUDY_LEVELS, refine_radius=DOMAIN_STUDY_RADIUS):
    """Workloads of the domain-size study, domain-major, finest level last."""
    out = []
    for L in half_widths:
        for k in levels:
            out.append(Workload(f"domain{int(2 * L)}_lev{k}", 2, float(L), int(round(2 * L)), l0=1.0,
                                levels=int(k), refine_radius=float(refine_radius), newton="loop",
                                description=f"2d Sneddon l0=1 in [-{L:g},{L:g}]^2, base h=1, {k} levels "
                                            f"within {refine_radius:g} of the crack, eps=2h_min"))
    return out


# COD convergence study (Section 4.4): one domain, l0 = 1, base cells of edge 1, adaptive levels
# within COD_STUDY_RADIUS of the crack against global meshes of the same h_min.
COD_STUDY = dict(half_width=5.0, levels=(3, 4, 5, 6, 7), refine_radius=2.0)


def cod_study():
    return dict(COD_STUDY)
