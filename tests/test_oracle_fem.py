"""Pins of the oracle's residual and Jacobian (Formulation 1, Section 2; blocks in Section 3).

Closed forms used here hold exactly for the Q1 / 2-point Gauss discretisation:
  * homogeneous strain e and constant phi: every integrand is constant on B and the
    nodal basis sums to one, so sums of residual entries are |B| times the integrand;
  * a linear displacement is reproduced, so its interior residual vanishes (patch test);
  * linear phi: (1 - phi) phi is quadratic, integrated exactly by the 2-point rule.
The finite-difference test then pins the Jacobian against the residual.
"""
import numpy as np
import pytest

from oracle import fem, mesh as omesh
from oracle.material import Params
from inputs import random_state


def _interior(m):
    return ~m.dirichlet


def _linear_u(m, G):
    return m.coords @ G.T


@pytest.mark.parametrize("dim", [2, 3])
def test_zero_residual_at_rest(dim):
    m = omesh.uniform(dim, -1.0, 1.0, 6 if dim == 2 else 3)
    prm = Params(eps=0.3, kappa=1e-3)
    u = np.zeros((m.n_nodes, dim))
    one = np.ones(m.n_nodes)
    Ru, Rp, _ = fem.residual_all(m, prm, u, one, one)
    # only rounding of the interpolated 1 - phi remains (scale Gc/eps * cell volume)
    assert np.abs(Rp).max() < 1e-14 * prm.Gc / prm.eps * m.cell_h[0] ** dim
    # p (div w) integrates to zero against interior basis functions
    assert np.abs(Ru[_interior(m)]).max() < 1e-18


@pytest.mark.parametrize("dim", [2, 3])
def test_patch_test_linear_displacement(dim):
    m = omesh.uniform(dim, -1.0, 2.0, 5 if dim == 2 else 3)
    prm = Params(eps=0.3, kappa=1e-2, p=0.0)
    rng = np.random.default_rng(3)
    G = rng.standard_normal((dim, dim))
    u = _linear_u(m, G)
    one = np.ones(m.n_nodes)
    Ru, _, _ = fem.residual_all(m, prm, u, one, one)
    assert np.abs(Ru[_interior(m)]).max() < 1e-13 * np.abs(Ru).max()


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("mode", ["shear", "dilation", "general"])
def test_elastic_energy_identity(dim, mode):
    """sum_a u_a . R_u[a] = int g sigma(e):e for u = G x, p = 0, phi_tilde = c."""
    lo, hi = -1.0, 1.5
    m = omesh.uniform(dim, lo, hi, 4 if dim == 2 else 3)
    prm = Params(E=2.0, nu=0.3, eps=0.3, kappa=0.05, p=0.0)
    G = np.zeros((dim, dim))
    if mode == "shear":
        G[0, 1] = 0.7
    elif mode == "dilation":
        G = 0.4 * np.eye(dim)
    else:
        G = np.random.default_rng(5).standard_normal((dim, dim))
    e = 0.5 * (G + G.T)
    mu, lam = prm.mu, prm.lam
    sig = 2 * mu * e + lam * np.trace(e) * np.eye(dim)
    c = 0.6
    g = (1 - prm.kappa) * c * c + prm.kappa
    u = _linear_u(m, G)
    Ru, _, _ = fem.residual_all(m, prm, u, np.ones(m.n_nodes), np.full(m.n_nodes, c))
    vol = (hi - lo) ** dim
    assert np.isclose((u * Ru).sum(), g * vol * np.sum(sig * e), rtol=1e-13)


@pytest.mark.parametrize("dim", [2, 3])
def test_pressure_term(dim):
    """u = 0, phi_tilde = c: sum_a x_a . R_u[a] = c^2 p int div x = c^2 p d |B|; phi plays no role."""
    lo, hi = -2.0, 1.0
    m = omesh.uniform(dim, lo, hi, 4 if dim == 2 else 2)
    prm = Params(eps=0.3, p=3e-3, kappa=1e-6)
    c = 0.7
    u = np.zeros((m.n_nodes, dim))
    rng = np.random.default_rng(0)
    Ru, _, _ = fem.residual_all(m, prm, u, rng.uniform(0, 1, m.n_nodes), np.full(m.n_nodes, c))
    vol = (hi - lo) ** dim
    assert np.isclose((m.coords * Ru).sum(), c * c * prm.p * dim * vol, rtol=1e-13)


@pytest.mark.parametrize("dim", [2, 3])
def test_phase_field_reaction_terms(dim):
    """u = G x, phi = c: sum_a R_phi[a] = |B| ((1-k) c s + 2 p c theta - Gc/eps (1-c))."""
    lo, hi = -1.0, 1.0
    m = omesh.uniform(dim, lo, hi, 4 if dim == 2 else 2)
    prm = Params(E=1.7, nu=0.25, Gc=1.3, eps=0.2, kappa=0.1, p=0.05)
    G = np.random.default_rng(7).standard_normal((dim, dim)) * 0.5
    e = 0.5 * (G + G.T)
    sig = 2 * prm.mu * e + prm.lam * np.trace(e) * np.eye(dim)
    s, th = np.sum(sig * e), np.trace(e)
    vol = (hi - lo) ** dim
    for c in (0.0, 0.35, 1.0):
        _, Rp, mass = fem.residual_all(m, prm, _linear_u(m, G), np.full(m.n_nodes, c),
                                       np.random.default_rng(1).uniform(0, 1, m.n_nodes))
        exact = vol * ((1 - prm.kappa) * c * s + 2 * prm.p * c * th - prm.Gc / prm.eps * (1 - c))
        assert np.isclose(Rp.sum(), exact, rtol=1e-13, atol=1e-15)
        assert np.isclose(mass.sum(), vol, rtol=1e-14)


@pytest.mark.parametrize("dim", [2, 3])
def test_phase_field_gradient_term(dim):
    """u = 0, phi = x_0: sum_a x_a R_phi[a] = -Gc/eps int (x - x^2) + Gc eps |B|."""
    lo, hi = -0.5, 1.5
    m = omesh.uniform(dim, lo, hi, 6 if dim == 2 else 3)
    prm = Params(Gc=2.0, eps=0.4)
    x = m.coords[:, 0]
    _, Rp, _ = fem.residual_all(m, prm, np.zeros((m.n_nodes, dim)), x.copy(), np.ones(m.n_nodes))
    side = (hi - lo) ** (dim - 1)
    int_x = (hi ** 2 - lo ** 2) / 2 * side
    int_x2 = (hi ** 3 - lo ** 3) / 3 * side
    exact = -prm.Gc / prm.eps * (int_x - int_x2) + prm.Gc * prm.eps * (hi - lo) ** dim
    assert np.isclose((x * Rp).sum(), exact, rtol=1e-13)


@pytest.mark.parametrize("dim", [2, 3])
def test_rigid_body_modes_in_kernel(dim):
    m = omesh.uniform(dim, -1.0, 1.0, 3 if dim == 2 else 2)
    prm = Params(eps=0.3, kappa=0.2)
    u0 = np.zeros((m.n_nodes, dim))
    rng = np.random.default_rng(2)
    J = fem.jacobian_all(m, prm, u0, rng.uniform(0, 1, m.n_nodes), rng.uniform(0, 1, m.n_nodes))
    nu = dim * m.n_nodes
    Kuu = J[:nu, :nu]
    x = m.coords
    modes = []
    for c in range(dim):
        t = np.zeros((m.n_nodes, dim))
        t[:, c] = 1.0
        modes.append(t)
    pairs = [(0, 1)] if dim == 2 else [(0, 1), (1, 2), (0, 2)]
    for i, j in pairs:
        r = np.zeros((m.n_nodes, dim))
        r[:, i] = -x[:, j]
        r[:, j] = x[:, i]
        modes.append(r)
    scale = abs(Kuu).max()
    for md in modes:
        assert np.abs(Kuu @ md.ravel()).max() < 1e-13 * scale
    # a non-rigid mode is not in the kernel
    st = np.zeros((m.n_nodes, dim))
    st[:, 0] = x[:, 0]
    assert np.abs(Kuu @ st.ravel()).max() > 1e-3 * scale


def _fd_jacobian(m, prm, u, phi, pt):
    d = m.dim
    n = m.n_nodes
    U = np.concatenate([u.ravel(), phi])
    def R(Uv):
        Ru, Rp, _ = fem.residual_all(m, prm, Uv[:d * n].reshape(n, d), Uv[d * n:], pt)
        return np.concatenate([Ru.ravel(), Rp])
    cols = []
    for j in range(U.size):
        t = 1e-6 * max(1.0, abs(U[j]))
        Up, Um = U.copy(), U.copy()
        Up[j] += t
        Um[j] -= t
        cols.append((R(Up) - R(Um)) / (2 * t))
    return np.stack(cols, axis=1)


@pytest.mark.parametrize("dim,n", [(2, 2), (2, 3), (3, 1), (3, 2)])
def test_jacobian_matches_finite_differences(dim, n):
    m = omesh.uniform(dim, -1.0, 1.0, n)
    prm = Params(E=1.0, nu=0.2, Gc=1.0, eps=0.5, kappa=1e-3, p=0.3)
    u, phi, _, pt = random_state(m.n_nodes, dim, seed=11 + n, u_scale=0.3)
    Jfd = _fd_jacobian(m, prm, u, phi, pt)
    J = fem.jacobian_all(m, prm, u, phi, pt).toarray()
    nu = dim * m.n_nodes
    blocks = {"uu": (slice(0, nu), slice(0, nu)), "pu": (slice(nu, None), slice(0, nu)),
              "pp": (slice(nu, None), slice(nu, None))}
    for name, (r, c) in blocks.items():
        err = np.abs(J[r, c] - Jfd[r, c]).max() / np.abs(Jfd[r, c]).max()
        assert err < 1e-7, (name, err)
    # the u-phi block is zero (phi_tilde, not phi, in E22ATW)
    assert np.abs(Jfd[:nu, nu:]).max() < 1e-9 * np.abs(Jfd).max()
    assert np.abs(J[:nu, nu:]).max() == 0.0
