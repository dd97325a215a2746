"""Pins of the oracle's adaptive meshes with hanging nodes (Section 3 adaptive Q1^c meshes)."""
import numpy as np
import pytest

from oracle import adaptive, fem
from oracle.material import Params
from inputs import random_state


def _mesh(dim):
    if dim == 2:
        return adaptive.adaptive(2, -1.0, 1.0, 4, 3, 0.15, (0.0, 0.0, 0.0), 0.3)
    return adaptive.adaptive(3, -1.0, 1.0, 2, 2, 0.1, (0.0, 0.0, 0.0), 0.3)


@pytest.mark.parametrize("dim", [2, 3])
def test_tiling_balance_and_constraints(dim):
    m = _mesh(dim)
    assert m.n_free < m.n_nodes
    assert np.isclose((m.cell_h ** dim).sum(), 2.0 ** dim)
    c = m.cell_lo + 0.5 * m.cell_h[:, None]
    for i in range(m.n_cells):
        near = np.all(np.abs(c - c[i]) <= 0.5 * (m.cell_h + m.cell_h[i])[:, None] + 1e-12, axis=1)
        assert m.cell_h[near].max() <= 2 * m.cell_h[i] + 1e-12
    a = np.random.default_rng(0).standard_normal(dim)
    f = m.coords @ a + 0.7
    assert np.allclose(m.C @ f[m.free], f, atol=1e-13)
    assert np.allclose(np.asarray(m.C.sum(axis=1)).ravel(), 1.0)


@pytest.mark.parametrize("dim", [2, 3])
def test_patch_and_mass_on_adaptive_mesh(dim):
    m = _mesh(dim)
    prm = Params(eps=0.3, kappa=1e-2, p=0.0)
    G = np.random.default_rng(3).standard_normal((dim, dim))
    uf = m.coords[m.free] @ G.T
    u = m.C @ uf
    one = np.ones(m.n_nodes)
    R, B = fem.residual(m, prm, u, one, one)
    nf = m.n_free
    Ru = R[:dim * nf].reshape(nf, dim)
    interior = ~m.dirichlet[m.free]
    assert np.abs(Ru[interior]).max() < 1e-12 * np.abs(Ru).max()
    assert np.isclose(B.sum(), 2.0 ** dim, rtol=1e-13)


def test_condensed_jacobian_matches_finite_differences():
    m = adaptive.adaptive(2, -1.0, 1.0, 2, 2, 0.05, (0.0, 0.0, 0.0), 0.2)
    assert m.n_free < m.n_nodes
    prm = Params(eps=0.5, kappa=1e-3, p=0.3)
    u, phi, _, pt = random_state(m.n_nodes, 2, seed=5, u_scale=0.3)
    U = fem.restrict(m, u, phi)
    u, phi = fem.expand(m, U)
    pt = m.C @ pt[m.free]
    J = fem.jacobian(m, prm, u, phi, pt).toarray()
    Jfd = np.zeros_like(J)
    for j in range(U.size):
        t = 1e-6 * max(1.0, abs(U[j]))
        Up, Um = U.copy(), U.copy()
        Up[j] += t
        Um[j] -= t
        Rp, _ = fem.residual(m, prm, *fem.expand(m, Up), pt)
        Rm, _ = fem.residual(m, prm, *fem.expand(m, Um), pt)
        Jfd[:, j] = (Rp - Rm) / (2 * t)
    assert np.abs(J - Jfd).max() < 1e-7 * np.abs(Jfd).max()
