"""Pins of the oracle's reference element, material law, meshes and functionals.

Each check compares the oracle with something the paper or textbook mathematics fixes,
never with the oracle's own formulas retyped.
"""
import os
import numpy as np
import pytest

from oracle import q1, material, mesh as omesh, functionals as ofun

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append(line.split())
    return rows


@pytest.mark.parametrize("dim", [2, 3])
def test_partition_of_unity_and_linear_reproduction(dim):
    rng = np.random.default_rng(1)
    xi = rng.uniform(-1, 1, (20, dim))
    N = q1.shape(dim, xi)
    dN = q1.shape_grad(dim, xi)
    s = q1.signs(dim)
    assert np.allclose(N.sum(axis=1), 1.0, atol=1e-15)
    assert np.allclose(dN.sum(axis=1), 0.0, atol=1e-15)
    # interpolating the vertex coordinates reproduces the point and a unit gradient
    assert np.allclose(N @ s, xi, atol=1e-15)
    assert np.allclose(np.einsum("pak,aj->pjk", dN, s), np.eye(dim)[None], atol=1e-15)


def _hamming(a, b):
    return bin(a ^ b).count("1")


@pytest.mark.parametrize("h", [1.0, 0.25])
def test_textbook_mass_and_laplacian_2d(h):
    N, dN, w = q1.reference(2)
    W = (h / 2) ** 2
    M = W * np.einsum("q,qa,qb->ab", w, N, N)
    K = W * (2 / h) ** 2 * np.einsum("q,qak,qbk->ab", w, dN, dN)
    # bilinear square: mass h^2/36 (4,2,1), stiffness 1/6 (4,-1,-2) by vertex distance
    Mref = np.array([[{0: 4, 1: 2, 2: 1}[_hamming(a, b)] for b in range(4)] for a in range(4)]) * h * h / 36
    Kref = np.array([[{0: 4, 1: -1, 2: -2}[_hamming(a, b)] for b in range(4)] for a in range(4)]) / 6
    assert np.allclose(M, Mref, rtol=1e-14, atol=0)
    assert np.allclose(K, Kref, rtol=1e-14, atol=1e-16)


def test_textbook_mass_and_laplacian_3d():
    h = 0.5
    N, dN, w = q1.reference(3)
    W = (h / 2) ** 3
    M = W * np.einsum("q,qa,qb->ab", w, N, N)
    K = W * (2 / h) ** 2 * np.einsum("q,qak,qbk->ab", w, dN, dN)
    Mref = np.array([[{0: 8, 1: 4, 2: 2, 3: 1}[_hamming(a, b)] for b in range(8)] for a in range(8)]) * h ** 3 / 216
    Kref = np.array([[{0: 4, 1: 0, 2: -1, 3: -1}[_hamming(a, b)] for b in range(8)] for a in range(8)]) * h / 12
    assert np.allclose(M, Mref, rtol=1e-14, atol=0)
    assert np.allclose(K, Kref, rtol=1e-14, atol=1e-16)


@pytest.mark.parametrize("E,nu", [(1.0, 0.2), (3.5, 0.3), (200.0, 0.45)])
def test_lame_relations(E, nu):
    mu, lam = material.lame(E, nu)
    assert np.isclose(lam / (2 * (lam + mu)), nu, rtol=1e-14)
    assert np.isclose(mu * (3 * lam + 2 * mu) / (lam + mu), E, rtol=1e-14)


def test_appendix_constants():
    mu, lam = material.lame(1.0, 0.2)
    assert np.isclose(mu, 5.0 / 12.0, rtol=1e-15) and np.isclose(lam, 5.0 / 18.0, rtol=1e-15)


def test_table1_dof_counts():
    rows = _golden("table1_dofs.txt")
    for ref, dofs in rows:
        ref, dofs = int(ref), int(dofs)
        n = 2 ** (ref + 3)
        if ref <= 6:
            m = omesh.uniform(2, -1.0, 1.0, n)
            assert m.n_all == dofs
            assert m.n_cells == n * n
        assert 3 * (n + 1) ** 2 == dofs


@pytest.mark.parametrize("dim", [2, 3])
def test_uniform_mesh_geometry(dim):
    m = omesh.uniform(dim, -2.0, 2.0, 4)
    s = (q1.signs(dim) + 1) / 2
    corners = m.cell_lo[:, None, :] + s[None] * m.cell_h[:, None, None]
    assert np.allclose(m.coords[m.cells], corners)
    on_bd = np.any(np.isclose(np.abs(m.coords), 2.0), axis=1)
    assert np.array_equal(on_bd, m.dirichlet)


def test_sneddon_closed_forms_against_paper():
    vals = {r[0]: float(r[1]) for r in _golden("sneddon_values.txt")}
    t2 = ofun.sneddon_tcv(2, 1e-3, 1.0, 1.0, 0.2)
    t3 = ofun.sneddon_tcv(3, 1e-3, 1.0, 1.0, 0.2)
    assert abs(t2 - vals["tcv2d_exact"]) < 0.5e-7
    assert abs(t3 - vals["tcv3d_exact"]) < 0.5e-7


def test_sneddon_cod_integrates_to_tcv():
    # 2d: TCV = int 2 u_n dx ; 3d: TCV = int int 2 u_n dx dy (Section 4 consistency)
    from scipy.integrate import quad
    p, l0, E, nu = 1e-3, 0.7, 1.3, 0.25
    i2, _ = quad(lambda x: 2 * ofun.sneddon_cod(2, p, l0, E, nu, x), -l0, l0, epsabs=1e-14)
    assert np.isclose(i2, ofun.sneddon_tcv(2, p, l0, E, nu), rtol=1e-10)
    i3, _ = quad(lambda r: 2 * ofun.sneddon_cod(3, p, l0, E, nu, r) * 2 * np.pi * r, 0, l0, epsabs=1e-14)
    assert np.isclose(i3, ofun.sneddon_tcv(3, p, l0, E, nu), rtol=1e-10)


@pytest.mark.parametrize("dim", [2, 3])
def test_tcv_exact_on_representable_fields(dim):
    lo, hi = -1.5, 2.5
    m = omesh.uniform(dim, lo, hi, 6 if dim == 2 else 3)
    u = np.zeros((m.n_nodes, dim))
    u[:, 0] = 1.0
    phi = (m.coords[:, 0] - lo) / (hi - lo)
    vol = (hi - lo) ** dim
    assert np.isclose(ofun.tcv(m, u, phi), vol / (hi - lo), rtol=1e-14)
    # u = x_0 e_0, phi = x_0: integral of x_0 over B
    u[:, 0] = m.coords[:, 0]
    phi = m.coords[:, 0].copy()
    exact = (hi ** 2 - lo ** 2) / 2 * (hi - lo) ** (dim - 1)
    assert np.isclose(ofun.tcv(m, u, phi), exact, rtol=1e-13)


@pytest.mark.parametrize("dim", [2, 3])
def test_cod_exact_on_representable_fields(dim):
    lo, hi = -1.0, 1.0
    m = omesh.uniform(dim, lo, hi, 8 if dim == 2 else 4)
    u = np.zeros((m.n_nodes, dim))
    u[:, dim - 1] = 2.0 + m.coords[:, 0]        # linear along the line's abscissa
    phi = m.coords[:, dim - 1] ** 1 * 0.5       # d phi / d x_last = 1/2
    x0 = np.full(dim - 1, 0.3125)
    # 1/2 int_{lo}^{hi} (2 + x0) * 1/2 dy
    exact = 0.5 * (2.0 + x0[0]) * 0.5 * (hi - lo)
    assert np.isclose(ofun.cod(m, u, phi, x0), exact, rtol=1e-14)
