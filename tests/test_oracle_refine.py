"""Pins of the oracle's refinement between loading steps, solution transfer and crack-region
marks (Section 3: refinement that keeps eps = 2h in the crack region)."""
import numpy as np
import pytest

from oracle import adaptive, mesh as omesh, refine


def _balanced_tiling(m, area):
    assert np.isclose((m.cell_h ** m.dim).sum(), area)
    c = m.cell_lo + 0.5 * m.cell_h[:, None]
    for i in range(m.n_cells):
        near = np.all(np.abs(c - c[i]) <= 0.5 * (m.cell_h + m.cell_h[i])[:, None] + 1e-12, axis=1)
        assert m.cell_h[near].max() <= 2 * m.cell_h[i] + 1e-12


def test_splitting_every_uniform_cell_halves_the_edge():
    for dim, n in ((2, 4), (3, 2)):
        m = omesh.uniform(dim, -1.0, 1.0, n)
        r = refine.refine(m, np.ones(m.n_cells, dtype=np.uint8))
        u = omesh.uniform(dim, -1.0, 1.0, 2 * n)
        assert r.n_nodes == u.n_nodes and r.n_cells == u.n_cells and r.n_free == u.n_free
        assert np.allclose(np.sort(r.cell_h), np.sort(u.cell_h))
        at = {tuple(q): x for q, x in zip(r.lattice, r.coords)}
        assert set(at) == set(map(tuple, u.lattice))
        assert max(np.abs(at[tuple(q)] - x).max() for q, x in zip(u.lattice, u.coords)) <= 1e-15


@pytest.mark.parametrize("dim", [2, 3])
def test_marked_cells_are_split_and_the_result_is_balanced(dim):
    if dim == 2:
        m = adaptive.adaptive(2, -1.0, 1.0, 4, 2, 0.3, (0.0, 0.0, 0.0), 0.25)
    else:
        m = adaptive.adaptive(3, -1.0, 1.0, 2, 1, 0.1, (0.0, 0.0, 0.0), 0.3)
    rng = np.random.default_rng(5 + dim)
    flags = (rng.random(m.n_cells) < 0.2).astype(np.uint8)
    flags[np.argmin(m.cell_h)] = 1                     # a finest cell: one more level
    r = refine.refine(m, flags)
    assert r.h_min == pytest.approx(m.h_min / 2)
    _balanced_tiling(r, 2.0 ** dim)
    centres = r.cell_lo + 0.5 * r.cell_h[:, None]
    for c in np.nonzero(flags)[0]:
        inside = np.all((centres > m.cell_lo[c]) & (centres < m.cell_lo[c] + m.cell_h[c]), axis=1)
        assert inside.sum() >= 2 ** dim
        assert r.cell_h[inside].max() <= m.cell_h[c] / 2 + 1e-15
    # unmarked cells are split only by the balance
    for c in np.nonzero(flags == 0)[0][:50]:
        inside = np.all((centres > m.cell_lo[c]) & (centres < m.cell_lo[c] + m.cell_h[c]), axis=1)
        assert inside.sum() in (1, 2 ** dim) or r.cell_h[inside].min() < m.cell_h[c] / 2


@pytest.mark.parametrize("dim", [2, 3])
def test_transfer_reproduces_the_old_function(dim):
    if dim == 2:
        m = adaptive.adaptive(2, -1.0, 1.0, 4, 2, 0.3, (0.0, 0.0, 0.0), 0.25)
    else:
        m = adaptive.adaptive(3, -1.0, 1.0, 2, 2, 0.1, (0.0, 0.0, 0.0), 0.3)
    assert m.n_free < m.n_nodes
    rng = np.random.default_rng(17)
    flags = (rng.random(m.n_cells) < 0.3).astype(np.uint8)
    r = refine.refine(m, flags)
    vals = rng.standard_normal(m.n_nodes)
    new = refine.transfer(m, r, vals)
    for x in rng.uniform(-1.0, 1.0, (40, dim)):
        assert abs(refine.evaluate(r, new, x) - refine.evaluate(m, vals, x)) <= 1e-13
    # a field that is Q1 on every cell (a + b.x + c x0 x1) is reproduced at every node
    a = rng.standard_normal(dim)

    def f(X):
        return 0.3 + X @ a + 0.7 * X[:, 0] * X[:, 1]

    assert np.abs(refine.transfer(m, r, f(m.coords)) - f(r.coords)).max() <= 1e-14


def test_crack_marks_against_a_direct_scan():
    m = adaptive.adaptive(2, -1.0, 1.0, 4, 2, 0.3, (0.0, 0.0, 0.0), 0.25)
    rng = np.random.default_rng(3)
    phi = m.C @ rng.uniform(0.0, 1.0, m.n_free)
    h_t = m.h_min * 1.5
    flags = refine.mark_crack(m, phi, 0.4, h_t)
    for c in range(m.n_cells):
        want = m.cell_h[c] > h_t and min(phi[m.cells[c, a]] for a in range(4)) < 0.4
        assert bool(flags[c]) == want
    assert flags.any() and not flags.all()


@pytest.mark.parametrize("dim", [2, 3])
def test_kelly_vanishes_for_linear_displacements(dim):
    if dim == 2:
        m = adaptive.adaptive(2, -1.0, 1.0, 4, 2, 0.3, (0.0, 0.0, 0.0), 0.25)
    else:
        m = adaptive.adaptive(3, -1.0, 1.0, 2, 2, 0.1, (0.0, 0.0, 0.0), 0.3)
    assert m.n_free < m.n_nodes
    A = np.random.default_rng(2).standard_normal((dim, dim))
    u = m.coords @ A.T + 0.3
    assert np.abs(refine.kelly(m, u)).max() <= 1e-24


def test_kelly_closed_form_at_a_kink():
    """u_0 = |x_0 - a| with a on a grid line: the normal derivative jumps by 2 across that line,
    so the cells on either side have eta^2 = h/24 * 4 * h = h^2/6 and all others 0."""
    n, L = 8, 1.0
    m = omesh.uniform(2, -L, L, n)
    h = 2 * L / n
    a = -L + 3 * h
    u = np.zeros((m.n_nodes, 2))
    u[:, 0] = np.abs(m.coords[:, 0] - a)
    eta2 = refine.kelly(m, u)
    touch = (np.abs(m.cell_lo[:, 0] - a) < 1e-12) | (np.abs(m.cell_lo[:, 0] + h - a) < 1e-12)
    assert touch.sum() == 2 * n
    assert np.allclose(eta2[touch], h * h / 6.0, rtol=1e-13)
    assert np.abs(eta2[~touch]).max() <= 1e-28
