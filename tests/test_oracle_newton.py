"""Pins of the oracle's active set, elimination, exact solve and Newton loop (Section 3),
and of the whole discrete problem against Sneddon's closed form (Section 4)."""
import itertools
import numpy as np
import pytest

from oracle import fem, newton, mesh as omesh, functionals as ofun
from oracle.material import Params
from inputs import crack_band_phi, random_state


def _sneddon(n, L=2.0, l0=0.25, kappa=1e-10, p=1e-3):
    m = omesh.uniform(2, -L, L, n)
    h = 2 * L / n
    prm = Params(eps=2 * h, kappa=kappa, p=p)
    phi0 = crack_band_phi(m.coords, l0, prm.eps)
    return m, prm, phi0


def test_dense_lu_matches_block_substitution():
    m, prm, phi0 = _sneddon(8, L=1.0, l0=0.3, kappa=1e-6)
    u0 = np.zeros((m.n_nodes, 2))
    st = newton.newton_step_system(m, prm, u0, phi0, phi0, phi0)
    a = newton.solve_block(m, st.Jm, st.F)
    b = newton.solve_dense(st.Jm, st.F)
    assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()
    assert st.active.sum() > 0
    # a generic state with nonzero elimination targets (phi != phi_old on active DoFs)
    u, phi, phi_old, pt = random_state(m.n_nodes, 2, seed=4, u_scale=1e-2)
    u[m.dirichlet] = 0.0
    st = newton.newton_step_system(m, prm, u, phi, phi_old, pt)
    a = newton.solve_block(m, st.Jm, st.F)
    b = newton.solve_dense(st.Jm, st.F)
    assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()
    assert np.any(st.target[st.fixed] != 0.0)
    # the fixed DoFs land exactly on their targets; J is block lower triangular
    assert np.allclose(a[st.fixed], st.target[st.fixed], rtol=1e-13, atol=0)
    nu = 2 * m.n_free
    assert abs(st.Jm[:nu, nu:]).max() == 0.0


def test_elimination_identity_small():
    """Z12 reading: fixed rows/cols zeroed, diagonal kept, column moved to the RHS."""
    import scipy.sparse as sp
    J = sp.csr_matrix(np.array([[4.0, 1.0, 0.5], [1.0, 3.0, 0.2], [0.5, 0.2, 2.0]]))
    R = np.array([1.0, -2.0, 0.5])
    fixed = np.array([False, True, False])
    target = np.array([0.0, 0.7, 0.0])
    Jm, F = newton.mask_system(J, R, fixed, target)
    x = np.linalg.solve(Jm.toarray(), F)
    # same as solving J x = -R with x_1 prescribed
    A = J.toarray()
    free = [0, 2]
    ref = np.linalg.solve(A[np.ix_(free, free)], -R[free] - A[free, 1] * 0.7)
    assert np.isclose(x[1], 0.7, rtol=1e-15)
    assert np.allclose(x[free], ref, rtol=1e-14)


def _check_kkt(m, prm, out, phi_old, pt, tol):
    d = m.dim
    nf = m.n_free
    u, phi = out["u"], out["phi"]
    R, B = fem.residual(m, prm, u, phi, pt)
    Ru = R[:d * nf].reshape(nf, d)[~m.dirichlet[m.free]]
    Rp = R[d * nf:]
    A = out["active"]
    scale = np.abs(R).max()
    assert np.abs(Ru).max() < tol * scale
    assert np.abs(Rp[~A]).max() < tol * scale            # stationarity off the active set
    assert np.all(phi[m.free] <= phi_old[m.free] + 1e-12)  # feasibility
    assert np.all(-Rp[A] / B[A] >= -tol * scale / B[A])  # lambda >= 0 on A
    assert np.allclose(phi[m.free][A], phi_old[m.free][A], atol=1e-12)   # complementarity


def test_kkt_at_newton_fixed_point():
    m, prm, phi0 = _sneddon(16, L=1.0, l0=0.25, kappa=1e-8)
    u0 = np.zeros((m.n_nodes, 2))
    out = newton.newton_loop(m, prm, u0, phi0, phi0, phi0)
    assert out["converged"]
    _check_kkt(m, prm, out, phi0, phi0, 1e-8)


def test_bruteforce_active_set_matches_pdas():
    """u = 0, p = 0: the phi problem is a QP; exactly one active set satisfies KKT."""
    m = omesh.uniform(2, -1.0, 1.0, 3)
    prm = Params(eps=0.35, kappa=1e-3, p=0.0, Gc=1.0)
    rng = np.random.default_rng(21)
    phi_old = np.where(rng.uniform(size=m.n_nodes) < 0.5, 1.0, rng.uniform(0.3, 0.99, m.n_nodes))
    u0 = np.zeros((m.n_nodes, 2))
    out = newton.newton_loop(m, prm, u0, phi_old.copy(), phi_old, np.ones(m.n_nodes), tol=1e-12)
    assert out["converged"]
    n = m.n_nodes
    zero = np.zeros(n)
    Jpp = fem.jacobian(m, prm, u0, zero, np.ones(n))[2 * n:, 2 * n:].toarray()
    R0, B = fem.residual(m, prm, u0, zero, np.ones(n))
    b = -R0[2 * n:]                  # R_phi(phi) = Jpp phi - b at u = 0
    hits = []
    for bits in itertools.product([False, True], repeat=n):
        S = np.array(bits)
        F = ~S
        phi = phi_old.copy()
        if F.any():
            phi[F] = np.linalg.solve(Jpp[np.ix_(F, F)], b[F] - Jpp[np.ix_(F, S)] @ phi_old[S])
        Rp = Jpp @ phi - b
        if np.all(phi[F] <= phi_old[F] + 1e-12) and np.all(Rp[S] <= 1e-12):
            hits.append(S)
    assert len(hits) == 1
    assert np.array_equal(hits[0], out["active"])
    assert 0 < hits[0].sum() < n


def test_symmetry_of_centred_crack():
    m, prm, phi0 = _sneddon(16, L=1.0, l0=0.25, kappa=1e-6)
    u0 = np.zeros((m.n_nodes, 2))
    st = newton.newton_step_system(m, prm, u0, phi0, phi0, phi0)
    U = fem.restrict(m, u0, phi0) + newton.solve_block(m, st.Jm, st.F)
    u, phi = fem.expand(m, U)
    n = 16
    I, J = m.lattice[:, 0], m.lattice[:, 1]
    mx = (n - I) + (n + 1) * J          # mirror x -> -x
    my = I + (n + 1) * (n - J)          # mirror y -> -y
    s = np.abs(u).max()
    assert np.allclose(u[mx, 0], -u[:, 0], atol=1e-12 * s) and np.allclose(u[my, 0], u[:, 0], atol=1e-12 * s)
    assert np.allclose(u[mx, 1], u[:, 1], atol=1e-12 * s) and np.allclose(u[my, 1], -u[:, 1], atol=1e-12 * s)
    assert np.allclose(phi[mx], phi, atol=1e-12) and np.allclose(phi[my], phi, atol=1e-12)
    assert u[np.argmin(np.abs(m.coords[:, 0]) + np.abs(m.coords[:, 1] - 2 * 2.0 / 16)), 1] > 0


@pytest.mark.slow
def test_sneddon_tcv_band_and_h_convergence():
    """Config-1 geometry: eps/l0 = 0.25 overestimates TCV, the finite domain (L/l0 = 8)
    underestimates it; halving h (eps = 2h) must shrink the error."""
    exact = ofun.sneddon_tcv(2, 1e-3, 0.25, 1.0, 0.2)
    errs = []
    for n in (64, 128):
        m, prm, phi0 = _sneddon(n)
        u0 = np.zeros((m.n_nodes, 2))
        st = newton.newton_step_system(m, prm, u0, phi0, phi0, phi0)
        U = fem.restrict(m, u0, phi0) + newton.solve_block(m, st.Jm, st.F)
        u, phi = fem.expand(m, U)
        errs.append(ofun.tcv(m, u, phi) / exact - 1.0)
        cod0 = ofun.cod(m, u, phi, [1.0 / n])
        assert 0.5 < cod0 / ofun.sneddon_cod(2, 1e-3, 0.25, 1.0, 0.2, 1.0 / n) < 1.5
    assert 0.0 < errs[1] < 0.4
    assert abs(errs[1]) < 0.75 * abs(errs[0])


def test_cycle_rule_on_membership_sequences():
    """Section 3 constrains alternating active-set indices: of the eight membership
    sequences over three iterates exactly in-out-in and out-in-out alternate; frozen DoFs are
    active from then on, whatever the later decisions."""
    seqs = np.array(list(itertools.product([False, True], repeat=3)))
    a0, a1, a2 = seqs[:, 0], seqs[:, 1], seqs[:, 2]
    flagged = newton.alternating(a0, a1, a2)
    expect = np.array([(x != y) and (y != z) for x, y, z in seqs])
    assert flagged.sum() == 2
    assert np.array_equal(flagged, expect)
    assert set(map(tuple, seqs[flagged].astype(int))) == {(1, 0, 1), (0, 1, 0)}
    none = np.zeros(8, dtype=bool)
    act, frz = newton.freeze(a0, a1, a2, none)
    assert np.array_equal(frz, flagged)
    assert np.array_equal(act, a2 | flagged)          # out-in-out ends active, not inactive
    assert act[np.where((seqs == [0, 1, 0]).all(1))[0][0]]
    # a DoF frozen earlier stays frozen and active even when every later decision is "out"
    earlier = np.zeros(8, dtype=bool)
    earlier[0] = True                                  # the out-out-out sequence
    act, frz = newton.freeze(a0, a1, a2, earlier)
    assert frz[0] and act[0]
    assert np.array_equal(frz, flagged | earlier)
    # the inputs are left alone
    assert not none.any()


def _alternating_problem():
    from inputs import alternating_case
    c = alternating_case()
    m = omesh.uniform(2, -c["L"], c["L"], c["n"])
    assert np.array_equal(m.dirichlet, c["boundary"])
    prm = Params(E=c["E"], nu=c["nu"], Gc=c["Gc"], kappa=c["kappa"], eps=c["eps"], p=c["p"])
    return m, prm, c


def test_cycle_rule_stops_an_alternating_active_set():
    m, prm, c = _alternating_problem()
    args = (m, prm, c["u0"], c["phi0"], c["phi_old"], c["phi_tilde"])
    out = newton.newton_loop(*args, tol=1e-8, max_it=20)
    assert out["status"] == "ok" and out["converged"]
    assert out["iterations"] == 4
    assert np.array_equal(np.nonzero(out["frozen"])[0], [0, 1])
    assert out["active"][[0, 1]].all()
    # without the rule the same loop alternates until the cap with a converged residual
    raw = newton.newton_loop(*args, tol=1e-8, max_it=20, freeze_cycles=False)
    assert raw["status"] == "cycle" and not raw["converged"]
    assert raw["iterations"] == 20
    assert raw["res"] <= 1e-8 * raw["r0"]
    assert all(e["changed"] > 0 for e in raw["log"][-6:])
    # a periodic orbit of the active set (period 3 here: DoFs 0 and 1 leave and re-enter)
    acts = [e["n_active"] for e in raw["log"][-6:]]
    assert acts[:3] == acts[3:] and len(set(acts)) == 3
