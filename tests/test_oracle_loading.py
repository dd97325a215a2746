"""Pins of the oracle's quasi-static loading steps (Formulation 1 per loading step n, with
phi_old = phi^{n-1} and phi_tilde the linear extrapolation in time)."""
import numpy as np

from oracle import adaptive, loading, mesh as omesh, newton as onewton, functionals as ofun
from oracle.material import Params
from inputs import crack_band_phi


def _uniform(n=16, L=1.0):
    m = omesh.uniform(2, -L, L, n)
    eps = 2 * (2 * L / n)
    return m, eps, crack_band_phi(m.coords, 0.25, eps)


def test_extrapolation_exact_for_fields_linear_in_time():
    """phi(t, x) = a(x) + b(x) t with a, b linear in x: the extrapolation to t_n from t_{n-1},
    t_{n-2} (unequal steps) is exact at every node, hanging nodes included (a field linear in
    space is reproduced by the edge-midpoint interpolation)."""
    m = adaptive.adaptive(2, -1.0, 1.0, 4, 2, 0.3, (0.0, 0.0, 0.0), 0.25)
    assert m.n_nodes > m.n_free                      # the mesh has hanging nodes
    x, y = m.coords[:, 0], m.coords[:, 1]
    a = 0.6 + 0.1 * x - 0.05 * y
    b = -0.04 - 0.01 * x + 0.02 * y

    def phi(t):
        return a + b * t

    t2, t1, tn = 0.3, 1.1, 2.6
    w = loading.step_weight(tn, t1, t2)
    assert abs(w - 1.5 / 0.8) < 1e-15
    pt = loading.extrapolate(m, phi(t1), phi(t2), w)
    assert np.all((phi(tn) > 0) & (phi(tn) < 1))
    assert np.abs(pt - phi(tn)).max() <= 1e-14


def test_extrapolation_clips_to_the_phase_field_range():
    m, _, _ = _uniform(4)
    one = np.ones(m.n_nodes)
    assert np.all(loading.extrapolate(m, 0.1 * one, 0.6 * one, 1.0) == 0.0)     # 0.1 - 0.5 < 0
    assert np.all(loading.extrapolate(m, 1.0 * one, 0.5 * one, 1.0) == 1.0)     # 1.0 + 0.5 > 1
    assert np.allclose(loading.extrapolate(m, 0.5 * one, 0.6 * one, 2.0), 0.3, rtol=0, atol=1e-15)


def test_first_step_is_linear_in_the_load():
    """At step 1 phi_tilde = phi^0 for any load, and the u-equation is linear in p for a fixed
    phi_tilde (M_uphi = 0), so the first step of a ramp p/3, 2p/3, p moves u by exactly 1/3
    of what one step at p does."""
    m, eps, phi0 = _uniform()
    P = 1e-3
    prms = [Params(eps=eps, kappa=1e-8, p=P * k / 3) for k in (1, 2, 3)]
    u0 = np.zeros((m.n_nodes, 2))
    steps = loading.loading(m, prms, [0.0, 1.0, 2.0, 3.0], u0, phi0, atol=1e-12)
    one = onewton.newton_loop(m, Params(eps=eps, kappa=1e-8, p=P), u0, phi0, phi0, phi0, atol=1e-12)
    assert all(r["converged"] for r in steps) and one["converged"]
    assert np.abs(3.0 * steps[0]["u"] - one["u"]).max() <= 1e-12 * np.abs(one["u"]).max()
    assert np.array_equal(steps[0]["phi_tilde"], phi0)


def test_irreversibility_across_steps():
    """phi^n <= phi^{n-1} at every node of every step, active DoFs held exactly at phi^{n-1}
    (a phi_old other than the previous step's field fails the second check: the first step
    moves phi by about 0.58)."""
    m, eps, phi0 = _uniform()
    prms = [Params(eps=eps, kappa=1e-8, p=1e-3 * k / 3) for k in (1, 2, 3)]
    steps = loading.loading(m, prms, [0.0, 1.0, 1.5, 3.0], np.zeros((m.n_nodes, 2)), phi0, atol=1e-12)
    prev = phi0
    for r in steps:
        assert r["converged"]
        assert np.array_equal(r["phi_old"], prev)
        assert (r["phi"] - prev).max() <= 0.0
        act = r["active"]
        assert act.any()
        assert np.array_equal(r["phi"][m.free][act], prev[m.free][act])
        prev = r["phi"]
    assert (phi0 - steps[0]["phi"]).max() > 0.5


def test_constant_load_reaches_a_stationary_state():
    """Repeated steps at one load converge: the phase field stops moving, phi_tilde tends to
    phi, a step from the stationary state takes one Newton iteration (absolute stop rule),
    and TCV settles."""
    m, eps, phi0 = _uniform()
    P = 1e-3
    N = 8
    prms = [Params(eps=eps, kappa=1e-8, p=P) for _ in range(N)]
    steps = loading.loading(m, prms, list(range(N + 1)), np.zeros((m.n_nodes, 2)), phi0, atol=1e-12)
    assert all(r["converged"] for r in steps)
    assert steps[-1]["iterations"] == 1 and steps[-2]["iterations"] == 1
    assert np.abs(steps[-1]["phi"] - steps[-2]["phi"]).max() <= 1e-13
    assert np.abs(steps[-1]["phi_tilde"] - steps[-1]["phi_old"]).max() <= 1e-13
    t = [ofun.tcv(m, r["u"], r["phi"]) for r in steps[-3:]]
    assert abs(t[-1] / t[0] - 1) <= 1e-9


def test_continuation_with_a_previous_state():
    """Three steps in one call equal two steps followed by one step that is given the state
    before it (phi^1 at t_1) for its extrapolation."""
    m, eps, phi0 = _uniform(12)
    prms = [Params(eps=eps, kappa=1e-8, p=1e-3 * k / 3) for k in (1, 2, 3)]
    times = [0.0, 1.0, 2.5, 3.0]
    u0 = np.zeros((m.n_nodes, 2))
    full = loading.loading(m, prms, times, u0, phi0, atol=1e-12)
    part = loading.loading(m, prms[:2], times[:3], u0, phi0, atol=1e-12)
    last = loading.loading(m, prms[2:], times[2:], part[-1]["u"], part[-1]["phi"],
                           phi_prev=part[0]["phi"], t_prev=times[1], atol=1e-12)
    assert np.array_equal(full[-1]["phi_tilde"], last[0]["phi_tilde"])
    assert np.array_equal(full[-1]["u"], last[0]["u"])
    assert np.array_equal(full[-1]["phi"], last[0]["phi"])


def test_absolute_stop_rule_at_a_converged_start():
    """Starting a step at its own converged state: with the relative rule alone the residual
    cannot fall tol times below a start that is already at rounding level; the absolute floor
    ends the loop after one iteration."""
    m, eps, phi0 = _uniform(8)
    prm = Params(eps=eps, kappa=1e-8, p=1e-3)
    u0 = np.zeros((m.n_nodes, 2))
    r = onewton.newton_loop(m, prm, u0, phi0, phi0, phi0, atol=1e-12)
    assert r["converged"]
    again = onewton.newton_loop(m, prm, r["u"], r["phi"], phi0, phi0, atol=1e-12)
    assert again["converged"] and again["iterations"] == 1
    stuck = onewton.newton_loop(m, prm, r["u"], r["phi"], phi0, phi0, max_it=4)
    assert not stuck["converged"]
