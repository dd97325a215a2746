"""Quasi-static loading steps n = 1, 2, 3, ... of Formulation 1 (Section 2) on a fixed mesh.

TEST INFRASTRUCTURE ONLY (see the package header).

Formulation 1 is posed per loading step n with phi_old the phase field of the previous
step and phi_tilde a linear extrapolation in time of the phase field (the convexification
the paper takes from its reference [HeWheWi15]).  Per step:
    phi_old   = phi^{n-1}
    phi_tilde = clip(phi^{n-1} + w_n (phi^{n-1} - phi^{n-2}), 0, 1),
                w_n = (t_n - t_{n-1}) / (t_{n-1} - t_{n-2}),
    (u^n, phi^n) = Newton / active-set loop of Section 3 from (u^{n-1}, phi^{n-1}).
Readings (the paper gives no formula for phi_tilde):
  * the line through (t_{n-2}, phi^{n-2}) and (t_{n-1}, phi^{n-1}) evaluated at t_n;
  * at the first step only one state is known, so phi_tilde = phi^0 (constant extrapolation),
    unless the caller passes a state before it (phi_prev at t_prev);
  * clipped to [0, 1], the range of a phase field;
  * applied to the free DoFs, hanging-node values then interpolated from them, since the
    discrete field is determined by its free values (clip and interpolation do not commute).
The pressure of step n is the caller's (a schedule p_n per step).

Pinned by tests/test_oracle_loading.py: exact extrapolation of fields linear in time on
unequal steps; the clip bounds; hanging values equal to the mean of their edge's ends; the
u-equation is linear in p for a fixed phi_tilde, so the first step of a pressure ramp gives
exactly p_1 / p times the displacement of one step at p; TCV_n / p_n constant along a ramp
below the critical pressure (the crack does not move); irreversibility phi^n <= phi^{n-1}
with active DoFs held exactly at phi^{n-1}.
"""
import numpy as np

from . import newton as onewton


def extrapolate(mesh, phi1, phi2, w):
    """phi_tilde on all nodes from the previous (phi1) and second previous (phi2) fields."""
    f = mesh.free
    pt = np.clip(phi1[f] + w * (phi1[f] - phi2[f]), 0.0, 1.0)
    return mesh.C @ pt


def step_weight(t_n, t_1, t_2):
    """w_n of the linear extrapolation to t_n from t_1 = t_{n-1} and t_2 = t_{n-2}."""
    return (t_n - t_1) / (t_1 - t_2)


def loading(mesh, prms, times, u0, phi0, phi_prev=None, t_prev=None, **newton_kw):
    """Steps n = 1 .. len(times) - 1; prms[n-1] holds step n's parameters (its pressure),
    times[0] is the time of (u0, phi0).  Returns one dict per step: the Newton result
    (u, phi, iterations, active, ...) plus phi_old, phi_tilde and tcv-ready state."""
    assert len(prms) == len(times) - 1
    u = np.array(u0, dtype=np.float64)
    phi = mesh.C @ np.asarray(phi0, dtype=np.float64)[mesh.free]
    before = None
    if phi_prev is not None:
        before = (mesh.C @ np.asarray(phi_prev, dtype=np.float64)[mesh.free], float(t_prev))
    out = []
    for n in range(1, len(times)):
        phi_old = phi.copy()
        if before is None:
            phi_tilde = phi_old.copy()
        else:
            phi_tilde = extrapolate(mesh, phi_old, before[0], step_weight(times[n], times[n - 1], before[1]))
        res = onewton.newton_loop(mesh, prms[n - 1], u, phi, phi_old, phi_tilde, **newton_kw)
        res["phi_old"] = phi_old
        res["phi_tilde"] = phi_tilde
        out.append(res)
        before = (phi_old, times[n - 1])
        u, phi = res["u"], res["phi"]
    return out
