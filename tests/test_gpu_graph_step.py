"""The captured FGMRES iteration (use_graphs): the Krylov index lives on the device, one Arnoldi
step (both V-cycles, J z, Gram-Schmidt, rotations, summary) is captured once per preconditioner
setup and replayed every iteration.  Replays must give bit for bit what direct launches give:
for one instance and a batch, FP64 and FP32 hierarchies, across restarts and basis growth, and
through a whole Newton loop."""
import numpy as np
import pytest
import torch

from paper_1806_09924_amd import binding as B
from gpu_util import Problem, dev, host

pytestmark = pytest.mark.gpu


def _solve_both(S, A, n, **kw):
    out = []
    for g in (0, 1):
        du = torch.empty(n, dtype=torch.float64, device="cuda")
        st = B.solve(S, A, du, B.solve_opts(use_graphs=g, **kw), raise_on_status=False)
        out.append((st, host(du)))
    return out


@pytest.mark.parametrize("precision", [64, 32])
def test_graph_step_bitwise_config1(precision):
    P = Problem(2, 2.0, 128)
    u, phi, po, pt = P.dstate()
    S = B.System(P.mesh).assemble(P.prm, u, phi, po, pt)
    A = B.Amg(S, B.amg_opts(precision=precision))
    (s0, d0), (s1, d1) = _solve_both(S, A, P.mesh.n_solve, rtol=1e-10)
    assert s0["status"] == s1["status"] == B.FR_OK
    assert s0["iters"] == s1["iters"] > 1
    assert np.array_equal(d0, d1)
    # short restarts: several cycles, the device index restarting at 0 in each; a basis that
    # grows past its first capacity (24 vectors) on the way
    (s0, d0), (s1, d1) = _solve_both(S, A, P.mesh.n_solve, rtol=1e-12, restart=7)
    assert s0["iters"] == s1["iters"] > 7
    assert np.array_equal(d0, d1)
    (s0, d0), (s1, d1) = _solve_both(S, A, P.mesh.n_solve, rtol=1e-13, restart=40)
    assert s0["iters"] == s1["iters"]
    assert np.array_equal(d0, d1)


def test_graph_step_bitwise_batch_and_newton():
    specs = [(0.75, 24, 5e-4), (1.0, 32, 1e-3), (1.2, 40, 1.5e-3)]
    from oracle import mesh as omesh
    from inputs import crack_band_phi
    descs = [B.mesh_desc(2, -L, L, n) for (L, n, _) in specs]
    prms, phis = [], []
    for (L, n, p) in specs:
        eps = 2 * 2 * L / n
        prms.append(B.params(eps=eps, kappa=1e-10, p=p))
        phis.append(crack_band_phi(omesh.uniform(2, -L, L, n).coords, 0.25, eps))
    phi0 = np.concatenate(phis)
    results = []
    for g in (0, 1):
        mesh = B.Mesh(descs)
        u = torch.zeros((mesh.n_nodes, 2), dtype=torch.float64, device="cuda")
        phi = dev(phi0)
        st = B.newton(mesh, prms, u, phi, dev(phi0), dev(phi0), solve=B.solve_opts(use_graphs=g))
        results.append((st, host(u), host(phi)))
    (st0, u0, p0), (st1, u1, p1) = results
    assert [s["linear_iters"] for s in st0] == [s["linear_iters"] for s in st1]
    assert [s["status"] for s in st1] == [B.FR_OK] * 3
    assert np.array_equal(u0, u1) and np.array_equal(p0, p1)


def test_graph_step_fresh_preconditioner_on_the_same_system():
    """A preconditioner made on a system after an earlier one was destroyed (it typically takes
    the same address): its solves must capture their own step, not replay the earlier one's
    (whose hierarchy buffers are gone).  Replay against direct launches, bit for bit."""
    import gc
    P = Problem(2, 2.0, 64)
    u, phi, po, pt = P.dstate()
    S = B.System(P.mesh).assemble(P.prm, u, phi, po, pt)
    for prec in (64, 32, 64):
        A = B.Amg(S, B.amg_opts(precision=prec))
        out = {}
        for g in (1, 0):
            du = torch.empty(P.mesh.n_solve, dtype=torch.float64, device="cuda")
            st = B.solve(S, A, du, B.solve_opts(use_graphs=g, rtol=1e-10))
            out[g] = (st["iters"], host(du))
        assert out[0][0] == out[1][0]
        assert np.array_equal(out[0][1], out[1][1])
        del A
        gc.collect()
