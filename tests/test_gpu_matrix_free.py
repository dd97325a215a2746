"""The matrix-free fine-level operators on uniform 2d meshes (fine_matrix_free, bit 0: M_uu from
phi_tilde; bit 1: the masked M_phiphi, and with bit 0 the phase-field rows of the J-SpMV, from the
assembly's u, phi and active set; bit 2: the finest displacement level's prolongation and
restriction from the aggregation; default all) equal the stored (masked) operators up to
rounding, in the smoothers, the fine-level residuals, the transfers and the J-SpMV; the FGMRES
solve and the Newton loop reach the same results with the same iteration counts either way."""
import numpy as np
import pytest
import torch

from paper_1806_09924_amd import binding as B
from oracle import newton as onewton
from inputs import random_state
from gpu_util import Problem, dev, host

pytestmark = pytest.mark.gpu


def _solve(S, mf, precision=64, rtol=1e-10):
    A = B.Amg(S, B.amg_opts(precision=precision, fine_matrix_free=mf))
    du = torch.empty(S.mesh.n_solve, dtype=torch.float64, device="cuda")
    st = B.solve(S, A, du, B.solve_opts(rtol=rtol))
    z = torch.empty_like(du)
    A.apply(dev(np.random.default_rng(5).standard_normal(S.mesh.n_solve)), z)
    return st, host(du), host(z)


def _rect_system(L, nx, ny, seed=11):
    """A rectangle of square cells and a generic state (every term of the blocks, both masks)."""
    d = B.mesh_desc(2, -L, L, nx)
    d.hi[1] = -L + 2 * L / nx * ny
    d.base[1] = ny
    mesh = B.Mesh(d)
    state = random_state(mesh.n_nodes, 2, seed)
    prm = B.params(eps=0.1, kappa=1e-6, p=2e-3)
    return mesh, prm, state


@pytest.mark.parametrize("mf", [1, 2, 3, 5, 7])
@pytest.mark.parametrize("precision", [64, 32])
@pytest.mark.parametrize("shape", [(2.0, 128, 128), (1.0, 40, 24)])
def test_matrix_free_fine_level_matches_stored_blocks(shape, precision, mf):
    L, nx, ny = shape
    if nx == ny:
        P = Problem(2, L, nx)
        state = P.state
        mesh, prm = P.mesh, P.prm
    else:
        mesh, prm, state = _rect_system(L, nx, ny)
    S = B.System(mesh).assemble(prm, *[dev(a) for a in state])
    st0, d0, z0 = _solve(S, 0, precision)
    st1, d1, z1 = _solve(S, mf, precision)
    # the V-cycle (matrix-free fine smoother and residual) equals the stored-block one to the
    # rounding of the hierarchy's precision
    assert np.abs(z1 - z0).max() <= (1e-11 if precision == 64 else 1e-5) * np.abs(z0).max()
    # the solve: same iterations (FP32: within one), same increment to the solver tolerance
    assert abs(st0["iters"] - st1["iters"]) <= (0 if precision == 64 else 1)
    assert st1["relres"] <= 1e-10
    nu = 2 * mesh.n_free
    for sl, bar in ((slice(0, nu), 5e-7), (slice(nu, None), 1e-8)):
        assert np.abs(d1[sl] - d0[sl]).max() <= bar * np.abs(d0[sl]).max()
    # its residual is the true one of the stored Jacobian
    rp, ci, vv = S.csr()
    import scipy.sparse as sp
    J = sp.csr_matrix((vv, ci, rp), shape=(mesh.n_solve, mesh.n_solve))
    _, F, _, _ = S.vectors()
    F = host(F)
    assert np.linalg.norm(F - J @ d1) / np.linalg.norm(F) <= 1.01e-10


@pytest.mark.parametrize("case", ["sneddon", "rect"])
def test_matrix_free_jspmv_equals_stored(case):
    """fracture_matvec_free (rows 1 and 3) against the stored masked Jacobian, element by element,
    on the Sneddon state (crack band active) and on a generic state (active and inactive nodes
    mixed, Dirichlet rows and columns, nonzero u), for several vectors."""
    if case == "sneddon":
        P = Problem(2, 2.0, 128)
        mesh, prm, state = P.mesh, P.prm, P.state
    else:
        mesh, prm, state = _rect_system(1.0, 40, 24, seed=3)
    S = B.System(mesh).assemble(prm, *[dev(a) for a in state])
    act = host(S.vectors()[3])
    nu = 2 * mesh.n_free
    assert 0 < act.sum() < mesh.n_free or case == "sneddon"
    rng = np.random.default_rng(7)
    for k in range(3):
        x = dev(rng.standard_normal(mesh.n_solve))
        y0 = torch.empty_like(x)
        S.matvec(x, y0)
        ref = host(y0)
        for rows in (1, 3):
            y = torch.empty_like(x)
            S.matvec_free(x, y, rows=rows)
            got = host(y)
            for sl in (slice(0, nu), slice(nu, None)):
                scale = np.abs(ref[sl]).max()
                assert np.abs(got[sl] - ref[sl]).max() <= 1e-13 * scale, (rows, sl)
            # rows whose whole product is one stored diagonal entry (active phase-field rows)
            # come out exactly
            a = np.flatnonzero(act)
            assert np.array_equal(got[nu + a], ref[nu + a]) or rows == 1


def test_matrix_free_newton_loop_config1():
    P = Problem(2, 2.0, 128)
    out = []
    for mf in (0, 7):
        u, phi, po, pt = P.dstate()
        st = B.newton(P.mesh, P.prm, u, phi, po, pt, amg=B.amg_opts(fine_matrix_free=mf))
        out.append((st, host(u), host(phi)))
    (s0, u0, p0), (s1, u1, p1) = out
    assert s0["status"] == s1["status"] == B.FR_OK
    assert s0["iterations"] == s1["iterations"] and s0["linear_iters"] == s1["linear_iters"]
    assert s0["n_active"] == s1["n_active"]
    _, t0 = B.functionals(P.mesh, dev(u0), dev(p0))
    _, t1 = B.functionals(P.mesh, dev(u1), dev(p1))
    assert abs(t1 / t0 - 1) <= 1e-8
