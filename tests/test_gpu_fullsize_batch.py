"""Parity on the full batched workload: 48 independent 2d Sneddon instances (domain
half-widths L ~ U[1, 20], eps in {2h, 4h}, p ~ U[5e-4, 2e-3], crack centre offsets, N up to
706 cells per axis; seed 9924) solved as one disjoint-union system with per-instance
parameters, per-instance FGMRES convergence and per-instance functionals, with the FP32 and
the FP64 preconditioner.

Per instance the oracle checks: the three smallest instances exactly (the oracle's exact
Newton step: relative residual of the GPU update evaluated by the oracle, TCV); the three
largest on sampled rows of the assembled residual that the oracle computes from the cells
around them; every instance through FP32-versus-FP64 agreement of TCV and the per-instance
convergence reports."""
import numpy as np
import pytest
import torch

from paper_1806_09924_amd import binding as B
from oracle import mesh as omesh, fem, newton as onewton, functionals as ofun
from oracle.material import Params as OParams
from inputs import batched_instances, crack_band_phi
from gpu_util import dev, host

pytestmark = pytest.mark.gpu

L0 = 0.25


@pytest.fixture(scope="module")
def batch():
    wl = batched_instances(48, 9924)
    descs = [B.mesh_desc(2, -w.L, w.L, w.n) for w in wl]
    mesh = B.Mesh(descs)
    assert mesh.n_inst == 48
    xyz = mesh.nodes()[0]
    inst = [mesh.instance(i) for i in range(48)]
    prm, oprm, phi = [], [], []
    for i, w in enumerate(wl):
        h = 2 * w.L / w.n
        eps = w.eps_factor * h
        prm.append(B.params(eps=eps, kappa=1e-10, p=w.p))
        oprm.append(OParams(eps=eps, kappa=1e-10, p=w.p))
        nd = inst[i]
        x = xyz[nd["node_offset"]:nd["node_offset"] + nd["n_nodes"]]
        phi.append(crack_band_phi(x, L0, eps, w.center))
    phi = np.concatenate(phi)
    sizes = np.array([(w.n + 1) ** 2 for w in wl])
    return dict(wl=wl, mesh=mesh, inst=inst, prm=prm, oprm=oprm, phi=phi, order=np.argsort(sizes))


def _split(batch, v, i):
    """Solve-order union vector -> instance i's solve-order vector."""
    nd, nf = batch["inst"][i], batch["mesh"].n_free
    f0, nfi = nd["free_offset"], nd["n_free"]
    return np.concatenate([v[2 * f0:2 * (f0 + nfi)], v[2 * nf + f0:2 * nf + f0 + nfi]])


def _nodes(batch, a, i):
    nd = batch["inst"][i]
    return a[nd["node_offset"]:nd["node_offset"] + nd["n_nodes"]]


@pytest.fixture(scope="module")
def solved(batch):
    m = batch["mesh"]
    assert m.n_all > 20_000_000
    u = torch.zeros((m.n_nodes, 2), dtype=torch.float64, device="cuda")
    phi = dev(batch["phi"])
    S = B.System(m).assemble(batch["prm"], u, phi, phi, phi)
    out = {"S": S}
    for prec in (32, 64):
        A = B.Amg(S, B.amg_opts(precision=prec))
        du = torch.empty(m.n_solve, dtype=torch.float64, device="cuda")
        stats = B.solve(S, A, du, B.solve_opts(rtol=1e-10))
        out[prec] = (host(du), stats)
        del A
    return out


def test_every_instance_converges(batch, solved):
    for prec in (32, 64):
        _, stats = solved[prec]
        assert len(stats) == 48
        for i, st in enumerate(stats):
            assert st["status"] == 0 and st["relres"] <= 1e-10, (prec, i, st)
            assert st["iters"] <= 100, (prec, i, st)


def test_smallest_instances_against_exact_oracle_step(batch, solved):
    for i in batch["order"][:3]:
        w = batch["wl"][i]
        om = omesh.uniform(2, -w.L, w.L, w.n)
        phi0 = _nodes(batch, batch["phi"], i)
        u0 = np.zeros((om.n_nodes, 2))
        o = onewton.newton_step_system(om, batch["oprm"][i], u0, phi0, phi0, phi0)
        ref = onewton.solve_block(om, o.Jm, o.F)
        U0 = fem.restrict(om, u0, phi0)
        ur, pr = fem.expand(om, U0 + ref)
        t_ref = ofun.tcv(om, ur, pr)
        for prec in (32, 64):
            d = _split(batch, solved[prec][0], i)
            assert np.linalg.norm(o.F - o.Jm @ d) / np.linalg.norm(o.F) <= 1.01e-10
            ug, pg = fem.expand(om, U0 + d)
            assert abs(ofun.tcv(om, ug, pg) / t_ref - 1) <= 1e-6


def test_largest_instances_sampled_rows(batch, solved):
    R, F, _, _ = solved["S"].vectors()
    R, F = host(R), host(F)
    rng = np.random.default_rng(48)
    for i in batch["order"][-3:]:
        w = batch["wl"][i]
        om = omesh.uniform(2, -w.L, w.L, w.n)
        n1 = w.n + 1
        phi0 = _nodes(batch, batch["phi"], i)
        # sampled nodes: random, and the rows around the crack centre
        cx = int(round((w.center[0] + w.L) / (2 * w.L) * w.n))
        cy = int(round((w.center[1] + w.L) / (2 * w.L) * w.n))
        ii, jj = np.meshgrid(np.arange(cx - 30, cx + 31), np.arange(cy - 5, cy + 6), indexing="ij")
        sample = np.unique(np.concatenate([rng.integers(0, n1 * n1, 600), (ii + n1 * jj).ravel()]))
        i0, j0 = sample % n1, sample // n1
        cells = []
        for di in (-1, 0):
            for dj in (-1, 0):
                ci, cj = i0 + di, j0 + dj
                ok = (ci >= 0) & (ci < w.n) & (cj >= 0) & (cj < w.n)
                cells.append((ci + w.n * cj)[ok])
        cells = np.unique(np.concatenate(cells))
        Ru, Rp, _ = fem.residual_all(om, batch["oprm"][i], np.zeros((om.n_nodes, 2)), phi0, phi0, cells_idx=cells)
        Ri = _split(batch, R, i)
        nf = om.n_free
        scale = np.abs(Ri).max()
        assert np.abs(Ri[2 * sample] - Ru[sample, 0]).max() <= 1e-12 * scale
        assert np.abs(Ri[2 * sample + 1] - Ru[sample, 1]).max() <= 1e-12 * scale
        assert np.abs(Ri[2 * nf + sample] - Rp[sample]).max() <= 1e-12 * scale


def test_fp32_and_fp64_functionals_agree(batch, solved):
    m = batch["mesh"]
    tc = {}
    for prec in (32, 64):
        d = solved[prec][0]
        nf = m.n_free
        u = np.zeros((m.n_nodes, 2))
        phi = batch["phi"].copy()
        free_nodes = np.nonzero(m.nodes()[3] >= 0)[0]
        u[free_nodes] = d[:2 * nf].reshape(-1, 2)
        phi[free_nodes] += d[2 * nf:]
        _, tcv = B.functionals(m, dev(u), dev(phi))
        tc[prec] = np.asarray(tcv)
    assert np.all(np.abs(tc[32] / tc[64] - 1) <= 1e-6)
    assert np.all(tc[64] > 0)
