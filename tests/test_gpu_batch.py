"""Batched instances (the domain-size / eps studies of Section 4 solved together): the union
mesh, per-instance parameters, per-instance convergence of FGMRES and per-instance
functionals, each instance checked against the oracle on that instance alone."""
import numpy as np
import pytest
import torch

from paper_1806_09924_amd import binding as B
from oracle import mesh as omesh, fem, newton as onewton, functionals as ofun
from oracle.material import Params as OParams
from inputs import crack_band_phi
from gpu_util import dev, host

pytestmark = pytest.mark.gpu

INST = [  # (L, N, eps factor, p, crack centre)
    (0.75, 24, 2.0, 5e-4, (0.02, -0.01)),
    (1.0, 32, 4.0, 1e-3, (-0.05, 0.03)),
    (1.2, 40, 2.0, 1.5e-3, (0.0, 0.0)),
    (1.5, 48, 4.0, 2e-3, (0.08, -0.06)),
]


class Batch:
    def __init__(self, kappa=1e-10, l0=0.25):
        self.descs = [B.mesh_desc(2, -L, L, N) for (L, N, _, _, _) in INST]
        self.mesh = B.Mesh(self.descs)
        assert self.mesh.n_inst == len(INST)
        self.inst = [self.mesh.instance(i) for i in range(len(INST))]
        self.om, self.prm, self.oprm, self.state = [], [], [], []
        xyz = self.mesh.nodes()[0]
        for i, (L, N, fac, p, c) in enumerate(INST):
            om = omesh.uniform(2, -L, L, N)
            eps = fac * 2 * L / N
            self.om.append(om)
            self.prm.append(B.params(eps=eps, kappa=kappa, p=p))
            self.oprm.append(OParams(eps=eps, kappa=kappa, p=p))
            nd = self.inst[i]
            assert np.allclose(xyz[nd["node_offset"]:nd["node_offset"] + nd["n_nodes"]], om.coords, atol=1e-14)
            phi0 = crack_band_phi(om.coords, l0, eps, (c[0], c[1], 0.0))
            self.state.append((np.zeros((om.n_nodes, 2)), phi0))
        self.nf = self.mesh.n_free

    def union(self, k):
        return dev(np.concatenate([s[k].ravel() for s in self.state]).reshape(-1, 2) if k == 0 else
                   np.concatenate([s[k] for s in self.state]))

    def split(self, v, i):
        """Solve-order union vector -> instance i's solve-order vector."""
        nd = self.inst[i]
        f0, nfi = nd["free_offset"], nd["n_free"]
        return np.concatenate([v[2 * f0:2 * (f0 + nfi)], v[2 * self.nf + f0:2 * self.nf + f0 + nfi]])

    def split_nodes(self, a, i):
        nd = self.inst[i]
        return a[nd["node_offset"]:nd["node_offset"] + nd["n_nodes"]]


def test_batched_assembly_matches_per_instance_oracle():
    bt = Batch()
    u, phi = bt.union(0), bt.union(1)
    S = B.System(bt.mesh).assemble(bt.prm, u, phi, phi, phi)
    R, F, _, _ = S.vectors()
    R, F = host(R), host(F)
    for i in range(len(INST)):
        o = onewton.newton_step_system(bt.om[i], bt.oprm[i], bt.state[i][0], bt.state[i][1], bt.state[i][1],
                                       bt.state[i][1])
        assert np.abs(bt.split(R, i) - o.R).max() <= 1e-12 * np.abs(o.R).max()
        assert np.abs(bt.split(F, i) - o.F).max() <= 1e-12 * np.abs(o.F).max()


@pytest.mark.parametrize("precision", [64, 32])
def test_batched_solve_per_instance(precision):
    bt = Batch()
    u, phi = bt.union(0), bt.union(1)
    S = B.System(bt.mesh).assemble(bt.prm, u, phi, phi, phi)
    A = B.Amg(S, B.amg_opts(precision=precision))
    du = torch.empty(bt.mesh.n_solve, dtype=torch.float64, device="cuda")
    for rtol, fbar in ((1e-8, 5e-6), (1e-10, 1e-6)):
        stats = B.solve(S, A, du, B.solve_opts(rtol=rtol))
        d = host(du)
        U = []
        for i in range(len(INST)):
            o = onewton.newton_step_system(bt.om[i], bt.oprm[i], bt.state[i][0], bt.state[i][1], bt.state[i][1],
                                           bt.state[i][1])
            di = bt.split(d, i)
            assert stats[i]["status"] == 0 and stats[i]["relres"] <= rtol
            assert np.linalg.norm(o.F - o.Jm @ di) / np.linalg.norm(o.F) <= 1.01 * rtol
            ref = onewton.solve_block(bt.om[i], o.Jm, o.F)
            U0 = fem.restrict(bt.om[i], bt.state[i][0], bt.state[i][1])
            ug, pg = fem.expand(bt.om[i], U0 + di)
            ur, pr = fem.expand(bt.om[i], U0 + ref)
            U.append((ug, pg, ofun.tcv(bt.om[i], ur, pr)))
        ug = dev(np.concatenate([x[0] for x in U]))
        pg = dev(np.concatenate([x[1] for x in U]))
        _, tcv = B.functionals(bt.mesh, ug, pg)
        for i in range(len(INST)):
            assert abs(tcv[i] / U[i][2] - 1) <= fbar, (i, rtol, tcv[i] / U[i][2] - 1)


def test_batched_cod_per_instance():
    bt = Batch()
    rng = np.random.default_rng(2)
    u = rng.standard_normal((bt.mesh.n_nodes, 2)) * 1e-3
    phi = rng.uniform(0, 1, bt.mesh.n_nodes)
    xs = np.array([[[0.0125], [0.3]] for _ in INST])
    cod, tcv = B.functionals(bt.mesh, dev(u), dev(phi), xs)
    for i in range(len(INST)):
        ui, pi = bt.split_nodes(u, i), bt.split_nodes(phi, i)
        assert abs(tcv[i] - ofun.tcv(bt.om[i], ui, pi)) <= 1e-13 * abs(tcv[i]) + 1e-18
        for k in range(2):
            ref = ofun.cod(bt.om[i], ui, pi, xs[i, k])
            assert abs(cod[i, k] - ref) <= 1e-13 * abs(ref) + 1e-18
