"""Parameter studies of Section 4 run on the batched path (every instance of a study in one
disjoint-union system, one Newton / active-set loop for all of them).

domain_size(): Section 4.2, the influence of the finite domain on the TCV of the 2d Sneddon
crack with l0 = 1.  For every domain the TCV is computed at several mesh levels (eps = 2 h)
and extrapolated in h; the paper reports the extrapolated value's error against the exact
6.0319E-03 as 5.6 %, 1.5 %, 0.5 % and 0.1 % for the domains 10x10 ... 80x80.

Run as `python -m paper_1806_09924_amd.studies` (prints one JSON object).
"""
import json
import sys
import time

import numpy as np
import torch

from . import binding as B


def domain_size(workloads, precision=64, rtol=1e-8, exact=None):
    """Solves every workload of the study in one batch; returns per-domain rows with the
    TCV per level, the extrapolated TCV and its relative error against `exact`."""
    from inputs import crack_band_phi   # the workloads' initial crack field
    descs = [B.mesh_desc(2, -w.L, w.L, w.n, levels=w.levels, refine_radius=w.refine_radius, crack_half_len=w.l0)
             for w in workloads]
    t0 = time.perf_counter()
    mesh = B.Mesh(descs)
    t_mesh = time.perf_counter() - t0
    xyz = mesh.nodes()[0]
    inst = [mesh.instance(i) for i in range(len(workloads))]
    phi0 = np.zeros(mesh.n_nodes)
    prms = []
    for i, w in enumerate(workloads):
        nd = inst[i]
        eps = w.eps_factor * nd["h_min"]
        sl = slice(nd["node_offset"], nd["node_offset"] + nd["n_nodes"])
        phi0[sl] = crack_band_phi(xyz[sl], w.l0, eps, w.center)
        prms.append(B.params(E=w.E, nu=w.nu, Gc=w.Gc, kappa=w.kappa, eps=eps, p=w.p))
    dev = torch.device("cuda")
    phi0_d = torch.as_tensor(phi0, device=dev)
    u = torch.zeros((mesh.n_nodes, 2), dtype=torch.float64, device=dev)
    phi = phi0_d.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = B.newton(mesh, prms, u, phi, phi0_d, phi0_d, amg=B.amg_opts(precision=precision),
                  solve=B.solve_opts(rtol=rtol))
    torch.cuda.synchronize()
    t_newton = time.perf_counter() - t0
    _, tcv = B.functionals(mesh, u, phi)
    rows = {}
    for i, w in enumerate(workloads):
        r = rows.setdefault(2 * w.L, dict(domain=2 * w.L, h=[], tcv=[], n_dofs=[], newton=[], fgmres=[]))
        r["h"].append(inst[i]["h_min"])
        r["tcv"].append(float(tcv[i]))
        r["n_dofs"].append(3 * inst[i]["n_nodes"])
        r["newton"].append(st[i]["iterations"])
        r["fgmres"].append(st[i]["linear_iters"])
        assert st[i]["status"] == 0, (w.name, st[i])
    for r in rows.values():
        h, t = np.array(r["h"]), np.array(r["tcv"])
        # eps = 2h: the functional converges linearly in eps; Richardson from the two finest
        # levels (h halves between levels)
        r["tcv_extrapolated"] = float(2 * t[-1] - t[-2])
        if exact:
            r["rel_error_extrapolated"] = float(r["tcv_extrapolated"] / exact - 1)
            r["rel_error_finest"] = float(t[-1] / exact - 1)
    return dict(rows=sorted(rows.values(), key=lambda r: r["domain"]), n_inst=len(workloads),
                n_dofs=int(3 * mesh.n_nodes), t_mesh=t_mesh, t_newton=t_newton, precision=precision)


def main(argv=None):
    from inputs import domain_study
    ws = domain_study()
    exact = 2 * np.pi * 1e-3 * 1.0 ** 2 * (1 - 0.2 ** 2) / 1.0
    out = domain_size(ws, precision=int(argv[0]) if argv else 64, exact=exact)
    out["exact"] = exact
    print(json.dumps(out))


if __name__ == "__main__":
    main(sys.argv[1:])
