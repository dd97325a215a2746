"""Parameter studies of Section 4 run on the batched path (every instance of a study in one
disjoint-union system, one Newton / active-set loop for all of them).

domain_size(): Section 4.2, the influence of the finite domain on the TCV of the 2d Sneddon
crack with l0 = 1.  For every domain the TCV is computed at several mesh levels (eps = 2 h)
and extrapolated in h; the paper reports the extrapolated value's error against the exact
6.0319E-03 as 5.6 %, 1.5 %, 0.5 % and 0.1 % for the domains 10x10 ... 80x80.

cod_convergence(): Section 4.4, the crack opening displacement on one domain under adaptive
and under global refinement (eps = 2 h_min on every mesh), each family's reference value by
Richardson extrapolation of its own three finest levels, and the observed orders of the errors
against h and against the number of DoFs.

convergence_3d(): Section 4.3, the TCV of the 3d penny crack (l0 = 1, 10 x 10 x 10 domain) on
adaptive meshes whose finest edge is 10 l0 / 2^ref, with eps = 2 x the finest cell's diameter
(the eps column of the Fig. 3 table), against Sneddon's 5.12E-03.

loading_refinement(): the algorithm around the Newton solve (Section 3) on one Sneddon mesh: a
loading step at half the load, crack-region and gradient-jump marks, refinement, transfer of u,
phi and the previous phase field, and the step at the full load on the refined mesh, each stage
timed.

launch_cost(): milliseconds per FGMRES iteration with the captured Arnoldi step and with direct
launches, on a launch-bound 50 k-DoF mesh and on the 48-instance batch.

Run as `python -m paper_1806_09924_amd.studies [domain|cod|3d|refine|launch] [64|32]` (prints one
JSON object).
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


def richardson(values):
    """Reference value and observed order from the last three entries of a sequence computed
    on meshes whose h halves from one entry to the next: with C_h = C* + a h^q,
    q = log2((C_2h - C_4h) / (C_h - C_2h)) and C* = C_h + (C_h - C_2h) / (2^q - 1)."""
    c4, c2, c1 = (float(v) for v in values[-3:])
    d_coarse, d_fine = c2 - c4, c1 - c2
    if d_fine == 0.0 or d_coarse / d_fine <= 0.0:
        raise ValueError("richardson: the last three values do not converge monotonically")
    q = float(np.log2(d_coarse / d_fine))
    return c1 + d_fine / (2.0 ** q - 1.0), q


def _solve_family(descs, l0, xs, precision, rtol):
    """One batched Newton loop over meshes of one family; COD at xs and DoFs per mesh."""
    from inputs import crack_band_phi   # the workloads' initial crack field
    mesh = B.Mesh(descs)
    xyz = mesh.nodes()[0]
    ni = len(descs)
    inst = [mesh.instance(i) for i in range(ni)]
    phi0 = np.zeros(mesh.n_nodes)
    prms = []
    for i, nd in enumerate(inst):
        eps = 2.0 * nd["h_min"]
        sl = slice(nd["node_offset"], nd["node_offset"] + nd["n_nodes"])
        phi0[sl] = crack_band_phi(xyz[sl], l0, eps)
        prms.append(B.params(eps=eps, kappa=1e-10, p=1e-3))
    dev = torch.device("cuda")
    p0 = torch.as_tensor(phi0, device=dev)
    u = torch.zeros((mesh.n_nodes, 2), dtype=torch.float64, device=dev)
    phi = p0.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = B.newton(mesh, prms, u, phi, p0, p0, amg=B.amg_opts(precision=precision), solve=B.solve_opts(rtol=rtol))
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    st = st if isinstance(st, list) else [st]
    cx = np.array([[[x] for x in xs]] * ni)
    cod, _ = B.functionals(mesh, u, phi, cx if ni > 1 else cx[0])
    for i in range(ni):
        assert st[i]["status"] == 0, (i, st[i])
    return dict(h=[nd["h_min"] for nd in inst], n_dofs=[3 * nd["n_nodes"] for nd in inst],
                cod=np.asarray(cod).reshape(ni, len(xs)).T.tolist(), newton=[s["iterations"] for s in st],
                t_newton=t)


def _orders(h, n, err):
    e = np.asarray(err, dtype=float)
    return dict(vs_h=np.log2(e[:-1] / e[1:]).tolist(),
                vs_dofs=(np.log(e[:-1] / e[1:]) / np.log(np.asarray(n[1:], float) / np.asarray(n[:-1], float))).tolist())


def cod_convergence(half_width, levels, refine_radius, l0=1.0, xs=(0.0, 0.5), precision=64, rtol=1e-10):
    """COD at the points xs along the crack (x_0 = xs, through the crack) under adaptive
    refinement (base cells of edge 1, `levels` within refine_radius of the crack) and global
    refinement of the same h_min, each with its Richardson reference from its three finest
    levels (the global family stops one level short of the adaptive one: the finest global
    mesh is the largest).  Returns the values, references, errors and observed orders."""
    L = float(half_width)
    n0 = int(round(2 * L))
    ad = _solve_family([B.mesh_desc(2, -L, L, n0, levels=k, refine_radius=refine_radius, crack_half_len=l0)
                        for k in levels], l0, xs, precision, rtol)
    gl = _solve_family([B.mesh_desc(2, -L, L, n0 << k) for k in levels[:-1]], l0, xs, precision, rtol)
    out = dict(domain=2 * L, l0=l0, xs=list(xs), refine_radius=refine_radius, adaptive=ad, global_=gl)
    for fam in (ad, gl):
        fam["reference"], fam["order_richardson"], fam["errors"], fam["orders"] = [], [], [], []
        for k in range(len(xs)):
            ref, q = richardson(fam["cod"][k])
            err = [abs(c - ref) for c in fam["cod"][k]]
            fam["reference"].append(ref)
            fam["order_richardson"].append(q)
            fam["errors"].append(err)
            fam["orders"].append(_orders(fam["h"][:-1], fam["n_dofs"][:-1], err[:-1]))
    return out


def convergence_3d(refs=(7, 8, 9), refine_radius=0.4, precision=32, rtol=1e-8, steps=1):
    """The refs' meshes in one batch: base 16^3 cells of edge 10/16 (ref 4), ref - 4 levels within
    refine_radius of the crack disk, eps = 2 sqrt(3) h_min.  steps = 1: one Newton loop from the
    sharp initial crack (phi_tilde = phi_old = phi_0).  steps > 1: that many quasi-static loading
    steps at the constant pressure (fracture_loading: phi_old the previous step's phase field,
    phi_tilde extrapolated in time), the phase field relaxing from the sharp initial band to its
    stationary profile; the later steps start at equilibrium, so their Newton stop test has the
    absolute floor 1e-8 x the smallest first-step residual.  Returns per ref the DoFs (4 per
    node), eps, the TCV after every step, and the final TCV's relative error against Sneddon's
    closed form."""
    from inputs import crack_band_phi   # the workloads' initial crack field
    descs = [B.mesh_desc(3, -5.0, 5.0, 16, levels=r - 4, refine_radius=refine_radius, crack_half_len=1.0)
             for r in refs]
    t0 = time.perf_counter()
    mesh = B.Mesh(descs)
    t_mesh = time.perf_counter() - t0
    xyz = mesh.nodes()[0]
    inst = [mesh.instance(i) for i in range(len(refs))]
    phi0 = np.zeros(mesh.n_nodes)
    prms, epss = [], []
    for i, nd in enumerate(inst):
        eps = 2.0 * np.sqrt(3.0) * nd["h_min"]
        sl = slice(nd["node_offset"], nd["node_offset"] + nd["n_nodes"])
        phi0[sl] = crack_band_phi(xyz[sl], 1.0, eps)
        prms.append(B.params(eps=eps, kappa=1e-10, p=1e-3))
        epss.append(eps)
    dev = torch.device("cuda")
    p0 = torch.as_tensor(phi0, device=dev)
    u = torch.zeros((mesh.n_nodes, 3), dtype=torch.float64, device=dev)
    phi = p0.clone()
    amg, sol = B.amg_opts(precision=precision), B.solve_opts(rtol=rtol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    one = lambda x: x if isinstance(x, list) else [x]  # one ref: the binding returns one dict
    st1, tcv1 = B.loading(mesh, [prms], [0.0, 1.0], u, phi, amg=amg, solve=sol)
    stats = [one(st1[0])]
    tcvs = [np.atleast_1d(tcv1)[:len(refs)] if len(refs) > 1 else np.atleast_1d(tcv1)]
    if steps > 1:
        atol = 1e-8 * min(s["res0"] for s in stats[0])
        st, tcv = B.loading(mesh, [prms] * (steps - 1), np.arange(1.0, steps + 1.0), u, phi, phi_prev=p0,
                            t_prev=0.0, amg=amg, solve=sol, newton=B.newton_opts(atol=atol))
        tcv = np.asarray(tcv).reshape(steps - 1, len(refs))
        for k in range(steps - 1):
            stats.append(one(st[k]))
            tcvs.append(tcv[k])
    torch.cuda.synchronize()
    t_newton = time.perf_counter() - t0
    exact = 16.0 * 1e-3 * 1.0 ** 3 * (1 - 0.2 ** 2) / (3.0 * 1.0)
    rows = []
    for i, r in enumerate(refs):
        for k in range(len(stats)):
            assert stats[k][i]["status"] == 0, (r, k, stats[k][i])
        t_steps = [float(np.asarray(t).reshape(-1)[i]) for t in tcvs]
        rows.append(dict(ref=r, ten_l0_over_h=2 ** r,
                         h_min=inst[i]["h_min"], n_dofs=4 * inst[i]["n_nodes"], eps=epss[i], tcv=t_steps[-1],
                         tcv_steps=t_steps, rel_error=float(t_steps[-1] / exact - 1),
                         rel_error_first_step=float(t_steps[0] / exact - 1),
                         newton=[s[i]["iterations"] for s in stats], fgmres=[s[i]["linear_iters"] for s in stats]))
    return dict(rows=rows, exact=exact, refine_radius=refine_radius, precision=precision, steps=steps,
                t_mesh=t_mesh, t_newton=t_newton, n_dofs=int(4 * mesh.n_nodes))


def loading_refinement(n=2048, L=10.0, l0=0.25, kelly_fraction=0.01, precision=64):
    """Two loading steps (p/2, then p) on the n x n Sneddon mesh with one refinement between them:
    crack-region marks (phi < 1/2 on cells coarser than h/2) and the cells in the top
    `kelly_fraction` of the gradient-jump indicator are split.  Returns per-stage seconds, the
    Newton / FGMRES counts and TCV of both steps, and the mesh sizes."""
    from inputs import crack_band_phi   # the workload's initial crack field
    dev = torch.device("cuda")

    def now():
        torch.cuda.synchronize()
        return time.perf_counter()

    out = {}
    t0 = now()
    m = B.Mesh(B.mesh_desc(2, -L, L, n))
    out["t_mesh"] = now() - t0
    h = 2 * L / n
    eps = 2 * h
    phi0 = torch.as_tensor(crack_band_phi(m.nodes()[0], l0, eps), device=dev)
    u = torch.zeros((m.n_nodes, 2), dtype=torch.float64, device=dev)
    phi = phi0.clone()
    prm = [B.params(eps=eps, kappa=1e-10, p=5e-4), B.params(eps=eps, kappa=1e-10, p=1e-3)]
    amg, so, no = B.amg_opts(precision=precision), B.solve_opts(rtol=1e-8), B.newton_opts(atol=1e-13)
    t0 = now()
    st1, tcv1 = B.loading(m, prm[:1], [0.0, 1.0], u, phi, amg=amg, solve=so, newton=no)
    out["t_step1"] = now() - t0
    eta = torch.empty(m.n_cells, dtype=torch.float64, device=dev)
    t0 = now()
    B.kelly(m, u, eta)
    crack, n_crack = B.mark_crack(m, phi, 0.5, h / 2)
    e = eta.cpu().numpy()
    flags = crack | (e > np.quantile(e, 1.0 - kelly_fraction)).astype(np.uint8)
    out["t_mark"] = now() - t0
    t0 = now()
    m2 = m.refine(flags)
    out["t_refine"] = now() - t0
    u2 = torch.empty((m2.n_nodes, 2), dtype=torch.float64, device=dev)
    phi2 = torch.empty(m2.n_nodes, dtype=torch.float64, device=dev)
    prev2 = torch.empty(m2.n_nodes, dtype=torch.float64, device=dev)
    t0 = now()
    B.transfer(m, m2, u, u2)
    B.transfer(m, m2, phi, phi2)
    B.transfer(m, m2, phi0, prev2)
    out["t_transfer"] = now() - t0
    t0 = now()
    st2, tcv2 = B.loading(m2, prm[1:], [1.0, 2.0], u2, phi2, phi_prev=prev2, t_prev=0.0, amg=amg, solve=so,
                          newton=no)
    out["t_step2"] = now() - t0
    for s_ in st1 + st2:
        assert s_["status"] == 0, s_
    out.update(cells=[m.n_cells, m2.n_cells], n_solve=[m.n_solve, m2.n_solve], hanging=m2.n_hanging,
               marked=int(flags.sum()), crack_marked=int(n_crack),
               newton=[st1[0]["iterations"], st2[0]["iterations"]],
               fgmres=[st1[0]["linear_iters"], st2[0]["linear_iters"]], tcv=[float(tcv1[0]), float(tcv2[0])])
    return out


def launch_cost(repeats=5, batch=True):
    """Time per FGMRES iteration with the captured Arnoldi step (one graph launch per iteration)
    and with direct launches, on the 128 x 128 mesh of [-2, 2]^2 (50 k DoFs: launch bound) and on
    the 48-instance batch of the batched studies (46.8 M DoFs): one Newton step's solve to 1e-8,
    FP64 hierarchy, repeated; wall and host CPU milliseconds per iteration (the best repeat;
    the first graph solve after a setup, which captures the step, is reported apart)."""
    from inputs import crack_band_phi, batched_instances

    def measure(mesh, prm, phi0):
        u = torch.zeros((mesh.n_nodes, mesh.dim), dtype=torch.float64, device="cuda")
        phi = torch.as_tensor(phi0, dtype=torch.float64, device="cuda")
        S = B.System(mesh).assemble(prm, u, phi, phi, phi)
        A = B.Amg(S)
        du = torch.empty(mesh.n_solve, dtype=torch.float64, device="cuda")
        row = {"n_solve": mesh.n_solve}
        for g in (0, 1):
            best = None
            for r in range(repeats + 1):
                if g == 1 and r == 0:
                    A.setup()            # a fresh setup: the first graph solve captures the step
                torch.cuda.synchronize()
                c0, t0 = time.process_time(), time.perf_counter()
                st = B.solve(S, A, du, B.solve_opts(use_graphs=g))
                torch.cuda.synchronize()
                t1, c1 = time.perf_counter(), time.process_time()
                its = st["iters"] if isinstance(st, dict) else max(x["iters"] for x in st)
                cur = (1e3 * (t1 - t0) / its, 1e3 * (c1 - c0) / its, its)
                if g == 1 and r == 0:
                    row["graph_first_solve_ms"] = 1e3 * (t1 - t0)
                    continue
                if best is None or cur[0] < best[0]:
                    best = cur
            key = "graph" if g else "direct"
            row[key] = {"wall_ms_per_iter": best[0], "host_cpu_ms_per_iter": best[1], "iters": best[2]}
        return row

    out = {}
    L, n = 2.0, 128
    m = B.Mesh(B.mesh_desc(2, -L, L, n))
    eps = 2 * 2 * L / n
    out["sneddon2d_128"] = measure(m, B.params(eps=eps), crack_band_phi(m.nodes()[0], 0.25, eps))
    if batch:
        ws = batched_instances()
        descs = [B.mesh_desc(2, -w.L, w.L, w.n) for w in ws]
        bm = B.Mesh(descs)
        xyz = bm.nodes()[0]
        phis = []
        for i, w in enumerate(ws):
            nd = bm.instance(i)
            phis.append(crack_band_phi(xyz[nd["node_offset"]:nd["node_offset"] + nd["n_nodes"]], w.l0, w.eps,
                                       (w.center[0], w.center[1], 0.0)))
        out["batch48"] = measure(bm, [B.params(**w.params()) for w in ws], np.concatenate(phis))
    return out


def main(argv=None):
    argv = list(argv or [])
    which = argv.pop(0) if argv and argv[0] in ("domain", "cod", "3d", "refine", "launch") else "domain"
    precision = int(argv[0]) if argv else 64
    if which == "launch":
        print(json.dumps(launch_cost()))
        return
    if which == "refine":
        print(json.dumps(loading_refinement(precision=precision)))
        return
    if which == "3d":
        refs = tuple(int(r) for r in argv[1].split(",")) if len(argv) > 1 else (7, 8, 9)
        steps = int(argv[2]) if len(argv) > 2 else 1
        print(json.dumps(convergence_3d(refs=refs, precision=precision, steps=steps)))
        return
    if which == "cod":
        from inputs import cod_study
        c = cod_study()
        out = cod_convergence(c["half_width"], c["levels"], c["refine_radius"], precision=precision)
        print(json.dumps(out))
        return
    from inputs import domain_study
    ws = domain_study()
    exact = 2 * np.pi * 1e-3 * 1.0 ** 2 * (1 - 0.2 ** 2) / 1.0
    out = domain_size(ws, precision=precision, exact=exact)
    out["exact"] = exact
    print(json.dumps(out))


if __name__ == "__main__":
    main(sys.argv[1:])
