"""Benchmark: the Newton / active-set loop of one loading step of the 2d Sneddon problem on a
uniform 2048 x 2048 Q1 mesh of [-10, 10]^2 (12,595,203 DoFs), on one MI355X.

One step = reset the state to (u = 0, phi = phi_0) and run the whole loop: assembly of the
residual and masked Jacobian, active set, AMG setup of both diagonal blocks, FGMRES to the
1e-8 relative residual, line search and stop test, repeated until the Newton loop stops.

value = N_solve * (FGMRES iterations summed over the K timed steps) / wall time / 1e6
        (MDoF-iter/s, the whole loop in the denominator).  Also printed: the FGMRES-only
rate, the same loop with the FP32 AMG hierarchy, the per-kernel roofline of the dominant
kernel from HIP events inside the timed region, and the FP64 oracle's rate on the host.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Newton linear-solve MDoF-iter/s + HBM GB/s; FP32-AMG vs FP64 at 1e-8 residual"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=2048, help="cells per axis (2048 is the benchmark workload)")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--cpu-n", type=int, default=512, help="cells per axis of the oracle's sample")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a 1 GiB device copy (reference for the HBM byte counters)")
    ap.add_argument("--refresh-phi", type=int, default=1, help="amg_opts.refresh_phi (0, 1, 2)")
    ap.add_argument("--tune-load", metavar="PATH",
                    help="launch shapes saved by --tune-save: used instead of timing candidates")
    ap.add_argument("--tune-save", metavar="PATH", help="write the tuner's launch shapes at the end")
    ap.add_argument("--levels", action="store_true", help="(kept for old command lines; the hierarchy is always reported)")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


PROFILE_OF = {"cheb_f64_b2_l0": "cheb_f64_b2_sneddon2d_2048.md", "cheb_f64_b2_i16_l0": "cheb_f64_b2_sneddon2d_2048.md",
              "mf_cheb_f64": "mf_cheb_f64_sneddon2d_2048.md", "mf_pcheb_f64": "mf_pcheb_f64_sneddon2d_2048.md",
              "cheb_f64_b3_g16_l1": "cheb_f64_b3_g16_l1_sneddon2d_2048.md",
              "cheb_f64_b3_g4_l1": "cheb_f64_b3_g4_l1_sneddon2d_2048.md"}


def kernel_digest(src_text, kernel):
    """sha256 of a kernel's template definition together with every __device__ helper of the
    same file that it reaches (so a change in a helper counts as a change of the kernel)."""
    import hashlib
    import re
    m = re.search(r"(template <[^\n]*>\n__global__ void __launch_bounds__\(\d+\) " + kernel + r"\(.*?\n\}\n)",
                  src_text, re.S)
    if not m:
        return None
    helpers = {}
    for d in re.finditer(r"((?:template <[^\n]*>\n)?__device__ __forceinline__ [^\n(]*?(\w+)\(.*?\n\}\n)", src_text,
                         re.S):
        helpers[d.group(2)] = d.group(1)
    seen, todo, text = set(), [m.group(1)], m.group(1)
    while todo:
        body = todo.pop()
        for name, h in helpers.items():
            if name not in seen and re.search(r"\b" + name + r"\b", body):
                seen.add(name)
                todo.append(h)
    text += "".join(helpers[n] for n in sorted(seen))
    return hashlib.sha256(text.encode()).hexdigest()


def counted_traffic(kernel):
    """HBM bytes per launch from the committed rocprofv3 PMC summary of this kernel, or None
    when there is none or the kernel's source changed since the counters were taken."""
    import re
    name = PROFILE_OF.get(kernel)
    if not name:
        return None
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    t = re.search(r"^traffic_bytes_per_launch:\s*([0-9.eE+]+)", txt, re.M)
    h = re.search(r"^source: (\S+) kernel (\w+) sha256 prefix ([0-9a-f]+)", txt, re.M)
    if not t or not h:
        return None
    src = os.path.join(ROOT, h.group(1))
    if not os.path.exists(src):
        return None
    cur = kernel_digest(open(src).read(), h.group(2))
    return float(t.group(1)) if cur and cur.startswith(h.group(3)) else None


def cpu_baseline(n_cpu, L_full, n_full):
    """The FP64 oracle as it stands (one exact Newton step: residual, active set, masked Jacobian,
    block forward substitution by sparse LU) on a square of the benchmark mesh with the same h,
    eps and crack, timed on this host.  value = N_solve of the sample / seconds of the step."""
    import numpy as np
    from oracle import mesh as omesh, newton as onewton
    from oracle.material import Params as OParams
    from inputs import crack_band_phi
    h = 2 * L_full / n_full
    L = 0.5 * n_cpu * h
    m = omesh.uniform(2, -L, L, n_cpu)
    prm = OParams(eps=2 * h, kappa=1e-10, p=1e-3)
    phi0 = crack_band_phi(m.coords, 0.25, prm.eps)
    u0 = np.zeros((m.n_nodes, 2))
    c0, t0 = time.process_time(), time.perf_counter()
    st = onewton.newton_step_system(m, prm, u0, phi0, phi0, phi0)
    onewton.solve_block(m, st.Jm, st.F)
    t1, c1 = time.perf_counter(), time.process_time()
    wall = t1 - t0
    cores = max(1, int(round((c1 - c0) / wall)))
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return dict(value=m.n_solve / wall / 1e6, unit="MDoF/s (exact Newton steps)", cores=cores, kind="oracle",
                nproc=os.cpu_count(), usable_cores=usable, seconds_per_newton_step=wall, n_solve=m.n_solve,
                sample=(f"one exact Newton step (assembly + active set + masked Jacobian + sparse-LU block forward "
                        f"substitution; numpy/scipy, SuperLU single-threaded) on [-{L:g},{L:g}]^2 with {n_cpu}^2 "
                        f"cells, the benchmark's h, eps and crack: N_solve={m.n_solve}, {wall:.2f} s; value = "
                        f"N_solve / seconds per exact Newton step (compare newton_step_mdof_per_s)"),
                full_size=(f"not reached: the {n_full}^2 step (16x the sample's DoFs; sparse-LU fill grows faster "
                           f"than the DoFs) is not attempted within the bench's few-minute budget"))


def stream_ceiling(dev, nbytes=2 << 30, reps=10):
    """GB/s of a device copy (read + write counted) and of a read-only reduction over nbytes,
    HIP events on the current stream, after two warm-up passes."""
    import torch
    x = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
    y = torch.empty_like(x)
    res = {}
    for name, fn, moved in (("copy_gbs", lambda: y.copy_(x), 2 * nbytes), ("read_gbs", lambda: x.sum(), nbytes)):
        for _ in range(2):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        e1.synchronize()
        res[name] = moved * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del x, y
    torch.cuda.empty_cache()
    return res


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path; independent instances "
              "would shard across GPUs with no exchange, one large instance by node slabs with one-layer "
              "halos and one all-reduce of the Gram-Schmidt coefficients per FGMRES iteration.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_1806_09924_amd import binding as B
    from inputs import crack_band_phi

    torch.cuda.set_device(0)
    if args.tune_load:
        # the counter runs take the shapes of the traced run: timing under collection can pick others
        with open(args.tune_load) as f:
            B.tune_load(f.read())
    L, n, l0 = 10.0, args.n, 0.25
    h = 2 * L / n
    eps = 2 * h
    log(f"mesh {n}x{n} on [-{L},{L}]^2")
    mesh = B.Mesh(B.mesh_desc(2, -L, L, n))
    xyz = mesh.nodes()[0]
    phi0_h = crack_band_phi(xyz, l0, eps)
    dev = torch.device("cuda:0")
    phi0 = torch.as_tensor(phi0_h, dtype=torch.float64, device=dev)
    u = torch.zeros((mesh.n_nodes, 2), dtype=torch.float64, device=dev)
    phi = phi0.clone()
    prm = B.params(E=1.0, nu=0.2, Gc=1.0, kappa=1e-10, eps=eps, p=1e-3)
    sopts = B.solve_opts(rtol=1e-8, restart=100, maxit=500)
    nopts = B.newton_opts(tol=1e-8, max_it=30, ls_max=8)

    def step(precision):
        u.zero_()
        phi.copy_(phi0)
        amg = B.amg_opts(precision=precision, refresh_phi=args.refresh_phi)
        return B.newton(mesh, prm, u, phi, phi0, phi0, amg=amg, solve=sopts, newton=nopts)

    def run(precision, steps, warmup, profile):
        for i in range(warmup):
            st = step(precision)
            log(f"warmup fp{precision}: newton={st['iterations']} fgmres={st['linear_iters']} "
                f"asm={st['t_assemble']:.3f}s setup={st['t_setup']:.3f}s solve={st['t_solve']:.3f}s")
        torch.cuda.synchronize()
        if profile:
            B.profile(True)
        stats = []
        t0 = time.perf_counter()
        for i in range(steps):
            stats.append(step(precision))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        prof = B.profile_read() if profile else {}
        if profile:
            B.profile(False)
        for st in stats:
            log(f"fp{precision}{' profiled' if profile else ''}: newton={st['iterations']} fgmres={st['linear_iters']} "
                f"asm={st['t_assemble']:.3f}s setup={st['t_setup']:.3f}s solve={st['t_solve']:.3f}s "
                f"other={st['t_other']:.3f}s status={st['status']}")
        return t1 - t0, stats, prof

    # the timed run records no events; the per-kernel table comes from a second, profiled run
    wall, stats, _ = run(64, args.steps, args.warmup, False)
    prof, pstats = {}, []
    if not args.no_profile:
        _, pstats, prof = run(64, args.steps, 0, True)
    iters = sum(s["linear_iters"] for s in stats)
    t_solve = sum(s["t_solve"] for s in stats)
    newton_its = sum(s["iterations"] for s in stats)
    value = mesh.n_solve * iters / wall / 1e6
    cod, tcv = B.functionals(mesh, u, phi, [[h / 2]])
    tcv_exact = 2 * np.pi * 1e-3 * l0 ** 2 * (1 - 0.2 ** 2)
    out = {
        "metric": METRIC, "value": value, "unit": "MDoF-iter/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * wall / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"sneddon2d_{n}: 2d Sneddon, [-10,10]^2, {n}x{n} Q1, eps=2h, l0=0.25, p=1e-3, E=1, "
                               f"nu=0.2, Gc=1, kappa=1e-10, full Newton/active-set loop, FGMRES rtol 1e-8, "
                               f"FP64 SA-AMG block preconditioner",
                   "n_solve": mesh.n_solve, "n_all": mesh.n_all},
        "newton_iterations_per_step": newton_its / args.steps,
        "fgmres_iterations_per_newton": iters / max(1, newton_its),
        "solve_only_mdof_iter_s": mesh.n_solve * iters / t_solve / 1e6,
        # iteration-count independent: DoFs brought to the converged Newton solution per second
        # (a better preconditioner lowers MDoF-iter/s while it shortens the loop)
        "loop_mdof_per_s": mesh.n_solve * args.steps / wall / 1e6,
        # N_solve per second of Newton steps (assembly, setup, solve, line search): the unit of
        # the oracle's cpu_baseline
        "newton_step_mdof_per_s": mesh.n_solve * newton_its / wall / 1e6,
        "phase_seconds_per_step": {k: sum(s[k] for s in stats) / args.steps
                                   for k in ("t_assemble", "t_setup", "t_solve", "t_other")},
        "tcv": tcv, "tcv_sneddon": tcv_exact, "tcv_rel_err_vs_sneddon": tcv / tcv_exact - 1,
        "cod_center": float(cod[0]),
    }
    if prof:
        kern = {k: v for k, v in prof.items() if not k.startswith(("vcycle", "setup_"))}
        dom = max(kern, key=lambda k: kern[k]["ms"])
        d = kern[dom]
        avg_ms = d["ms"] / d["launches"]
        bytes_per = d["bytes"] / d["launches"]
        ach = bytes_per / (avg_ms * 1e-3) / 1e9
        out["roofline"] = {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": ach / HBM_PEAK_GBS, "traffic": counted_traffic(dom),
                           "bytes_per_launch": bytes_per, "avg_launch_ms": avg_ms, "launches": d["launches"]}
        # the whole FGMRES iteration and the V-cycle pair: algorithmic bytes of every solve-phase
        # kernel (smoothers, transfers and coarse products of both hierarchies; J-SpMV;
        # Gram-Schmidt) per iteration of the profiled run, over the timed run's FGMRES time per
        # iteration and over the V-cycle window (the two cycles run on two streams at once: the
        # longer of the two per-cycle times)
        p_iters = sum(s_["linear_iters"] for s_ in pstats)
        vc_names = [k for k in kern if k.startswith(("cheb_", "spmv_", "mf_"))]
        vc_bytes = sum(kern[k]["bytes"] for k in vc_names) / p_iters
        it_bytes = sum(v["bytes"] for v in kern.values()) / p_iters
        vc_ms = max(prof[k]["ms"] / prof[k]["launches"] for k in ("vcycle_u", "vcycle_phi") if k in prof)
        it_ms = 1e3 * t_solve / iters
        out["roofline"]["vcycle"] = {"bytes_per_iteration": vc_bytes, "ms_per_iteration": vc_ms,
                                     "achieved": vc_bytes / (vc_ms * 1e-3) / 1e9,
                                     "frac": vc_bytes / (vc_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                     "kernels": sorted(vc_names)}
        out["roofline"]["iteration"] = {"bytes_per_iteration": it_bytes, "ms_per_iteration": it_ms,
                                        "achieved": it_bytes / (it_ms * 1e-3) / 1e9,
                                        "frac": it_bytes / (it_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        # what this device's HBM sustains for plain streams (context for frac; peak stays the
        # published 8 TB/s)
        out["roofline"]["measured_ceiling"] = stream_ceiling(dev)
        out["kernels"] = {k: {"launches": v["launches"], "ms_total": v["ms"],
                              "gbs": (v["bytes"] / (v["ms"] * 1e-3) / 1e9) if v["ms"] > 0 and v["bytes"] > 0 else None}
                          for k, v in sorted(prof.items(), key=lambda kv: -kv[1]["ms"])}
    if not args.no_fp32:
        w32, s32, _ = run(32, args.steps, 1, False)
        p32 = {} if args.no_profile else run(32, args.steps, 0, True)[2]
        it32 = sum(s["linear_iters"] for s in s32)
        ts32 = sum(s["t_solve"] for s in s32)
        v32 = mesh.n_solve * it32 / w32 / 1e6
        out["fp32_amg"] = {
            "value": v32, "ms_per_step": 1e3 * w32 / args.steps,
            "fgmres_iterations_per_newton": it32 / max(1, sum(s["iterations"] for s in s32)),
            "solve_only_mdof_iter_s": mesh.n_solve * it32 / ts32 / 1e6,
            "speedup_whole_step": (wall / args.steps) / (w32 / args.steps),
            "speedup_time_to_solution": t_solve / ts32,
            "vcycle_ms": {k: v["ms"] for k, v in p32.items() if k.startswith("vcycle")},
            "kernels": {k: {"launches": v["launches"], "ms_total": v["ms"],
                            "gbs": (v["bytes"] / (v["ms"] * 1e-3) / 1e9) if v["ms"] > 0 and v["bytes"] > 0 else None}
                        for k, v in sorted(p32.items(), key=lambda kv: -kv[1]["ms"]) if not k.startswith("setup_")},
        }
        if prof:
            out["fp32_amg"]["vcycle_ms_fp64"] = {k: v["ms"] for k, v in prof.items() if k.startswith("vcycle")}
    # the hierarchy of the first Newton step: level sizes and the launch shapes the tuner
    # picked (SELL slice height, lanes per row) for each level's A, P, R
    u.zero_()
    phi.copy_(phi0)
    S = B.System(mesh).assemble(prm, u, phi, phi0, phi0)
    A = B.Amg(S, B.amg_opts(precision=64))
    lv = {}
    for blk, nm in ((0, "u"), (1, "phi")):
        nl = A.n_levels(blk)
        lv[nm] = []
        for lev in range(nl):
            d = A.level_info(blk, lev)
            d["shape"] = {w: list(A.level_shape(blk, lev, i)) for i, w in enumerate("APR") if i == 0 or lev + 1 < nl}
            lv[nm].append(d)
    out["amg_levels"] = lv
    del A, S
    if args.calibrate_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = {"read": src.numel() * 8, "write": dst.numel() * 8}
    if args.tune_save:
        with open(args.tune_save, "w") as f:
            f.write(B.tune_table())
    if not args.no_cpu:
        log("oracle timing on the host")
        out["cpu_baseline"] = cpu_baseline(args.cpu_n, L, n)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
