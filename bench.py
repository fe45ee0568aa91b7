"""Benchmark: time-to-tolerance of the SGML solve on one MI355X.

One step = one full solve (every cycle of Algorithm 3 plus the FP64
residual recurrence) to relative residual 1e-12 on the 4097^2 2D Poisson
workload with mixed Dirichlet (x-walls) / Neumann (y-walls) faces and 64
Gaussian blobs, inputs resident in HBM.  The headline value is the mixed
precision solve (FP32 cycle, FP64 refinement); the plain FP64 solve of the
same workload is timed beside it.  The other workloads (129^2 sine Poisson,
257^3 sphere medium, 129^3 forward + adjoint, 513^3 charges forward +
adjoint) are timed after it and reported under "configs".  Prints one JSON
line.
"""
import argparse
import hashlib
import json
import os
import platform
import re
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GNodes/s to rel. residual 1e-12 (FP64 vs FP32+FP64-refine); % HBM peak"
HBM_PEAK_GBS = 8000.0
TOL = 1e-12


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-configs", action="store_true", help="time the headline workload only")
    ap.add_argument("--workload", default="poisson2d_blobs")
    ap.add_argument("--study", action="store_true",
                    help="only run the convergence study of Sec. 3.1 (eq. 8 at 1025^2)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of known size (for HBM counter calibration)")
    return ap.parse_args()


def copy_calibration():
    """A plain copy of 1 GiB, three times: FETCH_SIZE / WRITE_SIZE of these
    dispatches against the known 1 GiB give the counters' scale."""
    import torch
    a = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": a.numel() * 4, "copies": 3}), flush=True)


def kernel_source_hash():
    src = os.path.join(ROOT, "paper_1703_07206_amd", "csrc", "sgml_visit2d_impl.h")
    with open(src, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def measured_traffic(kernel, nodes):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (profiles/traffic_*.md), scaled by the copy calibration; None when the
    summary is missing or was taken on another version of the kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic_visit2d_poisson2d_blobs_4097.md")
    if not os.path.exists(path):
        return None
    m = re.search(r"```json\n(.*?)\n```", open(path).read(), re.S)
    if not m:
        return None
    rec = json.loads(m.group(1))
    if rec.get("source_sha256_16") != kernel_source_hash() or kernel not in rec.get("kernels", {}):
        return None
    k = rec["kernels"][kernel]
    fetch = k["fetch_kib"] * 1024 * rec["fetch_scale"]
    write = k["write_kib"] * 1024 * rec["write_scale"]
    return {"bytes_per_launch": fetch + write, "fetch_bytes": fetch, "write_bytes": write,
            "bytes_per_node": (fetch + write) / nodes}


def host_cpu():
    """Model name and logical CPU count of the host."""
    model = platform.processor() or "unknown"
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return model, os.cpu_count()


def cpu_baseline(wl, cycles):
    """The FP64 oracle on the host cores: one cycle of the same workload
    (about 5-30 s), scaled by the cycle count the solve needs."""
    from oracle.core import OracleProblem, threads
    P = OracleProblem(wl.dim, wl.n, wl.stencil, wl.faces, wl.a, wl.sigma)
    t0 = time.perf_counter()
    P.cycle(wl.f, G=wl.G)
    t_cycle = time.perf_counter() - t0
    t_solve = t_cycle * cycles
    model, ncpu = host_cpu()
    return {"value": wl.nodes / t_solve / 1e9, "unit": "GNodes/s", "cores": threads(),
            "kind": "oracle",
            "sample": f"one cycle of the FP64 oracle (literal full-grid Algorithms 1-3, gcc -O2, OpenMP "
                      f"with {threads()} threads) on the same {wl.N}^{wl.dim} input took {t_cycle:.2f} s; "
                      f"value extrapolates by the {cycles} cycles the FP64 solve needs "
                      f"(x{cycles}); host: {model}, {ncpu} logical CPUs"}


def timed_solves(plan, f, G, u, precision, steps, profile, **kw):
    import torch
    stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        _, st = plan.solve(f, G, u, tol=TOL, max_cycles=2000, precision=precision, profile=profile,
                           stall_window=-1, **kw)
        stats.append(st)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, stats


def bytes_per_node(wl, name, tb):
    """Algorithmic HBM bytes per node and launch of a level-0 kernel class,
    tb = bytes of the cycle's precision (4 mixed, 8 FP64).
      2D fused visit (interpolation prologue + relaxations): read e (stale),
        source, coarse e (1/4 of the nodes); write e; the visit with injection
        (the cycle's first visit of level 0, whose stale values are zero and
        not read) reads no stale e and also writes the coarse level (1/4)
      3D relaxation (sweep0): read e, source (and the FP32/FP64 coefficient
        when heterogeneous), write e; the paired sigma = 1 relaxation moves
        the same bytes for two relaxations
      cycle end: read e, u, s; write u, s (FP64); mixed: write the next source
        (FP32) and, in 2D, its restriction to level 1 (1/4 of the nodes); the
        FP64 coefficient when heterogeneous
      closing visit and cycle end in one pass (2D mixed): the visit's reads
        (stale e, source, coarse e) and the cycle end's bytes without e"""
    mixed = tb == 4
    sig = wl.sigma is not None
    if name == "visit0":
        return 3 * tb + tb / 4
    if name == "visit0_inject":
        return 2 * tb + tb / 2
    if name == "sweep0":
        return 3 * tb + (tb if sig else 0)
    if name == "visit0_end":
        return 2 * tb + tb / 4 + 32 + 4 + tb / 4
    if name == "cycle_end":
        return tb + 32 + (4 if mixed else 0) + (tb / 4 if mixed and wl.dim == 2 else 0) + (8 if sig else 0)
    raise KeyError(name)


def kernel_rates(wl, st, tb):
    out = {}
    for name, rec in st["prof"].items():
        if rec["launches"] == 0:
            continue
        us = 1e3 * rec["ms"] / rec["launches"]
        bpn = bytes_per_node(wl, name, tb)
        gbs = bpn * wl.nodes / (us * 1e-6) / 1e9
        out[name] = {"us": us, "launches_per_solve": rec["launches"],
                     "sweeps_per_launch": rec["sweeps"] / rec["launches"],
                     "bytes_per_node": bpn, "GBs": gbs, "frac": gbs / HBM_PEAK_GBS}
    return out


def dominant(rates):
    return max(rates, key=lambda k: rates[k]["us"] * rates[k]["launches_per_solve"])


def dev(x):
    import torch
    return None if x is None else torch.from_numpy(np.ascontiguousarray(x)).cuda()


def config_record(wl, precisions, steps, warmup, adjoint_target=None):
    """Time-to-1e-12 of one workload in the given precisions (and, with an
    adjoint target, the adjoint solve of 0.5 |u - u_t|^2 after the forward
    solve), with the level-0 kernel rates of a profiled solve."""
    import torch
    from paper_1703_07206_amd import sgml
    f, G, sigma = dev(wl.f), dev(wl.G), dev(wl.sigma)
    plan = sgml.Plan(wl.dim, wl.n, wl.stencil, wl.faces, wl.a, sigma, precision=sgml.MIXED)
    u = torch.empty_like(f)
    rec = {"workload": f"{wl.name} {wl.N}^{wl.dim}", "nodes": wl.nodes,
           "stencil": "radial" if wl.stencil else "axis", "faces": wl.faces, "tol": TOL}
    for name, prec in precisions:
        for _ in range(warmup):
            plan.solve(f, G, u, tol=TOL, max_cycles=2000, precision=prec, stall_window=-1)
        t, sts = timed_solves(plan, f, G, u, prec, steps, False)
        _, stp = timed_solves(plan, f, G, u, prec, 1, True)
        _, rmax, norm0 = plan.residual(f, u, G=G)
        rates = kernel_rates(wl, stp[-1], 4 if prec == sgml.MIXED else 8)
        r = {"ms": t * 1e3, "GNodes_s": wl.nodes / t / 1e9, "cycles": sts[-1]["cycles"],
             "relres": sts[-1]["relres"], "relres_true": rmax / norm0, "kernels": rates}
        if rates:
            d = dominant(rates)
            r["dominant_kernel"] = {"name": d, "GBs": rates[d]["GBs"], "frac": rates[d]["frac"]}
        if adjoint_target is not None:
            # dL/du of 0.5 |u - u_t|^2 over the unknowns, then the adjoint solve
            from paper_1703_07206_amd import workloads as W
            mask = torch.from_numpy(W.dirichlet_mask(wl.dim, wl.n, wl.faces)).cuda()
            ut = dev(adjoint_target)
            g = torch.where(mask, 0.0, u - ut)
            lam = torch.empty_like(g)
            plan.adjoint(g, lam, tol=TOL, max_cycles=2000, precision=prec, stall_window=-1)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                _, sa = plan.adjoint(g, lam, tol=TOL, max_cycles=2000, precision=prec, stall_window=-1)
            torch.cuda.synchronize()
            ta = (time.perf_counter() - t0) / steps
            r["adjoint"] = {"ms": ta * 1e3, "cycles": sa["cycles"], "relres": sa["relres"]}
            r["forward_plus_adjoint_ms"] = (t + ta) * 1e3
            del g, lam, ut, mask
        rec[name] = r
    del plan, f, G, sigma, u
    torch.cuda.empty_cache()
    return rec


def study(max_cycles=40):
    """Sec. 3.1's convergence experiment (Fig. 3): eq. 8 on 1025^2 with
    Dirichlet 0, the residual (max norm over the sources' max norm) and the
    normalised L1 error of eq. 9 against the closed form eq. 7 after every
    cycle, against full-mesh work units, for n_r in {1, 2, 4, full doubling},
    both nestings of Algorithm 3, several pseudo-time steps, and the 5-point
    and radial 9-point stencils.  Work units per cycle: one per call of
    Algorithm 2 and one per averaging step of Algorithm 1 (restriction(nu) is
    nu steps, called before every visit), plus the residual recurrence pass."""
    import torch
    from paper_1703_07206_amd import sgml
    from paper_1703_07206_amd import workloads as W
    wl = W.manufactured2d(n=10)
    f = dev(wl.f)
    ue = dev(wl.extra["u_exact"])
    w = torch.ones_like(ue)
    w[0, :] *= 0.5
    w[-1, :] *= 0.5
    w[:, 0] *= 0.5
    w[:, -1] *= 0.5
    l1_norm = float(torch.sum(w * ue.abs()))
    variants = []
    for stencil, theta_list in ((sgml.AXIS, (0.0, 0.6, 1.0)), (sgml.RADIAL, (0.0, 1.5))):
        for theta in theta_list:
            for n_r, sched in ((2, 0), (1, 0), (4, 0), (0, 0), (2, 1)):
                if theta != 0.0 and (n_r, sched) != (2, 0):
                    continue
                variants.append((stencil, theta, n_r, sched))
    out = []
    for stencil, theta, n_r, sched in variants:
        plan = sgml.Plan(2, wl.n, stencil, "DDDD", 0.0, None, precision=sgml.FP64, theta=theta)
        wu = sum(lv + c for lv, c in sgml.schedule(wl.n, n_r, sched)) + 1
        kw = dict(n_r=n_r, schedule=sched, precision=sgml.FP64, stall_window=-1, raise_on_failure=False)
        u, st = plan.solve(f, tol=TOL, max_cycles=max_cycles, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.solve(f, u=u, tol=TOL, max_cycles=max_cycles, **kw)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        hist = st["history"]
        l1 = []
        for k in range(1, st["cycles"] + 1):
            uk, _ = plan.solve(f, tol=0.0, max_cycles=k, **kw)
            l1.append(float(torch.sum(w * (uk - ue).abs())) / l1_norm)
        rates = [hist[i + 1] / hist[i] for i in range(len(hist) - 1) if hist[i] > 0]
        rec = {"stencil": "radial 9-point" if stencil else "axis 5-point",
               "theta": theta if theta > 0 else (1.0 if stencil else 0.8), "n_r": n_r if n_r > 0 else "full",
               "nesting": "closing level-0 visit once" if sched == 0 else "closing level-0 visit per tooth",
               "work_units_per_cycle": wu, "status": st["status"], "cycles": st["cycles"], "ms": t * 1e3,
               "median_rate": float(np.median(rates)) if rates else None,
               "residual": hist, "l1_error": l1}
        out.append(rec)
        print(f"# {rec['stencil']} theta={rec['theta']} n_r={rec['n_r']} {rec['nesting']}: "
              f"{rec['cycles']} cycles, {wu} WU/cycle, rate {rec['median_rate']}, "
              f"final L1 {l1[-1] if l1 else None:.3e}", file=sys.stderr, flush=True)
        del plan
    print(json.dumps({"study": "sec31_fig3", "grid": "1025^2", "variants": out}), flush=True)


def batch_record(wl, steps):
    """The vector Poisson problem (three right-hand sides, one operator):
    time to 1e-12 of the batch solve against three single solves, mixed."""
    import torch
    from paper_1703_07206_amd import sgml
    k = wl.f.shape[0]
    F = dev(wl.f)
    plan = sgml.Plan(wl.dim, wl.n, wl.stencil, wl.faces, wl.a, None, precision=sgml.MIXED, nrhs=k)
    single = sgml.Plan(wl.dim, wl.n, wl.stencil, wl.faces, wl.a, None, precision=sgml.MIXED)
    U = torch.empty_like(F)
    kw = dict(tol=TOL, max_cycles=2000, precision=sgml.MIXED, stall_window=-1)
    plan.solve_batch(F, U=U, **kw)
    for c in range(k):
        single.solve(F[c], u=U[c], **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        _, sts = plan.solve_batch(F, U=U, **kw)
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t0) / steps
    t0 = time.perf_counter()
    for _ in range(steps):
        for c in range(k):
            single.solve(F[c], u=U[c], **kw)
    torch.cuda.synchronize()
    ts = (time.perf_counter() - t0) / steps
    rec = {"workload": f"{wl.name} {wl.N}^{wl.dim} x {k} right-hand sides", "nodes": wl.nodes * k,
           "precision": "mixed", "batch_ms": tb * 1e3, "single_solves_ms": ts * 1e3,
           "speedup": ts / tb, "GNodes_s": wl.nodes * k / tb / 1e9,
           "cycles": [st["cycles"] for st in sts]}
    del plan, single, F, U
    torch.cuda.empty_cache()
    return rec


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.study:
        study()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "decomposition is a design, not part of this build", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1703_07206_amd import sgml
    from paper_1703_07206_amd import workloads as W

    wl = W.CONFIGS[args.workload]()
    f, G, sigma = dev(wl.f), dev(wl.G), dev(wl.sigma)
    plan = sgml.Plan(wl.dim, wl.n, wl.stencil, wl.faces, wl.a, sigma, precision=sgml.MIXED)
    u = torch.empty_like(f)
    u64 = torch.empty_like(f)

    for _ in range(args.warmup):
        plan.solve(f, G, u, tol=TOL, max_cycles=2000, precision=sgml.MIXED, stall_window=-1)
        plan.solve(f, G, u64, tol=TOL, max_cycles=2000, precision=sgml.FP64, stall_window=-1)
    # the timed steps run uninstrumented; the same number of steps then runs
    # again with HIP events around the level-0 launches (on the solve's
    # stream) for the per-kernel durations of the roofline
    t_mix, _ = timed_solves(plan, f, G, u, sgml.MIXED, args.steps, False)
    t_64, _ = timed_solves(plan, f, G, u64, sgml.FP64, args.steps, False)
    t_mix_p, st_mix = timed_solves(plan, f, G, u, sgml.MIXED, args.steps, True)
    t_64_p, st_64 = timed_solves(plan, f, G, u64, sgml.FP64, args.steps, True)
    print(f"# mixed: {t_mix * 1e3:.3f} ms/solve ({t_mix_p * 1e3:.3f} instrumented), {st_mix[-1]['cycles']} "
          f"cycles; fp64: {t_64 * 1e3:.3f} ms/solve ({t_64_p * 1e3:.3f} instrumented), "
          f"{st_64[-1]['cycles']} cycles", file=sys.stderr, flush=True)

    # accuracy of both results
    _, r_mix, norm0 = plan.residual(f, u, G=G)
    _, r_64, _ = plan.residual(f, u64, G=G)
    diff = float((u - u64).abs().max() / u64.abs().max())

    sm, s6 = st_mix[-1], st_64[-1]
    k_mix, k_64 = kernel_rates(wl, sm, 4), kernel_rates(wl, s6, 8)
    dom = dominant(k_mix)
    achieved = k_mix[dom]["GBs"]
    bytes_per_launch = k_mix[dom]["bytes_per_node"] * wl.nodes
    stencil = ("radial " + ("9" if wl.dim == 2 else "27") if wl.stencil
               else "axis " + ("5" if wl.dim == 2 else "7")) + "-point"

    traffic = measured_traffic(dom, wl.nodes) if args.workload == "poisson2d_blobs" else None
    out = {
        "metric": METRIC,
        "value": wl.nodes / t_mix / 1e9,
        "unit": "GNodes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_mix * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{wl.name} {wl.N}^{wl.dim}", "nodes": wl.nodes,
                   "stencil": "radial" if wl.stencil else "axis", "faces": wl.faces,
                   "tol": TOL, "precision": "fp32 cycle + fp64 refinement", "n_r": 2,
                   "env": {"HIP_FORCE_DEV_KERNARG": os.environ.get("HIP_FORCE_DEV_KERNARG")}},
        "ms_per_step_instrumented": t_mix_p * 1e3,
        "fp64": {"value": wl.nodes / t_64 / 1e9, "ms_per_step": t_64 * 1e3,
                 "cycles": s6["cycles"], "relres_true": r_64 / norm0, "kernels": k_64},
        "mixed": {"cycles": sm["cycles"], "relres": sm["relres"], "relres_true": r_mix / norm0,
                  "rel_diff_vs_fp64": diff, "kernels": k_mix},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic["bytes_per_launch"] if traffic else None,
                     "traffic_detail": traffic,
                     "kernel": f"level-0 {dom} (FP32 cycle, {stencil})",
                     "bytes_per_launch": bytes_per_launch,
                     # every level-0 kernel class, the fine-grid sweeps (fused
                     # visits) next to the cycle end
                     "per_kernel": {"mixed": {k: v["frac"] for k, v in k_mix.items()},
                                    "fp64": {k: v["frac"] for k, v in k_64.items()}}},
    }
    del plan, f, G, sigma, u, u64
    torch.cuda.empty_cache()

    if not args.no_configs and args.workload == "poisson2d_blobs":
        # the other workloads, each to 1e-12
        cfg = {}
        w = W.poisson2d_sine(n=7)
        cfg["poisson2d_sine_129"] = config_record(w, [("fp64", sgml.FP64)], max(args.steps, 5), 2)
        print("# poisson2d_sine 129^2 done", file=sys.stderr, flush=True)
        w = W.helmholtz3d_spheres(n=8)
        cfg["helmholtz3d_spheres_257"] = config_record(w, [("mixed", sgml.MIXED)], 3, 1)
        print("# helmholtz3d_spheres 257^3 done", file=sys.stderr, flush=True)
        w = W.helmholtz3d_adjoint(n=7)
        cfg["helmholtz3d_adjoint_129"] = config_record(w, [("fp64", sgml.FP64)], 3, 1,
                                                       adjoint_target=w.extra["u_target"])
        print("# helmholtz3d_adjoint 129^3 done", file=sys.stderr, flush=True)
        w = W.poisson3d_charges(n=9)
        cfg["poisson3d_charges_513"] = config_record(w, [("mixed", sgml.MIXED), ("fp64", sgml.FP64)], 3, 1,
                                                     adjoint_target=w.extra["u_target"])
        print("# poisson3d_charges 513^3 done", file=sys.stderr, flush=True)
        cfg["trifoil_vortex_257_x3"] = batch_record(W.trifoil_vortex(n=8), 3)
        print("# trifoil_vortex 257^3 x 3 done", file=sys.stderr, flush=True)
        del w
        out["configs"] = cfg
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, s6["cycles"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
