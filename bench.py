"""Benchmark: SA-AMG setup + PCG/V-cycle solve on the 128^3 z-stretched 7-point cube.

One step = one full pass of the hot path on one batch: sa_setup (strength, aggregation,
filtered matrix, eigenvalue estimate, smoothed prolongator, Galerkin products, smoother
setup, coarsest inverse) followed by sa_solve (CG + Chebyshev V-cycle to 1e-8), with the
matrix and right-hand side already resident in HBM.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = "fd7_128_a1000"
PRECISION_WORKLOAD = "fd7_160_a1000"
PEAK_HBM_GBS = 8000.0
# rocprofv3 counter summaries of the fine-level SpMV kernel, one per workload and precision
# (profiles/k_spmv_sell_<workload>_<f64|f32>_hbm_traffic.md); a traffic figure is reported only
# while the kernel's sources still hash to the value recorded with it
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_spmv_sell_{workload}_{dtype}_hbm_traffic.md")
# the SpMV kernel body and epilogues live in solve_device.hpp, its launch and row partition in
# solve_kernels.hip, the block-to-XCD mapping in common.hpp; build.py holds the compile flags
KERNEL_SOURCES = ["paper_2103_10476_amd/csrc/solve_device.hpp",
                  "paper_2103_10476_amd/csrc/solve_kernels.hip",
                  "paper_2103_10476_amd/csrc/common.hpp",
                  "paper_2103_10476_amd/build.py"]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def pct(a, q):
    return float(np.percentile(np.asarray(a), q))


def solve_bytes_model(info, precision="fp64"):
    """Algorithmic HBM bytes of one PCG iteration from the hierarchy sizes.

    SpMV on a CSR with n rows, nnz entries: nnz*(s + 4) + 4(n+1) + s*ncols (x, read once)
    + the epilogue's vector traffic.  V-cycle per level l < L: Chebyshev degree 2 from zero
    (vector pass 3 vectors; step 6 vectors), residual (3), restriction R, prolongation
    (add: 2 vectors), post-smoothing start (5) and step (7 vectors).  Coarsest: dense n^2
    inverse read + 2 vectors.  PCG (FP64): q = A p, 4 dots (2 vectors each), x/r update
    (6 vectors), p update (3 vectors).  All vectors s bytes per entry.
    """
    s = 4 if precision == "fp32" else 8
    L = info["levels"]
    tot = 0.0
    for l in range(L):
        n, nnz = info["n"][l], info["nnz"][l]
        if l == L - 1:
            tot += 8.0 * n * n + 16.0 * n
            continue
        nc = info["n"][l + 1]
        nnzp = info["nnz_p"][l]
        spmv_a = nnz * (s + 4) + 4 * (n + 1) + s * n
        spmv_p = nnzp * (s + 4) + 4 * (n + 1) + s * nc
        spmv_r = nnzp * (s + 4) + 4 * (nc + 1) + s * n
        vec = s * n
        tot += 3 * vec                     # d = invD f / theta (+ u)
        tot += spmv_a + 6 * vec            # step: reads d,f,invD; writes r,u (last)
        tot += spmv_a + 2 * vec            # residual r = f - A u
        tot += spmv_r + s * nc             # restriction
        tot += spmv_p + 2 * vec            # prolongation u += P uc
        tot += spmv_a + 4 * vec            # post start: r, d
        tot += spmv_a + 6 * vec            # post step
    n0, nnz0 = info["n"][0], info["nnz"][0]
    tot += nnz0 * 12 + 4 * (n0 + 1) + 16 * n0   # q = A p (FP64)
    tot += 8 * n0 * (2 * 3 + 1 + 6 + 3)          # dots p.q, r.r, r.z; updates
    if precision == "fp32":
        tot += 12.0 * n0 * 2                     # casts at the V-cycle boundary
    return tot


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default=WORKLOAD)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the timed FP32-vs-FP64 repetitions and the other legs "
                         "(profiling runs); the 160^3 roofline solves still run")
    ap.add_argument("--legs-out", default=None, metavar="PATH",
                    help="also write every leg's full results to PATH (JSON)")
    ap.add_argument("--serving-requests", type=int, default=256)
    ap.add_argument("--serving-rates", default="0.35,0.7,1.0",
                    help="open-loop arrival rates as fractions of the closed-loop rate")
    ap.add_argument("--serving-slots", type=int, default=4)
    ap.add_argument("--serving-budget-gib", type=float, default=8.0)
    ap.add_argument("--family-seeds", type=int, default=10,
                    help="perturbed-cube meshes in the mesh-family leg")
    ap.add_argument("--only-systems", action="store_true",
                    help="run only the systems-SA leg (elasticity, rigid-body modes)")
    ap.add_argument("--only-gmres", action="store_true",
                    help="run only the GMRES leg (nonsymmetric 128^3 cube, GMRES vs CG)")
    ap.add_argument("--only-families", action="store_true",
                    help="run only the mesh-family leg (perturbed and stretched cubes)")
    ap.add_argument("--only-serving", action="store_true",
                    help="run only the serving leg (prints its JSON object)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="first run a plain device copy of BYTES (3 times): the reference "
                         "kernel that calibrates rocprofv3 FETCH_SIZE/WRITE_SIZE counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark measures one GPU; --gpus must be 1 "
                          "(the multi-GPU decomposition is described, not implemented)"}))
        sys.exit(2)

    import torch
    from paper_2103_10476_amd import problems, solver

    torch.cuda.set_device(0)
    if args.only_systems:
        print(json.dumps(systems_leg(solver, problems)), flush=True)
        return
    if args.only_gmres:
        print(json.dumps(gmres_leg(solver, problems)), flush=True)
        return
    if args.only_families:
        print(json.dumps(families_leg(solver, problems, seeds=args.family_seeds)), flush=True)
        return
    if args.only_serving:
        print(json.dumps(serving_leg(solver, problems, args)), flush=True)
        return
    if args.copy_probe:
        src = torch.ones(args.copy_probe // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copy probe: {args.copy_probe} bytes read and written per copy")
        del src, dst
    p = problems.workload(args.workload)
    b = problems.random_rhs(p.n, problems.RHS_SEED.get(args.workload, 2))
    drp = torch.from_numpy(p.rp).cuda()
    dcol = torch.from_numpy(p.col).cuda()
    dval = torch.from_numpy(p.val).cuda()
    db = torch.from_numpy(b).cuda()
    x = torch.empty_like(db)
    torch.cuda.synchronize()
    opts = solver.Options(theta=0.02, rtol=1e-8)

    def step(o=opts):
        h = solver.Hierarchy(p.n, drp, dcol, dval, options=o)
        ts = time.perf_counter()
        _, it, rr, st = h.solve(db, x)
        torch.cuda.synchronize()
        te = time.perf_counter() - ts
        return h, it, rr, st, te

    log(f"[bench] {p.name} n={p.n} nnz={p.nnz}: warmup {args.warmup}")
    for _ in range(args.warmup):
        h, *_ = step()
        h.close()
    # timed steps: nothing instrumented inside the timed region
    times, setups, solves = [], [], []
    torch.cuda.synchronize()
    t_all = time.perf_counter()
    for k in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h, it, rr, st, tsolve = step()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        times.append(dt)
        solves.append(tsolve)
        setups.append(dt - tsolve)
        info = h.info()
        if k == 0:
            log(f"[bench] levels n={info['n']} nnz={info['nnz']} mis_rounds={info['mis_rounds']}")
        h.close()
        log(f"[bench] step {k}: {dt * 1e3:.2f} ms (setup {setups[-1] * 1e3:.2f}, solve "
            f"{tsolve * 1e3:.2f}, {it} its, {st})")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_all
    x_main = x.cpu().numpy()
    # one more pass, outside the timed region, with HIP events around the fine-level SpMVs
    h, *_ = step()
    h.profile(True)
    h.solve(db, x)
    torch.cuda.synchronize()
    prof_main = h.profile_read()
    h.close()
    value = pct(times, 50)
    legs = {}
    result = {
        "metric": "setup+solve s & HBM GB/s, 128³ stretched; FP32-Vcycle vs FP64; p50/p99",
        "value": round(value, 6),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded 7-point finite-volume cube, U(-1,1) right-hand side)",
        "config": {"workload": f"{args.workload}: 3-D 7-point FV Laplacian, 128^3 unknowns, "
                               "z-stretched 1:1000, plain SA theta=0.02, Chebyshev(2) V-cycle, "
                               "PCG to 1e-8",
                   "n": p.n, "nnz": p.nnz, "levels": info["levels"],
                   "operator_complexity": round(info["operator_complexity"], 4),
                   "iterations": it},
        "setup_s": {"p50": round(pct(setups, 50), 6), "p99": round(pct(setups, 99), 6)},
        "solve_s": {"p50": round(pct(solves, 50), 6), "p99": round(pct(solves, 99), 6)},
        "setup_plus_solve_s": {"p50": round(pct(times, 50), 6), "p99": round(pct(times, 99), 6),
                               "min": round(min(times), 6)},
    }
    sb = solve_bytes_model(info) * (it + 1)
    result["solve_hbm_gbs"] = round(sb / pct(solves, 50) / 1e9, 1)
    # the 128^3 fine operator (217-246 MB per launch) can stay in the 256 MB Infinity Cache
    # between launches; the headline roofline is taken on the 160^3 cube (424 MB per launch)
    c4 = c4_leg(solver, problems, PRECISION_WORKLOAD, reps=1 if args.no_extras else 5)
    legs["fp32_vcycle_vs_fp64"] = c4
    result["roofline"] = c4["roofline_fp64"]
    if result["roofline"] is not None:
        result["roofline"]["stream_probe_gbs"] = stream_probe()
    result["roofline_fp32"] = _slim(c4["roofline_fp32"])
    legs["roofline_128_mall_assisted"] = roofline(
        prof_main, args.workload, note="128^3 fine operator, small enough to be served "
        "partly from the 256 MB Infinity Cache")
    result["roofline_128_mall_assisted"] = _slim(legs["roofline_128_mall_assisted"])
    if not args.no_extras:
        legs["variants"] = variants_leg(solver, p, drp, dcol, dval, db)
        legs["numeric_resetup"] = resetup_leg(solver, p, drp, dcol, dval, db)
        legs["variant_sweep"] = variant_sweep_leg(solver, problems)
        legs["mesh_families"] = families_leg(solver, problems, seeds=args.family_seeds)
        legs["gmres"] = gmres_leg(solver, problems)
        legs["systems"] = systems_leg(solver, problems)
        legs["serving"] = serving_leg(solver, problems, args)
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(p, b, x_main, c4)
    for k in ("problem", "b"):  # inputs kept for the oracle comparison, not results
        c4.pop(k, None)
    for prec in ("fp64", "fp32"):
        c4[prec].pop("x", None)
    result["fp32_vcycle_vs_fp64"] = summarise_precision(c4)
    result.update(summarise_legs(legs))
    if args.legs_out:
        os.makedirs(os.path.dirname(os.path.abspath(args.legs_out)), exist_ok=True)
        with open(args.legs_out, "w") as f:
            json.dump({"headline": result, "legs": legs}, f, indent=1)
    log("[bench] legs " + json.dumps(legs))
    print(json.dumps(result, separators=(",", ":")), flush=True)


def _slim(roof):
    """A secondary roofline figure in a few fields (the full object goes to the legs)."""
    if roof is None:
        return None
    return {k: roof[k] for k in ("input", "achieved", "frac", "avg_us",
                                 "algorithmic_bytes_per_launch", "traffic")}


def summarise_precision(c4):
    """The FP32-vs-FP64 leg in a few numbers: p50 setup+solve and solve seconds, iterations,
    the speed-up and each solution's error against the FP64 oracle's (when computed)."""
    out = {"workload": c4["workload_short"]}
    for prec in ("fp64", "fp32"):
        r = c4[prec]
        out[prec] = {"setup_plus_solve_s_p50": r["setup_plus_solve_s"]["p50"],
                     "solve_s_p50": r["solve_s"]["p50"], "iterations": r["iterations"],
                     "true_rel_residual": float(f"{r['true_rel_residual']:.3e}"),
                     "rel_err_vs_oracle": r.get("rel_err_vs_oracle")}
    out["solve_speedup_fp32"] = c4["solve_speedup_fp32"]
    out["setup_plus_solve_speedup_fp32"] = c4["setup_plus_solve_speedup_fp32"]
    out["rel_err_fp32_vs_fp64"] = float(f"{c4['rel_err_fp32_vs_fp64']:.3e}")
    return out


def summarise_legs(legs):
    """One short entry per further leg (their full results go to --legs-out and stderr)."""
    out = {}
    if "variants" in legs:
        out["variants"] = {k: [v.get("iterations"), v.get("operator_complexity"),
                               v.get("setup_s"), v.get("solve_s")] if "iterations" in v
                           else v["status"] for k, v in legs["variants"].items()}
        out["variants_fields"] = "iterations, operator complexity, setup s, solve s"
    if "numeric_resetup" in legs:
        r = legs["numeric_resetup"]
        out["numeric_resetup"] = {"resetup_s_p50": r["resetup_s"]["p50"],
                                  "fresh_setup_s_p50": r["fresh_setup_same_values_s"]["p50"],
                                  "speedup": r["speedup_vs_setup"], "iterations": r["iterations"]}
    if "variant_sweep" in legs:
        sw = {}
        for case, v in legs["variant_sweep"].items():
            its = [t["iterations"] for t in v["table"].values() if "iterations" in t]
            sw[case] = {"combinations": len(v["table"]), "failed": len(v["table"]) - len(its),
                        "iterations_min": min(its) if its else None,
                        "iterations_max": max(its) if its else None}
        out["variant_sweep"] = sw
    if "mesh_families" in legs:
        mf = legs["mesh_families"]
        pc = mf["perturbed_cube"]
        fam = {}
        for w in ("weight_1/d^1", "weight_1/d^2"):
            t = pc[w]
            fam[f"perturbed_{w}"] = {k: [t[k]["mean_iterations"], t[k]["failures"]]
                                     for k in ("plain", "offlmp", "1norm", "offlmp+1norm")
                                     if k in t}
            sc = mf["stretched_cube"][w]
            fam[f"stretched_{w}"] = [sc["plain_failures"]] + [
                (sc["vs_plain"][k]["plain_minus_it"] or {}).get("more_than_plain")
                for k in ("1norm", "offlmp", "cnstrnt", "sprsfy") if k in sc["vs_plain"]]
        fam["fields"] = ("perturbed: [mean iterations, failures]; stretched: [plain failures, "
                         "problems with more iterations than plain: 1norm, offlmp, cnstrnt, "
                         "sprsfy]")
        out["mesh_families"] = fam
    if "gmres" in legs:
        out["gmres"] = {k: [v.get("steps", v.get("gmres_steps")),
                            v.get("solve_s_p50", v.get("gmres_solve_s_p50"))]
                        for k, v in legs["gmres"].items()}
    if "systems" in legs:
        out["systems"] = {k: [v["iterations"], v["setup_s_p50"], v["solve_s_p50"]]
                          for k, v in legs["systems"].items() if k != "problem"}
    if "serving" in legs:
        sv = legs["serving"]
        c = sv["closed_loop"]
        srv = {"closed_loop_solves_per_s": c["solves_per_s"], "failed": c["failed"],
               "closed_loop_latency_s": [c["latency_s"]["p50"], c["latency_s"]["p99"]]}
        for k, v in sv.items():
            if k.startswith("open_loop_"):
                srv[k + "_latency_s"] = [v["latency_s"]["p50"], v["latency_s"]["p99"],
                                         v["arrival_rate_per_s"]]
        t = sv["closed_loop_tight_budget"]
        srv["tight_budget_solves_per_s"] = t["solves_per_s"]
        if "closed_loop_copied_inputs" in sv:
            srv["copied_inputs_solves_per_s"] = sv["closed_loop_copied_inputs"]["solves_per_s"]
        srv["fields"] = "latency [p50, p99] (open loop: and arrivals per s)"
        out["serving"] = srv
    return out


def stream_probe(nbytes=512 << 20, reps=10):
    """Achievable HBM bandwidth on this device, for context beside the 8 TB/s spec: a device
    copy of 512 MiB (bytes read + written) and a full read (a sum over 512 MiB), timed with
    events on the current stream."""
    import torch
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    out = {}
    for name, fn, moved in (("copy_read_write", lambda: b.copy_(a), 2 * nbytes),
                            ("read", lambda: a.sum(), nbytes)):
        fn()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        e1.synchronize()
        out[name] = round(moved * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)
    del a, b
    torch.cuda.empty_cache()
    return out


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, dtype="f64"):
    """HBM bytes per fine-level SpMV launch from the committed counter summary, or None when
    the summary is missing, covers another workload, or the kernel has changed since."""
    kv = {}
    try:
        with open(TRAFFIC_PROFILE.format(workload=workload, dtype=dtype)) as f:
            for line in f:
                k, sep, v = line.partition(":")
                k = k.strip().strip("-*` ")
                if sep and k.isidentifier():
                    kv[k] = v.strip().strip("`")
    except OSError:
        return None
    if kv.get("workload") != workload or kv.get("kernel_source_sha256") != kernel_source_hash():
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def roofline(tot, workload=WORKLOAD, dtype="f64", note=None):
    """Fine-level SpMV (sliced ELL; the kernel with the largest share of the solve):
    algorithmic bytes per launch (entries x (value + 4 B index) + slice offsets + x once + the
    vectors its fused epilogue reads/writes; padding not counted) over the launch duration from
    HIP events recorded around every such launch of one profiled solve, on the library's
    stream."""
    if not tot["launches"]:
        return None
    avg_ms = tot["ms"] / tot["launches"]
    bytes_per = tot["bytes"] / tot["launches"]
    achieved = bytes_per / (avg_ms * 1e-3) / 1e9
    out = {"bound": "hbm",
           "kernel": ("k_spmv_sell<double>" if dtype == "f64" else
                      "k_spmv_sell<float> (V-cycle) and <double> (CG)") +
                     ", fine level, sliced ELL, fused epilogues",
           "input": workload,
           "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
           "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": measured_traffic(workload, dtype),
           "launches": tot["launches"], "avg_us": round(avg_ms * 1e3, 2),
           "algorithmic_bytes_per_launch": round(bytes_per)}
    if note:
        out["note"] = note
    return out


def c4_leg(solver, problems, workload, reps=5):
    """FP32-stored/applied V-cycle inside FP64 PCG against the all-FP64 solve on the 160^3
    z-stretched cube (4.1M unknowns), same GPU, same input, relative residual 1e-10 for both.
    One untimed setup+solve per precision first; then `reps` timed setup+solve pairs (p50 and
    p99 reported), with nothing instrumented; then one more solve with HIP events around the
    fine-level SpMV launches (the roofline: 424 MB per FP64 launch, more than the 256 MB
    Infinity Cache holds).  Accuracy: the true residual ||b - A x|| / ||b|| (host, scipy), the
    relative difference between the two solutions, and (added by the CPU-baseline leg) each
    one's error against the FP64 oracle's solution."""
    import torch
    import scipy.sparse as sp
    p = problems.workload(workload)
    b = problems.random_rhs(p.n, problems.RHS_SEED[workload])
    drp = torch.from_numpy(p.rp).cuda()
    dcol = torch.from_numpy(p.col).cuda()
    dval = torch.from_numpy(p.val).cuda()
    db = torch.from_numpy(b).cuda()
    A = sp.csr_matrix((p.val, p.col, p.rp), shape=(p.n, p.n))
    out = {"workload": f"{workload}: 3-D 7-point FV Laplacian, 160^3 unknowns, z-stretched "
                       "1:1000, plain SA theta=0.02, Chebyshev(2), rtol 1e-10",
           "workload_short": f"{workload}, rtol 1e-10", "n": p.n, "nnz": p.nnz,
           "problem": p, "b": b}
    xs = {}
    for prec in ("fp64", "fp32"):
        o = solver.Options(theta=0.02, rtol=1e-10, precision=prec)
        h = solver.Hierarchy(p.n, drp, dcol, dval, options=o)  # untimed warm-up pass
        h.solve(db)
        h.close()
        setups, solves = [], []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            h = solver.Hierarchy(p.n, drp, dcol, dval, options=o)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            x, it, rr, st = h.solve(db)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            setups.append(t1 - t0)
            solves.append(t2 - t1)
            info = h.info()
            if len(setups) < reps:
                h.close()
        h.profile(True)
        h.solve(db)
        torch.cuda.synchronize()
        dt = "f64" if prec == "fp64" else "f32"
        out[f"roofline_{prec}"] = roofline(
            h.profile_read(), workload, dt,
            note=f"matrix and x alone {'424' if dt == 'f64' else '277'} MB per launch, "
                 "over the 256 MB Infinity Cache")
        h.close()
        xs[prec] = x.clone()
        xh = x.cpu().numpy()
        res = np.linalg.norm(b - A @ xh) / np.linalg.norm(b)
        tot = [a + c for a, c in zip(setups, solves)]
        out[prec] = {"setup_s": {"p50": round(pct(setups, 50), 5), "p99": round(pct(setups, 99), 5)},
                     "solve_s": {"p50": round(pct(solves, 50), 5), "p99": round(pct(solves, 99), 5)},
                     "setup_plus_solve_s": {"p50": round(pct(tot, 50), 5),
                                            "p99": round(pct(tot, 99), 5)},
                     "iterations": it, "status": st, "true_rel_residual": float(res),
                     "levels": info["levels"],
                     "operator_complexity": round(info["operator_complexity"], 4),
                     "solve_hbm_gbs": round(solve_bytes_model(info, prec) * (it + 1)
                                            / pct(solves, 50) / 1e9, 1),
                     "x": xh}
    out["rel_err_fp32_vs_fp64"] = float(torch.linalg.norm(xs["fp32"] - xs["fp64"]) /
                                        torch.linalg.norm(xs["fp64"]))
    out["solve_speedup_fp32"] = round(out["fp64"]["solve_s"]["p50"] /
                                      out["fp32"]["solve_s"]["p50"], 3)
    out["setup_plus_solve_speedup_fp32"] = round(out["fp64"]["setup_plus_solve_s"]["p50"] /
                                                 out["fp32"]["setup_plus_solve_s"]["p50"], 3)
    log(f"[bench] 160^3: fp64 {out['fp64']['iterations']} its "
        f"{out['fp64']['setup_plus_solve_s']['p50'] * 1e3:.1f} ms, fp32 "
        f"{out['fp32']['iterations']} its {out['fp32']['setup_plus_solve_s']['p50'] * 1e3:.1f} ms")
    del drp, dcol, dval, db, xs
    torch.cuda.empty_cache()
    return out


def variants_leg(solver, p, drp, dcol, dval, db):
    """One setup per variant (plain, Sprsfy, OffLmp, 1Norm, Cnstrnt) with the solve to 1e-8."""
    import torch
    out = {}
    for name, var in (("plain", []), ("sprsfy", ["sprsfy"]), ("offlmp", ["offlmp"]),
                      ("1norm", ["1norm"]), ("cnstrnt", ["cnstrnt"])):
        o = solver.Options(theta=0.02, rtol=1e-8, variants=var)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        try:
            h = solver.Hierarchy(p.n, drp, dcol, dval, options=o)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            _, it, rr, st = h.solve(db)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            inf = h.info()
            out[name] = {"setup_s": round(t1 - t0, 5), "solve_s": round(t2 - t1, 5),
                         "iterations": it, "status": st, "levels": inf["levels"],
                         "operator_complexity": round(inf["operator_complexity"], 4)}
            h.close()
        except Exception as e:  # a variant may fail on a problem (reported, not fatal)
            out[name] = {"status": str(e)[:120]}
    return out


def variant_sweep_leg(solver, problems):
    """The 16 combinations of Sprsfy, OffLmp, 1Norm and Cnstrnt (the paper's Table 1 layout:
    CG iterations and operator complexity per combination), rtol 1e-10, on the Sec. 1.2
    stress problem (Q1 on 1x1x2 boxes, 24^3 unknowns, theta 0.15), the 128^3 z-stretched
    cube and the 100^3 random-kappa Q1 cube (theta 0.02).  A failing combination is reported
    with its status (the paper's negative-eigenvalue / small-diagonal failures)."""
    import itertools
    from fractions import Fraction
    import torch
    names = ("sprsfy", "offlmp", "1norm", "cnstrnt")
    cases = [("stress_box_24_theta0.15", problems.q1_stretched_box(24, Fraction(2)), 0.15, 7),
             ("fd7_128_a1000", problems.workload("fd7_128_a1000"), 0.02, 2),
             ("q1_100_randkappa", problems.workload("q1_100_randkappa"), 0.02, 4)]
    out = {}
    for cname, p, theta, seed in cases:
        b = torch.from_numpy(problems.random_rhs(p.n, seed)).cuda()
        drp = torch.from_numpy(p.rp).cuda()
        dcol = torch.from_numpy(p.col).cuda()
        dval = torch.from_numpy(p.val).cuda()
        table = {}
        for bits in itertools.product((0, 1), repeat=4):
            var = tuple(n for n, on in zip(names, bits) if on)
            key = "+".join(var) or "plain"
            o = solver.Options(theta=theta, rtol=1e-10, variants=var)
            try:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                h = solver.Hierarchy(p.n, drp, dcol, dval, options=o)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                _, it, _, st = h.solve(b)
                torch.cuda.synchronize()
                inf = h.info()
                table[key] = {"iterations": it, "operator_complexity":
                              round(inf["operator_complexity"], 4), "levels": inf["levels"],
                              "status": st, "setup_s": round(t1 - t0, 4),
                              "solve_s": round(time.perf_counter() - t1, 4)}
                h.close()
            except Exception as e:
                table[key] = {"status": str(e).split(":")[1].split("(")[0].strip()
                              if ":" in str(e) else str(e)[:80]}
        out[cname] = {"n": p.n, "nnz": p.nnz, "table": table}
        log(f"[bench] variant sweep {cname}: " + ", ".join(
            f"{k} {v.get('iterations', v['status'])}" for k, v in table.items()))
        del drp, dcol, dval, b
    return out


def _spawn():
    """Worker processes for host-side input generation are spawned, not forked: a fork of a
    process that has initialised the GPU runtime would inherit its state."""
    import multiprocessing
    return multiprocessing.get_context("spawn")


def _to_device(p, b, X):
    import torch
    return (p.n, torch.from_numpy(p.rp).cuda(), torch.from_numpy(p.col).cuda(),
            torch.from_numpy(p.val).cuda(), torch.from_numpy(b).cuda(),
            torch.from_numpy(np.ascontiguousarray(X)).cuda())


def _family_run(solver, dev, var, **kw):
    """One setup + solve with coordinates on the GPU (inputs already resident): a dict of
    iterations, operator complexity, times and status (or the failure status)."""
    import torch
    n, drp, dcol, dval, b, X = dev
    o = solver.Options(variants=var, **kw)
    try:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = solver.Hierarchy(n, drp, dcol, dval, options=o, coords=X)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, it, _, st = h.solve(b)
        torch.cuda.synchronize()
        inf = h.info()
        h.close()
        return {"iterations": it, "oc": inf["operator_complexity"], "status": st,
                "setup_s": t1 - t0, "solve_s": time.perf_counter() - t1}
    except Exception as e:  # the method's own failures (negative eigenvalue, zero diagonal)
        msg = str(e)
        return {"status": msg.split(":")[1].split("(")[0].strip() if ":" in msg else msg[:80]}


def _perturbed_mesh(args):
    from paper_2103_10476_amd import problems
    return problems.perturbed_cube(*args)


def _stretched_mesh(args):
    from paper_2103_10476_amd import problems
    return problems.stretched_cube(*args)


def _perturbed_table(runs):
    table = {}
    for key, rs in runs.items():
        ok = [r for r in rs if "iterations" in r]
        table[key] = {"failures": len(rs) - len(ok),
                      "failure_status": sorted({r["status"] for r in rs if "iterations" not in r}),
                      "mean_iterations": round(float(np.mean([r["iterations"] for r in ok])), 2)
                      if ok else None,
                      "operator_complexity": round(float(np.mean([r["oc"] for r in ok])), 4)
                      if ok else None,
                      "setup_plus_solve_s_p50": round(pct([r["setup_s"] + r["solve_s"]
                                                           for r in ok], 50), 4) if ok else None}
    return table


def _stretched_summary(res):
    plain = res["plain"]
    hist = {}
    for k, rs in res.items():
        if k == "plain":
            continue
        diffs = [a["iterations"] - r["iterations"] for a, r in zip(plain, rs)
                 if "iterations" in a and "iterations" in r]
        hist[k] = {"failures": sum("iterations" not in r for r in rs),
                   "compared": len(diffs),
                   "plain_minus_it": {"min": min(diffs), "max": max(diffs),
                                      "within_3": sum(abs(d) <= 3 for d in diffs),
                                      "at_least_15_fewer": sum(d >= 15 for d in diffs),
                                      "more_than_plain": sum(d < 0 for d in diffs)}
                   if diffs else None}
    ok = [r["iterations"] for r in plain if "iterations" in r]
    return {"plain_failures": len(plain) - len(ok),
            "plain_mean_iterations": round(float(np.mean(ok)), 2) if ok else None,
            "vs_plain": hist}


def families_leg(solver, problems, seeds=10, ne=60):
    """The paper's two mesh families on the GPU, with the distance-Laplacian strength
    (theta 0.025) for both weights 1/d (the paper's text) and 1/d^2, coarsening to <= 1000
    unknowns, Chebyshev(2) and CG to 1e-10 on the Dirichlet right-hand side.

    * Randomly perturbed cube (Table 1 layout): ``seeds`` meshes of ne^3 elements x all 16
      combinations; per combination the failures, and the mean iterations and operator
      complexity over the runs that did not fail.
    * Triaxially stretched reaction-diffusion cube (Fig. 2): the 10 (kx,ky,kz) x 5 sigma = 50
      problems at ne^3 elements, Chebyshev interval end 1.1 lambda; per adaptation the
      distribution of (plain SA iterations - its iterations) and its failures.
    Meshes are built on host worker processes; each is uploaded once."""
    import itertools
    from concurrent.futures import ProcessPoolExecutor
    names = ("sprsfy", "offlmp", "1norm", "cnstrnt")
    combos = [tuple(n for n, on in zip(names, bits) if on)
              for bits in itertools.product((0, 1), repeat=4)]
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    paper = dict(theta=0.025, max_coarse=1000, rtol=1e-10)
    powers = (1, 2)
    out = {}
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=workers, mp_context=_spawn()) as ex:
        meshes = list(ex.map(_perturbed_mesh, [(ne, s) for s in range(seeds)]))
    t_mesh = time.perf_counter() - t0
    runs = {pw: {"+".join(v) or "plain": [] for v in combos} for pw in powers}
    t0 = time.perf_counter()
    for mesh in meshes:
        dev = _to_device(*mesh)
        for pw in powers:
            for v in combos:
                runs[pw]["+".join(v) or "plain"].append(
                    _family_run(solver, dev, v, dist_power=pw, **paper))
        del dev
    t_gpu = time.perf_counter() - t0
    pc = {"elements": f"{ne}^3", "n": meshes[0][0].n, "nnz": meshes[0][0].nnz,
          "seeds": seeds, "mesh_build_s": round(t_mesh, 1), "gpu_runs_s": round(t_gpu, 1)}
    for pw in powers:
        pc[f"weight_1/d^{pw}"] = _perturbed_table(runs[pw])
        log(f"[bench] perturbed cube 1/d^{pw}: " + ", ".join(
            f"{k} {v['mean_iterations']}/{v['failures']}f"
            for k, v in pc[f"weight_1/d^{pw}"].items()))
    out["perturbed_cube"] = pc
    del meshes
    cases = [(kx, ky, kz, sg, ne) for (kx, ky, kz) in problems.STRETCH_CONFIGS
             for sg in problems.STRETCH_SIGMAS]
    variants = {"plain": (), "1norm": ("1norm",), "offlmp": ("offlmp",),
                "cnstrnt": ("cnstrnt",), "sprsfy": ("sprsfy",)}
    res = {pw: {k: [] for k in variants} for pw in powers}
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=workers, mp_context=_spawn()) as ex:
        for mesh in ex.map(_stretched_mesh, cases):
            dev = _to_device(*mesh)
            for pw in powers:
                for k, v in variants.items():
                    res[pw][k].append(_family_run(solver, dev, v, cheb_boost=1.1,
                                                  dist_power=pw, **paper))
            del dev
    sc = {"elements": f"{ne}^3", "problems": len(cases),
          "seconds": round(time.perf_counter() - t0, 1)}
    for pw in powers:
        sc[f"weight_1/d^{pw}"] = _stretched_summary(res[pw])
        log(f"[bench] stretched cube 1/d^{pw}: plain failures "
            f"{sc[f'weight_1/d^{pw}']['plain_failures']}; " + ", ".join(
                f"{k} {v['plain_minus_it']}"
                for k, v in sc[f"weight_1/d^{pw}"]["vs_plain"].items()))
    out["stretched_cube"] = sc
    return out


def gmres_leg(solver, problems, reps=3):
    """Restarted GMRES(30) with the V-cycle as right preconditioner (the paper's solver for
    nonsymmetric systems, Sec. 3.4) on a 128^3 graded upwind convection-diffusion cube
    (nonsymmetric, OffLmp + 1Norm, LU coarse solver), at the wind runs' tolerance 1e-5 and at
    1e-8, in FP64 and with the FP32 V-cycle; and GMRES next to CG on the symmetric 128^3
    benchmark cube.  p50 of setup and solve over ``reps`` runs, inputs resident in HBM."""
    import torch
    out = {}
    p = problems.cd7_upwind(128, 1000.0, (1.0, 0.5, 0.25))
    b = problems.random_rhs(p.n, 2)
    drp, dcol, dval = (torch.from_numpy(a).cuda() for a in (p.rp, p.col, p.val))
    db = torch.from_numpy(b).cuda()
    x = torch.empty_like(db)
    for prec in ("fp64", "fp32"):
        for rtol in (1e-5, 1e-8):
            o = solver.Options(variants=("offlmp", "1norm"), coarse_solver="lu", rtol=rtol,
                               precision=prec)
            se, so = [], []
            for _ in range(reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                h = solver.Hierarchy(p.n, drp, dcol, dval, options=o)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                _, it, rr, st = h.solve_gmres(db, x, restart=30)
                torch.cuda.synchronize()
                se.append(t1 - t0)
                so.append(time.perf_counter() - t1)
                h.close()
            out[f"cd7_128_nonsym_{prec}_rtol{rtol:g}"] = {
                "steps": it, "status": st, "rel_residual": rr,
                "setup_s_p50": round(pct(se, 50), 5), "solve_s_p50": round(pct(so, 50), 5),
                "solve_ms_per_step": round(pct(so, 50) / max(it, 1) * 1e3, 3)}
    log("[bench] gmres cd7 128^3: " + ", ".join(
        f"{k} {v['steps']} steps {v['solve_s_p50'] * 1e3:.1f} ms" for k, v in out.items()))
    del drp, dcol, dval, db, x
    q = problems.workload("fd7_128_a1000")
    bq = torch.from_numpy(problems.random_rhs(q.n, 2)).cuda()
    h = solver.Hierarchy(q.n, torch.from_numpy(q.rp).cuda(), torch.from_numpy(q.col).cuda(),
                         torch.from_numpy(q.val).cuda(), options=solver.Options(rtol=1e-8))
    xq = torch.empty_like(bq)
    cg, gm = [], []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, itc, _, _ = h.solve(bq, xq)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, itg, _, _ = h.solve_gmres(bq, xq, restart=30)
        torch.cuda.synchronize()
        cg.append(t1 - t0)
        gm.append(time.perf_counter() - t1)
    h.close()
    out["fd7_128_sym_cg_vs_gmres"] = {"cg_iterations": itc, "cg_solve_s_p50": round(pct(cg, 50), 5),
                                      "gmres_steps": itg,
                                      "gmres_solve_s_p50": round(pct(gm, 50), 5)}
    log(f"[bench] fd7 128^3: CG {itc} its {pct(cg, 50) * 1e3:.1f} ms, GMRES(30) {itg} steps "
        f"{pct(gm, 50) * 1e3:.1f} ms")
    return out


def systems_leg(solver, problems, reps=3):
    """Systems SA with a multi-vector nullspace (sa_setup_system) on a 3-D Q1 elasticity
    cantilever, 96 x 24 x 24 elements clamped at x = 0 (180,000 unknowns, 3 per node): the six
    rigid-body modes against the three translations, plain and OffLmp + 1Norm, Chebyshev
    interval end 1.1 lambda, CG to 1e-8; FP32 V-cycle for the rigid-body case.  p50 of setup
    and solve over ``reps`` runs, inputs resident in HBM."""
    import torch
    t0 = time.perf_counter()
    p, X, B = problems.elastic_beam(96, 24, 24)
    t_gen = time.perf_counter() - t0
    drp, dcol, dval = (torch.from_numpy(a).cuda() for a in (p.rp, p.col, p.val))
    db = torch.from_numpy(problems.random_rhs(p.n, 2)).cuda()
    x = torch.empty_like(db)
    out = {"problem": {"elements": "96x24x24", "n": p.n, "nnz": p.nnz, "block_size": 3,
                       "build_s": round(t_gen, 1)}}
    cases = [("rbm6_plain", 6, (), "fp64"), ("rbm6_offlmp_1norm", 6, ("offlmp", "1norm"), "fp64"),
             ("rbm6_plain_fp32", 6, (), "fp32"), ("translations3_plain", 3, (), "fp64")]
    for key, k, var, prec in cases:
        dB = torch.from_numpy(np.ascontiguousarray(B[:, :k])).cuda()
        o = solver.Options(variants=var, cheb_boost=1.1, rtol=1e-8, precision=prec)
        se, so = [], []
        for _ in range(reps):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            h = solver.Hierarchy(p.n, drp, dcol, dval, nullspace=dB, options=o, block_size=3)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            _, it, rr, st = h.solve(db, x)
            torch.cuda.synchronize()
            se.append(t2 - t1)
            so.append(time.perf_counter() - t2)
            inf = h.info()
            h.close()
        out[key] = {"iterations": it, "status": st, "levels": inf["n"],
                    "operator_complexity": round(inf["operator_complexity"], 4),
                    "setup_s_p50": round(pct(se, 50), 5), "solve_s_p50": round(pct(so, 50), 5)}
    log("[bench] systems (elastic beam): " + ", ".join(
        f"{k} {v['iterations']} its setup {v['setup_s_p50'] * 1e3:.1f} ms solve "
        f"{v['solve_s_p50'] * 1e3:.1f} ms" for k, v in out.items() if k != "problem"))
    return out


def resetup_leg(solver, p, drp, dcol, dval, db, reps=5):
    """Numeric re-setup on the same workload: new values D A D (D a seeded positive diagonal)
    on the setup's pattern, every symbolic decision of the setup kept; p50/p99 of the
    re-setup and of the following solve, next to a fresh setup on the same new values."""
    import torch
    rng = np.random.Generator(np.random.PCG64(31))
    d = rng.uniform(0.5, 2.0, size=p.n)
    rows = np.repeat(np.arange(p.n), np.diff(p.rp))
    val2 = torch.from_numpy((d[rows] * p.val) * d[p.col]).cuda()
    o = solver.Options(theta=0.02, rtol=1e-8)
    h = solver.Hierarchy(p.n, drp, dcol, dval, options=o)
    h.resetup(val2)  # warm-up
    re, so = [], []
    for k in range(reps):
        h.resetup(dval if k % 2 else val2)  # alternate between the two value sets
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h.resetup(val2)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, it, _, st = h.solve(db)
        torch.cuda.synchronize()
        re.append(t1 - t0)
        so.append(time.perf_counter() - t1)
    h.close()
    fr = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g = solver.Hierarchy(p.n, drp, dcol, val2, options=o)
        torch.cuda.synchronize()
        fr.append(time.perf_counter() - t0)
        g.close()
    return {"values": "D A D, D_i ~ U(0.5, 2) seeded", "iterations": it, "status": st,
            "resetup_s": {"p50": round(pct(re, 50), 5), "p99": round(pct(re, 99), 5)},
            "solve_s": {"p50": round(pct(so, 50), 5), "p99": round(pct(so, 99), 5)},
            "fresh_setup_same_values_s": {"p50": round(pct(fr, 50), 5),
                                          "p99": round(pct(fr, 99), 5)},
            "speedup_vs_setup": round(pct(fr, 50) / pct(re, 50), 3)}


def _build_requests(problems, count):
    """The serving workload's requests (seeded), built on host worker processes."""
    from concurrent.futures import ProcessPoolExecutor
    reqs = problems.serving_requests(count)
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    with ProcessPoolExecutor(max_workers=workers, mp_context=_spawn()) as ex:
        built = list(ex.map(problems.build_request, reqs, chunksize=4))
    return reqs, built


def _serve_run(solver, problems, reqs, built, budget, slots, arrivals=None, borrow=True):
    """Submits every request (all at once, or at the given arrival offsets in seconds) and
    collects the results.  Latency = completion - scheduled arrival.  borrow: the server reads
    the client's arrays (sa_server_submit_borrowed) instead of copying them at submission."""
    srv = solver.Server(hbm_budget=budget, max_slots=slots)
    tickets, lat_base = [], []
    t0 = time.perf_counter()
    for i, (req, (p, b)) in enumerate(zip(reqs, built)):
        if arrivals is not None:
            wait = t0 + arrivals[i] - time.perf_counter()
            if wait > 0:
                time.sleep(wait)
        sched = t0 + (arrivals[i] if arrivals is not None else 0.0)
        o = solver.Options(**problems.serving_method(req))
        tickets.append(srv.submit(p, b, o, borrow=borrow))
        lat_base.append(time.perf_counter() - sched)  # submission delay (host copy)
    lat, queue, its, fails, peaks, ests = [], [], [], [], [], []
    worst = (0.0, None)
    for t, req, (p, _), base in zip(tickets, reqs, built, lat_base):
        try:
            _, r = srv.wait(t, p.n)
        except Exception as e:
            fails.append({"request": req, "n": p.n, "nnz": p.nnz, "error": str(e)[:160]})
            continue
        ratio = r["peak_bytes"] / r["reserved_bytes"]
        if ratio > worst[0]:
            worst = (ratio, {"request": req, "n": p.n, "nnz": p.nnz, "peak": r["peak_bytes"],
                             "estimate": r["reserved_bytes"], "levels": r["levels"]})
        lat.append(base + r["latency_seconds"])
        queue.append(r["queue_seconds"])
        its.append(r["iterations"])
        peaks.append(r["peak_bytes"])
        ests.append(r["reserved_bytes"])
    wall = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    return {"requests": len(reqs), "failed": len(fails), "failures": fails,
            "wall_s": round(wall, 3),
            "solves_per_s": round((len(reqs) - len(fails)) / wall, 2),
            "latency_s": {"p50": round(pct(lat, 50), 4), "p99": round(pct(lat, 99), 4)},
            "queue_s": {"p50": round(pct(queue, 50), 4), "p99": round(pct(queue, 99), 4)},
            "iterations": {"p50": pct(its, 50), "max": int(max(its))},
            "budget_bytes": budget, "peak_reserved_bytes": st["peak_reserved_bytes"],
            "peak_measured_bytes": st["peak_measured_bytes"],
            "solve_ticks": st["solve_ticks"], "mean_requests_per_tick": round(st["mean_group"], 2),
            "max_requests_per_tick": st["max_group"],
            "max_peak_over_estimate": round(worst[0], 3), "max_peak_request": worst[1]}


def serving_leg(solver, problems, args):
    """Serving workload: seeded requests (7-point z-stretched cubes with aspect 10^U[1,3] or
    27-point random-kappa cubes, side 16..96), FP32 V-cycle in FP64 CG to 1e-10, on one GPU
    with `slots` concurrent requests under an HBM budget.  Closed loop (all submitted at
    t=0) gives the throughput; open loop runs use Poisson arrivals at the given fractions of
    it; a final closed-loop run uses a budget of 1.5 times the largest request's estimate.
    Setups overlap on `slots` streams; the solves of all set-up requests advance together,
    one grouped launch per CG/V-cycle step per tick.  The client keeps its arrays, so requests
    are submitted by reference; one more closed-loop run copies them at submission (about 13 GB
    of host copies for the 256 requests, done by the submitting thread)."""
    t = time.perf_counter()
    reqs, built = _build_requests(problems, args.serving_requests)
    log(f"[bench] serving: {len(reqs)} requests built in {time.perf_counter() - t:.1f} s")
    budget = int(args.serving_budget_gib * 2**30)
    slots = args.serving_slots
    # warm-up: one pass over a few requests (allocator cache, code paths)
    _serve_run(solver, problems, reqs[:8], built[:8], budget, slots)
    out = {"workload": f"{len(reqs)} seeded requests: 7-point z-stretched cube (aspect "
                       "10^U[1,3]) or 27-point random-kappa cube (u ~ U[-3,3]), side "
                       "U{16..96}; OffLmp+1Norm SA, Chebyshev(2) with the eigenvalue "
                       "estimate x1.1, FP32 V-cycle, FP64 CG, rtol 1e-10",
           "slots": slots,
           "nnz_total": int(sum(p.nnz for p, _ in built))}
    closed = _serve_run(solver, problems, reqs, built, budget, slots)
    log(f"[bench] serving closed loop: {closed['solves_per_s']} solves/s, latency p50 "
        f"{closed['latency_s']['p50']} s")
    out["closed_loop"] = closed
    rng = np.random.Generator(np.random.PCG64(60))
    gaps = rng.exponential(1.0, size=len(reqs))
    for frac in [float(f) for f in args.serving_rates.split(",") if f]:
        rate = frac * closed["solves_per_s"]
        arr = np.concatenate([[0.0], np.cumsum(gaps[:-1] / rate)])
        r = _serve_run(solver, problems, reqs, built, budget, slots, arrivals=arr)
        r["arrival_rate_per_s"] = round(rate, 2)
        log(f"[bench] serving open loop at {frac} x: latency p50 {r['latency_s']['p50']} s "
            f"p99 {r['latency_s']['p99']} s")
        out[f"open_loop_{frac:g}x"] = r
    big = max(solver.estimate_bytes(p.n, p.nnz) for p, _ in built)
    tight = _serve_run(solver, problems, reqs, built, int(1.5 * big), slots)
    log(f"[bench] serving tight budget: {tight['solves_per_s']} solves/s")
    out["closed_loop_tight_budget"] = tight
    copied = _serve_run(solver, problems, reqs, built, budget, slots, borrow=False)
    log(f"[bench] serving closed loop, inputs copied at submission: "
        f"{copied['solves_per_s']} solves/s")
    out["closed_loop_copied_inputs"] = copied
    return out


def cpu_baseline(p, b, x_gpu, c4):
    """The CPU oracle (plain single-threaded C++) on the same workload, timed: full setups and
    solves of the 128^3 cube (two, about 7 s on one core), in seconds per setup+solve.  The same
    runs give the reference solutions the GPU's are compared with: the 128^3 FP64 solve, and
    (one untimed oracle run on the 160^3 cube, rtol 1e-10) the FP64 and FP32-V-cycle solves of
    the precision leg, whose errors are written into `c4`."""
    from oracle import oracle as orc
    try:
        cores = len(os.sched_getaffinity(0))
    except Exception:
        cores = os.cpu_count()
    reps = 2
    ts, tso = [], []
    for _ in range(reps):
        t0 = time.perf_counter()
        h = orc.OracleHierarchy(p.n, p.rp, p.col, p.val, theta=0.02, rtol=1e-8)
        t1 = time.perf_counter()
        r = h.solve(b)
        t2 = time.perf_counter()
        ts.append(t2 - t0)
        tso.append(t2 - t1)
        del h
    err_main = float(np.linalg.norm(x_gpu - r["x"]) / np.linalg.norm(r["x"]))
    q, bq = c4.pop("problem"), c4.pop("b")
    h = orc.OracleHierarchy(q.n, q.rp, q.col, q.val, theta=0.02, rtol=1e-10)
    rq = h.solve(bq)
    del h
    for prec in ("fp64", "fp32"):
        xg = c4[prec].pop("x")
        c4[prec]["rel_err_vs_oracle"] = float(f"{np.linalg.norm(xg - rq['x']) / np.linalg.norm(rq['x']):.3e}")
    c4["oracle_iterations"] = rq["iterations"]
    log(f"[bench] oracle: 128^3 setup+solve {np.mean(ts):.2f} s ({r['iterations']} its), GPU "
        f"error {err_main:.2e}; 160^3: fp64 error {c4['fp64']['rel_err_vs_oracle']}, fp32 "
        f"error {c4['fp32']['rel_err_vs_oracle']}")
    return {"value": round(float(np.mean(ts)), 3), "unit": "s", "cores": 1, "kind": "oracle",
            "sample": f"{reps} full setups + PCG solves of the same workload on one thread "
                      f"({cores} host cores available); solve {np.mean(tso):.2f} s of it; "
                      f"{r['iterations']} iterations",
            "higher_is_better": False,
            "gpu_rel_err_vs_oracle": float(f"{err_main:.3e}"),
            "oracle_iterations": r["iterations"]}


if __name__ == "__main__":
    main()
