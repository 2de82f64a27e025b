#!/usr/bin/env python3
"""Throughput of adaptive-multilevel BDDC PCG solves on one MI355X.

Workload (default): Q1 diffusion on a 256 x 256 grid, 16 x 16 substructures
(H/h = 16), three levels with 4 x 4 groups, k = 10^U(0,6) per element plus 8
channels of k = 1e6, adaptive coarse dofs with tau = 10, f ~ U[-1, 1],
PCG to relative residual 1e-8, FP64 throughout.

One step is the whole hot path on one synthetic input: bddc_setup (local
matrices, weights, interior elimination, per-edge eigenproblems, constrained
factors, next level, coarsest factor), bddc_solve (PCG on the level-1
interface with the three-level preconditioner, interior recovery) and
bddc_destroy.  Coefficients and load are resident in HBM before timing; the
partition (integer topology input) is read on the host.

Prints one JSON line on stdout; progress goes to stderr.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

COPY_BYTES = 256 << 20
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6
METRIC = "PCG solves/s to rel. residual 1e-8, mixed vs FP64 BDDC; p50/p99 solve latency"

# which kernels are bound by HBM bytes and which by FP64 arithmetic
KERNEL_BOUND = {"partial_chol": "mfma", "partial_chol_l2": "mfma"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_0911_5730_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".hpp", ".cpp")):
            h.update(open(os.path.join(csrc, name), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when the kernels changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    data = json.load(open(path))
    ent = data.get(workload, {}).get(kernel)
    if not ent or ent.get("source_hash") != kernel_source_hash():
        return None
    return ent.get("bytes_per_launch")


def cpu_baseline(prob_full):
    """The oracle on a bounded sample of the same workload: the lower-left
    quarter of the 256 x 256 coefficient field (128 x 128 elements, 8 x 8
    substructures with H/h = 16, three levels with 2 x 2 groups, tau = 10),
    set up and solved to 1e-8; scaled by the substructure count (x4) to one
    full solve."""
    import numpy as np

    import synth
    from oracle import pcg
    from oracle.bddc import BDDC

    nx = prob_full.nx // 2
    k = prob_full.coeff.reshape(prob_full.ny, prob_full.nx)[:nx, :nx].reshape(-1).copy()
    sample = synth.square_problem(nx, 8, levels=3, groups=(2, 2), constraints="adaptive", tau=prob_full.tau,
                                  seed=2000)
    sample.coeff = k
    threads = 1
    try:
        from threadpoolctl import threadpool_info
        info = threadpool_info()
        if info:
            threads = max(int(p.get("num_threads", 1)) for p in info)
    except Exception:
        pass
    t0 = time.perf_counter()
    B = BDDC(sample)
    out = pcg.solve(B, sample.f[0], rtol=prob_full.rtol)
    t = time.perf_counter() - t0
    scale = prob_full.nsub / sample.nsub
    return {"value": 1.0 / (t * scale), "unit": "solves/s", "cores": threads, "kind": "oracle",
            "sample": f"oracle setup+PCG on the 128x128 lower-left quarter of the workload's coefficient "
                      f"field (64 substructures, 3 levels, tau=10): {t:.2f} s, {out['iters']} iterations; "
                      f"scaled x{scale:g} by substructure count to one full solve",
            "host_cpus": len(os.sched_getaffinity(0))}


def precision_forms(P, synth, torch, cid: int, stream, precs=("fp64", "fp32", "bf16")) -> dict:
    """Setup time, solves/s (preconditioner reused) and the level-1 apply
    kernels' HBM rates for each precision form of one workload.  The reduced
    forms store the level-1 T_rr and Psi in FP32 or BF16 (inverse Cholesky
    factor) and keep the outer PCG, S, averaging, deeper levels and coarsest
    factor in FP64."""
    prob = synth.config(cid)
    coeff = torch.tensor(prob.coeff, dtype=torch.float64, device="cuda")
    f = torch.tensor(prob.f[0], dtype=torch.float64, device="cuda")
    u = torch.empty_like(f)
    out = {}
    for prec in precs:
        P.Solver(prob, coeff=coeff, stream=stream, precision=prec).close()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            P.Solver(prob, coeff=coeff, stream=stream, precision=prec).close()
        torch.cuda.synchronize()
        setup_ms = (time.perf_counter() - t0) / 3 * 1e3
        S = P.Solver(prob, coeff=coeff, stream=stream, precision=prec)
        _, it, rr = S.solve(f, u=u, rtol=prob.rtol, stream=stream)
        torch.cuda.synchronize()
        ns = 8
        t0 = time.perf_counter()
        for _ in range(ns):
            S.solve(f, u=u, rtol=prob.rtol, stream=stream)
        torch.cuda.synchronize()
        solve_s = (time.perf_counter() - t0) / ns
        kern = {}
        for name, label in (("schur_local", "matvec"), ("apply_restrict", "update_restrict")):
            P.timing_start(name, 1)
            S.solve(f, u=u, rtol=prob.rtol, stream=stream)
            tm = P.timing_stop()
            us = tm["ms"] / max(1, tm["launches"]) * 1e3
            by = tm["bytes"] / max(1, tm["launches"])
            gbs = by / (us * 1e-6) / 1e9 if us > 0 else 0.0
            kern[label] = {"avg_launch_us": us, "algorithmic_bytes_per_launch": by, "achieved_GBs": gbs,
                           "frac_of_hbm_peak": gbs / PEAK_HBM_GBS, "launches": tm["launches"]}
        S.close()
        out[prec] = {"solves_per_s": 1.0 / solve_s, "solve_ms": solve_s * 1e3, "iterations": int(it[0]),
                     "relres": float(rr[0]), "setup_ms": setup_ms, "apply_kernels": kern}
        log(f"bench: config {cid} {prec}: {1.0 / solve_s:.1f} solves/s, {int(it[0])} iterations, "
            f"setup {setup_ms:.2f} ms")
    for prec in precs:
        out[prec]["solves_vs_fp64"] = out[prec]["solves_per_s"] / out["fp64"]["solves_per_s"]
    return out


def blocked_rhs(P, synth, torch, cid: int, stream, nrhs: int = 8, precs=("fp64", "fp32")) -> dict:
    """Right-hand sides solved per second (preconditioner set up once) with
    `nrhs` seeded loads in one blocked solve, against the same loads solved one
    at a time (BDDC_SOLVE_BLOCK=1); the iterates are the same bitwise."""
    prob = synth.config(cid, nrhs=nrhs)
    coeff = torch.tensor(prob.coeff, dtype=torch.float64, device="cuda")
    F = torch.tensor(prob.f, dtype=torch.float64, device="cuda")
    U = torch.empty_like(F)
    out = {}
    for prec in precs:
        S = P.Solver(prob, coeff=coeff, stream=stream, precision=prec)
        res = {}
        for mode in ("blocked", "one_at_a_time"):
            if mode == "one_at_a_time":
                os.environ["BDDC_SOLVE_BLOCK"] = "1"
            try:
                _, it, _ = S.solve(F, u=U, rtol=prob.rtol, stream=stream)
                torch.cuda.synchronize()
                reps = 5
                t0 = time.perf_counter()
                for _ in range(reps):
                    S.solve(F, u=U, rtol=prob.rtol, stream=stream)
                torch.cuda.synchronize()
                dt = (time.perf_counter() - t0) / reps
            finally:
                os.environ.pop("BDDC_SOLVE_BLOCK", None)
            res[mode] = {"rhs_per_s": nrhs / dt, "ms_per_solve_call": dt * 1e3, "iterations_max": int(max(it))}
        S.close()
        res["speedup"] = res["blocked"]["rhs_per_s"] / res["one_at_a_time"]["rhs_per_s"]
        out[prec] = res
        log(f"bench: config {cid} {prec}: {nrhs} rhs blocked {res['blocked']['rhs_per_s']:.1f}/s, one at a time "
            f"{res['one_at_a_time']['rhs_per_s']:.1f}/s")
    return out


def autotuned(P, synth, torch, cid: int, stream, nrhs: int) -> dict:
    """bddc_autotune on one workload (the preconditioner set up once): the
    configuration it chose and right-hand sides per second with the default
    launch configuration and with the tuned one (a fresh handle of the same
    shape starts from the remembered choice)."""
    prob = synth.config(cid, nrhs=nrhs)
    coeff = torch.tensor(prob.coeff, dtype=torch.float64, device="cuda")
    F = torch.tensor(prob.f, dtype=torch.float64, device="cuda")
    U = torch.empty_like(F)

    def rate(S):
        S.solve(F, u=U, rtol=prob.rtol, stream=stream)
        torch.cuda.synchronize()
        reps = 5
        t0 = time.perf_counter()
        for _ in range(reps):
            S.solve(F, u=U, rtol=prob.rtol, stream=stream)
        torch.cuda.synchronize()
        return nrhs * reps / (time.perf_counter() - t0)

    S = P.Solver(prob, coeff=coeff, stream=stream)
    default = S.tuning()
    r0 = rate(S)
    t = S.autotune(F, u=U, rtol=prob.rtol, reps=3, stream=stream)
    S.close()
    S = P.Solver(prob, coeff=coeff, stream=stream)
    r1 = rate(S)
    assert S.tuning()["deep_path"] == t["deep_path"]
    S.close()
    log(f"bench: config {cid}, {nrhs} rhs: default {r0:.1f}/s, tuned {r1:.1f}/s ({t})")
    return {"default": {k: default[k] for k in ("deep_path", "finalize", "graph", "check")}, "default_rhs_per_s": r0,
            "tuned": {k: t[k] for k in ("deep_path", "finalize", "graph", "check")}, "tuned_rhs_per_s": r1}


def batching_form(P, synth, torch, stream, precision: str = "fp32") -> dict:
    """Config 4 (2048 x 2048, 9216 uneven Voronoi regions, three levels,
    eight loads): set-up time, then the eight loads in one blocked solve
    (FP32 form, FP64 outer PCG) and the same loads one at a time."""
    prob = synth.config(4, nrhs=8)
    coeff = torch.tensor(prob.coeff, dtype=torch.float64, device="cuda")
    F = torch.tensor(prob.f, dtype=torch.float64, device="cuda")
    U = torch.empty_like(F)
    P.Solver(prob, coeff=coeff, stream=stream, precision=precision).close()   # first use of the sizes
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S = P.Solver(prob, coeff=coeff, stream=stream, precision=precision)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    out = {"setup_s": setup_s, "n_free": prob.n_free, "substructures": prob.nsub, "nc": S.info()["nc"],
           "precision": precision}
    for mode in ("blocked", "one_at_a_time"):
        if mode == "one_at_a_time":
            os.environ["BDDC_SOLVE_BLOCK"] = "1"
        try:
            _, it, rr = S.solve(F, u=U, rtol=prob.rtol, stream=stream)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            S.solve(F, u=U, rtol=prob.rtol, stream=stream)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
        finally:
            os.environ.pop("BDDC_SOLVE_BLOCK", None)
        out[mode] = {"rhs_per_s": 8 / dt, "ms_per_solve_call": dt * 1e3, "iterations_max": int(max(it)),
                     "relres_max": float(max(rr))}
    S.close()
    log(f"bench: config 4: setup {setup_s:.2f} s, 8 rhs blocked {out['blocked']['rhs_per_s']:.1f}/s, "
        f"one at a time {out['one_at_a_time']['rhs_per_s']:.1f}/s, {out['blocked']['iterations_max']} iterations")
    return out


def concurrent_steps(P, prob, coeff, f, torch, nsteps: int, nstreams: int = 2) -> float:
    """Whole steps (set-up, solve, destroy) of independent problems issued from
    `nstreams` host threads, each with a stream and handles of its own, so one
    problem's host set-up work overlaps another's kernels.  Returns steps/s."""
    import threading
    streams = [torch.cuda.Stream() for _ in range(nstreams)]
    outs = [torch.empty_like(f) for _ in range(nstreams)]
    errors = []

    def worker(k):
        try:
            for _ in range(k, nsteps, nstreams):
                S = P.Solver(prob, coeff=coeff, stream=streams[k])
                S.solve(f, u=outs[k], rtol=prob.rtol, stream=streams[k])
                S.close()
        except Exception as e:  # reported after the join
            errors.append(e)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    th = [threading.Thread(target=worker, args=(k,)) for k in range(nstreams)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if errors:
        raise errors[0]
    return nsteps / (t1 - t0)


def serving(synth, count: int = 40, rate: float = 200.0, slots: int = 2, precision: str = "fp32",
            problems=None, resident: bool = False) -> dict:
    """A seeded Poisson stream of requests (grid side 128 or 256, H/h 8 or 16,
    2-3 levels, k = 10^U(0,m), m in 0..6, 1-4 right-hand sides, adaptive
    tau = 10) submitted at their arrival times to the serving loop; with
    `problems`, the requests share that many problems (loads of their own),
    and with `resident` the server keeps set-up problems and merges the
    pending loads of one problem into one blocked solve."""
    from paper_0911_5730_amd.serve import Request, Server
    stream = synth.request_stream(count, rate=rate, problems=problems)
    srv = Server(slots=slots, resident=resident)
    try:
        t0 = srv.now()
        for t, prob in stream:
            wait = t - (srv.now() - t0)
            if wait > 0:
                time.sleep(wait)
            key = prob.meta.get("problem") if problems else None
            srv.submit(Request(prob=prob, rhs=prob.f, precision=precision, arrival=srv.now(), key=key))
        srv.drain()
    finally:
        srv.close()
    bad = [r for r in srv.finished if r.error is not None]
    if bad:
        raise bad[0].error
    st = srv.stats()
    st.update({"rate_per_s": rate, "precision": precision, "problems": problems,
               "rhs": int(sum(p.f.shape[0] for _, p in stream))})
    return st


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16"],
                    help="storage of the level-1 preconditioner operators in the timed steps")
    ap.add_argument("--roofline-kernel", default="deep",
                    help="library kernel timed for the roofline (default: the one with the largest share of a step)")
    ap.add_argument("--sample-every", type=int, default=8,
                    help="time one in this many launches of the roofline kernel")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true", help="skip the request-stream measurement")
    ap.add_argument("--no-blocked", action="store_true", help="skip the blocked right-hand-side measurement")
    ap.add_argument("--no-autotune", action="store_true", help="skip the autotuner measurement")
    ap.add_argument("--no-batching", action="store_true", help="skip the config-4 (uneven substructures) measurement")
    ap.add_argument("--no-precision-forms", action="store_true",
                    help="skip the FP64 / FP32 / BF16 comparison on configs 2 and 3")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy a 256 MiB device buffer three times (reference for the HBM byte counters)")
    args = ap.parse_args()
    ws = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or ws != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the substructures of one problem run on a single MI355X)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_0911_5730_amd as P
    import synth

    torch.cuda.set_device(0)
    if args.copy_calibration:
        n = COPY_BYTES // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration": {"bytes_read": COPY_BYTES, "bytes_written": COPY_BYTES, "copies": 3}}))
        return
    prob = synth.config(args.config)
    coeff = torch.tensor(prob.coeff, dtype=torch.float64, device="cuda")
    f = torch.tensor(prob.f[0], dtype=torch.float64, device="cuda")
    u = torch.empty_like(f)
    stream = torch.cuda.current_stream()

    def step():
        S = P.Solver(prob, coeff=coeff, stream=stream, precision=args.precision)
        _, it, rr = S.solve(f, u=u, rtol=prob.rtol, stream=stream)
        info = S.info()
        S.close()
        return it[0], rr[0], info

    log(f"bench: config {args.config} ({synth.CONFIG_NAMES[args.config]}), warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # ---- timed region: K whole steps
    P.timing_start(args.roofline_kernel, args.sample_every)
    lat = []
    iters = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        it, rr, info = step()
        lat.append(time.perf_counter() - ts)
        iters.append(it)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tm = P.timing_stop()
    elapsed = t1 - t0
    log(f"bench: {args.steps} steps in {elapsed:.3f} s, iterations {iters[0]}, relres {rr:.2e}")

    # ---- solve-only, apply-only and setup-only rates (outside the timed region)
    S = P.Solver(prob, coeff=coeff, stream=stream, precision=args.precision)
    S.solve(f, u=u)
    torch.cuda.synchronize()
    ns = max(5, args.steps)
    s0 = time.perf_counter()
    for _ in range(ns):
        S.solve(f, u=u)
    torch.cuda.synchronize()
    solve_s = (time.perf_counter() - s0) / ns
    # the full-space preconditioner z = M^-1 r (bddc_apply) on one vector
    z = torch.empty_like(f)
    S.apply(f, z, stream=stream)
    torch.cuda.synchronize()
    na = 20 * ns
    a0 = time.perf_counter()
    for _ in range(na):
        S.apply(f, z, stream=stream)
    torch.cuda.synchronize()
    apply_s = (time.perf_counter() - a0) / na
    S.close()
    # set-ups alone, with the interior elimination timed for its MFMA roofline
    P.timing_start("partial_chol", 1)
    su0 = time.perf_counter()
    for _ in range(ns):
        P.Solver(prob, coeff=coeff, stream=stream, precision=args.precision).close()
    torch.cuda.synchronize()
    setup_s = (time.perf_counter() - su0) / ns
    tch = P.timing_stop()
    ch_ms = tch["ms"] / max(1, tch["launches"])
    ch_tf = (tch["flops"] / max(1, tch["launches"])) / (ch_ms * 1e-3) / 1e12 if tch["launches"] else 0.0
    setup_roof = {"kernel": "partial_chol", "bound": "mfma", "achieved": ch_tf, "peak": PEAK_FP64_TFLOPS,
                  "unit": "TFLOP/s", "frac": ch_tf / PEAK_FP64_TFLOPS, "avg_launch_us": ch_ms * 1e3,
                  "flops_per_launch": tch["flops"] / max(1, tch["launches"]), "launches": tch["launches"]}

    # ---- roofline of the chosen kernel, from the events of the timed region
    kernel = args.roofline_kernel
    bound = KERNEL_BOUND.get(kernel, "hbm")
    per_launch_ms = tm["ms"] / max(1, tm["launches"])
    workload = f"config{args.config}"
    if bound == "hbm":
        achieved = (tm["bytes"] / max(1, tm["launches"])) / (per_launch_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": achieved / PEAK_HBM_GBS}
    else:
        achieved = (tm["flops"] / max(1, tm["launches"])) / (per_launch_ms * 1e-3) / 1e12
        roof = {"bound": bound, "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP64_TFLOPS}
    roof.update({"kernel": kernel, "launches": tm["launches"], "avg_launch_us": per_launch_ms * 1e3,
                 "algorithmic_bytes_per_launch": tm["bytes"] / max(1, tm["launches"]),
                 "traffic": measured_traffic(kernel, workload)})

    # the same steps from two host threads on two streams (independent problems in flight)
    conc = concurrent_steps(P, prob, coeff, f, torch, max(2 * args.steps, 8))
    log(f"bench: two streams: {conc:.1f} steps/s")
    lat_ms = np.array(lat) * 1e3
    out = {
        "metric": METRIC,
        "value": args.steps / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded coefficient field, partition and load)",
        "config": {"workload": workload + ": " + synth.CONFIG_NAMES[args.config], "n_free": prob.n_free,
                   "substructures": prob.nsub, "levels": prob.levels, "tau": prob.tau,
                   "precision": args.precision, "rtol": prob.rtol, "step": "setup + PCG solve + destroy"},
        "latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99))},
        "concurrent_steps_per_s": {"value": conc, "streams": 2,
                                   "note": "independent steps from two host threads, one stream each; a set-up's "
                                           "host work overlaps the other problem's kernels"},
        "solve_only_per_s": 1.0 / solve_s,
        "applies_per_s": 1.0 / apply_s,
        "setup_ms": setup_s * 1e3,
        "iterations": iters[0],
        "nc": info["nc"],
        "indicator": info["indicator"],
        "kappa": info["kappa"],
        "roofline": roof,
        "setup_roofline": setup_roof,
    }
    if not args.no_serving:
        out["serving"] = {"two_slots": serving(synth, slots=2), "one_slot": serving(synth, slots=1),
                          "shared_problems": serving(synth, count=120, rate=2000.0, slots=2, problems=4),
                          "shared_problems_resident": serving(synth, count=120, rate=2000.0, slots=2, problems=4,
                                                              resident=True),
                          "note": "requests/s over the stream and arrival-to-completion latency; each request is "
                                  "set up, solved to 1e-8 and released on a slot with its own stream; "
                                  "shared_problems: 120 requests at 2000/s over 4 problems (loads of their own), "
                                  "_resident: set-up problems kept and pending loads of one problem merged into "
                                  "one blocked solve"}
        sv = out["serving"]
        log(f"bench: serving {sv['two_slots']['solves_per_s']:.1f} req/s (two slots); shared problems "
            f"{sv['shared_problems']['solves_per_s']:.1f} req/s, resident {sv['shared_problems_resident']['solves_per_s']:.1f}"
            f" req/s (p99 {sv['shared_problems']['latency_ms']['p99']:.1f} -> "
            f"{sv['shared_problems_resident']['latency_ms']['p99']:.1f} ms)")
    if not args.no_precision_forms:
        out["precision_forms"] = {
            "note": "solves/s with the preconditioner set up once; FP32 / BF16 = reduced storage of the level-1 "
                    "T_rr and Psi streamed every iteration (BF16: inverse Cholesky factor), FP64 outer PCG",
            "config2": precision_forms(P, synth, torch, 2, stream),
            "config3": precision_forms(P, synth, torch, 3, stream),
        }
    if not args.no_blocked:
        out["blocked_rhs"] = {
            "note": "right-hand sides per second, 8 seeded loads in one blocked PCG (each launch applies its "
                    "operator block to every column still iterating) against the same loads one at a time",
            "config2": blocked_rhs(P, synth, torch, 2, stream),
            "config3": blocked_rhs(P, synth, torch, 3, stream),
        }
    if not args.no_batching:
        out["batching_form"] = dict(batching_form(P, synth, torch, stream),
                                    note="config 4: 2048x2048 Q1, 9216 jittered Voronoi regions (152-927 dofs) in "
                                         "576 groups, k = 10^U(0,4), adaptive tau = 10, 8 loads; regions smaller than "
                                         "the workload's 1500-6000 dofs (dense local factors, see the design notes)")
    if not args.no_autotune:
        out["autotune"] = {
            "note": "launch configuration chosen by bddc_autotune (deep-level path, partial-sum mode, graph, "
                    "iterations per chunk) and right-hand sides per second before and after",
            "config2_1rhs": autotuned(P, synth, torch, 2, stream, 1),
            "config3_8rhs": autotuned(P, synth, torch, 3, stream, 8),
        }
    if not args.no_cpu_baseline:
        log("bench: timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(prob)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
