#!/usr/bin/env python3
"""Throughput of adaptive-multilevel BDDC PCG solves on one MI355X.

Workload (default): Q1 diffusion on a 1024 x 1024 grid (1,046,529 unknowns),
64 x 64 substructures (H/h = 16), three levels with 16 x 16 groups, k = 1,
adaptive coarse dofs with tau = 10, f ~ U[-1, 1], PCG to relative residual
1e-8.

One step is one bddc_solve of the load with a set-up preconditioner: PCG on
the level-1 interface with the three-level preconditioner (substructure
corrections, stiffness-scaled averaging, the level-2 problem and the
coarsest solve every iteration) and the interior recovery.  The timed steps
run the mixed form (level-1 preconditioner operators stored in FP32, FP64
outer PCG); the FP64 path is timed beside it on the same load, and the
set-up (local matrices, interior elimination, per-edge eigenproblems,
constrained factors, next level, coarsest factor) is timed separately.
Coefficients and load are resident in HBM before timing.

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


def elasticity_form(P, synth, torch, stream, reps: int = 5) -> dict:
    """The paper's own experiment (Section 6, Tables 1-7): plane elasticity
    (lambda = 1, mu = 2), 768 x 768 Q1 mesh (1,176,578 free dofs, whole
    boundary clamped), 48 x 48 substructures (H/h = 16), 3 x 3 level-2
    substructures for three levels, one jagged edge on each level.  For two
    and three levels and constraints c, c+e and adaptive with tau = 10, 3, 2:
    coarse dofs per level, C (coarse problem size over a substructure's
    dofs), the indicator omega-tilde, the Lanczos condition estimate,
    iterations to 1e-8, and solves/s in the mixed form and in FP64; the pair
    eigenvalues of Table 3 (level 1, tau = 10) and Tables 4 and 5 (level 2,
    tau = 2 and 10)."""
    ns, groups, hh = 48, 3, 16

    def edge_eigs(S, level, pairs):
        want = {tuple(sorted(p)): None for p in pairs}
        e = 0
        while any(v is None for v in want.values()):
            lam, nsel, pr = S.edge_eigs(level, e)
            key = (int(pr[0]), int(pr[1]))
            if key in want:
                want[key] = [round(float(x), 3) for x in lam[:8]]
            e += 1
        return want

    rows = []
    eigs = {}
    for levels in (2, 3):
        for kind, tau in (("corners", float("inf")), ("corners_edges", float("inf")), ("adaptive", 10.0),
                          ("adaptive", 3.0), ("adaptive", 2.0)):
            prob = synth.paper_elasticity_problem(hh * ns, ns, levels=levels, groups=groups, constraints=kind,
                                                  tau=tau, seed=50)
            f = torch.tensor(prob.f[0], dtype=torch.float64, device="cuda")
            u = torch.empty_like(f)
            row = {"levels": levels, "constraints": kind, "tau": tau if kind == "adaptive" else None}
            for prec in ("fp32", "fp64"):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                S = P.Solver(prob, stream=stream, precision=prec)
                torch.cuda.synchronize()
                setup = time.perf_counter() - t0
                _, it, rr = S.solve(f, u=u, rtol=prob.rtol, stream=stream)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(reps):
                    S.solve(f, u=u, rtol=prob.rtol, stream=stream)
                torch.cuda.synchronize()
                dt = (time.perf_counter() - t0) / reps
                info = S.info()
                nc = list(info["nc"])
                if prec == "fp64":
                    nblk = 1 if levels == 2 else groups * groups
                    row.update(nc=nc, C=round(nc[0] / nblk / (prob.n_free / prob.nsub), 2),
                               omega=info["indicator"] if kind == "adaptive" else None, kappa=info["kappa"],
                               iterations=int(it[0]), relres=float(rr[0]))
                    if kind == "adaptive" and tau == 10.0 and levels == 2:
                        # substructures numbered from one, row by row
                        pairs = [(1, 2), (1, 49), (2, 3), (2, 50), (3, 4), (3, 51), (49, 50), (50, 51), (50, 98)]
                        got = edge_eigs(S, 1, [(a - 1, b - 1) for a, b in pairs])
                        eigs["table3_level1_tau10"] = {f"{a},{b}": got[(a - 1, b - 1)] for a, b in pairs}
                    if kind == "adaptive" and tau in (2.0, 10.0) and levels == 3:
                        pairs = [(1, 2), (1, 4), (2, 3), (2, 5), (3, 6), (4, 7), (5, 6), (5, 8), (8, 9)]
                        got = edge_eigs(S, 2, [(a - 1, b - 1) for a, b in pairs])
                        eigs[f"table{4 if tau == 2.0 else 5}_level2_tau{tau:g}"] = {
                            f"{a},{b}": got[(a - 1, b - 1)] for a, b in pairs}
                row[prec] = {"solves_per_s": 1.0 / dt, "solve_ms": dt * 1e3, "iterations": int(it[0]),
                             "setup_ms": setup * 1e3}
                S.close()
            row["mixed_vs_fp64"] = row["fp32"]["solves_per_s"] / row["fp64"]["solves_per_s"]
            log(f"bench: paper elasticity L={levels} {kind} tau={row['tau']}: nc {row['nc']}, C {row['C']}, "
                f"omega {row['omega']}, kappa {row['kappa']:.2f}, {row['iterations']} it; "
                f"fp32 {row['fp32']['solves_per_s']:.1f}/s, fp64 {row['fp64']['solves_per_s']:.1f}/s")
            rows.append(row)
    return {"workload": "768x768 Q1 plane elasticity (lambda 1, mu 2), 48x48 substructures (H/h = 16), "
                        "3x3 level-2 substructures, one jagged edge per level, whole boundary clamped, "
                        "f ~ U[-1, 1]", "n_free": 2 * 767 * 767, "rows": rows, "pair_eigenvalues": eigs}


def batching_form(P, synth, torch, stream, precs=("fp32", "fp64")) -> dict:
    """Config 4 (2048 x 2048, about 1024 uneven Voronoi regions, three levels,
    eight loads): for each precision form (set up one after the other), the
    set-up time and the eight loads in one blocked solve; the mixed form also
    one load at a time."""
    prob = synth.config(4, nrhs=8)
    coeff = torch.tensor(prob.coeff, dtype=torch.float64, device="cuda")
    F = torch.tensor(prob.f, dtype=torch.float64, device="cuda")
    U = torch.empty_like(F)
    out = {"n_free": prob.n_free, "substructures": prob.nsub}
    for prec in precs:
        P.Solver(prob, coeff=coeff, stream=stream, precision=prec).close()   # first use of the sizes
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S = P.Solver(prob, coeff=coeff, stream=stream, precision=prec)
        torch.cuda.synchronize()
        res = {"setup_s": time.perf_counter() - t0, "nc": S.info()["nc"],
               "device_gb": S.info()["device_bytes"] / 1e9}
        modes = ("blocked", "one_at_a_time") if prec == precs[0] else ("blocked",)
        for mode in modes:
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
            res[mode] = {"rhs_per_s": 8 / dt, "ms_per_solve_call": dt * 1e3, "iterations_max": int(max(it)),
                         "relres_max": float(max(rr))}
        S.close()
        out[prec] = res
        log(f"bench: config 4 {prec}: setup {res['setup_s']:.2f} s, 8 rhs blocked {res['blocked']['rhs_per_s']:.1f}/s, "
            f"{res['blocked']['iterations_max']} iterations")
    if "fp64" in out and precs[0] in out:
        out["mixed_vs_fp64"] = out[precs[0]]["blocked"]["rhs_per_s"] / out["fp64"]["blocked"]["rhs_per_s"]
    return out


def serving(synth, count: int = 40, rate: float = 200.0, slots: int = 4, precision: str = "fp32",
            problems=None, resident: bool = False, full: bool = False) -> dict:
    """A seeded Poisson stream of requests submitted at their arrival times to
    the continuous-batching server.  full: the serving workload (grid side
    128-1024, H/h 8-32, two or three levels, k = 10^U(0,m), m in 0..6, 1-16
    right-hand sides, adaptive tau = 10); else sides 128/256, H/h 8/16, 1-4
    right-hand sides, and with `problems` the requests share that many
    problems (loads of their own), kept set up with `resident`."""
    from paper_0911_5730_amd.serve import Request, Server
    stream = (synth.serving_stream(count, rate=rate) if full
              else synth.request_stream(count, rate=rate, problems=problems))
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


# kernels whose launches may dominate a PCG iteration (timed in a pre-pass;
# the one with the largest share is timed in the timed region)
ROOFLINE_CANDIDATES = ("schur_local", "apply_restrict", "apply_average", "deep", "wide_pre", "wide_restrict",
                       "wide_coarse", "wide_post")


def solve_rate(S, f, u, stream, torch, steps, rtol):
    """`steps` bddc_solve calls of one load on a set-up handle: solves/s and
    the per-solve wall times (each call synchronises its stream)."""
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its = None
    for _ in range(steps):
        ts = time.perf_counter()
        _, its, _ = S.solve(f, u=u, rtol=rtol, stream=stream)
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    return steps / (time.perf_counter() - t0), lat, its


def dominant_kernel(P, S, f, u, stream, rtol):
    """The library kernel with the largest summed time over one solve."""
    best, best_ms, shares = None, -1.0, {}
    for name in ROOFLINE_CANDIDATES:
        P.timing_start(name, 1)
        S.solve(f, u=u, rtol=rtol, stream=stream)
        tm = P.timing_stop()
        shares[name] = tm["ms"]
        if tm["launches"] and tm["ms"] > best_ms:
            best, best_ms = name, tm["ms"]
    return best, shares


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(gpu_rates: dict) -> dict:
    """The oracle timed on this host: the full config-2 problem (256 x 256,
    65,025 unknowns, three levels, adaptive tau = 10), set up and solved to
    1e-8 with every BLAS thread, and config 1 with every thread and with one.
    Configs 3 and 4 are not run (the oracle's set-up alone takes tens of
    minutes there) and are reported as not completed."""
    import synth
    from oracle import pcg
    from oracle.bddc import BDDC
    threads = 1
    limiter = None
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        info = threadpool_info()
        if info:
            threads = max(int(p.get("num_threads", 1)) for p in info)
        limiter = threadpool_limits
    except Exception:
        pass

    def run(cid):
        prob = synth.config(cid)
        t0 = time.perf_counter()
        B = BDDC(prob)
        t1 = time.perf_counter()
        out = pcg.solve(B, prob.f[0], rtol=prob.rtol)
        t2 = time.perf_counter()
        return {"setup_s": t1 - t0, "solve_s": t2 - t1, "total_s": t2 - t0, "iterations": out["iters"],
                "solves_per_s": 1.0 / (t2 - t0), "solve_only_per_s": 1.0 / (t2 - t1)}

    c2 = run(2)
    c1 = run(1)
    c1_1t = None
    if limiter is not None:
        with limiter(limits=1):
            c1_1t = run(1)
    return {"value": c2["solves_per_s"], "unit": "solves/s", "cores": threads, "kind": "oracle",
            "sample": f"the full config-2 problem (256x256 Q1, 65,025 unknowns, 16x16 substructures, 3 levels, "
                      f"adaptive tau=10): oracle set-up {c2['setup_s']:.1f} s + PCG {c2['solve_s']:.1f} s "
                      f"({c2['iterations']} iterations), no scaling; configs 3 and 4 not completed (oracle "
                      f"set-up beyond the bench's time budget)",
            "cpu_model": cpu_model(), "host_cpus": len(os.sched_getaffinity(0)), "blas_threads": threads,
            "config2": c2, "config1": c1, "config1_one_thread": c1_1t,
            "config3": "not completed", "config4": "not completed",
            "gpu_config2_fp64_solves_per_s": gpu_rates.get("config2_fp64"),
            "gpu_config2_setup_plus_solve_per_s": gpu_rates.get("config2_step")}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--precision", default="fp32", choices=["fp64", "fp32", "bf16"],
                    help="precision form of the timed solves (the FP64 path is timed beside it)")
    ap.add_argument("--roofline-kernel", default="auto",
                    help="library kernel timed for the roofline (auto: the one with the largest share of a solve)")
    ap.add_argument("--sample-every", type=int, default=8,
                    help="time one in this many launches of the roofline kernel")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true", help="skip the request-stream measurement")
    ap.add_argument("--no-blocked", action="store_true", help="skip the blocked right-hand-side measurement")
    ap.add_argument("--no-autotune", action="store_true", help="skip the autotuner measurement")
    ap.add_argument("--no-batching", action="store_true", help="skip the config-4 (uneven substructures) measurement")
    ap.add_argument("--no-elasticity", action="store_true", help="skip the plane-elasticity measurement")
    ap.add_argument("--elasticity-only", action="store_true",
                    help="only the plane-elasticity measurement (one JSON line)")
    ap.add_argument("--no-precision-forms", action="store_true",
                    help="skip the FP64 / FP32 / BF16 comparison on config 2")
    ap.add_argument("--batching-only", action="store_true",
                    help="only the config-4 (uneven substructures, eight loads) measurement, as one JSON line")
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
    if args.elasticity_only:
        print(json.dumps({"elasticity": elasticity_form(P, synth, torch, torch.cuda.current_stream())}))
        return
    if args.batching_only:
        print(json.dumps({"batching_form": batching_form(P, synth, torch, torch.cuda.current_stream())}))
        return
    prob = synth.config(args.config)
    coeff = torch.tensor(prob.coeff, dtype=torch.float64, device="cuda")
    f = torch.tensor(prob.f[0], dtype=torch.float64, device="cuda")
    u = torch.empty_like(f)
    stream = torch.cuda.current_stream()
    log(f"bench: config {args.config} ({synth.CONFIG_NAMES[args.config]}), {args.precision} against fp64")

    def setup(prec):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S = P.Solver(prob, coeff=coeff, stream=stream, precision=prec)
        torch.cuda.synchronize()
        return S, time.perf_counter() - t0

    P.Solver(prob, coeff=coeff, stream=stream, precision=args.precision).close()   # first use of the sizes
    S, setup_s = setup(args.precision)
    for _ in range(args.warmup):
        S.solve(f, u=u, rtol=prob.rtol, stream=stream)
    torch.cuda.synchronize()
    kernel = args.roofline_kernel
    shares = None
    if kernel == "auto":
        kernel, shares = dominant_kernel(P, S, f, u, stream, prob.rtol)
        log(f"bench: kernel time per solve (ms): " + ", ".join(f"{k} {v:.3f}" for k, v in shares.items() if v))

    # ---- timed region: K solves of the load with the set-up preconditioner
    P.timing_start(kernel, args.sample_every)
    rate, lat, its = solve_rate(S, f, u, stream, torch, args.steps, prob.rtol)
    tm = P.timing_stop()
    elapsed = args.steps / rate
    info = S.info()
    log(f"bench: {args.steps} {args.precision} solves in {elapsed:.4f} s ({rate:.1f}/s), {its[0]} iterations")

    # the full-space preconditioner z = M^-1 r (bddc_apply) on one vector
    z = torch.empty_like(f)
    S.apply(f, z, stream=stream)
    torch.cuda.synchronize()
    na = max(20, 4 * args.steps)
    a0 = time.perf_counter()
    for _ in range(na):
        S.apply(f, z, stream=stream)
    torch.cuda.synchronize()
    apply_s = (time.perf_counter() - a0) / na
    S.close()
    # ---- the FP64 path on the same load (outside the timed region; set up
    # after the mixed form is released, so the largest workloads fit)
    S64, setup64_s = setup("fp64")
    for _ in range(args.warmup):
        S64.solve(f, u=u, rtol=prob.rtol, stream=stream)
    # under the same conditions as the timed region above (the sampled
    # kernel timing armed: its events keep the iterations out of HIP graphs)
    P.timing_start(kernel, args.sample_every)
    rate64, lat64, its64 = solve_rate(S64, f, u, stream, torch, args.steps, prob.rtol)
    tm64 = P.timing_stop()
    S64.close()
    log(f"bench: fp64 {rate64:.1f} solves/s, {its64[0]} iterations; {args.precision}/fp64 = {rate / rate64:.3f}")
    # whole steps: set-up, solve, destroy
    nst = max(3, args.steps // 4)
    torch.cuda.synchronize()
    e0 = time.perf_counter()
    for _ in range(nst):
        S1, _ = setup(args.precision)
        S1.solve(f, u=u, rtol=prob.rtol, stream=stream)
        S1.close()
    torch.cuda.synchronize()
    step_s = (time.perf_counter() - e0) / nst
    # set-ups alone, with the level-1 interior elimination timed for its MFMA roofline
    P.timing_start("partial_chol", 1)
    su0 = time.perf_counter()
    for _ in range(nst):
        P.Solver(prob, coeff=coeff, stream=stream, precision=args.precision).close()
    torch.cuda.synchronize()
    setup_avg_s = (time.perf_counter() - su0) / nst
    tch = P.timing_stop()
    ch_ms = tch["ms"] / max(1, tch["launches"])
    ch_tf = (tch["flops"] / max(1, tch["launches"])) / (ch_ms * 1e-3) / 1e12 if tch["launches"] else 0.0
    setup_roof = {"kernel": "partial_chol", "bound": "mfma", "achieved": ch_tf, "peak": PEAK_FP64_TFLOPS,
                  "unit": "TFLOP/s", "frac": ch_tf / PEAK_FP64_TFLOPS, "avg_launch_us": ch_ms * 1e3,
                  "flops_per_launch": tch["flops"] / max(1, tch["launches"]), "launches": tch["launches"]}

    # ---- roofline of the dominant kernel, from the events of the timed region
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
                 "traffic": measured_traffic(kernel, f"{workload}_{args.precision}"),
                 "kernel_ms_per_solve": shares})
    lat_ms = np.array(lat) * 1e3
    lat64_ms = np.array(lat64) * 1e3
    out = {
        "metric": METRIC,
        "value": rate,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else f"{'f32' if args.precision == 'fp32' else 'bf16'}+f64",
        "data": "synthetic (seeded coefficient field, partition and load)",
        "config": {"workload": workload + ": " + synth.CONFIG_NAMES[args.config], "n_free": prob.n_free,
                   "substructures": prob.nsub, "levels": prob.levels, "tau": prob.tau,
                   "precision": args.precision, "rtol": prob.rtol,
                   "step": "one bddc_solve of one load to relative residual 1e-8 (PCG with the set-up "
                           "multilevel preconditioner, interior recovery); set-up excluded, reported beside"},
        "latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99))},
        "fp64": {"solves_per_s": rate64, "latency_ms": {"p50": float(np.percentile(lat64_ms, 50)),
                                                          "p99": float(np.percentile(lat64_ms, 99))},
                 "iterations": int(its64[0]), "setup_ms": setup64_s * 1e3,
                 "roofline_kernel_avg_launch_us": 1e3 * tm64["ms"] / max(1, tm64["launches"])},
        "mixed_vs_fp64": rate / rate64,
        "iterations": int(its[0]),
        "setup_ms": setup_s * 1e3,
        "setup_avg_ms": setup_avg_s * 1e3,
        "end_to_end_steps_per_s": 1.0 / step_s,
        "applies_per_s": 1.0 / apply_s,
        "nc": info["nc"],
        "indicator": info["indicator"],
        "kappa": info["kappa"],
        "roofline": roof,
        "setup_roofline": setup_roof,
    }
    gpu_rates = {}
    if not args.no_serving:
        out["serving"] = {"config5": serving(synth, count=60, full=True),
                          "config5_one_slot": serving(synth, count=60, full=True, slots=1),
                          "shared_problems": serving(synth, count=120, rate=2000.0, problems=4),
                          "shared_problems_resident": serving(synth, count=120, rate=2000.0, problems=4,
                                                              resident=True),
                          "note": "requests/s (and right-hand sides/s) over the stream and arrival-to-completion "
                                  "latency; config5: 60 requests of the serving workload at 200/s, set up when "
                                  "their HBM footprint fits, solved stepwise (up to 4 solves in flight, new ones "
                                  "joining between chunks of 8 iterations), mixed precision, rtol 1e-8; one_slot: "
                                  "one solve in flight; shared_problems: 120 requests at 2000/s over 4 problems, "
                                  "_resident: set-up problems kept and pending loads of one problem merged into "
                                  "one blocked solve"}
        sv = out["serving"]
        log(f"bench: serving config 5: {sv['config5']['solves_per_s']:.1f} req/s, p50/p99 "
            f"{sv['config5']['latency_ms']['p50']:.1f}/{sv['config5']['latency_ms']['p99']:.1f} ms (one solve in "
            f"flight: {sv['config5_one_slot']['solves_per_s']:.1f} req/s); shared problems "
            f"{sv['shared_problems']['solves_per_s']:.1f} req/s, resident "
            f"{sv['shared_problems_resident']['solves_per_s']:.1f} req/s")
    if not args.no_precision_forms:
        c2 = precision_forms(P, synth, torch, 2, stream)
        gpu_rates["config2_fp64"] = c2["fp64"]["solves_per_s"]
        gpu_rates["config2_step"] = 1.0 / (1e-3 * (c2["fp64"]["setup_ms"] + c2["fp64"]["solve_ms"]))
        out["precision_forms"] = {
            "note": "solves/s with the preconditioner set up once; FP32 / BF16 = reduced storage of the level-1 "
                    "T_rr and Psi streamed every iteration (BF16: inverse Cholesky factor), FP64 outer PCG",
            "config2": c2,
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
                                    note="config 4: " + synth.CONFIG_NAMES[4])
    if not args.no_elasticity:
        out["elasticity"] = elasticity_form(P, synth, torch, stream)
    if not args.no_autotune:
        out["autotune"] = {
            "note": "launch configuration chosen by bddc_autotune (deep-level path, partial-sum mode, graph, "
                    "iterations per chunk) and right-hand sides per second before and after",
            "config2_1rhs": autotuned(P, synth, torch, 2, stream, 1),
            "config3_8rhs": autotuned(P, synth, torch, 3, stream, 8),
        }
    if not args.no_cpu_baseline:
        log("bench: timing the CPU oracle (full config 2, config 1 with all threads and with one)")
        out["cpu_baseline"] = cpu_baseline(gpu_rates)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
