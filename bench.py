"""Benchmark: CholeskyQR2 of the 1048576 x 128 FP64 matrix (cond 1e6) on one MI355X.

One step = one full CholeskyQR2 (both passes and R = R2 R1) through the C ABI
(cqr2_factor) on a device-resident synthetic matrix A = G diag(logspace(0,-6,128)) V.
Prints one JSON line.  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]

--workload / --mixed time the other named problems (cqr2_factor_ex with the
given flags) with the same JSON layout; the default is the 1048576 x 128 one.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP64_PEAK_TFLOPS = 78.6        # MI355X dense FP64 (vector and matrix)
METRIC = "CQR2 GFLOP/s + HBM roofline % (1M\u00d7128 FP64); served solves/s, p99 latency"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_tall_1Mx128.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def flops_cqr2(m: int, n: int) -> float:
    """CholeskyQR2 flop count along its critical path: 4 m n^2 + 5 n^3 / 3."""
    return 4.0 * m * n * n + 5.0 * n ** 3 / 3.0


def flops_householder(m: int, n: int) -> float:
    """The paper's GFLOP/s numerator (Householder QR): 2 m n^2 - 2 n^3 / 3."""
    return 2.0 * m * n * n - 2.0 * n ** 3 / 3.0


# Timer classes of the library (cqr2_timing_read order) grouped by the kernel
# they time, per path.  64 < n <= 128: the MFMA 16x16x4 streaming kernels,
# pass 2's Gram fused into pass 1's Q1 (k_fused16).  n <= 64: the MFMA 4x4x4
# kernels, two Grams and two Q products.
KERNEL_CLASSES_S16 = {
    "k_fused16": ("q_pass1",),
    "k_apply16": ("q_pass2",),
    "k_gram16": ("gram",),
    "k_gram16_reduce": ("gram_reduce",),
    "k_cholinv": ("cholinv",),
    "k_upper_product_final": ("upper_product",),
}
KERNEL_CLASSES_SMALL = {
    "k_apply_rinv": ("q_pass1", "q_pass2"),
    "k_gram_partials": ("gram",),
    "k_gram_reduce": ("gram_reduce",),
    "k_cholinv": ("cholinv",),
    "k_upper_product_final": ("upper_product",),
}


def kernel_units(kernel: str, m: int, n: int):
    """Algorithmic work of ONE launch of `kernel` at (m, n): (flops, bytes).

    Flops count multiply-adds of the triangle actually needed (2 per product);
    bytes are the minimum HBM traffic: each operand read once, each output
    written once.
    """
    tri = m * n * (n + 1)            # 2 flops x (n (n+1) / 2 products per row)
    if kernel in ("k_gram_partials", "k_gram16"):
        return float(tri), 8.0 * m * n                  # reads A once
    if kernel in ("k_apply_rinv", "k_apply16"):
        return float(tri), 16.0 * m * n                 # reads A, writes Q
    if kernel == "k_fused16":
        return 2.0 * tri, 16.0 * m * n                  # Q1 = A U1 and the Gram of Q1: reads A, writes Q1
    if kernel == "k_gram16_reduce":
        return 0.0, 8.0 * 256 * 36 * 256                # partial Grams read once
    if kernel == "k_gram_reduce":
        ng = 1
        while ng < (n + 3) // 4:
            ng *= 2
        return 0.0, 8.0 * 256 * 16 * (ng * (ng + 1) // 2)
    if kernel == "k_cholinv":
        return 2.0 * n ** 3 / 3.0, 8.0 * n * n
    return 2.0 * n ** 3 / 3.0, 24.0 * n * n


def read_traffic(kernel: str):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they
    were taken on the current kernel source; else None."""
    from paper_1710_08471_amd.profiling import source_sha
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    k = t.get("kernels", {}).get(kernel)
    if k is None or k.get("source_sha") != source_sha(kernel):
        return None
    return float(k["bytes_per_launch"])


def cpu_baseline(a, budget_s: float):
    """The CPU oracle (plain FP64 CholeskyQR2, numpy) on this host."""
    import oracle
    try:
        from threadpoolctl import threadpool_info
    except ImportError:
        threadpool_info = None
    m, n = a.shape
    times = []
    t_start = time.perf_counter()
    while True:
        t0 = time.perf_counter()
        oracle.cqr2(a)
        times.append(time.perf_counter() - t0)
        if time.perf_counter() - t_start + times[-1] > budget_s or len(times) >= 25:
            break
    cores = os.cpu_count()
    if threadpool_info is not None:
        blas = [p for p in threadpool_info() if p.get("user_api") == "blas"]
        if blas:
            cores = int(blas[0].get("num_threads", cores))
    t = statistics.median(times)
    return {
        "value": round(flops_cqr2(m, n) / t / 1e9, 3),
        "unit": "GFLOP/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"the full {m}x{n} matrix, median of {len(times)} oracle CholeskyQR2 runs "
                  f"({t:.3f} s each, {sum(times):.1f} s of CPU work)",
    }


# Served stream (2000 requests of uneven shape, Poisson arrivals at a fixed
# rate); the rate is pinned well below the measured closed-loop capacity.
SERVE_REQUESTS = 2000
SERVE_SEED = 5
SERVE_RATE = 2500.0            # requests per second (open loop), about 0.2 of the closed-loop capacity
SERVE_ARENA = 16 << 30         # workspace arena of the server, bytes
SERVE_BUDGET = 64 << 30        # in-flight footprint budget (A, Q, R, workspace), bytes
SERVE_SLOTS = 256
SERVE_SUBMIT_PER_STEP = 64     # submissions between two server steps, at most


def device_checks(torch, a, q, r, x=None, b=None):
    """Invariants of a served result, computed on the device in FP64 (the
    comparison with the CPU oracle is the GPU tests' job): orthogonality,
    residual, R upper triangular with a positive diagonal, and for a
    least-squares request the optimality of X (Aᵀ(AX - B) = 0, relative)."""
    n = q.shape[1]
    qt = q.t().contiguous()
    eye = torch.eye(n, dtype=torch.float64, device=q.device)
    orth = float(torch.linalg.norm(qt @ q - eye))
    resid = float(torch.linalg.norm(a - q @ r) / torch.linalg.norm(a))
    upper = bool(torch.equal(r, torch.triu(r))) and bool((torch.diagonal(r) > 0).all())
    out = {"orthogonality": orth, "residual": resid,
           "ok": bool(orth <= 1e-12 and resid <= 1e-13 and upper)}
    if x is not None:
        at = a.t().contiguous()
        g = at @ (a @ x - b)
        scale = float(torch.linalg.norm(at @ a) * torch.linalg.norm(x) + torch.linalg.norm(at @ b))
        opt = float(torch.linalg.norm(g)) / scale
        out["normal_eq_rel"] = opt
        out["ok"] = bool(out["ok"] and opt <= 1e-12)
    return out


def serve_stream(cq, torch, count: int, rate: float, seed: int):
    """Closed-loop capacity and open-loop latency of the continuous-batching
    server on the request mix; a sample of results is checked on the device
    (device_checks)."""
    import numpy as np

    from synth import gdv_matrix_device, request_mix

    reqs = request_mix(count, rate, seed)
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    mats = [gdv_matrix_device(r.m, r.n, r.kappa, r.seed, device=dev) for r in reqs]
    qs = [cq.empty_colmajor(r.m, r.n, device=dev) for r in reqs]
    rs = [cq.empty_colmajor(r.n, r.n, device=dev) for r in reqs]
    torch.cuda.synchronize()
    total_a = sum(r.m * r.n * 8 for r in reqs)
    log(f"serving: {count} requests generated on the device in {time.perf_counter() - t0:.1f} s "
        f"({total_a / 1e9:.1f} GB of A)")

    # least-squares requests for the mixed-type run: every 4th request, nrhs 1..8
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed + 1)
    lsq = {r.idx: (torch.randn((1 + r.idx % 8, r.m), generator=gen, device=dev, dtype=torch.float64).t(),
                   cq.empty_colmajor(r.n, 1 + r.idx % 8, device=dev)) for r in reqs if r.idx % 4 == 0}

    def run(arrivals_ms, with_lstsq=False):
        done = {}
        steps = 0
        with cq.Server(SERVE_ARENA, SERVE_BUDGET, SERVE_SLOTS) as sv:
            sv.clock()
            h0 = time.perf_counter()
            i = 0
            while len(done) < count:
                now = (time.perf_counter() - h0) * 1e3
                batch_end = i + SERVE_SUBMIT_PER_STEP   # the first launch need not wait for every submission
                while i < min(count, batch_end) and arrivals_ms[i] <= now:
                    if with_lstsq and i in lsq:
                        sv.submit_lstsq(i, mats[i], lsq[i][0], lsq[i][1], qs[i], rs[i])
                    else:
                        sv.submit(i, mats[i], qs[i], rs[i])
                    i += 1
                sv.step()
                steps += 1
                for tag, ms in sv.poll():
                    done[tag] = ms
        lat = np.array([done[k] - arrivals_ms[k] for k in range(count)])
        span = max(done.values()) - min(arrivals_ms)
        return {"solves_per_s": round(count / (span / 1e3), 1), "p50_ms": round(float(np.percentile(lat, 50)), 3),
                "p99_ms": round(float(np.percentile(lat, 99)), 3), "makespan_ms": round(span, 2),
                "host_steps": steps}

    closed = run([0.0] * count)
    log(f"serving closed loop: {closed}")
    opened = run([r.arrival_s * 1e3 for r in reqs])
    log(f"serving open loop at {rate:.0f}/s: {opened}")
    # the same stream time-scaled to 0.5 and 0.8 of the measured capacity C
    at_frac = {}
    for frac in (0.5, 0.8):
        r_frac = round(frac * closed["solves_per_s"], -2)
        scale = rate / r_frac if r_frac > 0 else 1.0
        res = run([r.arrival_s * 1e3 * scale for r in reqs])
        res["rate_per_s"] = r_frac
        at_frac[frac] = res
        log(f"serving open loop at {r_frac:.0f}/s ({frac} C): {res}")

    # mixed request types: a quarter of the stream are least-squares solves
    mixed = run([r.arrival_s * 1e3 for r in reqs], with_lstsq=True)
    mixed["lstsq_requests"] = len(lsq)
    log(f"serving open loop at {rate:.0f}/s, 1 in 4 requests least squares: {mixed}")

    # device-side checks on the first request of every n in the mix (the last
    # run served the least-squares requests: their X is checked too)
    checked = []
    for nn in sorted({r.n for r in reqs}):
        k = next(r.idx for r in reqs if r.n == nn)
        c = device_checks(torch, mats[k], qs[k], rs[k])
        checked.append({"request": k, "m": reqs[k].m, "n": nn, **c})
    for nn in sorted({r.n for r in reqs}):
        k = next((r.idx for r in reqs if r.n == nn and r.idx in lsq), None)
        if k is None:
            continue
        c = device_checks(torch, mats[k], qs[k], rs[k], x=lsq[k][1], b=lsq[k][0])
        checked.append({"request": k, "m": reqs[k].m, "n": nn, "lstsq_nrhs": int(lsq[k][0].shape[1]), **c})
    return {
        "requests": count, "rate_per_s": rate, "seed": seed,
        "mix": "m log-uniform [1024,131072], n in {16,32,64,128,256}, kappa log-uniform [1e1,1e6]",
        "solves_per_s": opened["solves_per_s"], "p50_ms": opened["p50_ms"], "p99_ms": opened["p99_ms"],
        "closed_loop": closed, "open_loop": opened, "open_loop_0.5C": at_frac[0.5], "open_loop_0.8C": at_frac[0.8], "open_loop_lstsq_mix": mixed,
        "device_check_sample": checked,
        "slots": SERVE_SLOTS, "arena_bytes": SERVE_ARENA, "footprint_budget": SERVE_BUDGET,
    }


BATCHED_SHAPES = ((256, 4096, 128), (64, 16384, 256), (512, 2048, 32))  # (count, m, n)


def batched_leg(cq, torch, steps: int = 5, warmup: int = 2):
    """cqr2_factor_batched on sets of equal-shape problems (A = randn, column-major,
    generated on the device): ms per call, problems/s and CholeskyQR2 GFLOP/s of the
    whole batch, and the device checks of its first and last problem."""
    lib = cq.load()
    dev = torch.device("cuda:0")
    sp = cq.ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rows = []
    for count, m, n in BATCHED_SHAPES:
        gen = torch.Generator(device=dev)
        gen.manual_seed(7 * m + n)
        mats = [torch.randn((n, m), generator=gen, device=dev, dtype=torch.float64).t() for _ in range(count)]
        qs = [cq.empty_colmajor(m, n, device=dev) for _ in range(count)]
        rs = [cq.empty_colmajor(n, n, device=dev) for _ in range(count)]
        probs = [cq.problem(a, q, r, None) for a, q, r in zip(mats, qs, rs)]
        arr = (cq.Problem * count)(*probs)
        wb = lib.cqr2_batched_workspace_size(arr, count, cq.CQR2_FP64)
        work = torch.empty(max(int(wb), 256), dtype=torch.uint8, device=dev)

        def call():
            rc = lib.cqr2_factor_batched(arr, count, cq._ptr(work), work.numel(), cq.CQR2_FP64, sp)
            if rc != 0:
                raise cq.CQR2Error(rc, "cqr2_factor_batched")
        for _ in range(warmup):
            call()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            call()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        flops = count * (4.0 * m * n * n + 5.0 * n ** 3 / 3.0)
        checks = [device_checks(torch, mats[i], qs[i], rs[i]) for i in (0, count - 1)]
        rows.append({"problems": count, "m": m, "n": n, "ms_per_call": round(ms, 4),
                     "problems_per_s": round(count / (ms / 1e3), 1), "gflops": round(flops / (ms / 1e3) / 1e9, 1),
                     "checks": checks})
        log(f"batched {count} x {m}x{n}: {ms:.3f} ms per call")
        del mats, qs, rs, work
    return rows


def mixed_sweep(cq, torch, steps: int, warmup: int):
    """The 262144 x 256 comparison problem (A = G D V, generated on the device)
    at each condition number of the sweep: CholeskyQR2 in plain FP64 and with pass 1's Q1 in FP32
    (CQR2_MIXED_P1_FP32), each timed over `steps` calls; orthogonality and
    residual of both, and the mixed R against the FP64 R (both on the device)."""
    from synth import WORKLOADS, gdv_matrix_device
    from synth.matrices import MIXED_KAPPAS

    wl = WORKLOADS["mixed_262144x256"]
    m, n = wl.m, wl.n
    lib = cq.load()
    dev = torch.device("cuda:0")
    sp = cq.ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    wbytes = max(lib.cqr2_workspace_size(m, n, f) for f in (cq.CQR2_FP64, cq.CQR2_MIXED_P1_FP32))
    work = torch.empty(wbytes, dtype=torch.uint8, device=dev)
    rows = []
    for kappa in sorted(MIXED_KAPPAS):
        # generated on the device (same recipe, torch's seeded generator): the
        # two forms factor the same bytes
        a = gdv_matrix_device(m, n, kappa, MIXED_KAPPAS[kappa], device=dev)
        res = {}
        for name, flags in (("fp64", cq.CQR2_FP64), ("mixed", cq.CQR2_MIXED_P1_FP32)):
            q = cq.empty_colmajor(m, n, device=dev)
            r = cq.empty_colmajor(n, n, device=dev)

            def step():
                rc = lib.cqr2_factor_ex(cq._ptr(a), m, n, m, cq._ptr(q), m, cq._ptr(r), n, cq._ptr(work), wbytes,
                                        None, flags, sp)
                if rc != 0:
                    raise cq.CQR2Error(rc, "cqr2_factor_ex")
            for _ in range(warmup):
                step()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                step()
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / steps
            c = device_checks(torch, a, q, r)
            res[name] = {"ms": round(ms, 4), "orthogonality": c["orthogonality"], "residual": c["residual"], "r": r}
        r_rel = float(torch.linalg.norm(res["mixed"]["r"] - res["fp64"]["r"]) / torch.linalg.norm(res["fp64"]["r"]))
        rows.append({
            "kappa": kappa,
            "fp64_ms": res["fp64"]["ms"], "mixed_ms": res["mixed"]["ms"],
            "speedup": round(res["fp64"]["ms"] / res["mixed"]["ms"], 4),
            "fp64_orthogonality": res["fp64"]["orthogonality"], "mixed_orthogonality": res["mixed"]["orthogonality"],
            "fp64_residual": res["fp64"]["residual"], "mixed_residual": res["mixed"]["residual"],
            "mixed_r_rel_to_fp64": r_rel,
            "equal_orthogonality_gate": bool(res["fp64"]["orthogonality"] <= 1e-12
                                             and res["mixed"]["orthogonality"] <= 1e-12),
        })
        log(f"mixed sweep kappa {kappa:g}: {rows[-1]}")
    return {"workload": "mixed_262144x256", "m": m, "n": n, "steps": steps, "per_kappa": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="tall_1Mx128",
                    help="tall_1Mx128 (default), tall_4096x64, rect_65536x4096 or mixed_262144x256")
    ap.add_argument("--kappa", type=float, default=None, help="condition number (mixed_262144x256 sweep)")
    ap.add_argument("--mixed", action="store_true", help="CQR2_MIXED_P1_FP32 (pass-1 Q1 in FP32)")
    ap.add_argument("--shifted", action="store_true", help="CQR2_SHIFTED_CQR3 (shifted CholeskyQR3)")
    ap.add_argument("--inverse-depth", type=int, default=0,
                    help="CQR2_INVERSE_DEPTH(d): partial inverse, Q by block substitution (n > 128)")
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle time for the CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy-gib", type=float, default=0.0,
                    help="also run a device copy of this many GiB (counter calibration under rocprofv3)")
    ap.add_argument("--no-serve", action="store_true", help="skip the served-stream measurement")
    ap.add_argument("--no-mixed-sweep", action="store_true",
                    help="skip the FP64-vs-mixed comparison at 262144 x 256 over the condition numbers")
    ap.add_argument("--serve-only", action="store_true", help="only the served-stream measurement")
    ap.add_argument("--serve-requests", type=int, default=SERVE_REQUESTS)
    ap.add_argument("--serve-rate", type=float, default=SERVE_RATE)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1710_08471_amd as cq
    from synth import WORKLOADS, workload_matrix

    if args.serve_only:
        cq.load()
        out = {"metric": "served solves/s, p99 latency", "unit": "solves/s", "n_gpus": 1, "data": "synthetic",
               "higher_is_better": True, "dtype": "f64"}
        sv = serve_stream(cq, torch, args.serve_requests, args.serve_rate, SERVE_SEED)
        out["value"] = sv["solves_per_s"]
        out["serving"] = sv
        print(json.dumps(out), flush=True)
        return

    wl = WORKLOADS[args.workload]
    m, n = wl.m, wl.n
    flags = cq.CQR2_MIXED_P1_FP32 if args.mixed else (cq.CQR2_SHIFTED_CQR3 if args.shifted else cq.CQR2_FP64)
    flags |= cq.CQR2_INVERSE_DEPTH(args.inverse_depth)
    default_run = (args.workload == "tall_1Mx128" and not args.mixed and not args.shifted
                   and args.inverse_depth == 0)
    log(f"generating {wl.description} (seed {wl.seed}) on the host ...")
    t0 = time.perf_counter()
    a_host = workload_matrix(args.workload, args.kappa)
    log(f"  generated in {time.perf_counter() - t0:.1f} s")

    lib = cq.load()
    dev = torch.device("cuda:0")
    a = cq.colmajor(torch.from_numpy(a_host).to(dev))
    q = cq.empty_colmajor(m, n, device=dev)
    r = cq.empty_colmajor(n, n, device=dev)
    stream = torch.cuda.current_stream()
    sp = cq.ctypes.c_void_p(stream.cuda_stream)
    if default_run:
        def step():
            rc = lib.cqr2_factor(cq._ptr(a), m, n, m, cq._ptr(q), cq._ptr(r), sp)
            if rc != 0:
                raise cq.CQR2Error(rc, "cqr2_factor")
    else:
        wbytes = lib.cqr2_workspace_size(m, n, flags)
        work = torch.empty(max(wbytes, 256), dtype=torch.uint8, device=dev)

        def step():
            rc = lib.cqr2_factor_ex(cq._ptr(a), m, n, m, cq._ptr(q), m, cq._ptr(r), n, cq._ptr(work), wbytes,
                                    None, flags, sp)
            if rc != 0:
                raise cq.CQR2Error(rc, "cqr2_factor_ex")

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"warmup {args.warmup} done")

    # Timed region: K whole CholeskyQR2 steps.
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed * 1e3 / args.steps
    log(f"timed {args.steps} steps: {ms_per_step:.4f} ms/step")

    # The same K steps again with a HIP event pair around every kernel, recorded
    # by the library on the stream the kernels run on.
    cq.timing_reset()
    cq.timing_enable(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    inst_ms = (time.perf_counter() - t1) * 1e3 / args.steps
    cq.timing_enable(False)
    kt = cq.timing_read()
    log("per-class (HIP events): " + ", ".join(
        f"{k} {v[0] / max(v[1], 1) * 1e3:.1f} us x{v[1] // args.steps}" for k, v in kt.items() if v[1]))

    if args.calib_copy_gib > 0:
        nb = int(args.calib_copy_gib * (1 << 30)) // 8
        src = torch.ones(nb, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # Correctness of the last timed result (device-side check, FP64).
    qt = q.t().contiguous()
    orth = float(torch.linalg.norm(qt @ qt.t() - torch.eye(n, dtype=torch.float64, device=dev)))
    resid = float(torch.linalg.norm(a - q @ r) / torch.linalg.norm(a))
    log(f"orthogonality {orth:.3e}, residual {resid:.3e}")

    t_step = ms_per_step / 1e3
    value = flops_cqr2(m, n) / t_step / 1e9
    hbm_bytes_6mn = 6.0 * m * n * 8

    out = {
        "metric": METRIC if default_run else
        f"CQR2 GFLOP/s ({args.workload}{' mixed' if args.mixed else ''}{' shifted CQR3' if args.shifted else ''}"
        f"{f' inverse depth {args.inverse_depth}' if args.inverse_depth else ''})",
        "value": round(value, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32" if args.mixed else "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "m": m, "n": n, "lda": m,
                   "kappa": args.kappa if args.kappa is not None else wl.kappa, "seed": wl.seed,
                   "flags": "CQR2_MIXED_P1_FP32" if args.mixed else
                   ("CQR2_SHIFTED_CQR3" if args.shifted else "CQR2_FP64")
                   + (f" | CQR2_INVERSE_DEPTH({args.inverse_depth})" if args.inverse_depth else ""),
                   "matrix": wl.description},
        "hbm_roofline_pct_6mn": round(100.0 * hbm_bytes_6mn / t_step / 1e9 / HBM_PEAK_GBS, 2),
        "paper_convention_gflops": round(flops_householder(m, n) / t_step / 1e9, 2),
        "class_ms": {k: round(v[0] / v[1], 5) for k, v in kt.items() if v[1]},
        "instrumented_ms_per_step": round(inst_ms, 5),
        "orthogonality": orth,
        "residual": resid,
    }

    # Dominant kernel (largest total time over the K instrumented steps) and its
    # roofline; only the n <= 128 FP64 path has one kernel per timer class.  The
    # bound is the roof the kernel's algorithmic work meets first: HBM bytes
    # at 8 TB/s against FP64 flops at 78.6 TF/s.
    if n <= 128 and not args.mixed and not args.shifted:
        classes = KERNEL_CLASSES_S16 if n > 64 else KERNEL_CLASSES_SMALL
        tot = {k: sum(kt[c][0] for c in cls if kt.get(c, (0, 0))[1]) for k, cls in classes.items()}
        cnt = {k: sum(kt[c][1] for c in cls if kt.get(c, (0, 0))[1]) for k, cls in classes.items()}
        dom = max(tot, key=tot.get)
        avg_ms = tot[dom] / cnt[dom]
        fl, by = kernel_units(dom, m, n)
        bound = "hbm" if by / (HBM_PEAK_GBS * 1e9) >= fl / (FP64_PEAK_TFLOPS * 1e12) else "mfma"
        if bound == "hbm":
            achieved = by / (avg_ms / 1e3) / 1e9
            roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4)}
        else:
            achieved = fl / (avg_ms / 1e3) / 1e12
            roof = {"bound": "mfma", "achieved": round(achieved, 2), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(achieved / FP64_PEAK_TFLOPS, 4)}
        roof["traffic"] = read_traffic(dom) if default_run else None
        roof["kernel"] = dom
        roof["launches_per_step"] = cnt[dom] // args.steps
        roof["avg_launch_ms"] = round(avg_ms, 5)
        roof["algorithmic_per_launch"] = by if bound == "hbm" else fl
        out["roofline"] = roof
    if default_run and not args.no_mixed_sweep:
        out["mixed_vs_fp64"] = mixed_sweep(cq, torch, steps=10, warmup=2)
    if default_run and not args.no_serve:
        out["batched"] = batched_leg(cq, torch)
        out["serving"] = serve_stream(cq, torch, args.serve_requests, args.serve_rate, SERVE_SEED)
    if default_run and not args.no_cpu_baseline:
        log("timing the CPU oracle ...")
        out["cpu_baseline"] = cpu_baseline(a_host, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
