"""Throughput benchmark of the condensation log-determinant on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--path blocked|plain]
                    [--b B] [--workload NAME] [--no-plain] [--no-cpu]

A step is one whole log-determinant of the workload matrix (every stage of
the path: pivot searches, row factoring, updates, log/sign accumulation),
with the matrix resident in HBM before the timed region starts.  The
headline is the panel-blocked path (MFMA trailing updates) on the dense
N = 8000 FP64 N(0,1) matrix; the plain unblocked FP64 GPU path is timed on
the same matrix beside it.  Prints ONE JSON line with the metric, a
roofline object for the kernel that dominates the timed steps (HIP events
the library records on the stream each kernel runs on), and the CPU oracle
timed on a bounded sample of the same workload.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "log-dets/s and GFLOP/s (2N³/3) vs plain FP64 GPU at stated rel. error"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6
FP32_PEAK_TFS = 157.3
BF16_PEAK_TFS = 2500.0  # dense MFMA
# Matrix condensation, Table 3: best time for N = 8000 (FP64, 128 Haswell
# cores over MPI) = 7.17 s.  Another machine's number: context, not a target.
PAPER_BEST_N8000_S = 7.17

# Round trip of a store by one compute unit to its load by another through
# one XCD's L2 (sc0|nt loads), measured on MI355X with a probe kernel; a
# panel step needs at least two (the candidate record, then the winner's
# column), which sets the floor of the column-split panel chain per step.
L2_ROUND_TRIP_US = 0.52

# Source file of each timed kernel kind (a stored HBM-traffic measurement is
# used only while the source it was taken on is unchanged).
KERNEL_SOURCE = {
    "panel": "paper_1811_08057_amd/csrc/mc_blocked.hip",
    "update": "paper_1811_08057_amd/csrc/mc_gemm.hip",
    "plain_step": "paper_1811_08057_amd/csrc/mc_plain.hip",
}
KERNEL_NAME = {
    "panel": ("panel chain: blk_panel_split (one XCD, column slices; the "
              "row-per-block blk_panel_x / blk_panel for panels wider than "
              "8192 columns)"),
    "update": ("gemm_scalar (trailing update, FP64 MFMA; beside a panel, "
               "gemm_scalar_spare on the XCDs the panel leaves free)"),
    "update_f32": "gemm_scalar (trailing update, FP32 MFMA)",
    "update_bf16x3": "gemm_bf16x3 (trailing update, split-BF16x3 MFMA)",
    "plain_step": "plain_step (unblocked condensation step)",
}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=None)
    p.add_argument("--warmup", type=int, default=None)
    p.add_argument("--path", default="blocked", choices=["plain", "blocked"])
    p.add_argument("--b", type=int, default=-1,
                   help="panel width of the blocked path (-1: library default)")
    p.add_argument("--workload", default="normal_n8000")
    p.add_argument("--precision", default="f64", choices=["f64", "f32", "bf16x3"],
                   help="f64: FP64 storage and MFMA updates; f32 / bf16x3: "
                        "FP32 storage with FP32 or split-BF16x3 MFMA updates")
    p.add_argument("--no-plain", action="store_true",
                   help="skip timing the plain FP64 GPU path beside it")
    p.add_argument("--plain-steps", type=int, default=2)
    p.add_argument("--lookahead", default="on", choices=["on", "off"],
                   help="blocked path: run each trailing update beside the "
                        "next panel on a second stream (on) or keep one "
                        "stream (off)")
    p.add_argument("--profile-steps", type=int, default=3,
                   help="steps of the separate kernel-timing pass")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                   help="only run a device-to-device copy of BYTES bytes "
                        "three times (the reference kernel for scaling the "
                        "HBM counters FETCH_SIZE / WRITE_SIZE)")
    p.add_argument("--cpu-seconds", type=float, default=12.0)
    p.add_argument("--no-tune", action="store_true",
                   help="batch workloads: keep the library's default tuning "
                        "table instead of the autotuned one (cached per device)")
    p.add_argument("--grad", action="store_true",
                   help="batch workloads: time forward + backward (one "
                        "batched factor launch, the blocked factor call for "
                        "the largest members, one batched backward launch) "
                        "instead of the forward graph")
    p.add_argument("--study", default=None, choices=["pivot-rules"],
                   help="pivot-rules: accuracy of the three pivot-column "
                        "rules (Section 1, Section 2.2) on the GPU's plain "
                        "path against exact determinants; prints one JSON "
                        "line and exits")
    return p.parse_args()


def sha256_of(rel: str) -> str:
    with open(os.path.join(ROOT, rel), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def stored_traffic(kind: str, workload: str, b: int):
    """HBM bytes per launch of the kernel kind, from the committed rocprofv3
    counter summary for this workload, if its recorded source hash still
    matches the kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kind}_{workload}.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    fields = dict(re.findall(r"^- (\w+): (\S+)\s*$", text, re.M))
    try:
        if fields.get("source_sha256") != sha256_of(KERNEL_SOURCE[kind]):
            return None
        if int(fields.get("b", -2)) != b:
            return None
        return float(fields["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or platform.machine()


def host_threads() -> int:
    """Threads the oracle may use on this host: the processors it is allowed
    to run on, at most 16 (a GPU machine's CPU share)."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _oracle_sample(O, a, target_s: float):
    """(seconds, steps) of the oracle's first condensation steps, grown
    until they take about target_s (or the whole run)."""
    n = a.shape[0]
    steps = max(2, min(n, 16))
    while True:
        t0 = time.perf_counter()
        O.slogdet_steps(a, steps)
        dt = time.perf_counter() - t0
        if dt >= target_s or steps >= n:
            return dt, steps
        grow = max(1.5, min(8.0, target_s / max(dt, 1e-3)))
        steps = min(n, int(steps * grow) + 1)


def cpu_baseline(a, target_s: float, max_full_s: float = 40.0):
    """The oracle on the host's cores, timed two ways:

    * threads (the reported value): one OpenMP thread per allowed processor
      over the rows of each step (Figure 6's row distribution, on threads;
      results do not depend on the count) -- the whole log-determinant when
      the single-thread sample predicts it takes under max_full_s, else a
      sample scaled like the next one;
    * single thread: the first S condensation steps, scaled to a whole
      log-determinant by the step-work ratio sum (m-1)^2 -- the analogue of
      the paper's one-process column (the early steps are the widest, so
      the scaling errs on the slow side)."""
    from oracle import oracle as O
    import numpy as np

    n = a.shape[0]

    def work(steps):
        m = n - np.arange(steps, dtype=np.float64)
        return float(np.sum((m - 1.0) ** 2))

    threads = host_threads()
    prev = O.set_threads(1)
    try:
        dt1, s1 = _oracle_sample(O, a, target_s)
        full_1 = dt1 * work(n) / work(s1)
        O.set_threads(threads)
        if full_1 / threads <= max_full_s:
            t0 = time.perf_counter()
            O.slogdet(a)
            full_mt = time.perf_counter() - t0
            sample = f"one whole log-det of the same matrix on {threads} threads ({full_mt:.1f} s)"
        else:
            dtm, sm = _oracle_sample(O, a, target_s)
            full_mt = dtm * work(n) / work(sm)
            sample = (f"first {sm} of {n} condensation steps on {threads} threads "
                      f"({dtm:.1f} s), scaled by the step-work ratio to a whole "
                      f"log-det ({full_mt:.1f} s)")
    finally:
        O.set_threads(prev)
    flops = 2.0 * n ** 3 / 3.0
    multi = {"value": 1.0 / full_mt, "cores": threads, "sample": sample,
             "gflops": flops / full_mt / 1e9}
    single = {"value": 1.0 / full_1, "cores": 1,
              "sample": (f"first {s1} of {n} condensation steps "
                         f"({dt1:.1f} s on 1 thread), scaled by the "
                         f"step-work ratio to a whole log-det ({full_1:.1f} s)"),
              "gflops": flops / full_1 / 1e9}
    # the reported value is the faster of the two (small matrices run
    # faster on one thread than with a fork and join per step)
    best, other = (multi, single) if full_mt < full_1 else (single, multi)
    out = {"value": best["value"], "unit": "log-dets/s", "cores": best["cores"],
           "kind": "oracle", "sample": best["sample"], "gflops": best["gflops"],
           "cpu_model": cpu_model()}
    out["single_thread" if best is multi else "threads"] = other
    return out


def expected_for(workload: str):
    path = os.path.join(ROOT, "tests", "golden", f"expected_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def check_input(exp, key: str, data) -> None:
    """Fail loudly if the generated input is not the bytes the stored
    oracle values were computed on."""
    import synth

    if exp is None or key not in exp:
        return
    got = synth.sha256_of(data)
    if got != exp[key]:
        print(json.dumps({"error": f"input bytes differ from the stored "
                          f"oracle values' ({key}: {got} != {exp[key]})"}))
        sys.exit(3)


def timed(mc, torch, a, b, steps, warmup, stream, profile=False,
          update="native"):
    """ms per log-det over `steps` calls after `warmup`; returns
    (ms_per_step, last result, library kernel profiles by kind or None).
    The library's kernel timing puts an event pair around every timed
    launch, which perturbs the schedule, so the headline pass runs without
    it and the kernel averages come from a separate pass."""
    n = a.shape[0]
    dev = a.device
    work = mc.new_workspace(n, dev, a.dtype, update, b)
    res = mc.new_result(dev, 1)
    for _ in range(warmup):
        mc.logdet_async(a, res, work, b=b, update=update)
    torch.cuda.synchronize()
    if profile:
        mc.profile_enable(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        mc.logdet_async(a, res, work, b=b, update=update)
    e1.record(stream)
    torch.cuda.synchronize()
    prof = None
    if profile:
        prof = {k: mc.profile_read(k) for k in ("update", "panel")}
        mc.profile_enable(False)
    return e0.elapsed_time(e1) / steps, mc.read_result(res)[0], prof


def roofline_of(kind, p, workload, b, prec="f64"):
    """Roofline entry for one timed kernel kind (p: library profile)."""
    if p.launches == 0 or p.elapsed_ms <= 0:
        return None
    avg_us = p.elapsed_ms * 1e3 / p.launches
    if kind == "update":
        peak, mult = mfma_peak(prec)
        ach = mult * p.alg_flops / (p.elapsed_ms * 1e-3) / 1e12
        r = {"bound": "mfma", "achieved": ach, "peak": peak,
             "unit": "TFLOP/s", "frac": ach / peak}
    else:
        ach = p.alg_bytes / (p.elapsed_ms * 1e-3) / 1e9
        r = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
             "unit": "GB/s", "frac": ach / HBM_PEAK_GBS}
    r["traffic"] = stored_traffic(kind, workload, b)
    if kind == "panel":
        # the chain is a sequence of dependent steps: its bound is latency
        steps = b if b > 0 else 1
        us = avg_us / steps
        floor = 2.0 * L2_ROUND_TRIP_US
        r["latency"] = {"steps_per_launch": steps, "us_per_step": us,
                        "floor_us_per_step": floor, "frac": floor / us,
                        "floor": "two L2 round trips per step (record, then column)"}
    name = KERNEL_NAME[kind if kind != "update" or prec == "f64"
                       else f"update_{prec}"]
    r.update({"kernel": name, "launches": p.launches,
              "avg_launch_us": avg_us,
              "alg_bytes_per_launch": p.alg_bytes / p.launches,
              "alg_flops_per_launch": p.alg_flops / p.launches,
              "share_of_step": None})
    return r


def gpu_gram(torch, dev):
    """X^T X in FP64 on the GPU for the Wishart inputs (the draws are the
    seeded host draws; only the product runs on the device)."""
    def gram(x):
        xd = torch.from_numpy(x).to(dev)
        return torch.matmul(xd.t().contiguous(), xd).cpu().numpy()
    return gram


def cpu_baseline_batch(mats, target_s: float):
    """The oracle on the host's cores (OpenMP over the rows of each step) on
    the first members of the batch until about target_s, scaled to the
    whole batch by sum n^3."""
    from oracle import oracle as O

    threads = host_threads()
    prev = O.set_threads(threads)
    done, t_used = 0, 0.0
    while done < len(mats) and t_used < target_s:
        t0 = time.perf_counter()
        O.slogdet(mats[done])
        t_used += time.perf_counter() - t0
        done += 1
    O.set_threads(prev)
    w_all = sum(float(m.shape[0]) ** 3 for m in mats)
    w_done = sum(float(m.shape[0]) ** 3 for m in mats[:done])
    full = t_used * w_all / w_done
    return {"value": len(mats) / full, "unit": "log-dets/s", "cores": threads,
            "kind": "oracle", "cpu_model": cpu_model(),
            "sample": (f"first {done} of {len(mats)} matrices of the batch "
                       f"({t_used:.1f} s on {threads} threads), scaled by "
                       f"sum n^3 to the whole batch ({full:.1f} s)")}


def mfma_peak(prec: str):
    """(peak TFLOP/s, MFMA products per useful flop) of a precision."""
    return {"f64": (FP64_PEAK_TFS, 1), "f32": (FP32_PEAK_TFS, 1),
            "bf16x3": (BF16_PEAK_TFS, 3)}[prec]


def run_batch_grad(args, mc, torch, sizes, mats, devs, allexp, update, stream):
    """Forward + backward of sum_k log|det A_k| through the batched autograd
    function: the batched factor launch for the members below
    BatchedPlan.BLOCKED_MIN_N rows, the blocked factor call for each larger
    one, and one batched backward launch for all members."""
    import numpy as np

    prec = args.precision
    leaves = [d.clone().requires_grad_(True) for d in devs]

    def step():
        for x in leaves:
            x.grad = None
        signs, logabs = mc.slogdet_batched_autograd(leaves, update=update)
        logabs.sum().backward()
        return signs, logabs

    steps = args.steps if args.steps is not None else 10
    warmup = args.warmup if args.warmup is not None else 2
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        signs, logabs = step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    fwd_flops = sum(2.0 * n ** 3 / 3.0 for n in sizes)
    bwd_flops = sum(4.0 * n ** 3 / 3.0 for n in sizes)
    worst = gworst = None
    signs_ok = None
    if allexp is not None:
        exp = allexp["f64" if prec == "f64" else "f32"]
        la = logabs.detach().cpu().numpy()
        sg = signs.cpu().numpy()
        worst = max(abs(float(g) - e["logabsdet"]) / max(abs(e["logabsdet"]), 1.0)
                    for g, e in zip(la, exp))
        signs_ok = all(float(g) == e["sign"] for g, e in zip(sg, exp))
        if "grad_samples" in allexp:
            key = "f64" if prec == "f64" else "f32"
            gworst = 0.0
            for x, smp in zip(leaves, allexp["grad_samples"]):
                g = x.grad.double().cpu().numpy()
                ref = np.array(smp[key])
                got = np.array([g[i, j] for i, j in smp["ij"]])
                gworst = max(gworst, float(np.abs(got - ref).max() / np.abs(ref).max()))
    peak, mult = mfma_peak(prec)
    ach = mult * (fwd_flops + bwd_flops) / (ms * 1e-3) / 1e12
    out = {
        "metric": METRIC, "value": len(sizes) / (ms * 1e-3), "unit": "log-dets/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == "f64" else "f32", "data": "synthetic",
        "config": {"workload": args.workload, "batch": len(sizes),
                   "n_min": min(sizes), "n_max": max(sizes), "precision": prec,
                   "path": "batched forward + backward (autograd)"},
        "gflops": (fwd_flops + bwd_flops) / (ms * 1e-3) / 1e9,
        "rel_err_vs_oracle": worst, "sign_matches_oracle": signs_ok,
        "grad_sampled_rel_err_vs_oracle": gworst,
        "roofline": {"bound": "mfma", "achieved": ach, "peak": peak,
                     "unit": "TFLOP/s", "frac": ach / peak, "traffic": None,
                     "note": "forward 2n^3/3 + backward 4n^3/3 flops per member "
                             "over the whole step"},
    }
    print(json.dumps(out), flush=True)


def run_gmm(args, mc, torch, synth, spec, dev, stream):
    """Mixture log-likelihood: one step factors the k covariances (one
    batched factor launch) and scores every point (mc_gmm_loglik)."""
    import numpy as np

    prec = args.precision if args.precision != "bf16x3" else "f32"
    dtype = torch.float64 if prec == "f64" else torch.float32
    print(f"# generating {args.workload}", file=sys.stderr, flush=True)
    w, means, covs, x = synth.make(args.workload)
    k, d, m = len(covs), x.shape[1], x.shape[0]
    cv = [torch.from_numpy(c).to(dev, dtype) for c in covs]
    xl = torch.from_numpy(x).to(dev, dtype)
    mu = torch.from_numpy(means).to(dev, dtype)
    lw = torch.from_numpy(np.log(w)).to(dev)

    def step():
        fac = mc.gmm_factor(cv)
        return mc.gmm_loglik(xl, lw, mu, fac)

    steps = args.steps if args.steps is not None else 10
    warmup = args.warmup if args.warmup is not None else 2
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        ll, tot = step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    # the factor launch alone, for the split
    e0.record(stream)
    for _ in range(steps):
        fac = mc.gmm_factor(cv)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_fac = e0.elapsed_time(e1) / steps
    fac_flops = k * 2.0 * d ** 3 / 3.0
    solve_flops = k * m * 2.0 * d ** 2
    peak, _ = mfma_peak(prec)
    ach = solve_flops / ((ms - ms_fac) * 1e-3) / 1e12
    out = {
        "metric": "mixture log-likelihood: points/s (k log-dets + k*m Mahalanobis terms per step)",
        "value": m / (ms * 1e-3), "unit": "points/s", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": prec, "data": "synthetic",
        "config": {"workload": args.workload, "k": k, "d": d, "m": m,
                   "path": "batched factor + mc_gmm_loglik"},
        "ms_factor": ms_fac, "ms_loglik": ms - ms_fac,
        "gflops": (fac_flops + solve_flops) / (ms * 1e-3) / 1e9,
        "total_loglik": float(tot.cpu()),
        "roofline": {"bound": "mfma", "achieved": ach, "peak": peak, "unit": "TFLOP/s",
                     "frac": ach / peak, "traffic": None,
                     "note": "the mixture kernels: 2 d^2 flops per point and component "
                             "(two triangular substitutions) over the step time minus "
                             "the factor launch"},
    }
    print(json.dumps(out), flush=True)


def run_batch(args, mc, torch, synth, spec, dev, stream):
    """The batch as one captured graph, replayed: one persistent batched
    launch for the members below BatchedPlan.BLOCKED_MIN_N rows and the
    blocked path for each larger member; the plain FP64 GPU path beside
    it, one call per member."""
    prec = args.precision
    dtype = torch.float64 if prec == "f64" else torch.float32
    update = {"f64": "native", "f32": "f32", "bf16x3": "bf16x3"}[prec]
    print(f"# generating {args.workload}", file=sys.stderr, flush=True)
    sizes, mats = synth.make(args.workload, gram=gpu_gram(torch, dev))
    allexp = expected_for(args.workload)
    check_input(allexp, "sha256_f64", mats)
    if prec != "f64":
        check_input(allexp, "sha256_f32", [m.astype("float32") for m in mats])
    devs = [torch.from_numpy(m).to(dev, dtype) for m in mats]
    tune = None
    if not args.no_tune:
        # the panel widths and tiles of the batched launch from the
        # library's autotuner (cached per device), up to the largest member
        # the batched launch takes
        small_max = max([n for n in sizes if n < mc.BatchedPlan.BLOCKED_MIN_N], default=0)
        if small_max > 0:
            print("# autotuning the batched path", file=sys.stderr, flush=True)
            tb, tt, src = mc.autotune_cached(dtype, update, min(small_max, 4096), dev)
            tune = {"b": tb, "tile": tt, "source": src}
    if args.grad:
        run_batch_grad(args, mc, torch, sizes, mats, devs, allexp, update, stream)
        return
    plan = mc.BatchedPlan(devs, b=-1, update=update)
    plan.capture()
    steps = args.steps if args.steps is not None else 20
    warmup = args.warmup if args.warmup is not None else 2
    for _ in range(warmup):
        plan.replay()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        plan.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    got = plan.results()
    flops = sum(2.0 * n ** 3 / 3.0 for n in sizes)
    value = len(sizes) / (ms * 1e-3)

    worst, signs = None, None
    if allexp is not None:
        exp = allexp["f64" if prec == "f64" else "f32"]
        worst = max(abs(g.logabsdet - e["logabsdet"]) / max(abs(e["logabsdet"]), 1.0)
                    for g, e in zip(got, exp))
        signs = all(g.sign == e["sign"] for g, e in zip(got, exp))
    peak, mult = mfma_peak(prec)
    ach = mult * flops / (ms * 1e-3) / 1e12
    launches = len(plan.large) + (1 if plan.small else 0)
    roof = {"bound": "mfma", "achieved": ach, "peak": peak, "unit": "TFLOP/s",
            "frac": ach / peak, "traffic": None,
            "kernel": ("batched_persistent (one launch for the members below "
                       f"{plan.BLOCKED_MIN_N} rows) + the blocked path for each "
                       "larger member"),
            "launches": launches, "avg_launch_us": ms * 1e3 / max(launches, 1),
            "note": (f"achieved = {mult} x the useful 2n^3/3 flops per "
                     "member over the graph replay")}
    out = {
        "metric": METRIC, "value": value, "unit": "log-dets/s", "n_gpus": 1,
        "steps": steps, "warmup": warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == "f64" else "f32", "data": "synthetic",
        "config": {"workload": args.workload, "batch": len(sizes),
                   "n_min": min(sizes), "n_max": max(sizes),
                   "precision": prec, "path": "batched", "graph": True,
                   "blocked_members": len(plan.large),
                   "tune": tune or "library defaults"},
        "gflops": flops / (ms * 1e-3) / 1e9,
        "rel_err_vs_oracle": worst, "sign_matches_oracle": signs,
        "roofline": roof,
    }
    if not args.no_plain:
        print("# plain FP64 GPU path, member by member", file=sys.stderr, flush=True)
        a64 = [torch.from_numpy(m).to(dev) for m in mats]
        work = mc.new_workspace(max(sizes), dev, torch.float64, "native", 0)
        res = mc.new_result(dev, len(a64))
        for a in a64[:2]:
            mc.logdet_async(a, res[0:1], work, b=0)
        torch.cuda.synchronize()
        e0.record(stream)
        for i, a in enumerate(a64):
            mc.logdet_async(a, res[i:i + 1], work, b=0)
        e1.record(stream)
        torch.cuda.synchronize()
        pms = e0.elapsed_time(e1)
        out["plain_fp64_gpu"] = {"ms_per_batch": pms,
                                 "value": len(a64) / (pms * 1e-3)}
        out["speedup_vs_plain_fp64_gpu"] = pms / ms
    if not args.no_cpu:
        print("# cpu baseline (oracle sample)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline_batch(mats, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def _bareiss_logabs(a) -> tuple:
    """(sign, log|det|) of a float matrix exactly: its doubles scaled to
    integers by one power of two, then fraction-free (Bareiss) elimination
    with exact integer divisions."""
    import math
    from fractions import Fraction

    n = a.shape[0]
    fr = [[Fraction(float(x)) for x in row] for row in a]
    scale = 1
    for row in fr:
        for x in row:
            scale = max(scale, x.denominator)
    m = [[int(x * scale) for x in row] for row in fr]
    sign, prev = 1, 1
    for k in range(n - 1):
        if m[k][k] == 0:
            for i in range(k + 1, n):
                if m[i][k] != 0:
                    m[k], m[i] = m[i], m[k]
                    sign = -sign
                    break
            else:
                return 0, -math.inf
        for i in range(k + 1, n):
            for j in range(k + 1, n):
                m[i][j] = (m[i][j] * m[k][k] - m[i][k] * m[k][j]) // prev
        prev = m[k][k]
    d = m[n - 1][n - 1] * sign
    if d == 0:
        return 0, -math.inf
    # log|d| of a big integer, then undo the scaling (scale^n)
    bits = abs(d).bit_length()
    shift = max(0, bits - 60)
    la = math.log(abs(d) >> shift) + shift * math.log(2.0)
    return (1 if d > 0 else -1), la - n * math.log(scale)


def run_pivot_study(args, mc, torch, dev):
    """The three pivot-column rules on the GPU's plain FP64 path (Section 1:
    first non-zero, closest to 1; Section 2.2: largest |a|), relative error
    of log|det| against the exact determinant, over seeded matrix
    families."""
    import numpy as np

    families = {
        "sec22": ("rows drawn from {+-1e-10, +-2.01} plus 1e-3 N(0,1) noise "
                  "(the Section 2.2 example)",
                  lambda g, n: g.choice([1e-10, 2.01, -2.01, -1e-10], (n, n))
                  + 1e-3 * g.standard_normal((n, n))),
        "uniform": ("i.i.d. U[-1, 1]",
                    lambda g, n: g.uniform(-1.0, 1.0, (n, n))),
        "graded": ("U[-1, 1] with each row scaled by 10^U[-6, 6]",
                   lambda g, n: 10.0 ** g.uniform(-6.0, 6.0, (n, 1))
                   * g.uniform(-1.0, 1.0, (n, n))),
    }
    rules = ["maxabs", "first_nonzero", "closest_to_one"]
    sizes = [8, 32, 64]
    trials = args.steps if args.steps is not None else 10
    rows = []
    for fam, (desc, make) in families.items():
        for n in sizes:
            errs = {r: [] for r in rules}
            for t in range(trials):
                g = np.random.default_rng(1000 * n + t)
                a = make(g, n)
                sgn, ref = _bareiss_logabs(a)
                ad = torch.from_numpy(a).to(dev)
                for r in rules:
                    got, _ = mc.slogdet_rule(ad, r)
                    bad = got.sign != sgn or not np.isfinite(got.logabsdet)
                    errs[r].append(float("inf") if bad else
                                   abs(got.logabsdet - ref) / max(abs(ref), 1.0))
            for r in rules:
                e = np.array(errs[r])
                rows.append({"family": fam, "n": n, "rule": r, "trials": trials,
                             "median_rel_err": float(np.median(e)),
                             "max_rel_err": float(e.max())})
            print(f"# {fam} n={n} done", file=sys.stderr, flush=True)
    print(json.dumps({"study": "pivot-rules", "path": "plain FP64 (mc_logdet_rule)",
                      "reference": "exact determinant (Bareiss on the doubles' exact values)",
                      "families": {k: v[0] for k, v in families.items()},
                      "rows": rows}), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this engine runs on one GPU; "
                          f"--gpus {args.gpus} is not supported (use 1)"}))
        sys.exit(2)

    import torch

    import paper_1811_08057_amd as mc
    import synth

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    dev = torch.device("cuda:0")
    if args.calibrate_copy > 0:
        nb = args.calibrate_copy // 8 * 8
        src = torch.ones(nb // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": nb, "copy_bytes_written": nb,
                          "launches": 3}), flush=True)
        return
    if args.study == "pivot-rules":
        run_pivot_study(args, mc, torch, dev)
        return
    spec = synth.CONFIGS[args.workload]
    stream = torch.cuda.current_stream(dev)
    if spec["kind"] == "wishart_batch":
        run_batch(args, mc, torch, synth, spec, dev, stream)
        return
    if spec["kind"] == "gmm":
        run_gmm(args, mc, torch, synth, spec, dev, stream)
        return
    n = spec["n"]
    prec = args.precision
    update = {"f64": "native", "f32": "f32", "bf16x3": "bf16x3"}[prec]
    plain = args.path == "plain"
    if plain and prec != "f64":
        print(json.dumps({"error": "the plain path is FP64 only"}))
        sys.exit(2)
    b = 0 if plain else args.b
    if b < 0:
        b = mc.default_panel(n)
    steps = args.steps if args.steps is not None else (3 if plain else 20)
    warmup = args.warmup if args.warmup is not None else 1

    print(f"# generating {args.workload}", file=sys.stderr, flush=True)
    if spec["kind"] == "wishart":
        a_np = synth.make(args.workload, gram=gpu_gram(torch, dev))
    else:
        a_np = synth.make(args.workload)
    allexp = expected_for(args.workload)
    check_input(allexp, "sha256_f64", a_np)
    if prec != "f64":
        check_input(allexp, "sha256_f32", a_np.astype("float32"))
    a64 = torch.from_numpy(a_np).to(dev)
    a = a64 if prec == "f64" else a64.to(torch.float32)

    if not plain:
        mc.lookahead_enable(args.lookahead == "on")
    print(f"# {args.path} b={b}: warmup {warmup}, timing {steps}",
          file=sys.stderr, flush=True)
    ms_per_step, got, _ = timed(mc, torch, a, b, steps, warmup, stream,
                                update=update)
    prof_ms, prof = None, None
    if args.profile_steps > 0:  # 0: no kernel-timing pass (counter runs)
        print(f"# kernel timing pass: {args.profile_steps} steps",
              file=sys.stderr, flush=True)
        prof_ms, _, prof = timed(mc, torch, a, b, args.profile_steps, 0, stream,
                                 profile=True, update=update)
    value = 1000.0 / ms_per_step
    gflops = (2.0 * n ** 3 / 3.0) / (ms_per_step * 1e-3) / 1e9

    # accuracy against the stored oracle value for this workload: FP32
    # storage against the oracle on the FP32-rounded input where stored,
    # else against the FP64 value (named in rel_err_reference)
    exp, rel_err, sign_ok, ref_name = None, None, None, None
    if allexp is not None:
        exp = allexp["f64"]
        mine, ref_name = exp, "oracle, FP64 input"
        if prec != "f64" and "f32" in allexp:
            mine, ref_name = allexp["f32"], "oracle, FP32-rounded input"
        rel_err = abs(got.logabsdet - mine["logabsdet"]) / max(
            abs(mine["logabsdet"]), 1.0)
        sign_ok = got.sign == mine["sign"]

    # roofline of the dominant kernel (largest timed share of the step)
    entries = {}
    for k in (["plain_step"] if plain else ["panel", "update"]) if prof else []:
        p = prof["update" if k == "plain_step" else k]
        r = roofline_of(k, p, args.workload, b, prec)
        if r is not None:
            r["share_of_step"] = p.elapsed_ms / args.profile_steps / prof_ms
            r["timing_pass_ms_per_step"] = prof_ms
            entries[k] = r
    roof = None
    if entries:
        dominant = max(entries, key=lambda k: entries[k]["share_of_step"])
        roof = dict(entries[dominant])

    out = {
        "metric": METRIC, "value": value, "unit": "log-dets/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": (value * PAPER_BEST_N8000_S
                        if args.workload == "normal_n8000" else None),
        "dtype": "f64" if prec == "f64" else "f32", "data": "synthetic",
        "config": {"workload": args.workload, "n": n,
                   "dist": spec["kind"], "seed": spec.get("seed"),
                   "path": args.path, "b": b, "precision": prec,
                   "lookahead": None if plain else args.lookahead},
        "gflops": gflops,
        "rel_err_vs_oracle": rel_err, "rel_err_reference": ref_name,
        "sign_matches_oracle": sign_ok,
        "roofline": roof,
        "kernels": entries,
    }

    if not plain and not args.no_plain:
        print(f"# plain FP64 GPU path: {args.plain_steps} steps",
              file=sys.stderr, flush=True)
        pms, pgot, pprof = timed(mc, torch, a64, 0, args.plain_steps, 1, stream,
                                 profile=True)
        p = pprof["update"]
        pach = p.alg_bytes / (p.elapsed_ms * 1e-3) / 1e9
        out["plain_fp64_gpu"] = {
            "ms_per_step": pms, "value": 1000.0 / pms,
            "gflops": (2.0 * n ** 3 / 3.0) / (pms * 1e-3) / 1e9,
            "rel_err_vs_oracle": (abs(pgot.logabsdet - exp["logabsdet"]) /
                                  max(abs(exp["logabsdet"]), 1.0)
                                  if exp else None),
            "hbm_achieved_gbs": pach, "hbm_frac": pach / HBM_PEAK_GBS}
        out["speedup_vs_plain_fp64_gpu"] = pms / ms_per_step

    if not args.no_cpu:
        print("# cpu baseline (oracle sample)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(a_np, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
