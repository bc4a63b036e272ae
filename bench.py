"""Benchmark: batched full-MSG solves of the 256x256 separable lognormal workload.

One step = the whole hot path over one batch: coefficient-field synthesis at
every face of every grid, the full-MSG solve of every sample to a relative
residual of 1e-10 on all 64 grids, and the multi-index differences.  Inputs
(the standard normal KL coefficients) are resident in HBM before timing.

Prints one JSON line.  Beside the headline value it reports, under "extra":
  * the plain per-sample FP64 GPU MSG (the same library, one sample per
    call) on a few samples, for the batched-vs-plain ratio;
  * the 1024x64 strongly anisotropic workload in mixed precision (FP32
    cycles, FP64 refinement to 1e-8) and in FP64 on the same samples, with
    the mixed result's error against the FP64 one, and the plain per-sample
    FP64 rate on that workload;
  * the ragged multi-index batch {l1+l2 <= 8} in one call;
  * the request loop (Poisson arrivals, HBM-budget admission, continuous
    batching) with p50/p99 latency;
and the smoother's achieved bandwidth from HIP events around its launches in
the timed region (roofline), and the oracle timed on host cores.
"""
import argparse
import dataclasses
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# HIP events around one launch in this many (hash-picked) in the timed steps:
# an event pair around every launch costs about 6% of the step
PROFILE_EVERY = 8


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--samples", type=int, default=None, help="batch size (default: the preset's 4096)")
    ap.add_argument("--plain-samples", type=int, default=2)
    ap.add_argument("--cpu-samples", type=int, default=None, help="default: one per oracle thread")
    ap.add_argument("--mixed-oracle-samples", type=int, default=8,
                    help="1024x64 mixed results compared with the oracle in the CPU leg")
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--skip-plain", action="store_true")
    ap.add_argument("--skip-mixed", action="store_true")
    ap.add_argument("--skip-ragged", action="store_true")
    ap.add_argument("--skip-serve", action="store_true")
    ap.add_argument("--skip-mimc", action="store_true")
    ap.add_argument("--skip-factors", action="store_true", help="no MG-versus-MSG convergence-factor study")
    ap.add_argument("--skip-one-stream", action="store_true", help="no extra one-stream profiled step")
    ap.add_argument("--no-tune", action="store_true", help="library default plan instead of the autotuner's")
    ap.add_argument("--tune-cycles", type=int, default=1, help="cycles per stage in each autotuner trial")
    ap.add_argument("--mixed-workload-samples", type=int, default=None, help="default: the preset's 1024")
    ap.add_argument("--serve-requests", type=int, default=20000,
                    help="window of the 200000-request trace replayed per offered rate")
    ap.add_argument("--serve-rates", type=float, nargs="+", default=[5000.0, 2000.0, 1000.0, 500.0])
    ap.add_argument("--serve-oracle-requests", type=int, default=12,
                    help="served answers compared with the oracle in the CPU leg")
    ap.add_argument("--no-profile", action="store_true", help="no HIP events around launches")
    ap.add_argument("--overlap", type=int, default=None,
                    help="overlap mode of the timed steps (msg_solve_opts.overlap; default: the library's choice)")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "traffic_k_rbgs_se-256x256-s4096_one_stream.md"))
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run one device copy of this many bytes (calibrates the HBM byte counters)")
    return ap.parse_args()


def kernel_source_digest():
    """sha256 of the HIP kernel source: traffic counters taken on other code do not apply."""
    import hashlib
    with open(os.path.join(ROOT, "paper_1907_12334_amd", "csrc", "msg_kernels.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def read_traffic(path):
    """HBM bytes per smoother launch from a counter summary (lines 'key: value'),
    or None when it is absent or was measured on another kernel source."""
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            kv[k.strip()] = v.strip().strip("`")
    if kv.get("kernel_source_sha256") != kernel_source_digest():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_calibration(nbytes):
    """One elementwise device copy of nbytes (read nbytes, write nbytes)."""
    import torch
    n = nbytes // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    torch.add(src, 0.0, out=dst)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n * 8, "kernel": "elementwise add(src, 0) -> dst, float64"}), flush=True)


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.copy_bytes:
        copy_calibration(args.copy_bytes)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1",
                          "n_gpus_requested": args.gpus}))
        sys.exit(2)
    import torch
    from paper_1907_12334_amd import inputs as I
    from paper_1907_12334_amd import msg

    w = I.config(2)
    if args.samples:
        w = w.subset(args.samples)
    S = w.n_samples
    opts = msg.SolveOpts(tol=w.tol, max_cycles=w.max_cycles)
    h = msg.Handle(0)
    batch = msg.Batch(w.c, w.P, w.Q)
    log(f"workload {w.name}: S={S}, c={w.c}, (P,Q)=({w.P[0]},{w.Q[0]}), tol={w.tol}")
    xi_h = w.xi()
    xi = torch.tensor(xi_h, dtype=torch.float64, device="cuda:0")
    tune = None
    if not args.no_tune:
        from paper_1907_12334_amd import autotune as AT
        opts, tune = AT.autotune(h, w, opts, samples=S, cycles=args.tune_cycles, reps=1, log=log)
        torch.cuda.empty_cache()
        log(f"autotuned plan: {tune['params']}")
    if args.overlap is not None:
        opts = dataclasses.replace(opts, overlap=args.overlap)
    bufs = msg.Buffers(batch, opts)
    log(f"device buffers {sum(t.numel() * t.element_size() for t in [bufs.kx, bufs.ky, bufs.u, bufs.ws]) / 1e9:.1f} GB")

    def step():
        msg.run(h, w.field, batch, opts, xi, bufs)

    for k in range(args.warmup):
        t0 = time.perf_counter()
        step()
        torch.cuda.synchronize()
        log(f"warmup {k}: {time.perf_counter() - t0:.2f} s")

    h.set_profiling(not args.no_profile, every=PROFILE_EVERY)
    times = []
    torch.cuda.synchronize()
    t_all = time.perf_counter()
    for k in range(args.steps):
        t0 = time.perf_counter()
        step()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        log(f"step {k}: {times[-1]:.2f} s")
    elapsed = time.perf_counter() - t_all
    prof = h.profile()
    h.set_profiling(False)

    status = bufs.status.cpu().numpy()
    cycles = bufs.cycles.cpu().numpy()
    split = status_split(status)
    converged = split["converged"]
    # only samples solved to the tolerance on every grid count; a failed
    # sample also skips the stages above the level where it failed
    value = converged * args.steps / elapsed
    ms = 1000.0 * elapsed / args.steps
    log(f"status {split}, max cycles per grid {cycles.max()}, {value:.1f} solved samples/s")

    traffic = read_traffic(args.traffic)
    kernel_share = {k: round((v[1] / 1000.0) / elapsed, 4) for k, v in prof.items() if not k.endswith("_stage")}
    extra = {"kernel_time_share": kernel_share, "status": split, "autotune": tune,
             "event_timing": f"HIP events around one launch in {PROFILE_EVERY}, picked by a hash of the launch "
                             "counter; time shares scaled to all launches",
             "max_cycles_per_grid": int(cycles.max()),
             "cycles_per_grid_mean": round(float(cycles.mean()), 2),
             "roofline_timed_step_shared": {
                 "note": "smoother launches of the timed steps, whose three concurrent parts share the device: "
                         "each launch's duration includes the others' kernels",
                 "smooth": roofline_of(prof["smooth"], SMOOTH_KERNEL)}}
    roofline = None
    if not args.no_profile and not args.skip_one_stream:
        # the same step with every launch on one stream: each smoother
        # launch has the device to itself, so its duration is its own
        h.set_profiling(True, every=PROFILE_EVERY)
        o0 = dataclasses.replace(opts, overlap=0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        msg.run(h, w.field, batch, o0, xi, bufs)
        torch.cuda.synchronize()
        t_iso = time.perf_counter() - t0
        p0 = h.profile()
        h.set_profiling(False)
        roofline = roofline_of(p0["smooth"], SMOOTH_KERNEL, traffic)
        roofline["measured_on"] = ("one step with overlap = 0 after the timed steps (same inputs, every launch on "
                                   "one stream, no concurrent kernels)")
        sm_s = p0["smooth"][1] / 1000.0
        extra["one_stream_step"] = {
            "step_s": round(t_iso, 3), "solved_samples_per_s": round(status_split(bufs.status.cpu().numpy())
                                                                      ["converged"] / t_iso, 2),
            "smoother_seconds": round(sm_s, 3), "smoother_share_of_step": round(sm_s / t_iso, 4),
            "kernel_time_share": {k: round((v[1] / 1000.0) / t_iso, 4) for k, v in p0.items()
                                  if not k.endswith("_stage")},
            "smooth_stage_level": roofline_of(p0["smooth_stage"], SMOOTH_KERNEL)}
        log(f"one-stream step: {t_iso:.2f} s, smoother {roofline['achieved']} GB/s per-step model, "
            f"{roofline['achieved_minimal']} GB/s minimal ({sm_s:.2f} s of smoother time)")
    else:
        roofline = roofline_of(prof["smooth"], SMOOTH_KERNEL, traffic)
        roofline["measured_on"] = ("the timed steps, every launch on one stream" if args.overlap == 0 else
                                   "the timed steps (concurrent parts share the device)")

    cpu_threads = cpu_share()[0]
    head = take_samples(bufs, w, range(min(S, args.cpu_samples or cpu_threads)))

    # plain per-sample FP64 GPU MSG: one sample per call, same kernels
    if not args.skip_plain:
        n = min(args.plain_samples, S)
        b1 = msg.Batch(w.c, w.P[:1], w.Q[:1])
        bp = msg.Buffers(b1, opts)
        msg.run(h, w.field, b1, opts, xi[0:1], bp)          # warm
        torch.cuda.synchronize()
        st = []
        t0 = time.perf_counter()
        for s in range(n):
            msg.run(h, w.field, b1, opts, xi[s:s + 1], bp)
            st.append(int(bp.status.cpu().numpy()[0]))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        plain = st.count(0) / dt
        extra["plain_fp64_per_sample"] = {"value": round(plain, 3), "unit": "solved samples/s", "samples": n,
                                          "status": st}
        extra["batched_over_plain"] = round(value / plain, 1) if st.count(0) == n and split["converged"] == S \
            else None
        log(f"plain per-sample FP64: {plain:.3f} solved samples/s (status {st})")

    del bufs                       # the other legs allocate their own buffers
    torch.cuda.empty_cache()
    mixed_head = None
    if not args.skip_mixed:
        extra["mixed_1024x64"], mixed_head = mixed_leg(h, msg, I, torch, args)

    if not args.skip_ragged:
        extra["ragged"] = ragged_leg(h, msg, I, torch)

    served = None
    if not args.skip_serve:
        extra["serving"], served = serve_leg(msg, I, args)

    if not args.skip_mimc:
        extra["msg_mimc"] = mimc_leg(h, msg, I)

    if not args.skip_factors:
        extra["convergence_factors"] = factors_leg(h)

    cpu = None
    if not args.skip_cpu:
        cpu = cpu_baseline(w, head, I.config(4), mixed_head, served)
        log(f"cpu oracle: {cpu}")

    out = {
        "metric": "MSG solved samples/sec at 1e-8 rel. residual + p50/p99 latency, vs plain FP64",
        "value": round(value, 3),
        "unit": "solved samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic: seeded N(0,1) KL coefficients, separable squared-exponential field",
        "config": {"workload": w.name, "samples": S, "grid": "256x256 finest, 2x2 coarsest, 64 grids",
                   "field": "separable SE 50x50, lx=0.3, ly=0.03, sigma2=1, face-mean coefficients", "tol": w.tol,
                   "tol_note": "a sample counts as solved when every one of its 64 grids reaches a relative "
                               "residual of 1e-10, so it also meets the metric's 1e-8",
                   "cycle": "W(2,2)", "precision": "fp64", "status": split},
        "latency_ms": {"p50": round(float(np.percentile(times, 50)) * 1000, 1),
                       "p99": round(float(np.percentile(times, 99)) * 1000, 1),
                       "note": "batch mode: every sample completes with its batch"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(out), flush=True)


SMOOTH_KERNEL = ("k_rbgs<double,2|4> (red-black Gauss-Seidel passes: 2 fused sweeps, or 4 where two consecutive "
                 "W-cycle visits of a level share a pass)")


def status_split(status):
    st = np.asarray(status)
    return {"converged": int(np.sum(st == 0)), "maxiter": int(np.sum(st == 1)), "nonfinite": int(np.sum(st == 2))}


def roofline_of(stats, kernel, traffic=None):
    """HBM roofline of one kernel kind from (launches, ms, algorithmic bytes,
    per-step model bytes).  `achieved` counts the algorithmic bytes of the
    unblocked method: every red-black sweep reads v, b and the four
    conductances of a cell and writes v (5 values, 40 B in FP64), and so do the
    residual with its restriction and the coarse-grid correction; a pass that
    fuses several of them counts each.  The fused passes keep the intermediate
    iterates in LDS, so the HBM traffic they measure (`traffic`) can be below
    that count.  `achieved_minimal` counts every value a launch needs once
    (the least any implementation of the launch must move)."""
    launches, kms, kbytes = stats[:3]
    mbytes = stats[3] if len(stats) > 3 and stats[3] else kbytes
    achieved = mbytes / (kms * 1e-3) / 1e9 if kms > 0 else None
    minimal = kbytes / (kms * 1e-3) / 1e9 if kms > 0 else None
    avg_s = kms * 1e-3 / launches if launches else None
    return {
        "kernel": kernel,
        "bound": "hbm",
        "achieved": round(achieved, 1) if achieved else None,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
        "traffic": traffic,
        "bytes_model": ("per cell: 40 B (FP64) for each red-black sweep (read v, b, kx, ky; write v), 40 B for "
                        "the residual with its restriction, 40 B for the coarse-grid correction; a fused pass "
                        "counts each step it fuses"),
        "algorithmic_bytes_per_launch": mbytes / launches if launches else None,
        "achieved_minimal": round(minimal, 1) if minimal else None,
        "frac_minimal": round(minimal / HBM_PEAK_GBS, 4) if minimal else None,
        "minimal_bytes_per_launch": kbytes / launches if launches else None,
        "minimal_model": "every value a launch needs, read or written once",
        "achieved_hbm_counters": round(traffic / avg_s / 1e9, 1) if (traffic and avg_s) else None,
        "launches": launches,
        "avg_launch_us": round(1000.0 * kms / launches, 3) if launches else None,
    }


def grids_of(u, c, P, Q):
    """Split one sample's packed cells into its grids (p-major, q-minor)."""
    out, off = [], 0
    for p in range(P + 1):
        for q in range(Q + 1):
            n = (c << p) * (c << q)
            out.append(u[off:off + n])
            off += n
    return out


def timed_run(h, msg, torch, w, opts, xi, bufs=None):
    batch = msg.Batch(w.c, w.P, w.Q)
    bufs = bufs or msg.Buffers(batch, opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    msg.run(h, w.field, batch, opts, xi, bufs)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, bufs


def take_samples(bufs, w, ids):
    """Host copies of the results of the listed samples."""
    lay = bufs.layout
    u, q, dq = bufs.u.cpu().numpy(), bufs.q.cpu().numpy(), bufs.dq.cpu().numpy()
    st, cyc = bufs.status.cpu().numpy(), bufs.cycles.cpu().numpy()
    out = []
    for s in ids:
        c0, c1, g0, g1 = lay["cell"][s], lay["cell"][s + 1], lay["grid"][s], lay["grid"][s + 1]
        out.append({"sample": int(s), "P": int(w.P[s]), "Q": int(w.Q[s]), "u": u[c0:c1].copy(),
                    "q": q[g0:g1].copy(), "dq": dq[g0:g1].copy(), "cycles": cyc[g0:g1].copy(),
                    "status": int(st[s])})
    return out


def result_errors(c, P, Q, a, b):
    """Errors of result a against reference b: largest per-grid relative L2
    error of u, largest relative error of Q, largest error of Delta Q over the
    largest |Q| among the four quantities it combines."""
    eu = 0.0
    for x, y in zip(grids_of(a["u"], c, P, Q), grids_of(b["u"], c, P, Q)):
        eu = max(eu, float(np.linalg.norm(x - y) / max(np.linalg.norm(y), 1e-300)))
    eq = float(np.max(np.abs(a["q"] - b["q"]) / np.maximum(np.abs(b["q"]), 1e-300)))
    qm = np.abs(b["q"].reshape(P + 1, Q + 1))
    scale = qm.copy()
    scale[1:, :] = np.maximum(scale[1:, :], qm[:-1, :])
    scale[:, 1:] = np.maximum(scale[:, 1:], qm[:, :-1])
    scale[1:, 1:] = np.maximum(scale[1:, 1:], qm[:-1, :-1])
    edq = float(np.max(np.abs(a["dq"] - b["dq"]) / np.maximum(scale.ravel(), 1e-300)))
    return {"u_per_grid_l2": eu, "Q": eq, "dQ": edq}


def mixed_leg(h, msg, I, torch, args):
    """1024x64 workload: batched mixed precision and batched FP64 on the same
    samples (each run once warm), the mixed error against the FP64 GPU run,
    and plain per-sample FP64 on a few samples.  Rates count solved samples;
    a ratio is reported only when every sample of the runs it compares was
    solved (a failed sample skips the stages above its failure, which would
    flatter the rate).  Returns (summary, host copies of the first mixed
    results for the oracle check of the CPU-baseline leg)."""
    w = I.config(4)
    if args.mixed_workload_samples:
        w = w.subset(args.mixed_workload_samples)
    S = w.n_samples
    xi = torch.tensor(w.xi(), dtype=torch.float64, device="cuda:0")
    om = msg.SolveOpts(tol=w.ir_tol, max_cycles=w.max_cycles, precision=msg.MIXED)
    od = msg.SolveOpts(tol=w.ir_tol, max_cycles=w.max_cycles)
    w1 = w.subset(min(8, S))
    timed_run(h, msg, torch, w1, om, xi[:w1.n_samples])          # warm the code paths
    tm, bm = timed_run(h, msg, torch, w, om, xi)
    sm = status_split(bm.status.cpu().numpy())
    log(f"mixed {w.name}: {sm['converged'] / tm:.1f} solved samples/s, {sm}")
    mixed_head = take_samples(bm, w, range(min(S, args.mixed_oracle_samples)))
    td, bd = timed_run(h, msg, torch, w, od, xi)
    sd = status_split(bd.status.cpu().numpy())
    log(f"fp64 {w.name}: {sd['converged'] / td:.1f} solved samples/s, {sd}")
    both = np.flatnonzero((bm.status.cpu().numpy() == 0) & (bd.status.cpu().numpy() == 0))
    mres = take_samples(bm, w, both)
    dres = take_samples(bd, w, both)
    worst = {"u_per_grid_l2": 0.0, "Q": 0.0, "dQ": 0.0}
    for a, b in zip(mres, dres):
        e = result_errors(w.c, a["P"], a["Q"], a, b)
        worst = {k: max(worst[k], e[k]) for k in worst}
    del bm, bd
    # plain per-sample FP64 at the same tolerance, one sample per call
    n = min(args.plain_samples, S)
    st = []
    t0 = time.perf_counter()
    for s in range(n):
        one = dataclasses.replace(w, name=f"{w.name}[{s}]", P=w.P[s:s + 1], Q=w.Q[s:s + 1])
        _, b1 = timed_run(h, msg, torch, one, od, xi[s:s + 1])
        st.append(int(b1.status.cpu().numpy()[0]))
    plain = st.count(0) / (time.perf_counter() - t0)
    full = sm["converged"] == S and sd["converged"] == S and st.count(0) == n
    mixed_value, fp64_value = sm["converged"] / tm, sd["converged"] / td
    return {"workload": w.name, "samples": S, "tol": w.ir_tol, "unit": "solved samples/s",
            "mixed_value": round(mixed_value, 2), "fp64_batched_value": round(fp64_value, 2),
            "plain_fp64_per_sample_value": round(plain, 3), "plain_samples": n, "plain_status": st,
            "mixed_over_plain_fp64": round(mixed_value / plain, 1) if full else None,
            "mixed_over_batched_fp64": round(td / tm, 2) if full else None,
            "ratios": "measured: every sample of the compared runs was solved" if full else
                      "unmeasured: some sample failed, and failed samples skip work",
            "status_mixed": sm, "status_fp64": sd, "compared_samples": int(len(both)),
            "max_rel_err_mixed_vs_gpu_fp64": worst}, mixed_head


def ragged_leg(h, msg, I, torch):
    """The ragged multi-index batch {l1+l2 <= 8} (32416 samples) in one call."""
    from paper_1907_12334_amd import autotune as AT
    w = I.config(3)
    base = msg.SolveOpts(tol=w.tol, max_cycles=w.max_cycles)
    # plan autotuned on the whole batch (full solves): tail budget, then overlap mode
    opts, tune = AT.autotune(h, w, base, samples=w.n_samples, cycles=w.max_cycles, reps=1, log=log,
                             budgets=AT.WIDE_TAIL_BUDGETS, overlaps=(1, 2))
    xi = torch.tensor(w.xi(), dtype=torch.float64, device="cuda:0")
    _, bufs = timed_run(h, msg, torch, w, opts, xi)          # warm
    t, bufs = timed_run(h, msg, torch, w, opts, xi, bufs)
    log(f"ragged {w.name}: {w.n_samples / t:.0f} samples/s with {tune['params']}")
    _, bufs0 = timed_run(h, msg, torch, w, base, xi)
    t0, bufs0 = timed_run(h, msg, torch, w, base, xi, bufs0)
    same = bool(np.array_equal(bufs.cycles.cpu().numpy(), bufs0.cycles.cpu().numpy()))
    return {"workload": w.name, "samples": w.n_samples, "value": round(w.n_samples / t, 1), "unit": "samples/s",
            "seconds": round(t, 3), "converged": int(np.sum(bufs.status.cpu().numpy() == 0)),
            "max_cycles_per_grid": int(bufs.cycles.cpu().numpy().max()), "plan": tune["params"],
            "autotune_trials": tune["trials"], "default_plan_value": round(w.n_samples / t0, 1),
            "same_cycle_counts_as_default_plan": same,
            "max_rel_q_diff_vs_default_plan": float(np.max(np.abs(bufs.q.cpu().numpy() - bufs0.q.cpu().numpy()) /
                                                           np.maximum(np.abs(bufs0.q.cpu().numpy()), 1e-300)))}


def mimc_leg(h, msg, I):
    """Algorithm MSG-MIMC to a fixed RMSE for the point value and the boundary
    flux (KL-10, c = 4, mixed precision to 1e-8), batches of 512 samples."""
    from paper_1907_12334_amd import mimc as M
    out = {"field": "KL-10", "c": 4, "precision": "mixed, refined to 1e-8", "batch": 512}
    # the geometric pmf re-fitted from the rates, and the learned pmf of the
    # paper's experiments (sample sizes ~ sqrt(V/C) per index)
    for name, kind, tol, pmf in (("Q1_point", msg.QOI_POINT, 3e-4, "geometric"),
                                 ("Q1_point_learned_pmf", msg.QOI_POINT, 3e-4, "learned"),
                                 ("Q3_flux", msg.QOI_FLUX, 3e-3, "geometric"),
                                 ("Q3_flux_learned_pmf", msg.QOI_FLUX, 3e-3, "learned")):
        est = M.MSGMIMC(h, I.KL10, c=4, kind=kind, pmf=pmf)
        r = est.run(tol=tol, batch=512)
        top = sorted(r.index_counts.items(), key=lambda kv: -kv[1])[:6]
        out[name] = {"pmf": pmf, "tol": tol, "E": r.E, "rmse": r.rmse, "samples": r.N, "batches": r.batches,
                     "seconds": round(r.seconds, 3), "samples_per_s": round(r.N / r.seconds, 1),
                     "cell_visits": float(sum(t for _, t in est.work.values())),
                     "learned_rates": [round(x, 3) for x in r.rates],
                     "fitted_work_rates_gamma": [round(x, 3) for x in r.gamma],
                     "most_drawn_indices": [[list(k), v] for k, v in top]}
        log(f"MSG-MIMC {name}: E={r.E:.6f} rmse={r.rmse:.2e} N={r.N} in {r.seconds:.1f} s")
    # the paper's own field model: Matern (lambda = 1/4, nu = 1/2) with eta and
    # theta uniform per sample, exact fields by circulant embedding per sample;
    # indices capped at 7 (512 cells per direction, the paper's 2^18 unknowns;
    # embeddings of 16384 points per direction, rows by the four-step FFT)
    est = M.MSGMIMC(h, c=4, kind=msg.QOI_POINT, lmax=7, prior=I.MATERN_PAPER)
    r = est.run(tol=1e-3, batch=512, max_samples=1 << 17)
    top = sorted(r.index_counts.items(), key=lambda kv: -kv[1])[:6]
    out["Q1_point_matern_prior"] = {
        "field": "Matern lambda=1/4 nu=1/2, eta~U[1/16,1/4], theta~U[-30,30] deg, per-sample circulant embedding",
        "lmax": 7, "tol": 1e-3, "E": r.E, "rmse": r.rmse, "samples": r.N, "batches": r.batches,
        "seconds": round(r.seconds, 3), "samples_per_s": round(r.N / r.seconds, 1),
        "learned_rates": [round(x, 3) for x in r.rates], "fitted_work_rates_gamma": [round(x, 3) for x in r.gamma],
        "min_embedding_eig_ratio": est.min_eig_ratio,
        "samples_at_index_7": int(sum(v for k, v in r.index_counts.items() if max(k) == 7)),
        "most_drawn_indices": [[list(k), v] for k, v in top]}
    log(f"MSG-MIMC Q1 Matern prior: E={r.E:.6f} rmse={r.rmse:.2e} N={r.N} in {r.seconds:.1f} s")
    return out


def factors_leg(h):
    """Standard multigrid against MSG on the paper's Matern fields (lambda =
    1/4, nu = 1/2): plain cycles from zero, h = 1, 100 samples, 50 cycles,
    c = 2.  (a) 64 x 64 cells, W(2,2), eta in {1/4, 1/8, 1/16}, theta in {0,
    10, 20, 30} degrees: expected factor and median residual ratio after 10
    cycles; (b) eta = 1/16: W(nu,nu), nu = 1..5, on 8^2 .. 128^2 cells.
    Entries are [MG, MSG]; a factor is null where some sample did not
    converge."""
    from paper_1907_12334_amd.factors import Experiment
    ex = Experiment(h, c=2, samples=100, cycles=50)
    t0 = time.perf_counter()
    thetas = (0, 10, 20, 30)
    a = ex.table((0.25, 0.125, 0.0625), thetas, [5], [2])
    b = ex.table((0.0625,), thetas, [2, 3, 4, 5, 6], [1, 2, 3, 4, 5])
    secs = time.perf_counter() - t0

    def r(x, d=4):
        return None if x is None else float(f"{x:.{d}g}")

    out = {"setup": "Matern lambda=1/4, nu=1/2 (circulant embedding), c=2, 100 samples, 50 cycles from zero, h=1; "
                    "factor = (r_k/r_0)^(1/k) at the last k with r_k >= 1e-10; [MG, MSG]",
           "seconds": round(secs, 2), "min_embedding_eig_ratio": ex.min_eig_ratio,
           "fields_seconds": round(ex.field_seconds, 3), "field_samples": ex.field_samples,
           "64x64_W(2,2)_factor": {}, "64x64_W(2,2)_median_r10": {}, "eta=1/16_factor_by_cells": {}}
    for row in a:
        k1, k2 = f"eta={row['eta']:g}", f"theta={row['theta']}"
        out["64x64_W(2,2)_factor"].setdefault(k1, {})[k2] = [r(row["MG"]), r(row["MSG"])]
        out["64x64_W(2,2)_median_r10"].setdefault(k1, {})[k2] = [r(row["MG_median_r10"], 2),
                                                                  r(row["MSG_median_r10"], 2)]
    for row in b:
        d = out["eta=1/16_factor_by_cells"].setdefault(f"theta={row['theta']}", {}).setdefault(
            f"W({row['nu']},{row['nu']})", {})
        d[row["cells"]] = [r(row["MG"], 3), r(row["MSG"], 3)]
    log(f"convergence factors ({secs:.1f} s): {out['64x64_W(2,2)_factor']}")
    return out


def serve_leg(msg, I, args):
    """Request loop on a window of the 200 000-request Poisson trace (5000/s):
    its first `serve_requests` requests at the trace's rate, and the same
    requests at lower offered rates (arrival times scaled), to find the
    sustained capacity and the load at which latency degrades.  Returns
    (summary, served answers of small requests for the oracle check of the
    CPU leg)."""
    from paper_1907_12334_amd.serve import Engine, replay, summarize
    opts = msg.SolveOpts(tol=1e-8, max_cycles=200, precision=msg.MIXED)
    t, P, Q, ids = I.request_trace(200000, 5000.0)
    n = min(args.serve_requests, len(t))
    t, P, Q, ids = t[:n] - t[0], P[:n], Q[:n], ids[:n]
    out = {"field": "KL-10, normals drawn on the device per request", "c": 4,
           "precision": "mixed, refined to 1e-8", "trace": f"first {n} of 200000 requests, Poisson at 5000/s",
           "admission": "80% of free HBM in one arena per worker, 3 small-request workers + 1 large-request worker",
           "runs": {}}
    kept = []
    for rate in args.serve_rates:
        eng = Engine(I.KL10, 4, opts, workers=3, big_workers=1)
        try:
            reqs = replay(eng, t * (5000.0 / rate), P, Q, ids, timeout=900)
        finally:
            eng.close()
        s = summarize(reqs, rate)
        s["max_batches_in_flight"] = eng.max_inflight
        s["batches"] = len(eng.batches)
        out["runs"][f"{rate:g}_per_s"] = s
        log(f"serving at {rate:g}/s: {s}")
        if rate == 5000.0:
            kept = [{"sample": r.sample_id, "P": r.P, "Q": r.Q, "q": r.q, "dq": r.dq, "status": r.status}
                    for r in reqs if r.P + r.Q <= 6][:args.serve_oracle_requests]
        del eng
        import torch
        torch.cuda.empty_cache()
    sat = [float(k.split("_")[0]) for k, v in out["runs"].items() if v.get("saturated")]
    out["capacity_samples_per_s"] = max((v["samples_per_s"] for v in out["runs"].values() if v.get("saturated")),
                                        default=None)
    out["lowest_saturating_offered_per_s"] = min(sat) if sat else None
    out["highest_kept_up_offered_per_s"] = max((float(k.split("_")[0]) for k, v in out["runs"].items()
                                                if not v.get("saturated")), default=None)
    return out, kept


def cpu_share():
    """(threads for the oracle, CPUs in the affinity set): every CPU of the
    affinity set, within the process's CPU share where the environment
    states one (OMP_NUM_THREADS)."""
    aff = len(os.sched_getaffinity(0))
    share = os.environ.get("OMP_NUM_THREADS")
    threads = min(aff, int(share)) if share and share.isdigit() and int(share) > 0 else aff
    return threads, aff


def cpu_baseline(w, head, w4=None, mixed_head=None, served=None):
    """The oracle (field + full-MSG solve + differences) on host cores, one
    sample per thread, on the first samples of the same workload (as many as
    threads): its rate is the CPU baseline.  Its results are also compared
    with the GPU's on those samples, and the oracle is run (untimed) on the
    first samples of the 1024x64 workload to state the error of the GPU's
    mixed-precision results against it."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import binding as O
    threads, aff = cpu_share()
    n = len(head)

    def one(wl, s, tol=None):
        spec = wl.field.as_dict()
        xi = wl.xi([s])[0]
        kx, ky = O.hierarchy_field(wl.c, wl.P[s], wl.Q[s], spec, xi)
        r = O.fmsg_solve(wl.c, wl.P[s], wl.Q[s], kx, ky, O.opts(tol=tol or wl.tol, max_cycles=wl.max_cycles))
        r["dq"] = O.delta_q(wl.P[s], wl.Q[s], r["q"])
        return r

    O.lib()
    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        res = list(ex.map(lambda g: one(w, g["sample"]), head))
    dt = time.perf_counter() - t0
    t1 = time.perf_counter()
    one(w, head[0]["sample"])
    d1 = time.perf_counter() - t1
    solved = sum(1 for r in res if r["status"] == 0)
    worst = {"u_per_grid_l2": 0.0, "Q": 0.0, "dQ": 0.0}
    same_cycles = True
    for g, r in zip(head, res):
        same_cycles &= bool(np.array_equal(g["cycles"], r["cycles"]))
        e = result_errors(w.c, g["P"], g["Q"], g, r)
        worst = {k: max(worst[k], e[k]) for k in worst}
    out = {"value": round(solved / dt, 4), "unit": "solved samples/s", "cores": threads, "kind": "oracle",
           "sample": f"first {n} samples of {w.name}, one per thread", "seconds": round(dt, 2),
           "affinity_cpus": aff, "status": {"converged": solved, "failed": n - solved},
           "one_core": {"value": round(1.0 / d1, 4), "unit": "samples/s", "sample": "the first sample alone"},
           "cpu_model": cpu_model(),
           "gpu_vs_oracle_headline": {"samples": n, "same_cycle_counts": same_cycles, "max_err": worst}}
    if w4 is not None and mixed_head:
        with ThreadPoolExecutor(threads) as ex:
            res4 = list(ex.map(lambda g: one(w4, g["sample"], 1e-10), mixed_head))
        worst4 = {"u_per_grid_l2": 0.0, "Q": 0.0, "dQ": 0.0}
        per = []
        for g, r in zip(mixed_head, res4):
            e = result_errors(w4.c, g["P"], g["Q"], g, r)
            per.append({"sample": g["sample"], "gpu_status": g["status"], "oracle_status": int(r["status"]), **e})
            worst4 = {k: max(worst4[k], e[k]) for k in worst4}
        out["gpu_mixed_vs_fp64_oracle_1024x64"] = {
            "note": "mixed precision refined to 1e-8 on the GPU against the FP64 oracle run to 1e-10",
            "samples": len(per), "max_err": worst4, "per_sample": per}
    if served:
        from oracle import normals as N
        from paper_1907_12334_amd import inputs as I
        seed = I.BASE_SEED + 5

        def ora(r):
            xi = N.kl_normals(I.KL10.n_terms, [r["sample"]], seed)[0]
            kx, ky = O.hierarchy_field(4, r["P"], r["Q"], I.KL10.as_dict(), xi)
            res = O.fmsg_solve(4, r["P"], r["Q"], kx, ky, O.opts(tol=1e-10, max_cycles=200))
            return res["status"], res["q"], O.delta_q(r["P"], r["Q"], res["q"])
        with ThreadPoolExecutor(threads) as ex:
            res5 = list(ex.map(ora, served))
        eq = edq = 0.0
        for r, (st, q, dq) in zip(served, res5):
            eq = max(eq, float(np.max(np.abs(r["q"] - q) / np.abs(q))))
            edq = max(edq, float(np.max(np.abs(r["dq"] - dq)) / np.max(np.abs(q))))
        out["served_vs_fp64_oracle"] = {
            "note": "requests served at 5000/s (mixed precision, refined to 1e-8) against the FP64 oracle at 1e-10",
            "requests": len(served), "all_converged": all(r["status"] == 0 for r in served) and
            all(st == 0 for st, _, _ in res5), "max_err": {"Q": eq, "dQ_over_max_Q": edq}}
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


if __name__ == "__main__":
    main()
