"""Benchmark: batched full-MSG solves of the 256x256 separable lognormal workload.

One step = the whole hot path over one batch: coefficient-field synthesis at
every face of every grid, the full-MSG solve of every sample to a relative
residual of 1e-10 on all 64 grids, and the multi-index differences.  Inputs
(the standard normal KL coefficients) are resident in HBM before timing.

Prints one JSON line.  Beside the headline value it reports:
  * the plain per-sample FP64 GPU MSG (the same library, one sample per
    call) on a few samples, for the batched-vs-plain ratio;
  * the mixed-precision path on a slice of the batch, with its error against
    the FP64 result of the same samples;
  * the smoother's achieved bandwidth from HIP events around its launches in
    the timed region (roofline), and the oracle timed on host cores.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--samples", type=int, default=None, help="batch size (default: the preset's 4096)")
    ap.add_argument("--plain-samples", type=int, default=2)
    ap.add_argument("--mixed-samples", type=int, default=512)
    ap.add_argument("--cpu-samples", type=int, default=None)
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--skip-plain", action="store_true")
    ap.add_argument("--skip-mixed", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="no HIP events around launches")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "traffic_rbgs.json"))
    return ap.parse_args()


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
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
    bufs = msg.Buffers(batch, opts)
    log(f"device buffers {sum(t.numel() * t.element_size() for t in [bufs.kx, bufs.ky, bufs.u, bufs.ws]) / 1e9:.1f} GB")

    def step():
        msg.run(h, w.field, batch, opts, xi, bufs)

    for k in range(args.warmup):
        t0 = time.perf_counter()
        step()
        torch.cuda.synchronize()
        log(f"warmup {k}: {time.perf_counter() - t0:.2f} s")

    h.set_profiling(not args.no_profile)
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
    converged = int(np.sum(status == 0))
    value = S * args.steps / elapsed
    ms = 1000.0 * elapsed / args.steps
    log(f"converged {converged}/{S}, max cycles per grid {cycles.max()}, {value:.1f} samples/s")

    # roofline of the dominant kernel (the smoother), from the timed region
    launches, kms, kbytes = prof["smooth"]
    achieved = kbytes / (kms * 1e-3) / 1e9 if kms > 0 else None
    kernel_share = {k: (v[1] / 1000.0) / elapsed for k, v in prof.items()}
    traffic = None
    if os.path.exists(args.traffic):
        try:
            traffic = json.load(open(args.traffic)).get("bytes_per_launch")
        except Exception:
            traffic = None
    roofline = {
        "kernel": "k_rbgs<double,2> (red-black Gauss-Seidel, 2 fused sweeps)",
        "bound": "hbm",
        "achieved": round(achieved, 1) if achieved else None,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
        "traffic": traffic,
        "launches": launches,
        "avg_launch_us": round(1000.0 * kms / launches, 3) if launches else None,
        "algorithmic_bytes_per_launch": kbytes / launches if launches else None,
    }

    extra = {"kernel_time_share": {k: round(v, 4) for k, v in kernel_share.items()},
             "samples_converged": converged, "max_cycles_per_grid": int(cycles.max())}

    # plain per-sample FP64 GPU MSG: one sample per call, same kernels
    if not args.skip_plain:
        n = min(args.plain_samples, S)
        b1 = msg.Batch(w.c, w.P[:1], w.Q[:1])
        bp = msg.Buffers(b1, opts)
        msg.run(h, w.field, b1, opts, xi[0:1], bp)          # warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(n):
            msg.run(h, w.field, b1, opts, xi[s:s + 1], bp)
        torch.cuda.synchronize()
        plain = n / (time.perf_counter() - t0)
        extra["plain_fp64_per_sample"] = {"value": round(plain, 3), "unit": "samples/s", "samples": n}
        extra["batched_over_plain"] = round(value / plain, 1)
        log(f"plain per-sample FP64: {plain:.3f} samples/s")

    # mixed precision on a slice, error against the FP64 result of those samples
    if not args.skip_mixed:
        n = min(args.mixed_samples, S)
        wm = w.subset(n)
        bm = msg.Batch(wm.c, wm.P, wm.Q)
        om = msg.SolveOpts(tol=1e-8, max_cycles=w.max_cycles, precision=msg.MIXED)
        bufm = msg.Buffers(bm, om)
        msg.run(h, wm.field, bm, om, xi[:n], bufm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        msg.run(h, wm.field, bm, om, xi[:n], bufm)
        torch.cuda.synchronize()
        tm = time.perf_counter() - t0
        u64 = bufs.u[: bufm.u.numel()]
        lay = bufm.layout
        # worst per-grid relative difference to the FP64 solve over the slice (sampled grids)
        err = 0.0
        uc, um = u64.cpu().numpy(), bufm.u.cpu().numpy()
        for s in range(0, n, max(1, n // 16)):
            a = grids_of(uc[lay["cell"][s]:lay["cell"][s + 1]], wm.c, wm.P[s], wm.Q[s])
            b = grids_of(um[lay["cell"][s]:lay["cell"][s + 1]], wm.c, wm.P[s], wm.Q[s])
            for x, y in zip(a, b):
                err = max(err, float(np.linalg.norm(x - y) / np.linalg.norm(x)))
        extra["mixed"] = {"value": round(n / tm, 2), "unit": "samples/s", "samples": n, "tol": 1e-8,
                          "max_rel_err_vs_fp64": err,
                          "converged": int(np.sum(bufm.status.cpu().numpy() == 0))}
        log(f"mixed: {n / tm:.1f} samples/s, max rel err vs FP64 {err:.2e}")

    cpu = None
    if not args.skip_cpu:
        cpu = cpu_baseline(w, args.cpu_samples)
        log(f"cpu oracle: {cpu}")

    out = {
        "metric": "MSG solved samples/sec at 1e-8 rel. residual + p50/p99 latency, vs plain FP64",
        "value": round(value, 3),
        "unit": "samples/s",
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
                   "field": "separable SE 50x50, lx=0.3, ly=0.03, sigma2=1", "tol": w.tol,
                   "cycle": "W(2,2)", "precision": "fp64"},
        "latency_ms": {"p50": round(float(np.percentile(times, 50)) * 1000, 1),
                       "p99": round(float(np.percentile(times, 99)) * 1000, 1),
                       "note": "batch mode: every sample completes with its batch"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(out), flush=True)


def grids_of(u, c, P, Q):
    """Split one sample's packed cells into its grids (p-major, q-minor)."""
    out, off = [], 0
    for p in range(P + 1):
        for q in range(Q + 1):
            n = (c << p) * (c << q)
            out.append(u[off:off + n])
            off += n
    return out


def cpu_baseline(w, n=None):
    """The oracle (field + full-MSG solve + differences) on host cores, one
    sample per thread, on the first n samples of the same workload."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import binding as O
    cores = len(os.sched_getaffinity(0))
    cores = min(cores, 16)
    n = n or cores
    xi = w.xi(range(n))
    spec = w.field.as_dict()

    def one(s):
        kx, ky = O.hierarchy_field(w.c, w.P[s], w.Q[s], spec, xi[s])
        r = O.fmsg_solve(w.c, w.P[s], w.Q[s], kx, ky, O.opts(tol=w.tol, max_cycles=w.max_cycles))
        O.delta_q(w.P[s], w.Q[s], r["q"])
        return r["status"]

    O.lib()
    t0 = time.perf_counter()
    with ThreadPoolExecutor(cores) as ex:
        list(ex.map(one, range(n)))
    dt = time.perf_counter() - t0
    return {"value": round(n / dt, 4), "unit": "samples/s", "cores": cores, "kind": "oracle",
            "sample": f"first {n} samples of {w.name}, one per thread", "seconds": round(dt, 2)}


if __name__ == "__main__":
    main()
