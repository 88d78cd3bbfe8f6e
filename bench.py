"""Benchmark: batched plain VDAMP (Algorithm 1, SURE soft thresholding) on one MI355X.

Workload: a batch of B independent 256x256 slices of the single-256 recipe (16-ellipse
phantoms with smooth phase, polynomial variable density with a 16x16 fully sampled
centre, R = 4, 6, 8 in turn, 40 dB, 4-level Haar), 50 iterations per solve.  One
step = one complete solve of the batch (every pass of every iteration plus the output
step).  Inputs are resident in HBM before the timed region.

Prints ONE JSON line.  `value` is slice-iterations per second over the timed steps.
`roofline` reports the dominant kernel class (largest share of kernel time, from HIP
events recorded around every launch on the solve's stream inside the timed region):
algorithmic bytes it must move per launch / its average launch time, against the
MI355X HBM peak; `traffic` is the HBM bytes per launch that rocprofv3's FETCH_SIZE and
WRITE_SIZE counters measured for that kernel (scaled by a copy of known size), taken
from profiles/ while the kernel's sources are unchanged, else null.  `cpu_baseline` is the FP64 oracle timed on the host on a bounded
sample of the same workload.
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

METRIC = "VDAMP iters/sec and time-to-NMSE (256² batch); learned vs plain at equal NMSE"
HBM_PEAK_GBS = 8000.0
ITERS = 50
LEVELS = 4

# Algorithmic HBM bytes per pixel of each kernel class, per launch mode (complex64 = 8 B,
# float32 = 4 B).  rows_synth: read r, write X.  cols: read X, y, m/p, write X (first
# iteration: no X read).  rows_anal: read X and r, write r (first: no r read; output:
# read X, write x_hat).  sure: read r.
BYTES = {
    "rows_synth": 16.0,
    "cols": 28.0, "cols_first": 20.0,
    "rows_anal": 24.0, "rows_anal_first": 16.0, "rows_anal_out": 16.0,
    "sure": 8.0,
}


def algorithmic_bytes_per_solve(npx, iters):
    """Per kernel class: total algorithmic bytes over one solve and the launch count."""
    rs = (iters - 1 + 1) * BYTES["rows_synth"] * npx          # K-1 iterations + output
    cols = ((iters - 1) * BYTES["cols"] + BYTES["cols_first"] + BYTES["cols"]) * npx
    ra = ((iters - 1) * BYTES["rows_anal"] + BYTES["rows_anal_first"] + BYTES["rows_anal_out"]) * npx
    su = iters * BYTES["sure"] * npx
    return {"rows_synth": (rs, iters), "cols": (cols, iters + 1),
            "rows_anal": (ra, iters + 1), "sure": (su, iters)}


def make_batch(B):
    from paper_1911_01234_amd import synth
    slices, s, K = synth.workload_batch256(B)
    return slices, s, K


def nmse_db_batch(x_hat, x0, seg, batch):
    """Per-slice NMSE (dB) of a packed batch; seg holds each pixel's slice index."""
    import torch
    d = torch.zeros(batch, dtype=torch.float64, device=x0.device)
    n = torch.zeros_like(d)
    d.index_add_(0, seg, (x_hat - x0).abs().pow(2).double())
    n.index_add_(0, seg, x0.abs().pow(2).double())
    return (10.0 * torch.log10(d / n)).cpu().numpy()


KERNEL_SOURCES = {"cols": ["paper_1911_01234_amd/csrc/vdamp_passes.hip",
                           "paper_1911_01234_amd/csrc/vdamp_device.hpp",
                           "paper_1911_01234_amd/csrc/vdamp_internal.h"]}


def measured_traffic(kernel_class):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken
    on the kernel sources as they are now (else None)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_k_{kernel_class}_b256_256x256.md")
    if kernel_class not in KERNEL_SOURCES or not os.path.exists(path):
        return None
    rec = None
    for line in open(path):
        if line.startswith("TRAFFIC_RECORD "):
            rec = json.loads(line[len("TRAFFIC_RECORD "):])
    if rec is None:
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel_class]:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return rec["traffic_bytes_per_launch"] if h.hexdigest()[:16] == rec["source_sha"] else None


def cpu_baseline(slices, s, iters, budget_s):
    """FP64 oracle on the host, one slice at a time, until about budget_s seconds."""
    from oracle import vdamp_ref as o
    t0 = time.perf_counter()
    done = 0
    for sl in slices:
        o.vdamp(sl.y, sl.mask, sl.p, sl.sigma2, s, iters)
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": done * iters / dt, "unit": "slice-iterations/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} of the batch's 256x256 slices x {iters} iterations, FP64 NumPy, "
                      f"one process (pocketfft and sort single-threaded), {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--graph", action="store_true", help="time hipGraph replays instead of eager launches")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB device-to-device three times (a kernel of known traffic "
                         "for scaling hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: slices are independent, so a multi-GPU run "
              "would assign whole slices to GPUs with no communication; --gpus must be 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1911_01234_amd import vdamp as V

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    t_gen = time.perf_counter()
    slices, s, K = make_batch(args.batch)
    t_gen = time.perf_counter() - t_gen
    B = len(slices)
    ny = [sl.y.shape[0] for sl in slices]
    nx = [sl.y.shape[1] for sl in slices]
    npx = int(sum(a * b for a, b in zip(ny, nx)))
    print(f"[bench] generated {B} slices of 256x256 in {t_gen:.1f} s", file=sys.stderr, flush=True)

    stream = torch.cuda.Stream()
    flags = V.VDAMP_FLAG_USE_GRAPH if args.graph else V.VDAMP_FLAG_TIMING
    t_plan = time.perf_counter()
    plan = V.Plan(ny, nx, LEVELS, flags)
    t_plan = time.perf_counter() - t_plan
    ws = plan.workspace()
    y, mask, p, sigma2 = V.to_device(plan, slices)
    x_hat = torch.empty(plan.ntot, dtype=torch.complex64, device="cuda")
    x0 = torch.from_numpy(plan.pack([sl.x0 for sl in slices], np.complex64)).cuda()
    seg = torch.from_numpy(np.repeat(np.arange(B), [a * b for a, b in zip(ny, nx)])).cuda()

    def step(iters=K):
        with torch.cuda.stream(stream):
            plan.vdamp_solve(ws, y, mask, p, sigma2, iters, x_hat, None, stream=stream)

    for _ in range(args.warmup):
        step()
    stream.synchronize()
    if flags & V.VDAMP_FLAG_TIMING:
        plan.vdamp_pass_times()  # reset counters
    print(f"[bench] warmup done, timing {args.steps} steps", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    stream.synchronize()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = 1e3 * dt / args.steps
    value = B * K * args.steps / dt

    roofline = None
    pass_ms = None
    if flags & V.VDAMP_FLAG_TIMING:
        times = plan.vdamp_pass_times()
        pass_ms = {k: v[0] / args.steps for k, v in times.items()}
        alg = algorithmic_bytes_per_solve(npx, K)
        dom = max(alg, key=lambda k: times[k][0])
        tot_ms, launches = times[dom]
        bytes_total = alg[dom][0] * args.steps
        avg_launch_s = tot_ms / 1e3 / launches
        achieved = bytes_total / launches / avg_launch_s / 1e9
        traffic = measured_traffic(dom)
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                    "kernel": dom, "avg_launch_us": round(1e6 * avg_launch_s, 2),
                    "alg_bytes_per_launch": int(bytes_total / launches)}
        allb = sum(v[0] for v in alg.values()) * args.steps
        allt = sum(times[k][0] for k in alg) / 1e3
        roofline["all_passes_achieved_GBs"] = round(allb / allt / 1e9, 1)

    # time-to-NMSE: smallest iteration count whose batch-mean NMSE is within 0.1 dB of
    # the 50-iteration value (monitored runs), timed unmonitored
    step(K)
    stream.synchronize()
    target = float(nmse_db_batch(x_hat, x0, seg, B).mean()) + 0.1
    k_hit = K
    for k in range(1, K + 1):
        step(k)
        stream.synchronize()
        if float(nmse_db_batch(x_hat, x0, seg, B).mean()) <= target:
            k_hit = k
            break
    reps = 3
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(reps):
        step(k_hit)
    stream.synchronize()
    t_nmse = (time.perf_counter() - t1) / reps
    if flags & V.VDAMP_FLAG_TIMING:
        plan.vdamp_pass_times()

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        cpu = cpu_baseline(slices, s, K, args.cpu_budget)

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "slice-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"batched plain VDAMP, {B} slices of 256x256 (16-ellipse phantoms, "
                               f"R=4/6/8, 40 dB), 4-level Haar, {K} iterations per solve",
                   "batch": B, "ny": 256, "nx": 256, "levels": LEVELS, "iters": K,
                   "launch": "hipGraph" if args.graph else "eager, HIP events per kernel"},
        "mpx_iterations_per_s": round(value * 65536 / 1e6, 1),
        "time_to_nmse": {"target_db": round(target, 3), "iters": k_hit, "seconds": round(t_nmse, 5)},
        "plan_seconds": round(t_plan, 4),
        "roofline": roofline,
        "pass_ms_per_step": {k: round(v, 4) for k, v in pass_ms.items()} if pass_ms else None,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    plan.close()


if __name__ == "__main__":
    main()
