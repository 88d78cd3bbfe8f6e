"""Benchmark: batched plain VDAMP (Algorithm 1, SURE soft thresholding) on one MI355X,
and the learned-denoiser form against it.

Workload: a batch of B independent 256x256 slices of the single-256 recipe (16-ellipse
phantoms with smooth phase, polynomial variable density with a 16x16 fully sampled
centre, R = 4, 6, 8 in turn, 40 dB, 4-level Haar), 50 iterations per solve.  One
step = one complete solve of the batch (every pass of every iteration plus the output
step).  Inputs are resident in HBM before the timed region.

Prints ONE JSON line.  `value` is slice-iterations per second over the timed steps
(eager launches, nothing else on the stream).  `roofline` reports the dominant kernel
class (largest share of kernel time, from HIP events recorded around every pass on the
solve's stream during a second timed run of the same steps, `kernel_event_run`, whose
rate the events lower by about 7 %):
algorithmic bytes it must move per launch / its average launch time, against the
MI355X HBM peak; `traffic` is the HBM bytes per launch that rocprofv3's FETCH_SIZE and
WRITE_SIZE counters measured for that kernel (scaled by a copy of known size), taken
from profiles/ while the kernel's sources are unchanged, else null.  `cpu_baseline` is the FP64 oracle timed on the host on a bounded
sample of the same workload.

`learned` (unless --no-learned): the CNN denoiser is trained on the GPU by the library's
own kernels on (Psi^H r_k, tau_k, x0) pairs from plain-VDAMP solves of a disjoint set
of 256x256 slices (same generator), then 64 held-out slices of the timed batch are
solved with plain VDAMP and with the SURE-judged learned form: mean NMSE at 50
iterations, the learned form's NMSE at the wall-clock of the plain 50-iteration solve,
and each form's time to reach the plain form's 50-iteration NMSE.  `cnn_roofline`: the
network pass of a learned iteration (input packing, forward and JVP) against its binding
roofline, HBM (algorithmic activation bytes per pixel, CNN_BYTES_PER_PX, at 8 TB/s take
about 2.3x as long as its FLOPs at the dense BF16 MFMA peak), with the MFMA rate beside.
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
BF16_PEAK_TFLOPS = 2500.0
# FLOPs per pixel of the network's forward pass: 3x3 convolutions 2->48, 4 x 48->48, 48->2
CNN_FLOP_PER_PX = 2 * 9 * (2 * 48 + 4 * 48 * 48 + 48 * 2)
# Algorithmic HBM bytes per pixel of one learned iteration's network pass (forward + JVP),
# activations BF16 [pixel][channel]: packing the image and the probe into 8-channel
# inputs (read 8, write 16, twice); forward: layer 1 reads 16 and writes 96, layers 2-5
# read and write 96, layers 1-5 also write their 8-byte ReLU pattern, layer 6 reads 96
# plus the 8-byte residual and writes 8; JVP: the same with the pattern read instead
# of written.
CNN_BYTES_PER_PX = 2 * 24 + 2 * ((16 + 96 + 8) + 4 * (96 + 96 + 8) + (96 + 8 + 8))
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


def pass_rooflines(times, npx, iters, steps):
    """Per kernel class: average launch time and algorithmic bytes / time against the
    HBM peak (times from the plan's per-kernel HIP events over `steps` solves)."""
    alg = algorithmic_bytes_per_solve(npx, iters)
    out = {}
    for k, (b, _) in alg.items():
        ms, launches = times[k]
        if launches == 0:
            continue
        gbs = b * steps / (ms / 1e3) / 1e9
        out[k] = {"us_per_launch": round(1e3 * ms / launches, 2), "achieved_GBs": round(gbs, 1),
                  "frac": round(gbs / HBM_PEAK_GBS, 4)}
    return out


def other_workloads(stream, reps=3):
    """Throughput of the other batch shapes the library is built for: 64 and 512 slices of
    256^2, the ragged batch of 512 slices (128 each of 128^2, 192^2, 256^2, 320^2) and 128
    slices of 512^2 (whose finest bands take the large-band threshold search), each
    planned with the plan-time tuner.  One warm-up solve, then `reps` timed solves of 50 iterations each, eager with
    per-kernel events."""
    import torch
    from paper_1911_01234_amd import synth, vdamp as V
    res = {}
    for name, gen in (("batch_64_slices_256x256", lambda: synth.workload_batch256(64)),
                      ("batch_512_slices_256x256", lambda: synth.workload_batch256(512)),
                      ("mixed_512_slices_128_to_320", lambda: synth.workload_mixed(128)),
                      ("batch_128_slices_512x512", lambda: synth.workload_batch512(128))):
        t = time.perf_counter()
        slices, s, K = gen()
        tg = time.perf_counter() - t
        ny = [sl.y.shape[0] for sl in slices]
        nx = [sl.y.shape[1] for sl in slices]
        npx = int(sum(u * v for u, v in zip(ny, nx)))
        with torch.cuda.stream(stream):
            t = time.perf_counter()
            plan = V.Plan(ny, nx, s, V.VDAMP_FLAG_TIMING | V.VDAMP_FLAG_AUTOTUNE)
            t_plan = time.perf_counter() - t
            desc = plan.describe()
            ws = plan.workspace()
            y, mask, p, sigma2 = V.to_device(plan, slices)
            xh = torch.empty(plan.ntot, dtype=torch.complex64, device="cuda")
            x0 = torch.from_numpy(plan.pack([sl.x0 for sl in slices], np.complex64)).cuda()
            seg = torch.from_numpy(np.repeat(np.arange(len(slices)), [u * v for u, v in zip(ny, nx)])).cuda()
            plan.vdamp_solve(ws, y, mask, p, sigma2, K, xh, stream=stream)
            stream.synchronize()
            plan.vdamp_pass_times()
            t = time.perf_counter()
            for _ in range(reps):
                plan.vdamp_solve(ws, y, mask, p, sigma2, K, xh, stream=stream)
            stream.synchronize()
            dt = (time.perf_counter() - t) / reps
            times = plan.vdamp_pass_times()
            nm = float(nmse_db_batch(xh, x0, seg, len(slices)).mean())
            plan.close()
        del ws, y, mask, p, sigma2, xh, x0, seg
        torch.cuda.empty_cache()
        res[name] = {"slices": len(slices), "pixels": npx, "iters": K,
                     "seconds_per_solve": round(dt, 5),
                     "slice_iterations_per_s": round(len(slices) * K / dt, 1),
                     "mpx_iterations_per_s": round(npx * K / dt / 1e6, 1),
                     "nmse_db_mean": round(nm, 3),
                     "passes": pass_rooflines(times, npx, K, reps),
                     "plan_seconds_with_autotune": round(t_plan, 3),
                     "autotune": desc[desc.index("autotune:") + 10:] if "autotune:" in desc else None}
        print(f"[bench] {name}: generated in {tg:.1f} s, {res[name]['slice_iterations_per_s']} slice-it/s",
              file=sys.stderr, flush=True)
    return res


def make_batch(B):
    from paper_1911_01234_amd import synth
    slices, s, K = synth.workload_batch256(B)
    return slices, s, K


def nmse_db_batch(x_hat, x0, seg, batch):
    """Per-slice NMSE (dB) of a packed batch; seg holds each pixel's slice index (slices
    of equal size are reduced as rows of a matrix, others by an indexed sum)."""
    import torch
    n = x0.numel()
    if n % batch == 0 and bool((seg.view(batch, -1) == torch.arange(batch, device=seg.device)[:, None]).all()):
        d = (x_hat - x0).abs().pow(2).double().view(batch, -1).sum(1)
        s = x0.abs().pow(2).double().view(batch, -1).sum(1)
    else:
        d = torch.zeros(batch, dtype=torch.float64, device=x0.device)
        s = torch.zeros_like(d)
        d.index_add_(0, seg, (x_hat - x0).abs().pow(2).double())
        s.index_add_(0, seg, x0.abs().pow(2).double())
    return (10.0 * torch.log10(d / s)).cpu().numpy()


_PASS_SRC = ["paper_1911_01234_amd/csrc/vdamp_passes.hip", "paper_1911_01234_amd/csrc/vdamp_device.hpp",
             "paper_1911_01234_amd/csrc/vdamp_internal.h"]
KERNEL_SOURCES = {"cols": _PASS_SRC, "rows_synth": _PASS_SRC, "rows_anal": _PASS_SRC,
                  "sure": ["paper_1911_01234_amd/csrc/vdamp_sure.hip", "paper_1911_01234_amd/csrc/vdamp_device.hpp",
                           "paper_1911_01234_amd/csrc/vdamp_internal.h"]}


def measured_traffic(kernel_class):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken
    on the kernel sources as they are now (else None)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel_class}_b256_256x256.md")
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


def cpu_baseline(slices, s, iters, budget_s, gpu_nmse=None):
    """FP64 oracle on the host, one slice at a time, until about budget_s seconds.  With
    the GPU's per-slice NMSE after the same iteration count, the sample's oracle NMSE is
    reported beside it."""
    from oracle import vdamp_ref as o
    t0 = time.perf_counter()
    done = 0
    nm = []
    for sl in slices:
        xr = o.vdamp(sl.y, sl.mask, sl.p, sl.sigma2, s, iters)["x_hat"]
        done += 1
        nm.append(10.0 * np.log10(np.sum(np.abs(xr - sl.x0) ** 2) / np.sum(np.abs(sl.x0) ** 2)))
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    out = {"value": done * iters / dt, "unit": "slice-iterations/s", "cores": 1, "kind": "oracle",
           "sample": f"{done} of the batch's 256x256 slices x {iters} iterations, FP64 NumPy, "
                     f"one process (pocketfft and sort single-threaded), {dt:.1f} s"}
    if gpu_nmse is not None:
        g = np.asarray(gpu_nmse[:done], dtype=np.float64)
        d = g - np.asarray(nm)
        out["nmse_check"] = {"slices": done, "oracle_db_mean": round(float(np.mean(nm)), 3),
                             "gpu_db_mean": round(float(np.mean(g)), 3),
                             "median_abs_diff_db": round(float(np.median(np.abs(d))), 4),
                             "max_abs_diff_db": round(float(np.max(np.abs(d))), 4)}
    return out


def learned_section(args, test, s, K, stream):
    """Train the denoiser on the GPU, then compare learned and plain VDAMP on `test`."""
    import torch
    from paper_1911_01234_amd import synth, train as T, vdamp as V

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    tr, _, _ = synth.workload_batch256(args.train_slices, first_slice=10000)
    log(f"generated {len(tr)} training slices in {time.perf_counter() - t0:.1f} s")
    ks = (1, 2, 3, 5, 8, 12, 20, 30, 45)
    with torch.cuda.stream(stream):
        plan = V.Plan([256] * len(tr), [256] * len(tr), s)
        ws = plan.workspace()
        y, mask, p, sigma2 = V.to_device(plan, tr)
        cnn = V.Cnn(plan.nbands)
        cnn.set_params(torch.from_numpy(T.init_flat(plan.nbands, 0)).cuda(), stream=stream)
        s0 = T.input_scales(plan, cnn, ws, y, mask, p, sigma2, stream=stream)
        pairs = T.make_pairs(plan, ws, y, mask, p, sigma2, ks, stream=stream)
        x0 = torch.from_numpy(plan.pack([sl.x0 for sl in tr], np.complex64)).cuda()
        del ws, y, mask, p, sigma2
        stream.synchronize()
        log(f"{len(pairs) * len(tr)} training pairs ready; training {args.train_steps} steps")
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        losses = T.train(cnn, plan, pairs, s0, x0, args.train_steps, 1e-3, stream=stream, lr_final=1e-4)
        e1.record(stream)
        stream.synchronize()
        train_ms = e0.elapsed_time(e1)
        del pairs, x0, plan
        torch.cuda.empty_cache()

        B = len(test)
        plan = V.Plan([256] * B, [256] * B, s, V.VDAMP_FLAG_TIMING)
        ws = plan.workspace()
        cws = cnn.workspace(plan, V.VDAMP_CNN_WS_SOLVE)
        y, mask, p, sigma2 = V.to_device(plan, test)
        x0 = torch.from_numpy(plan.pack([sl.x0 for sl in test], np.complex64)).cuda()
        seg = torch.from_numpy(np.repeat(np.arange(B), 65536)).cuda()
        xh = torch.empty(plan.ntot, dtype=torch.complex64, device="cuda")

        def plain(k):
            plan.vdamp_solve(ws, y, mask, p, sigma2, k, xh, stream=stream)

        def learn(k):
            plan.vdamp_solve_learned(cnn, ws, cws, y, mask, p, sigma2, k, 7, xh, stream=stream)

        def nmse():
            stream.synchronize()
            return float(nmse_db_batch(xh, x0, seg, B).mean())

        def timed(fn, k, reps=3):
            fn(k)
            stream.synchronize()
            plan.vdamp_pass_times()
            t = time.perf_counter()
            for _ in range(reps):
                fn(k)
            stream.synchronize()
            dt = (time.perf_counter() - t) / reps
            return dt, plan.vdamp_pass_times()

        plain(K)
        n_plain = nmse()
        learn(K)
        n_learn = nmse()
        sel = torch.empty(B * plan.nbands, dtype=torch.int32, device="cuda")
        cnn.learned_export(plan, cws, sel=sel, stream=stream)
        stream.synchronize()
        sel_frac = sel.view(B, plan.nbands).float().mean(0).cpu().numpy()
        t_plain, _ = timed(plain, K)
        t_learn, times = timed(learn, K)
        # learned form within the plain 50-iteration wall-clock: soft thresholding for
        # the first kp iterations and the network in the last L.  (kp, L) is chosen on a
        # separate validation batch among the schedules whose estimated cost (from the
        # measured per-iteration times) fits the budget, then measured on the test batch.
        t_pi, t_li = t_plain / K, t_learn / K
        cands = []
        for L in (1, 2, 3):
            kmax = int((t_plain - L * t_li) / t_pi)
            for kp in range(4, kmax + 1, 4):
                cands.append((kp, L))
        val, _, _ = synth.workload_batch256(32, first_slice=20000)
        vplan = V.Plan([256] * len(val), [256] * len(val), s)
        vws = vplan.workspace()
        vcws = cnn.workspace(vplan, V.VDAMP_CNN_WS_SOLVE)
        vy, vm, vp, vs2 = V.to_device(vplan, val)
        vx0 = torch.from_numpy(vplan.pack([sl.x0 for sl in val], np.complex64)).cuda()
        vseg = torch.from_numpy(np.repeat(np.arange(len(val)), 65536)).cuda()
        vx = torch.empty(vplan.ntot, dtype=torch.complex64, device="cuda")
        vbest = None
        for kp, L in cands:
            vplan.vdamp_solve_learned(cnn, vws, vcws, vy, vm, vp, vs2, kp + L, 7, vx, learned_from=kp,
                                      stream=stream)
            stream.synchronize()
            n_v = float(nmse_db_batch(vx, vx0, vseg, len(val)).mean())
            if vbest is None or n_v < vbest[0]:
                vbest = (n_v, kp, L)
        del vws, vcws, vy, vm, vp, vs2, vx0, vx, vplan
        eq = None
        if vbest is not None:
            _, kp, L = vbest

            def hyb(k, _lf=kp):
                plan.vdamp_solve_learned(cnn, ws, cws, y, mask, p, sigma2, k, 7, xh, learned_from=_lf,
                                         stream=stream)
            hyb(kp + L)
            n_h = nmse()
            t_h = timed(hyb, kp + L)[0]
            eq = {"plain_iters_first": kp, "learned_iters": L, "seconds": round(t_h, 5), "nmse_db": round(n_h, 3),
                  "chosen_on": f"{len(val)} validation slices, {len(cands)} schedules within the budget"}
        k_eq = max(1, min(K, int(t_plain / t_li)))
        learn(k_eq)
        n_learn_eq = nmse()
        # time to reach the plain 50-iteration NMSE
        k_hit = None
        for k in range(1, K + 1):
            learn(k)
            if nmse() <= n_plain:
                k_hit = k
                break
        t_hit = timed(learn, k_hit)[0] if k_hit else None
        kp_hit = K
        for k in range(1, K + 1):
            plain(k)
            if nmse() <= n_plain + 1e-9:
                kp_hit = k
                break
        tp_hit = timed(plain, kp_hit)[0]
    cnn_ms, cnn_launch = times["cnn"]
    reps = 3
    flop = 2 * CNN_FLOP_PER_PX * plan.ntot  # forward + JVP per learned iteration
    cnn_bytes = CNN_BYTES_PER_PX * plan.ntot
    per_iter_s = cnn_ms / 1e3 / (reps * K)
    ach = flop / per_iter_s / 1e12
    out = {
        "train": {"slices": len(tr), "pairs": len(tr) * len(ks), "iteration_counts": list(ks),
                  "steps": args.train_steps, "seconds": round(train_ms / 1e3, 3),
                  "loss_first": float(np.mean(losses[:len(ks)])), "loss_last": float(np.mean(losses[-len(ks):]))},
        "test_slices": B,
        "nmse_db_at_50": {"plain": round(n_plain, 3), "learned": round(n_learn, 3)},
        "seconds_50_iters": {"plain": round(t_plain, 5), "learned": round(t_learn, 5)},
        "equal_wallclock": {"plain_seconds": round(t_plain, 5), "plain_nmse_db": round(n_plain, 3),
                            "learned_every_iteration": {"iters": k_eq, "nmse_db": round(n_learn_eq, 3)},
                            "learned_last_iterations": eq,
                            "gain_db": round(n_plain - eq["nmse_db"], 3) if eq else None},
        "time_to_plain50_nmse": {"target_db": round(n_plain, 3),
                                 "plain": {"iters": kp_hit, "seconds": round(tp_hit, 5)},
                                 "learned": {"iters": k_hit, "seconds": round(t_hit, 5) if t_hit else None}},
        "learned_band_fraction_last_iter": [round(float(v), 3) for v in sel_frac],
        "pass_ms_per_learned_solve": {k: round(v[0] / reps, 3) for k, v in times.items()},
        # the binding roofline of the network pass: HBM (its bytes at 8 TB/s take longer
        # than its FLOPs at the dense BF16 peak); the MFMA rate is reported beside it
        "cnn_roofline": {"bound": "hbm" if cnn_bytes / HBM_PEAK_GBS / 1e9 > flop / BF16_PEAK_TFLOPS / 1e12 else "mfma",
                         "achieved": round(cnn_bytes / per_iter_s / 1e9, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(cnn_bytes / per_iter_s / 1e9 / HBM_PEAK_GBS, 4),
                         "bytes_per_learned_iter": int(cnn_bytes),
                         "mfma": {"achieved": round(ach, 2), "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                                  "frac": round(ach / BF16_PEAK_TFLOPS, 4), "flop_per_learned_iter": int(flop)},
                         "ms_per_learned_iter": round(per_iter_s * 1e3, 3)},
    }
    log(f"learned: {json.dumps(out['nmse_db_at_50'])}, equal wall-clock {json.dumps(out['equal_wallclock'])}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--graph", action="store_true", help="time hipGraph replays instead of eager launches")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-denoiser section")
    ap.add_argument("--no-extra", action="store_true", help="skip the mixed and 512x512 batches")
    ap.add_argument("--train-slices", type=int, default=64)
    ap.add_argument("--train-steps", type=int, default=400)
    ap.add_argument("--test-slices", type=int, default=64)
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
    flags = V.VDAMP_FLAG_USE_GRAPH if args.graph else 0
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
    nmse_k = nmse_db_batch(x_hat, x0, seg, B)  # after the K-iteration solves

    # Per-kernel durations: the same K-iteration solves again, timed the same way, on a
    # plan that records a HIP event pair around every pass on the solve's stream
    # (VDAMP_FLAG_TIMING).  The events cost about 7 % of throughput, so `value` comes
    # from the run above and this run's rate is reported beside it.
    roofline = None
    pass_ms = None
    passes = None
    events_run = None
    if not args.graph:
        with torch.cuda.stream(stream):
            tplan = V.Plan(ny, nx, LEVELS, V.VDAMP_FLAG_TIMING)
            tws = tplan.workspace()
            tx = torch.empty_like(x_hat)
            for _ in range(max(1, args.warmup)):
                tplan.vdamp_solve(tws, y, mask, p, sigma2, K, tx, None, stream=stream)
            stream.synchronize()
            tplan.vdamp_pass_times()  # reset counters
            t0t = time.perf_counter()
            for _ in range(args.steps):
                tplan.vdamp_solve(tws, y, mask, p, sigma2, K, tx, None, stream=stream)
            stream.synchronize()
            dtt = time.perf_counter() - t0t
            times = tplan.vdamp_pass_times()
            same_t = bool(torch.equal(tx, x_hat))
            tplan.close()
        del tws, tx
        events_run = {"slice_iterations_per_s": round(B * K * args.steps / dtt, 1),
                      "ms_per_step": round(1e3 * dtt / args.steps, 3), "steps": args.steps,
                      "bitwise_equal_to_timed_run": same_t}
        print(f"[bench] kernel-event run: {events_run['slice_iterations_per_s']} slice-it/s", file=sys.stderr,
              flush=True)
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
        passes = pass_rooflines(times, npx, K, args.steps)

    # the same solves replayed from one hipGraph per solve (VDAMP_FLAG_USE_GRAPH): no
    # per-launch host work and no timing events; reported beside `value`
    graph = None
    if not args.graph:
        with torch.cuda.stream(stream):
            gplan = V.Plan(ny, nx, LEVELS, V.VDAMP_FLAG_USE_GRAPH)
            gws = gplan.workspace()
            gx = torch.empty_like(x_hat)
            for _ in range(max(1, args.warmup)):
                gplan.vdamp_solve(gws, y, mask, p, sigma2, K, gx, None, stream=stream)
            stream.synchronize()
            t0g = time.perf_counter()
            for _ in range(args.steps):
                gplan.vdamp_solve(gws, y, mask, p, sigma2, K, gx, None, stream=stream)
            stream.synchronize()
            dtg = time.perf_counter() - t0g
            same = bool(torch.equal(gx, x_hat))
            gplan.close()
        del gws, gx
        graph = {"slice_iterations_per_s": round(B * K * args.steps / dtg, 1),
                 "ms_per_step": round(1e3 * dtg / args.steps, 3), "bitwise_equal_to_eager": same}

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

    extra = None
    if not args.no_extra:
        extra = other_workloads(stream)

    learned = None
    if not args.no_learned:
        learned = learned_section(args, slices[:args.test_slices], s, K, stream)

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        cpu = cpu_baseline(slices, s, K, args.cpu_budget, nmse_k)

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
                   "launch": "hipGraph" if args.graph else "eager"},
        "mpx_iterations_per_s": round(value * 65536 / 1e6, 1),
        "hipgraph": graph,
        "kernel_event_run": events_run,
        "time_to_nmse": {"target_db": round(target, 3), "iters": k_hit, "seconds": round(t_nmse, 5)},
        "plan_seconds": round(t_plan, 4),
        "roofline": roofline,
        "pass_ms_per_step": {k: round(v, 4) for k, v in pass_ms.items()} if pass_ms else None,
        "passes": passes,
        "other_workloads": extra,
        "cpu_baseline": cpu,
        "learned": learned,
    }
    print(json.dumps(out), flush=True)
    plan.close()


if __name__ == "__main__":
    main()
