"""Benchmark of the live WDD per-frame update on one MI355X.

A step is one pass of the whole hot path over one batch of frames: decode and
project the batch onto the reduced basis, phase-weight and accumulate it into
the spectrum, Wiener-reduce, inverse DFT, and copy the displayed object to the
host.  Frames are resident in HBM before the timed region starts.  Prints one
JSON line (rank 0, one GPU).
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "live-update frames/s + p99 frame-to-snapshot latency; % MFMA/HBM peak"
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="medium")
    ap.add_argument("--order", default="object", choices=["spectrum", "object"],
                    help="accumulate the spectrum A (Wiener filter at snapshot) or the object spectrum D "
                         "(Wiener filter per frame)")
    ap.add_argument("--basis", default="hermite-gauss", choices=["hermite-gauss", "fourier"],
                    help="reduced Hermite-Gauss basis of K functions, or the full Fourier basis (K = N^2: "
                         "conventional WDD; detectors up to 64x64)")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16_hilo", "fp16_hilo", "bf16", "fp16"],
                    help="arithmetic of the projection's first stage (FP32 accumulation throughout)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the CPU oracle baseline (0: skip)")
    ap.add_argument("--profile-period", type=int, default=8,
                    help="time the dominant stage with HIP events on one step in every N of the timed region")
    ap.add_argument("--no-profile", action="store_true", help="skip the per-stage HIP event timing")
    ap.add_argument("--display", default="deferred", choices=["deferred", "async"],
                    help="pipelined steps: each image written by the next push's first launch (deferred) or "
                         "queued at once (async)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MB",
                    help="only run 5 plain device copies of MB megabytes (reference for HBM byte counters) and exit")
    ap.add_argument("--serving", action="store_true", help="run the serving mix instead of the single acquisition")
    ap.add_argument("--serving-acquisitions", type=int, default=24)
    ap.add_argument("--serving-budget-mb", type=int, default=1024)
    ap.add_argument("--serving-precision", default="bf16_hilo")
    ap.add_argument("--serving-order", default="object", choices=["spectrum", "object"])
    ap.add_argument("--serving-saturate", action="store_true", help="submit frames as fast as possible")
    ap.add_argument("--serving-limit-s", type=float, default=150.0)
    ap.add_argument("--pool-batches", type=int, default=128,
                    help="distinct batches generated (steps cycle through them); the medium workload has 128")
    return ap.parse_args()


def workload_label(wl, n_freq, k, fourier=False):
    kind = "uint16 Poisson %.0e e/frame" % wl.dose if wl.dose else "float32 noiseless"
    basis = (f"full Fourier basis K={k} (conventional WDD)" if fourier else f"K={k} Hermite-Gauss functions")
    return (f"{wl.name}: {wl.sy}x{wl.sx} raster scan, {wl.n}x{wl.n} detector ({kind}), aperture radius "
            f"{wl.radius:g} px, {basis}, {n_freq} kept frequencies, "
            f"batches of {wl.batch} in raster order, snapshot after every batch")


def measured_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` from the calibrated rocprofv3 counter passes recorded in
    profiles/hbm_traffic.md, or None when that record is missing or the kernel source has
    changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic.md")
    src = os.path.join(ROOT, "paper_2212_01309_amd", "csrc", "kernels.hip")
    if not os.path.exists(path):
        return None
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    for line in open(path):
        if line.startswith("traffic:"):
            f = dict(kv.split("=", 1) for kv in line.split()[1:])
            if f.get("workload") == workload and f.get("kernel") == kernel and f.get("kernels_sha") == digest:
                return float(f["bytes_per_launch"])
    return None


def roofline(wl, n_freq, k, dom, us, factored, fused, order="spectrum", fourier=False):
    """Roofline entry of stage `dom` (mean launch time `us`), from its algorithmic work."""
    if dom == "accumulate" and fourier:
        # one workgroup per kept frequency streams its W row (object order) or its A row
        # (read and write; W too when the Wiener reduction is fused)
        nbytes = (8.0 if order == "object" else (24.0 if fused else 16.0)) * n_freq * k
        kernel = "k_update_c<%d>" % (0 if order == "object" else (2 if fused else 1))
        bound = "hbm"
    elif dom == "accumulate" and order == "object":
        # object order: stream W once per row pass (D, the frames' projections and the
        # twiddles are a few hundred kB)
        nbytes, kernel, bound = 8.0 * n_freq * k, "k_row_fused_obj", "hbm"
    elif dom == "accumulate" and factored:
        # row-factored update: read and write A, read W when the Wiener reduction is fused
        nbytes = (24.0 if fused else 16.0) * n_freq * k
        kernel, bound = "k_row_update" + ("<true>" if fused else "<false>"), "hbm"
    elif dom == "accumulate":
        flops = 4.0 * n_freq * k * wl.batch            # complex phase x real coefficient per (v, k, frame)
        ach = flops / (us * 1e-6) / 1e12
        return {"kernel": "k_accumulate", "bound": "mfma", "achieved": ach, "peak": PEAK_FP32_MFMA_TFLOPS,
                "unit": "TFLOP/s", "frac": ach / PEAK_FP32_MFMA_TFLOPS, "traffic": None, "avg_us": us}
    elif dom == "wiener":
        nbytes, kernel, bound = 16.0 * n_freq * k, "k_wiener", "hbm"
    elif dom == "project":
        nbytes = (2.0 if wl.dose else 4.0) * wl.n * wl.n * wl.batch + 4.0 * k * wl.batch
        kernel, bound = "k_project", "hbm"
    else:
        nbytes = 3 * 8.0 * wl.sy * wl.sx
        kernel, bound = "k_dft_rows (x2)", "hbm"
    ach = nbytes / (us * 1e-6) / 1e9
    return {"kernel": kernel, "bound": bound, "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": ach / PEAK_HBM_GBS, "traffic": measured_traffic(wl.name, kernel), "avg_us": us,
            "algorithmic_bytes": nbytes}


def cpu_baseline(wl, frames, pos, seconds, fourier=False):
    """The FP64 oracle's live path (same step: push one batch, then snapshot) on the host cores."""
    import oracle.wdd as O
    try:
        from threadpoolctl import threadpool_info
        cores = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        cores = os.cpu_count() or 1
    t0 = time.perf_counter()
    plan = O.make_plan(wl.sy, wl.sx, wl.n, wl.n, wl.radius, None if fourier else wl.k,
                       amplitude=wl.aperture_amplitude(), defocus_edge=wl.defocus_edge, step=wl.step,
                       phi=O.fourier_basis(wl.n, wl.n) if fourier else None)
    plan_s = time.perf_counter() - t0

    def run(budget):
        live = O.Live(plan, "N")
        done = 0
        t0 = time.perf_counter()
        while True:
            b = (done * wl.batch) % len(pos)
            live.push(frames[b:b + wl.batch], pos[b:b + wl.batch])
            live.snapshot()
            done += 1
            el = time.perf_counter() - t0
            if el >= budget or done * wl.batch >= len(pos):
                return done, el

    done, el = run(seconds)
    out = {"value": done * wl.batch / el, "unit": "frames/s", "cores": int(cores), "kind": "oracle",
           "sample": f"{done} steps of {wl.batch} frames (push + snapshot each) of the same workload, FP64 NumPy, "
                     f"{el:.1f} s; plan build {plan_s:.1f} s excluded"}
    try:  # the same on one thread, a third of the time budget
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            d1, e1 = run(seconds / 3)
        out["value_1_thread"] = d1 * wl.batch / e1
    except ImportError:
        pass
    return out


def serving(args):
    """Serving mix: acquisitions arriving as a Poisson process, each streaming frames at its
    own rate in random delivery sizes, admitted by an HBM budget, served by one server with
    continuous batching.  Prints one JSON line."""
    import torch

    import paper_2212_01309_amd as wdd
    import synth

    rng = np.random.default_rng(2024)
    n_acq = args.serving_acquisitions
    arrivals = np.cumsum(rng.exponential(0.5, size=n_acq))          # mean 2 arrivals per second
    if args.serving_saturate:
        arrivals[:] = 0.0                                              # everything is there at once
    pools = {}
    for n in (64, 128, 256):                                          # frame pools per detector size
        radius = n / 4 if n <= 128 else 48.0
        wl = synth.Workload(f"pool{n}", 32, 32, n, radius, 64, 256, 2 * n, 30, (1.0, 3.0), (0.2, 0.5), 5e3, seed=n)
        fr = wl.frames(synth.raster_positions(16, 32))               # 512 frames
        pools[n] = torch.from_numpy(fr.view(np.int16)).to("cuda")
    torch.cuda.synchronize()
    acqs = []
    for i in range(n_acq):
        s = int(rng.choice([64, 128, 256, 512]))
        n = int(rng.choice([64, 128, 256]))
        acqs.append(dict(i=i, t_arrive=float(arrivals[i]), s=s, n=n, k=64 if n <= 128 else 128,
                         radius=n / 4 if n <= 128 else 48.0, rate=float(rng.uniform(1e4, 5e4)),
                         dose=float(rng.uniform(1e3, 1e4)), total=s * s, sent=0, id=None, t_start=None,
                         next_chunk=int(rng.integers(1, 513)), pos=synth.raster_positions(s, s)))
    srv = wdd.Server(hbm_budget_bytes=args.serving_budget_mb << 20, snapshot_interval_us=1000.0, batch_frames=512)
    waiting, active, done = list(acqs), [], []
    deferred = 0
    t0 = time.perf_counter()
    last_print = t0
    while waiting or active:
        t = time.perf_counter() - t0
        while waiting and waiting[0]["t_arrive"] <= t:
            a = waiting[0]
            aid = srv.open(a["radius"], a["s"], a["s"], a["n"], a["n"], a["k"], precision=args.serving_precision,
                           order=wdd.WDD_ORDER_OBJECT if args.serving_order == "object" else wdd.WDD_ORDER_SPECTRUM)
            if aid is None:
                if not a.get("deferred"):
                    a["deferred"] = True
                    deferred += 1
                break                                              # admitted in arrival order once memory frees
            a["id"], a["t_start"] = aid, t
            active.append(waiting.pop(0))
        for a in list(active):
            due = a["total"] if args.serving_saturate else min(a["total"], int((t - a["t_start"]) * a["rate"]))
            while a["sent"] < a["total"] and a["sent"] + min(a["next_chunk"], a["total"] - a["sent"]) <= due:
                nb = min(a["next_chunk"], a["total"] - a["sent"])
                pool = pools[a["n"]]
                off = a["sent"] % len(pool)
                nb = min(nb, len(pool) - off)                        # a delivery does not wrap the pool
                srv.submit(a["id"], pool[off:off + nb], a["pos"][a["sent"]:a["sent"] + nb])
                a["sent"] += nb
                a["next_chunk"] = int(rng.integers(1, 513))
            if a["sent"] >= a["total"]:
                srv.snapshot(a["id"])
                srv.close(a["id"])
                a["t_end"] = time.perf_counter() - t0
                active.remove(a)
                done.append(a)
        srv.step()
        if time.perf_counter() - last_print > 5.0:
            st = srv.stats()
            print(f"[serving] t={t:.1f}s open={st['open']} done={len(done)} frames={st['frames']} "
                  f"pending={st['pending_frames']}", file=sys.stderr, flush=True)
            last_print = time.perf_counter()
        if time.perf_counter() - t0 > args.serving_limit_s:
            break
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = srv.stats()
    srv.destroy()
    offered = sum(a["rate"] for a in acqs)
    out = {
        "metric": "serving mix: aggregate frames/s and frame-to-snapshot latency",
        "value": st["frames"] / wall, "unit": "frames/s", "n_gpus": 1, "higher_is_better": True,
        "dtype": f"{args.serving_precision} projection, f32 accumulate", "data": "synthetic",
        "config": {"workload": f"{n_acq} acquisitions, {'arriving together' if args.serving_saturate else 'Poisson arrivals (mean 2/s)'}, scans 64^2..512^2, detectors "
                               f"64^2..256^2, {'all frames available at t=0' if args.serving_saturate else '10k-50k frames/s each'}, "
                               f"deliveries of 1-512 frames, HBM budget {args.serving_budget_mb} MiB, "
                               f"snapshot every >= 1 ms per acquisition",
                   "wiener_order": args.serving_order,
                   "acquisitions_done": len(done), "deferred_admissions": deferred,
                   "offered_frames_per_s_sum_of_rates": offered},
        "frames": st["frames"], "wall_s": wall, "batches": st["batches"], "snapshots": st["snapshots"],
        "latency_ms": {"p50": st["latency_p50_us"] / 1e3, "p99": st["latency_p99_us"] / 1e3,
                       "max": st["latency_max_us"] / 1e3},
    }
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.serving:
        if args.gpus != 1:
            print("bench.py measures one GPU only", file=sys.stderr)
            sys.exit(2)
        serving(args)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: --gpus {args.gpus} is not supported (sharding the update "
              f"over several GPUs is not built).", file=sys.stderr)
        sys.exit(2)
    import torch

    if args.copy_calibration:
        src = torch.ones(args.copy_calibration * (1 << 20) // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": src.numel() * 4, "copies": 5}))
        return

    import paper_2212_01309_amd as wdd
    import synth

    wl = synth.WORKLOADS[args.workload]
    pos = synth.raster_positions(wl.sy, wl.sx)[:args.pool_batches * wl.batch]
    t0 = time.perf_counter()
    frames = wl.frames(pos)
    gen_s = time.perf_counter() - t0
    host = frames.view(np.int16) if frames.dtype == np.uint16 else frames
    dev = torch.from_numpy(host).to("cuda")
    torch.cuda.synchronize()
    dtype = wdd.WDD_U16 if frames.dtype == np.uint16 else wdd.WDD_F32
    fourier = args.basis == "fourier"
    plan = wdd.Plan(wl.radius, wl.sy, wl.sx, wl.n, wl.n, wl.n * wl.n if fourier else wl.k, dtype=dtype,
                    defocus=wl.defocus_edge, amplitude=wl.aperture_amplitude(), step=wl.step, max_batch=wl.batch,
                    precision=args.precision,
                    order=wdd.WDD_ORDER_OBJECT if args.order == "object" else wdd.WDD_ORDER_SPECTRUM,
                    basis=wdd.WDD_BASIS_FOURIER if fourier else wdd.WDD_BASIS_HERMITE_GAUSS)
    nb = len(pos) // wl.batch
    batches = [(dev[i * wl.batch:(i + 1) * wl.batch], pos[i * wl.batch:(i + 1) * wl.batch]) for i in range(nb)]

    # the displayed image stays in HBM (as the frames do); steps pipeline on the plan's stream
    shown = torch.empty((wl.sy, wl.sx), dtype=torch.complex64, device="cuda")

    def step(i, wait=False):
        fr, ps = batches[i % nb]
        plan.push_snapshot(fr, ps, out=shown, wait=wait, defer=not wait and args.display == "deferred")

    for i in range(args.warmup):
        step(i)
    stage_bits = {"project": wdd.STAGE_PROJECT, "rowdft": wdd.STAGE_ROWDFT, "accumulate": wdd.STAGE_ACCUMULATE,
                  "wiener": wdd.STAGE_WIENER, "display": wdd.STAGE_DISPLAY}
    stages = None
    if not args.no_profile:
        # untimed pass over every stage to find the dominant one; the timed region then brackets
        # only that stage with events (each timed launch costs two event records)
        plan.profile_enable(wdd.STAGE_ALL)
        for i in range(min(args.warmup, 100) or 20):
            step(i)
        pre = plan.profile_read()
        stages = {s: (pre[f"{s}_ms"] / pre[f"{s}_launches"] * 1e3 if pre[f"{s}_launches"] else 0.0)
                  for s in stage_bits}
        # the roofline entry is the accumulation kernel (the method's O(S^2 L^2) loop, the largest
        # kernel in the rocprofv3 summaries); the others are reported per launch beside it
        per_kernel = {s: stages[s] / (2.0 if s == "display" else 1.0) for s in stages}
        dominant = "accumulate"
        factored, fused = pre["factored_launches"] > 0, pre["wiener_launches"] == 0
        # events on one step in every `period` of the timed region (each timed launch costs two
        # event records, about 6 us of a 30 us step)
        plan.profile_period(args.profile_period)
        plan.profile_enable(stage_bits[dominant])
    plan.sync()
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        step(args.warmup + i)
    plan.sync()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    prof = plan.profile_read() if not args.no_profile else None
    if not args.no_profile:
        plan.profile_enable(0)
        plan.profile_period(1)
    # untimed: latency of one step (push to image complete in HBM), and the rate when every
    # image is also brought to the host through the plan's pinned buffer (PCIe included)
    nlat = min(args.steps, 500)
    lat = np.empty(nlat)
    for i in range(nlat):
        t = time.perf_counter()
        step(i, wait=True)
        lat[i] = time.perf_counter() - t
    pinned = plan.snapshot_buffer()
    t = time.perf_counter()
    for i in range(nlat):
        fr, ps = batches[i % nb]
        plan.push_snapshot(fr, ps, out=pinned)
    host_fps = nlat * wl.batch / (time.perf_counter() - t)
    # frames streamed from host memory instead (the library stages them through pinned
    # memory and copies them over PCIe), display kept in HBM
    host_frames = [frames[i * wl.batch:(i + 1) * wl.batch] for i in range(nb)]
    plan.sync()
    t = time.perf_counter()
    for i in range(nlat):
        plan.push_snapshot(host_frames[i % nb], batches[i % nb][1], out=shown, wait=False)
    plan.sync()
    host_frames_fps = nlat * wl.batch / (time.perf_counter() - t)
    n_freq, k = plan.n_freq, plan.k
    plan.close()

    fps = args.steps * wl.batch / elapsed
    out = {
        "metric": METRIC, "value": fps, "unit": "frames/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else f"{args.precision} projection, f32 accumulate",
        "data": "synthetic",
        "config": {"workload": workload_label(wl, n_freq, k, fourier), "scan": [wl.sy, wl.sx], "detector": [wl.n, wl.n],
                   "batch": wl.batch, "k": k, "n_freq": n_freq, "frames_dtype": str(frames.dtype),
                   "wiener_order": args.order, "basis": args.basis,
                   "display": "hbm" + (", each image's last pass deferred to the next push's projection launch "
                                       "where the plan allows it (FP32 Hermite-Gauss projection, detector rows "
                                       "<= 128, power-of-two scan width)" if args.display == "deferred" else "")},
        "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3), "p99": float(np.percentile(lat, 99) * 1e3),
                       "steps": nlat},
        "host_display_fps": host_fps,
        "host_frames_fps": host_frames_fps,
    }
    if prof is not None:
        # the dominant stage's mean launch time over the timed region replaces the pre-pass value
        stages[dominant] = prof[f"{dominant}_ms"] / max(prof[f"{dominant}_launches"], 1) * 1e3
        out["stages_us"] = stages
        out["largest_kernel_stage"] = max(per_kernel, key=per_kernel.get)
        out["roofline"] = roofline(wl, n_freq, k, dominant, stages[dominant], factored, fused, args.order, fourier)
    if args.cpu_seconds > 0:
        out["cpu_baseline"] = cpu_baseline(wl, frames, pos, args.cpu_seconds, fourier)
    out["generation_s"] = gen_s
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
