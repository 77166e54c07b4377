"""Benchmark of the live WDD per-frame update on one MI355X.

A step is one pass of the whole hot path over one batch of frames: decode and project
the batch onto the reduced basis, phase-weight it and add it to the spectrum (with the
Wiener filter applied per frame in the object order, the default, or at the snapshot in
the spectrum order), inverse DFT and display.  Frames are resident in HBM before the
timed region starts, and the displayed image is written to a buffer in HBM (steps
pipeline on the plan's stream); the rate with every image brought to host memory is
reported beside it.  The default workload is the largest single acquisition (512 x 512
scan, 256 x 256 uint16 detector, K = 128).  Prints one JSON line (one GPU).
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
    ap.add_argument("--workload", default="large")
    ap.add_argument("--order", default="object", choices=["spectrum", "object"],
                    help="accumulate the spectrum A (Wiener filter at snapshot) or the object spectrum D "
                         "(Wiener filter per frame)")
    ap.add_argument("--basis", default="hermite-gauss", choices=["hermite-gauss", "fourier"],
                    help="reduced Hermite-Gauss basis of K functions, or the full Fourier basis (K = N^2: "
                         "conventional WDD; detectors up to 64x64)")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16_hilo", "fp16_hilo", "bf16", "fp16"],
                    help="arithmetic of the projection's first stage (FP32 accumulation throughout)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="budget of the CPU oracle baseline (0: skip)")
    ap.add_argument("--no-profile", action="store_true", help="skip the untimed per-stage HIP event pass")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the side measurements (other Wiener order, snapshot cadence, precision, serving)")
    ap.add_argument("--display", default="deferred", choices=["deferred", "async"],
                    help="pipelined steps: each image written by the next push's first launch (deferred) or "
                         "queued at once (async)")
    ap.add_argument("--pipeline", default="auto", choices=["auto", "on", "two", "off"],
                    help="pipelined pushes (on: each batch's update in the next push's launch, beside that "
                         "push's projection; two: also the batch's x-DFT one launch ahead of its update); auto: "
                         "two stages where the plan supports them (object order, uint16 frames of 32..256 "
                         "columns in multiples of 32 and <= 256 rows, <= 128 with a reduced precision)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MB",
                    help="only run 5 plain device copies of MB megabytes (reference for HBM byte counters) and exit")
    ap.add_argument("--serving", action="store_true", help="run the Poisson-paced serving mix instead")
    ap.add_argument("--serving-acquisitions", type=int, default=24)
    ap.add_argument("--serving-budget-mb", type=int, default=1024)
    ap.add_argument("--serving-precision", default="bf16_hilo")
    ap.add_argument("--serving-order", default="object", choices=["spectrum", "object"])
    ap.add_argument("--serving-saturate", action="store_true", help="submit frames as fast as possible")
    ap.add_argument("--serving-mode", default="grouped", choices=["streams", "grouped", "graph"],
                    help="server launch mode: per-acquisition streams, grouped rounds, grouped rounds from a HIP graph")
    ap.add_argument("--serving-limit-s", type=float, default=150.0)
    ap.add_argument("--pool-batches", type=int, default=4,
                    help="distinct batches generated (steps cycle through them; the work per step does not "
                         "depend on the frame values)")
    return ap.parse_args()


def workload_label(wl, n_freq, k, fourier=False):
    kind = "uint16 Poisson %.0e e/frame" % wl.dose if wl.dose else "float32 noiseless"
    basis = (f"full Fourier basis K={k} (conventional WDD)" if fourier else f"K={k} Hermite-Gauss functions")
    return (f"{wl.name}: {wl.sy}x{wl.sx} raster scan, {wl.n}x{wl.n} detector ({kind}), aperture radius "
            f"{wl.radius:g} px, {basis}, {n_freq} kept frequencies, "
            f"batches of {wl.batch} in raster order, snapshot after every batch")


def _kernels_sha():
    import hashlib
    src = os.path.join(ROOT, "paper_2212_01309_amd", "csrc", "kernels.hip")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def profile_record(kind, workload, kernel):
    """A machine-readable line `<kind>: workload=.. kernel=.. ... kernels_sha=..` from the
    rocprofv3 summaries under profiles/, valid only while kernels.hip is unchanged."""
    digest = _kernels_sha()
    pdir = os.path.join(ROOT, "profiles")
    for name in sorted(os.listdir(pdir)) if os.path.isdir(pdir) else []:
        for line in open(os.path.join(pdir, name)):
            if line.startswith(kind + ":"):
                f = dict(kv.split("=", 1) for kv in line.split()[1:])
                if f.get("workload") == workload and f.get("kernel") == kernel and f.get("kernels_sha") == digest:
                    f["file"] = "profiles/" + name
                    return f
    return None


def roofline(wl, n_freq, k, order, fourier, precision, event_us, display_bytes=0.0, pipelined=False, rec=None):
    """Roofline entry of the accumulation kernel (the method's O(S^2 L^2) term and the
    largest kernel of every workload's kernel trace): algorithmic bytes per launch over the
    kernel's average duration from the rocprofv3 kernel trace recorded under profiles/ for
    this kernel source (the launches of the timed steps), with the live HIP-event mean from
    the untimed stage pass beside it (events include the launch's dispatch latency).
    display_bytes: the previous image's column pass when it rides in this launch (partial
    rows read, image written).  pipelined: the launch also projects the next batch (frames
    read, h written): k_row_fused_obj_next."""
    if fourier:
        nbytes = (8.0 if order == "object" else 24.0) * n_freq * k
        kernel = "k_update_c<%d>" % (0 if order == "object" else 2)
        rule = ("8" if order == "object" else "24") + " * n_freq * K"
    elif order == "object":
        # stream W once per row pass (D, the projections and the twiddles are a few hundred kB)
        nbytes, kernel = 8.0 * n_freq * k + display_bytes, "k_row_fused_obj"
        rule = "8 * n_freq * K (W read once)" + (" + 8 * Sy * Sx * (slots + 1) (the previous image's column "
                                                 "pass in the same launch)" if display_bytes else "")
        if pipelined:
            nbytes += (2.0 if wl.dose else 4.0) * wl.n * wl.n * wl.batch + 4.0 * k * wl.batch
            if pipelined == 2:   # as recorded: precision, and frames of more than 128 rows
                kernel = "k_row_fused_obj_next2<%d,%s>" % (PRECISION_CODES[precision],
                                                         "true" if wl.n > 128 else "false")
            else:
                kernel = "k_row_fused_obj_next<%d>" % PRECISION_CODES[precision]
            rule += " + frames + 4 * K * batch (the next batch's projection in the same launch)"
    else:
        # read and write A, read W (the Wiener reduction fused in before a snapshot)
        nbytes, kernel = 24.0 * n_freq * k, "k_row_update<true>"
        rule = "24 * n_freq * K (A read and written, W read)"
    rec = rec or wl.name + ("" if order == "object" else "_spectrum")
    trace = profile_record("kernel_trace", rec, kernel)
    if trace is not None:
        us, source = float(trace["avg_us"]), f"rocprofv3 kernel trace, {trace['file']}"
    else:
        us, source = event_us, "HIP events (untimed stage pass; no kernel trace recorded for this kernel source)"
    ach = nbytes / (us * 1e-6) / 1e9
    traffic = profile_record("traffic", rec, kernel)
    return {"kernel": kernel, "bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": ach / PEAK_HBM_GBS, "traffic": float(traffic["bytes_per_launch"]) if traffic else None,
            "avg_us": us, "avg_us_source": source, "hip_event_us": event_us, "algorithmic_bytes": nbytes,
            "algorithmic_bytes_rule": rule}


def projection_roofline(wl, k, order, display_bytes=0.0, rec=None):
    """The projection kernel against HBM: frame bytes + h written per launch (+ the previous
    image's column pass when it rides in the same launch), over the kernel-trace average
    recorded for this source (None without one)."""
    kernel = ("k_project_display" if display_bytes else "k_project") + (
        "<unsignedshort,0>" if wl.dose else "<float,0>")  # as recorded: no spaces
    trace = profile_record("kernel_trace", rec or wl.name + ("" if order == "object" else "_spectrum"), kernel)
    if trace is None:
        return None
    nbytes = (2.0 if wl.dose else 4.0) * wl.n * wl.n * wl.batch + 4.0 * k * wl.batch + display_bytes
    us = float(trace["avg_us"])
    return {"kernel": kernel, "bound": "hbm", "achieved": nbytes / (us * 1e-6) / 1e9, "peak": PEAK_HBM_GBS,
            "unit": "GB/s", "frac": nbytes / (us * 1e-6) / 1e9 / PEAK_HBM_GBS, "avg_us": us,
            "avg_us_source": f"rocprofv3 kernel trace, {trace['file']}", "algorithmic_bytes": nbytes,
            "algorithmic_bytes_rule": "frames + 4 * K * batch (h)" + (
                " + 8 * Sy * Sx * (slots + 1) (the previous image's column pass)" if display_bytes else "")}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, frames, pos, seconds, fourier=False):
    """The FP64 oracle's live path on the host cores, for the same step (push one batch,
    then snapshot).  The oracle's per-step work is linear in the number of kept frequencies
    except for the projection and the display's inverse FFT, so on workloads with many
    frequencies its plan is built on a random sample of them and the frequency-dependent
    part scaled by n_freq / sample: each part is timed with the oracle's own functions."""
    import oracle.wdd as O
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        threads = None
    cores = len(os.sched_getaffinity(0))
    all_f = O.nonzero_frequencies(wl.sy, wl.sx, wl.n, wl.n, wl.radius, wl.step)
    n_freq = len(all_f)
    sample = min(n_freq, 2048)
    rng = np.random.default_rng(5)
    pick = np.sort(rng.choice(n_freq, size=sample, replace=False)) if sample < n_freq else np.arange(n_freq)
    t0 = time.perf_counter()
    plan = O.make_plan(wl.sy, wl.sx, wl.n, wl.n, wl.radius, None if fourier else wl.k,
                       amplitude=wl.aperture_amplitude(), defocus_edge=wl.defocus_edge, step=wl.step,
                       phi=O.fourier_basis(wl.n, wl.n) if fourier else None, freqs=all_f[pick])
    plan_s = time.perf_counter() - t0
    scale = n_freq / sample
    nb = len(pos) // wl.batch

    def one_run(budget):
        live = O.Live(plan, "N")
        t_proj = t_push = t_extract = t_snap = 0.0
        steps = 0
        t_start = time.perf_counter()
        while True:
            b = (steps % nb) * wl.batch
            fr, ps = frames[b:b + wl.batch], pos[b:b + wl.batch]
            t = time.perf_counter()
            O.project(fr, plan.phi)
            t_proj += time.perf_counter() - t
            t = time.perf_counter()
            live.push(fr, ps)                      # projection + phases + accumulation
            t_push += time.perf_counter() - t
            t = time.perf_counter()
            live.spectrum()                        # the Wiener reduction
            t_extract += time.perf_counter() - t
            t = time.perf_counter()
            live.snapshot()                        # reduction + scatter + inverse FFT + normalisation
            t_snap += time.perf_counter() - t
            steps += 1
            if time.perf_counter() - t_start >= budget:
                break
        # full-size step: projection + scaled accumulation + scaled reduction + display
        step_s = (t_proj + (t_push - t_proj) * scale + t_extract * scale + (t_snap - t_extract)) / steps
        return wl.batch / step_s, steps

    runs = [one_run(seconds / 3) for _ in range(3)]
    vals = sorted(r[0] for r in runs)
    out = {"value": vals[1], "unit": "frames/s", "cores": cores, "kind": "oracle",
           "sample": (f"median of 3 runs of ~{seconds / 3:.0f} s ({', '.join(str(r[1]) for r in runs)} steps of "
                      f"{wl.batch} frames: push, then snapshot) on the same workload, FP64 NumPy; plan on "
                      f"{sample} of {n_freq} kept frequencies, frequency-dependent time scaled by "
                      f"{scale:.2f}; plan build {plan_s:.1f} s excluded"),
           "runs": vals, "blas_threads": threads, "cpu_model": cpu_model()}
    try:  # the same on one thread, one short run
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            out["value_1_thread"] = one_run(seconds / 6)[0]
    except ImportError:
        pass
    return out


PRECISION_CODES = {"fp32": 0, "bf16_hilo": 1, "fp16_hilo": 2, "bf16": 3, "fp16": 4}  # wdd_precision


# Pipeline stages of --pipeline auto: two.  With the longer chunks of two-stage plans the second
# stage measured faster than one on every workload here (per step: large 35.5 against 35.6 us,
# medium 11.0 against 12.1 us, defocus 13.1 against 13.5 us).
AUTO_STAGES = 2


def pipeline_supported(wl, order, precision, fourier):
    pow2 = (wl.sy & (wl.sy - 1)) == 0 and (wl.sx & (wl.sx - 1)) == 0
    return (order == "object" and not fourier and bool(wl.dose) and wl.n % 32 == 0 and pow2 and wl.sy <= 1024
            and 32 <= wl.n <= (256 if precision == "fp32" else 128))


def make_plan(wdd, wl, order, precision="fp32", fourier=False, max_batch=None, pipeline=False):
    return wdd.Plan(wl.radius, wl.sy, wl.sx, wl.n, wl.n, wl.n * wl.n if fourier else wl.k,
                    dtype=wdd.WDD_U16 if wl.dose else wdd.WDD_F32, defocus=wl.defocus_edge,
                    amplitude=wl.aperture_amplitude(), step=wl.step, max_batch=max_batch or wl.batch,
                    precision=precision,
                    order=wdd.WDD_ORDER_OBJECT if order == "object" else wdd.WDD_ORDER_SPECTRUM,
                    basis=wdd.WDD_BASIS_FOURIER if fourier else wdd.WDD_BASIS_HERMITE_GAUSS, pipeline=pipeline)


def run_steps(plan, batches, shown, first, count, defer, snapshot_every=1):
    """`count` pipelined steps from step number `first`; returns the host time spent issuing."""
    nb = len(batches)
    issue = 0.0
    for i in range(first, first + count):
        fr, ps = batches[i % nb]
        t = time.perf_counter()
        if (i + 1) % snapshot_every == 0:
            plan.push_snapshot(fr, ps, out=shown, wait=False, defer=defer)
        else:
            plan.push(fr, ps)
        issue += time.perf_counter() - t
    return issue


def timed(torch, plan, batches, shown, warmup, steps, defer, snapshot_every=1):
    run_steps(plan, batches, shown, 0, warmup, defer, snapshot_every)
    plan.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    issue = run_steps(plan, batches, shown, warmup, steps, defer, snapshot_every)
    plan.sync()
    torch.cuda.synchronize()
    return time.perf_counter() - t0, issue


DEVICE_FRAME_BYTES = 1 << 30   # frames held in HBM for the timed steps: 4x the 256 MB last-level cache


def load_batches(torch, wl, pool_batches):
    """Frames of `pool_batches` batches generated on the host, copied into HBM as many times
    as it takes to fill DEVICE_FRAME_BYTES (at most the whole acquisition), so that steps read
    frames from HBM rather than from the last-level cache; a step's positions walk the whole
    raster."""
    import synth
    total = (wl.sy * wl.sx) // wl.batch
    nb = max(1, min(pool_batches, total))
    pos_all = synth.raster_positions(wl.sy, wl.sx)
    pos = pos_all[:nb * wl.batch]
    t0 = time.perf_counter()
    frames = wl.frames(pos)
    gen_s = time.perf_counter() - t0
    host = frames.view(np.int16) if frames.dtype == np.uint16 else frames
    pool = torch.from_numpy(host).to("cuda")
    batch_bytes = host[:wl.batch].nbytes
    ndev = max(nb, min(total, -(-DEVICE_FRAME_BYTES // batch_bytes)))
    reps = -(-ndev // nb)
    dev = pool.repeat((reps,) + (1,) * (pool.dim() - 1))[:ndev * wl.batch].contiguous()
    del pool
    torch.cuda.synchronize()
    batches = [(dev[(i % ndev) * wl.batch:((i % ndev) + 1) * wl.batch], pos_all[i * wl.batch:(i + 1) * wl.batch])
               for i in range(total)]
    return frames, pos, batches, gen_s


def precision_lines(torch, wdd, synth, steps, warmup):
    """The reduced-precision projections beside FP32 on the precision workload (256 x 256
    scan, 128 x 128 uint16 detector with a defocused probe, K = 64), same steps."""
    wl = synth.WORKLOADS["defocus"]
    _, _, batches, _ = load_batches(torch, wl, 4)
    shown = torch.empty((wl.sy, wl.sx), dtype=torch.complex64, device="cuda")
    out = {"workload": "defocus: 256x256 scan, 128x128 uint16 detector (1e3 e/frame, pi rad defocus at the rim), "
                       "K=64, 51167 kept frequencies, object order, batches of 256, snapshot after every batch, "
                       "two pipeline stages",
           "steps": steps}
    for prec in ("fp32", "bf16_hilo", "fp16_hilo"):
        with make_plan(wdd, wl, "object", prec,
                       pipeline=AUTO_STAGES if pipeline_supported(wl, "object", prec, False) else 0) as plan:
            el, _ = timed(torch, plan, batches, shown, warmup, steps, True)
        out[prec] = {"frames_per_s": steps * wl.batch / el, "us_per_step": el / steps * 1e6}
    return out


def serving_line(torch, wdd, synth, limit_s=20.0):
    """A short serving mix beside the single acquisition, under each launch mode of the
    server: 8 acquisitions of different scan and detector sizes, every frame available at
    the start (saturated), BF16 hi+lo projection, object order, 1 GiB budget; aggregate
    frames/s and submit-to-snapshot latency."""
    rng = np.random.default_rng(7)
    pools = {}
    for n in (64, 128, 256):
        radius = n / 4 if n <= 128 else 48.0
        wl = synth.Workload(f"pool{n}", 32, 32, n, radius, 64, 256, 2 * n, 30, (1.0, 3.0), (0.2, 0.5), 5e3, seed=n)
        fr = wl.frames(synth.raster_positions(8, 32))               # 256 frames per detector size
        pools[n] = torch.from_numpy(fr.view(np.int16)).to("cuda")
    torch.cuda.synchronize()
    out = {"workload": "8 acquisitions, scans 64^2..256^2, detectors 64^2..256^2, all frames available at t=0, "
                       "deliveries of 1-512 frames, bf16 hi+lo projection, object order, snapshot every >= 1 ms; "
                       "plans made before the timed region, one untimed pass first"}
    serving_mode(torch, wdd, synth, pools, np.random.default_rng(7), "grouped", limit_s)  # warm-up
    for mode in ("streams", "grouped", "graph"):
        out[mode] = serving_mode(torch, wdd, synth, pools, np.random.default_rng(7), mode, limit_s)
    return out


def serving_mode(torch, wdd, synth, pools, rng, mode, limit_s):
    geoms = [(64, 64), (128, 64), (128, 128), (256, 128), (128, 256), (256, 64), (64, 256), (256, 256)]
    srv = wdd.Server(hbm_budget_bytes=1 << 30, snapshot_interval_us=1000.0, batch_frames=512, launch_mode=mode)
    todo = []
    for s, n in geoms:
        aid = srv.open(n / 4 if n <= 128 else 48.0, s, s, n, n, 64 if n <= 128 else 128, precision="bf16_hilo",
                       order=wdd.WDD_ORDER_OBJECT)
        todo.append(dict(id=aid, s=s, n=n, sent=0, total=s * s, pos=synth.raster_positions(s, s)))
    for a in todo:
        if a["id"] is not None:
            srv.wait_open(a["id"])
    t0 = time.perf_counter()
    while todo and time.perf_counter() - t0 < limit_s:
        for a in list(todo):
            if a["id"] is None:
                todo.remove(a)
                continue
            nb = int(rng.integers(1, 513))
            nb = min(nb, a["total"] - a["sent"], 256 - a["sent"] % 256)
            if nb > 0:
                srv.submit(a["id"], pools[a["n"]][a["sent"] % 256:a["sent"] % 256 + nb],
                           a["pos"][a["sent"]:a["sent"] + nb])
                a["sent"] += nb
        srv.step()
        for a in list(todo):  # the last snapshot once the server has pushed all of its frames
            if a["id"] is not None and a["sent"] >= a["total"] and srv.state(a["id"]) == (True, 0):
                srv.snapshot(a["id"])
                srv.close(a["id"])
                todo.remove(a)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = srv.stats()
    srv.destroy()
    return {"frames_per_s": st["frames"] / wall, "frames": st["frames"], "wall_s": wall,
            "grouped_rounds": st["group_rounds"], "graph_replays": st["graph_replays"],
            "latency_ms": {"p50": st["latency_p50_us"] / 1e3, "p99": st["latency_p99_us"] / 1e3}}


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
    srv = wdd.Server(hbm_budget_bytes=args.serving_budget_mb << 20, snapshot_interval_us=1000.0, batch_frames=512,
                     launch_mode=args.serving_mode)
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
            a["id"], a["t_open"] = aid, t
            active.append(waiting.pop(0))
        for a in list(active):
            if a["t_start"] is None:
                # the scan starts streaming once the acquisition's plan is made (on the server's
                # worker thread; the time from open to ready is reported separately)
                if not srv.state(a["id"])[0]:
                    continue
                a["t_start"] = t
            due = a["total"] if args.serving_saturate else min(a["total"], int((t - a["t_start"]) * a["rate"]))
            while a["sent"] < a["total"] and a["sent"] + min(a["next_chunk"], a["total"] - a["sent"]) <= due:
                nb = min(a["next_chunk"], a["total"] - a["sent"])
                pool = pools[a["n"]]
                off = a["sent"] % len(pool)
                nb = min(nb, len(pool) - off)                        # a delivery does not wrap the pool
                srv.submit(a["id"], pool[off:off + nb], a["pos"][a["sent"]:a["sent"] + nb])
                a["sent"] += nb
                a["next_chunk"] = int(rng.integers(1, 513))
        srv.step()
        for a in list(active):  # the last snapshot once the server has pushed all of its frames
            if a["sent"] >= a["total"] and srv.state(a["id"]) == (True, 0):
                srv.snapshot(a["id"])
                srv.close(a["id"])
                a["t_end"] = time.perf_counter() - t0
                active.remove(a)
                done.append(a)
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
    ready_ms = [1e3 * (a["t_start"] - a["t_open"]) for a in acqs if a.get("t_start") is not None and "t_open" in a]
    out = {
        "metric": "serving mix: aggregate frames/s and frame-to-snapshot latency",
        "value": st["frames"] / wall, "unit": "frames/s", "n_gpus": 1, "higher_is_better": True,
        "dtype": f"{args.serving_precision} projection, f32 accumulate", "data": "synthetic",
        "config": {"workload": f"{n_acq} acquisitions, {'arriving together' if args.serving_saturate else 'Poisson arrivals (mean 2/s)'}, scans 64^2..512^2, detectors "
                               f"64^2..256^2, {'all frames available at t=0' if args.serving_saturate else '10k-50k frames/s each'}, "
                               f"deliveries of 1-512 frames, HBM budget {args.serving_budget_mb} MiB, "
                               f"snapshot every >= 1 ms per acquisition",
                   "wiener_order": args.serving_order, "launch_mode": args.serving_mode,
                   "open_to_ready_ms": {"p50": float(np.percentile(ready_ms, 50)) if ready_ms else None,
                                        "max": float(max(ready_ms)) if ready_ms else None,
                                        "definition": "wdd_server_open returned to the plan ready (tables, "
                                                      "allocations and W upload on the server's worker thread)"},
                   "acquisitions_done": len(done), "deferred_admissions": deferred,
                   "offered_frames_per_s_sum_of_rates": offered},
        "frames": st["frames"], "wall_s": wall, "batches": st["batches"], "snapshots": st["snapshots"],
        "grouped_rounds": st["group_rounds"], "graph_replays": st["graph_replays"],
        "latency_ms": {"p50": st["latency_p50_us"] / 1e3, "p99": st["latency_p99_us"] / 1e3,
                       "max": st["latency_max_us"] / 1e3},
    }
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: --gpus {args.gpus} is not supported (sharding the update "
              f"over several GPUs is not built).", file=sys.stderr)
        sys.exit(2)
    if args.serving:
        serving(args)
        return
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
    fourier = args.basis == "fourier"
    frames, pos, batches, gen_s = load_batches(torch, wl, args.pool_batches)
    shown = torch.empty((wl.sy, wl.sx), dtype=torch.complex64, device="cuda")
    defer = args.display == "deferred"
    can_pipe = pipeline_supported(wl, args.order, args.precision, fourier)
    if args.pipeline in ("on", "two") and not can_pipe:
        sys.exit(f"--pipeline {args.pipeline}: this workload / order / precision has no pipelined form")
    chosen = AUTO_STAGES if can_pipe else 0   # the form --pipeline auto takes
    pipe_stages = {"off": 0, "on": 1, "two": 2}.get(args.pipeline, chosen)
    plan = make_plan(wdd, wl, args.order, args.precision, fourier, pipeline=pipe_stages)
    pipelined = pipe_stages > 0
    n_freq, k = plan.n_freq, plan.k
    plan_info = plan.info()

    stages = None
    if not args.no_profile:
        # untimed pass over every stage with HIP events on the plan stream (each timed launch
        # costs two event records, so none are recorded in the timed region)
        plan.profile_enable(wdd.STAGE_ALL)
        run_steps(plan, batches, shown, 0, max(20, min(args.warmup, 100)), defer)
        pre = plan.profile_read()
        plan.profile_enable(0)
        stages = {s: (pre[f"{s}_ms"] / pre[f"{s}_launches"] * 1e3 if pre[f"{s}_launches"] else 0.0)
                  for s in ("project", "rowdft", "accumulate", "wiener", "display")}

    elapsed, issue = timed(torch, plan, batches, shown, args.warmup, args.steps, defer)

    # untimed: latency from a push's call to its image ready in host memory (blocking push +
    # snapshot into the plan's pinned buffer), the rate with every image brought to the host,
    # and frames streamed from host memory instead (staged through pinned memory over PCIe)
    nlat = max(100, min(args.steps, 500))
    pinned = plan.snapshot_buffer()
    lat = np.empty(nlat)
    for i in range(nlat):
        fr, ps = batches[i % len(batches)]
        t = time.perf_counter()
        plan.push_snapshot(fr, ps, out=pinned)
        lat[i] = time.perf_counter() - t
    host_fps = nlat * wl.batch / lat.sum()
    nb = len(frames) // wl.batch
    host_frames = [frames[i * wl.batch:(i + 1) * wl.batch] for i in range(nb)]
    plan.sync()
    t = time.perf_counter()
    for i in range(nlat):
        plan.push_snapshot(host_frames[i % nb], batches[i % len(batches)][1], out=shown, wait=False)
    plan.sync()
    host_frames_fps = nlat * wl.batch / (time.perf_counter() - t)
    extras = {}
    if not args.no_extras and wl.snapshot_every:
        # the configuration's own snapshot cadence (every snapshot_every frames)
        every = max(1, wl.snapshot_every // wl.batch)
        el, _ = timed(torch, plan, batches, shown, args.warmup, max(args.steps, 2 * every), defer, every)
        steps_c = max(args.steps, 2 * every)
        extras["snapshot_every_%d_frames" % wl.snapshot_every] = {
            "frames_per_s": steps_c * wl.batch / el, "us_per_batch": el / steps_c * 1e6, "steps": steps_c}
    plan.close()

    if not args.no_extras and can_pipe:
        # the same steps with the other push form (pipelined or not)
        with make_plan(wdd, wl, args.order, args.precision, fourier, pipeline=0 if pipelined else AUTO_STAGES) as p2:
            el, _ = timed(torch, p2, batches, shown, args.warmup, args.steps, defer)
        extras["unpipelined" if pipelined else "pipelined"] = {
            "frames_per_s": args.steps * wl.batch / el, "us_per_step": el / args.steps * 1e6}
        if pipelined:  # and with the other number of pipeline stages
            other = 3 - pipe_stages
            with make_plan(wdd, wl, args.order, args.precision, fourier, pipeline=other) as p2:
                el, _ = timed(torch, p2, batches, shown, args.warmup, args.steps, defer)
            extras["pipeline_stages_%d" % other] = {
                "frames_per_s": args.steps * wl.batch / el, "us_per_step": el / args.steps * 1e6}

    if not args.no_extras and not fourier:
        other = "spectrum" if args.order == "object" else "object"
        with make_plan(wdd, wl, other, args.precision) as p2:
            el, _ = timed(torch, p2, batches, shown, args.warmup, args.steps, defer)
        extras[f"{other}_order"] = {"frames_per_s": args.steps * wl.batch / el, "us_per_step": el / args.steps * 1e6,
                                    "note": ("A resident in HBM, Wiener filter at each snapshot (the sufficient "
                                             "statistic kept)" if other == "spectrum" else
                                             "Wiener filter per frame, D accumulated")}

    fps = args.steps * wl.batch / elapsed
    out = {
        "metric": METRIC, "value": fps, "unit": "frames/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else f"{args.precision} projection, f32 accumulate",
        "data": "synthetic",
        "config": {"workload": workload_label(wl, n_freq, k, fourier), "scan": [wl.sy, wl.sx], "detector": [wl.n, wl.n],
                   "batch": wl.batch, "k": k, "n_freq": n_freq, "frames_dtype": str(frames.dtype),
                   "wiener_order": args.order, "basis": args.basis, "pipelined": pipelined,
                   "pipeline_stages": pipe_stages,
                   "display": "hbm" + ((", each batch's x-DFT in the next push's launch and its update in the "
                                        "one after (beside those pushes' projections), each image's last pass in "
                                        "the launch after that" if pipe_stages == 2 else
                                        ", each batch's update in the next push's launch (with that push's "
                                        "projection), each image's last pass in the launch after" if pipelined else
                                        ", each image's last pass deferred to the next push's first launch "
                                        "(its projection for detectors of <= 128 rows, else its first update; "
                                        "Hermite-Gauss basis, power-of-two scan width)") if defer else "")},
        "host_issue_us_per_step": issue / args.steps * 1e6,
        "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3), "p99": float(np.percentile(lat, 99) * 1e3),
                       "samples": nlat, "definition": "wdd_push_snapshot call to the image complete in host memory"},
        "host_display_fps": host_fps,
        "host_frames_fps": host_frames_fps,
    }
    if stages is not None:
        out["stages_us_hip_events"] = stages
        # where the deferred column pass of each image rides (see the plan's can_defer rules)
        info = plan_info
        pow2x = (wl.sx & (wl.sx - 1)) == 0
        slots = info.display_slots if args.order == "object" and info.display_slots else 1
        disp = 8.0 * wl.sy * wl.sx * (slots + 1)
        in_update = (defer and not fourier and args.order == "object" and (wl.n > 128 or pipelined)
                     and info.display_slots > 0)
        in_proj = defer and not fourier and wl.n <= 128 and pow2x and not pipelined
        # records of the profiles: per workload and order, unpipelined runs of pipelinable ones apart
        rec = wl.name + ("_spectrum" if args.order == "spectrum" else "_unpipelined" if can_pipe and not pipelined
                         else "_stages%d" % pipe_stages if pipelined and pipe_stages != chosen else "")
        out["roofline"] = roofline(wl, n_freq, k, args.order, fourier, args.precision, stages["accumulate"],
                                   disp if in_update else 0.0, pipe_stages, rec)
        # (pipelined: the projection has no launch of its own in the timed steps)
        proj = (None if fourier or args.precision != "fp32" or pipelined
                else projection_roofline(wl, k, args.order, disp if in_proj else 0.0, rec))
        if proj is not None:
            out["roofline_projection"] = proj
    out.update(extras)
    if not args.no_extras and args.workload == "large" and not fourier:
        out["precision_variants"] = precision_lines(torch, wdd, synth, max(args.steps, 500), args.warmup)
        out["serving"] = serving_line(torch, wdd, synth)
    if args.cpu_seconds > 0:
        out["cpu_baseline"] = cpu_baseline(wl, frames, pos, args.cpu_seconds, fourier)
    out["generation_s"] = gen_s
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
