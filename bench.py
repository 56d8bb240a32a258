"""Throughput of the FGBD per-frame path on one MI355X.

One step = one fgbd_denoise call (scan-line graph + noise estimate + filter
selection and sweeps) on a synthetic 1M-point frame already resident in HBM.
Prints one JSON line with points/s, frames/s, the roofline of the dominant
kernel (per-kernel HIP event timing from a profiled pass over the same steps)
and the CPU oracle timed on the host.  Beside the headline it reports the
three usage patterns on their own workloads: a batch of 8 uneven clouds in one
call, a stream of 30 moving frames replayed from one captured HIP graph
(frames/s and p50/p99 frame latency), and forward+backward of the polynomial
filter on 4 x 500k points inside 50 Adam steps.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "points/s (SLG+noise est+filter) at 1M pts, frames/s; HBM GB/s fraction; fwd+bwd pts/s"
HBM_PEAK_GBS = 8000.0


def algorithmic_bytes(kind: str, n: int, L: int, K: int, P: int) -> float:
    """Compulsory HBM bytes per launch of each kernel kind: every array a launch
    must read or write, read or written once, neighbour gathers counted as cache
    hits.  Codes of at most 32 bits (grids up to 2^10, every workload here) sort
    with one top-digit pass and the local sorts: the upsweep and the downsweep
    read the int32 coordinates once (12 B/point for all L directions), the
    downsweep writes the 8-byte items, and the local sort reads them and writes
    the sorted items and the 4-byte rank."""
    if kind == "radix_upsweep":
        return 12 * n
    if kind == "radix_downsweep":
        return (12 + 8 * L) * n
    if kind == "local_sort":
        return (8 + 8 + 4) * L * n
    if kind == "merge":     # xyz, rank, sorted items once, col + dist2 out
        return (12 + 4 * L + 8 * L + 8 * K) * n
    if kind == "weights":   # col + dist2 in, p out
        return 12 * K * n
    if kind == "noise":     # fused per-frame path (K = P): col + dist2 in, own colour, spread, p and float4 x1 out
        return (4 * K + 12 + 8 + 4 * K + 4 * K + 16) * n
    if kind == "sweep":     # col + p, float4 x in and out
        return (8 * K + 16 + 16) * n
    if kind == "sweep_first_fused":  # float4 x1 in and out (FSLR flag added), y (12 B) and spread in
        return (16 + 16 + 12 + 8) * n
    if kind == "sweep_first_merged":  # x1, y and spread in, col + p in, float4 x2 out
        return (16 + 12 + 8 + 8 * K + 16) * n
    if kind == "finalize":  # float4 in, float32 x3 out (plus the last sweep partials)
        return (16 + 12) * n
    return 0.0


def sweep_kind_sum(sweeps: int, K: int, tail_finalises: bool, per_launch):
    """Bytes the sweep launches of one fused-path call (K = P = 8: the noise
    launch computes x_1) move for a cloud whose selection computed `sweeps`
    iterates, from per_launch(record kind) -> bytes or None.  x_1's bytes are
    the noise kind's; the first sweep launch adds x_1's flags and sums and,
    with K = 8, computes x_2 in the same launch ("sweep_first_merged"); every
    later iterate is one plain sweep (a launch of its own or a pass of the
    tail's loop); launches that find the selection stopped move nothing; the
    tail launch finalises ("sweep_tail") when no separate finalize launch ran.
    None when a needed figure is missing."""
    merged = K == 8 and sweeps >= 2
    first = per_launch("sweep_first_merged" if merged else "sweep_first_fused")
    later = max(sweeps - (2 if merged else 1), 0)
    plain = per_launch("sweep") if later else 0.0
    tail = per_launch("sweep_tail") if tail_finalises else 0.0
    if first is None or plain is None or tail is None:
        return None
    return first + later * plain + tail


def sweep_kind_bytes(n: int, sweeps: int, L: int, K: int, P: int, tail_finalises: bool) -> float:
    """Algorithmic bytes of sweep_kind_sum (the tail's are the finalize kind's)."""
    return sweep_kind_sum(sweeps, K, tail_finalises,
                          lambda k: algorithmic_bytes("finalize" if k == "sweep_tail" else k, n, L, K, P))


# Source files each kernel kind is compiled from: a traffic figure measured
# with hardware counters is only reported while these are unchanged.
KIND_SOURCES = {
    "radix_upsweep": ("fgbd_sort.hip",), "radix_scan": ("fgbd_sort.hip",), "radix_downsweep": ("fgbd_sort.hip",),
    "merge": ("fgbd_graph.hip",), "weights": ("fgbd_graph.hip",),
    "noise": ("fgbd_noise.hip",), "noise_solve": ("fgbd_noise.hip",),
    "sweep": ("fgbd_filter.hip",), "finalize": ("fgbd_filter.hip",), "relabel": ("fgbd_graph.hip",),
    "local_sort": ("fgbd_sort.hip",), "sweep_first_merged": ("fgbd_filter.hip",),
    "sweep_first": ("fgbd_filter.hip",), "sweep_tail": ("fgbd_filter.hip",),
}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_fgbd_1M_frame.md")


def source_digest(kind: str) -> str:
    import hashlib

    h = hashlib.sha256()
    for f in KIND_SOURCES[kind] + ("fgbd_internal.h",):
        with open(os.path.join(ROOT, "paper_2401_09721_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _counter_record(kind: str, config: dict):
    """The committed counter record of `kind`, or None when the summary is
    missing, was taken on another workload, or the kernel's sources changed
    since."""
    try:
        with open(TRAFFIC_FILE) as fh:
            text = fh.read()
        rec = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    except (OSError, IndexError, ValueError):
        return None
    k = rec.get("kernels", {}).get(kind)
    if not k or rec.get("config") != config or k.get("source_sha256") != source_digest(kind):
        return None
    return k


def measured_traffic(kind: str, config: dict):
    """HBM bytes per launch of `kind` from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE, each scaled by what the counter reads for a
    plain device copy), or None (see _counter_record)."""
    k = _counter_record(kind, config)
    return k["hbm_bytes_per_launch"] if k else None


# VALU issue peak: 256 compute units, each issuing one 64-lane vector
# instruction per cycle (four SIMDs, four cycles each), at 2.4 GHz.
VALU_ISSUE_PEAK = 256 * 2.4e9


def measured_valu(kind: str, config: dict, us_per_launch: float):
    """Vector instructions per launch of `kind` (SQ_INSTS_VALU, wave level) from
    the committed counter summary, and the fraction of the VALU issue peak
    they take at the measured duration; None when there is no record."""
    k = _counter_record(kind, config)
    if not k or not k.get("valu_insts"):
        return None
    insts = k["valu_insts"]
    return {"insts_per_launch": insts, "issue_peak_per_s": VALU_ISSUE_PEAK,
            "frac": insts / (us_per_launch * 1e-6) / VALU_ISSUE_PEAK}


def roofline_object(kind: str, k: dict, bytes_per_step: float, traffic, valu) -> dict:
    """The roofline of the dominant kind from its per-step time `k`
    (ms_per_step, launches_per_step, us_per_launch), its algorithmic bytes per
    step, its counter-measured HBM bytes per step (or None) and measured_valu
    (or None).  HBM view by default; when the VALU issue fraction is the
    larger, the instruction rate against the issue peak ("bound": "alu") with
    the HBM view under "hbm".  The instruction count is the counter-measured
    one (a ballot ranking has no algorithmic flop count), so that fraction
    says how busy the issue port is, not how little work the kernel does."""
    gbs = bytes_per_step / (k["ms_per_step"] / 1e3) / 1e9
    hbm = {"kernel": kind, "bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": gbs / HBM_PEAK_GBS, "traffic": traffic,
           "traffic_basis": "HBM bytes per step of the same launches as bytes_per_step",
           "bytes_per_step": bytes_per_step, "ms_per_step": k["ms_per_step"],
           "launches_per_step": k["launches_per_step"],
           "timing": "HIP events around each launch on the library's stream"}
    if valu is None or valu["frac"] <= hbm["frac"]:
        return dict(hbm, valu=valu)
    rate = valu["insts_per_launch"] / (k["us_per_launch"] * 1e-6)
    return {"kernel": kind, "bound": "alu", "achieved": rate / 1e9, "peak": VALU_ISSUE_PEAK / 1e9,
            "unit": "G wave instructions/s", "frac": rate / VALU_ISSUE_PEAK, "traffic": traffic,
            "peak_basis": "256 CUs x one 64-lane vector instruction per cycle x 2.4 GHz",
            "work": "SQ_INSTS_VALU per launch from the committed counter record",
            "insts_per_launch": valu["insts_per_launch"], "us_per_launch": k["us_per_launch"], "hbm": hbm}


def _gen(job):
    from paper_2401_09721_amd import synth

    kind, kw = job
    if kind == "body":
        return synth.body_cloud(**kw)
    return synth.moved_body_frame(**kw)  # (cloud, fitted scale)


def selected_patterns(args) -> set:
    return set() if args.no_patterns else {p.strip() for p in args.patterns.split(",") if p.strip()}


def make_inputs(args, synth) -> dict:
    """The headline frame plus the workloads of the selected patterns: 8 uneven
    clouds (200k-1.2M points, sigma uniform in [5, 35]), a sequence of moving
    ~1M-point frames (sigma 20) and 4 clouds of 500k points (sigma 25) with
    clean colours."""
    import multiprocessing as mp

    pats = selected_patterns(args)
    want_batch = "batched" in pats
    want_diff = "fwd_bwd" in pats
    want_stream = bool(pats & {"streaming", "streaming_periodic"})
    jobs = [("body", dict(seed=synth.config_seed(1), target=args.points, sigma=args.sigma))]
    stream_seed = synth.config_seed(3)
    if want_batch:
        jobs += [("body", dict(bits=10, **kw)) for kw in synth.batched_specs(synth.config_seed(2), 8)]
    if want_diff:
        jobs += [("body", dict(seed=synth.config_seed(4, c), target=500_000, sigma=25.0)) for c in range(4)]
    if want_stream:
        jobs += [("frame", dict(seed=stream_seed, frame=0, target=args.points, sigma=20.0))]
    workers = max(1, min(16, os.cpu_count() or 1, len(jobs) + args.stream_frames))
    # The pool is closed and joined rather than terminated: a worker that ends
    # on SIGTERM runs whatever signal handler a preloaded profiler installed,
    # and one that deadlocks there leaves this process waiting forever.
    pool = mp.get_context("fork").Pool(workers)
    try:
        clouds = pool.map(_gen, jobs, chunksize=1)
        out = {"frame": clouds[0]}
        k = 1
        if want_batch:
            out["batch"] = clouds[k:k + 8]
            k += 8
        if want_diff:
            out["diff"] = clouds[k:k + 4]
            k += 4
        if want_stream:
            first, scale = clouds[k]  # later frames reuse the scale fitted on frame 0
            rest = pool.map(_gen, [("frame", dict(seed=stream_seed, frame=f, target=args.points, sigma=20.0,
                                                  scale=scale)) for f in range(1, args.stream_frames)],
                            chunksize=1)
            out["stream"] = [first] + [c for c, _ in rest]
    finally:
        pool.close()
        pool.join()
    return out


def _events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def bench_batched(clouds, prm, dev, args, fgbd, torch) -> dict:
    """One fgbd_denoise_batched call over 8 uneven clouds per step."""
    import numpy as np

    sizes = [c.n for c in clouds]
    offsets = torch.as_tensor(np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64), device=dev)
    xyz = torch.as_tensor(np.concatenate([c.xyz for c in clouds]), device=dev)
    rgb = torch.as_tensor(np.concatenate([c.noisy for c in clouds]), device=dev)
    total = int(xyz.shape[0])
    ctx = fgbd.Context(dev)
    ctx.reserve(prm, total, len(clouds))
    out = torch.empty_like(rgb)
    res = fgbd.new_result(dev, len(clouds))
    default = ctx.schedule()
    fgbd.denoise_batched(xyz, rgb, offsets, prm, ctx=ctx, out=out, res=res)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    schedule = ctx.autotune(xyz, rgb, offsets, prm, reps=2, out=out, res=res)
    tune_s = time.perf_counter() - t0
    for _ in range(max(1, args.warmup)):
        fgbd.denoise_batched(xyz, rgb, offsets, prm, ctx=ctx, out=out, res=res)
    steps = max(1, args.steps // 2)
    e0, e1 = _events(torch)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        fgbd.denoise_batched(xyz, rgb, offsets, prm, ctx=ctx, out=out, res=res)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    rs = fgbd.read_results(res)
    out_line = {"workload": f"{len(clouds)} body clouds of {min(sizes)}-{max(sizes)} points (sizes uniform in "
                            f"200k-1.2M), noise sigma uniform in [5, 35], 2^10 grid, one batched call",
                "n_points": total, "clouds": len(clouds), "sizes": sizes, "steps": steps,
                "ms_per_batch": ms, "points_per_s": total / (ms / 1e3), "clouds_per_s": len(clouds) / (ms / 1e3),
                "schedule": schedule, "default_schedule": default, "autotune_s": tune_s,
                "q": [r["q"] for r in rs], "sigma_est": [round(r["sigma_est"], 3) for r in rs]}
    if not args.no_profile:
        P = prm.patch if prm.patch > 0 else prm.k
        # Per-kernel HIP events over the same calls.  A sweep launch moves the
        # sweep's bytes for each cloud whose selection is still running, so
        # the sweep kind's bytes per batch are the sum over the clouds.
        ctx.profile(True)
        ctx.profile_read()
        for _ in range(steps):
            fgbd.denoise_batched(xyz, rgb, offsets, prm, ctx=ctx, out=out, res=res)
        torch.cuda.synchronize()
        prof = ctx.profile_read()
        ctx.profile(False)
        rs = fgbd.read_results(res)
        tail_fin = prof.get("finalize", (0.0, 0))[1] == 0
        sweep_bytes = sum(sweep_kind_bytes(n_s, r["sweeps"], prm.num_dirs, prm.k, P, tail_fin)
                          for n_s, r in zip(sizes, rs))
        kernels = {}
        for kind, (kms, launches) in prof.items():
            if launches == 0:
                continue
            per_step = kms / steps
            b = (sweep_bytes if kind == "sweep"
                 else algorithmic_bytes(kind, total, prm.num_dirs, prm.k, P) * launches / steps)
            kernels[kind] = {"ms_per_step": per_step, "launches_per_step": launches / steps,
                             "us_per_launch": 1e3 * kms / launches,
                             "algo_GBs": (b / (per_step / 1e3) / 1e9) if b else None}
        out_line["kernels"] = kernels
        out_line["sweeps"] = [r["sweeps"] for r in rs]
        # Active sweeps on the whole batch (its sweep arrays exceed the
        # 256 MB last-level cache): every cloud filtered at a fixed q, one
        # event pair around q = 32 and one around q = 0, difference / 32.
        qf = 32
        fgbd.denoise_batched_fixed_q(xyz, rgb, offsets, qf, prm, ctx=ctx, out=out, res=res)
        torch.cuda.synchronize()
        times = {}
        for q in (qf, 0):
            a0, a1 = _events(torch)
            a0.record()
            for _ in range(steps):
                fgbd.denoise_batched_fixed_q(xyz, rgb, offsets, q, prm, ctx=ctx, out=out, res=res)
            a1.record()
            torch.cuda.synchronize()
            times[q] = a0.elapsed_time(a1) / steps
        per_sweep = (times[qf] - times[0]) / qf
        b = algorithmic_bytes("sweep", total, prm.num_dirs, prm.k, P)
        out_line["roofline_sweep"] = {"kernel": "sweep (fixed q, every launch active)", "bound": "hbm",
                                      "achieved": b / (per_sweep / 1e3) / 1e9, "peak": HBM_PEAK_GBS,
                                      "unit": "GB/s", "frac": b / (per_sweep / 1e3) / 1e9 / HBM_PEAK_GBS,
                                      "bytes_per_launch": b, "us_per_launch": 1e3 * per_sweep,
                                      "timing": f"(batch at q={qf} - batch at q=0) / {qf}, one event pair each"}
    ctx.close()
    return out_line


def bench_streaming(frames, prm, dev, fgbd, torch, np) -> dict:
    """Frames resident in HBM; per frame a device copy into the static input
    buffers and one replay of the captured per-frame graph (the frame size is
    read from device memory).  Three passes over the sequence."""
    cap = max(f.n for f in frames)
    dxyz = [torch.as_tensor(f.xyz, device=dev) for f in frames]
    drgb = [torch.as_tensor(f.noisy, device=dev) for f in frames]
    doff = [torch.tensor([0, f.n], dtype=torch.int64, device=dev) for f in frames]
    ctx = fgbd.Context(dev)
    ctx.reserve(prm, cap, 1)
    xyz_s = torch.zeros((cap, 3), dtype=torch.int32, device=dev)
    rgb_s = torch.zeros((cap, 3), dtype=torch.float32, device=dev)
    off_s = torch.zeros(2, dtype=torch.int64, device=dev)
    out_s = torch.zeros((cap, 3), dtype=torch.float32, device=dev)
    res_s = fgbd.new_result(dev, 1)

    def load(f):
        n = frames[f].n
        xyz_s[:n].copy_(dxyz[f])
        rgb_s[:n].copy_(drgb[f])
        off_s.copy_(doff[f])

    load(0)
    side = torch.cuda.Stream(dev)
    side.wait_stream(torch.cuda.current_stream(dev))
    with torch.cuda.stream(side):
        fgbd.denoise_batched(xyz_s, rgb_s, off_s, prm, ctx=ctx, out=out_s, res=res_s)
    torch.cuda.current_stream(dev).wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        fgbd.denoise_batched(xyz_s, rgb_s, off_s, prm, ctx=ctx, out=out_s, res=res_s)
    torch.cuda.synchronize()
    for f in range(min(3, len(frames))):  # warm replays
        load(f)
        graph.replay()
    torch.cuda.synchronize()
    passes = 3
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(passes * len(frames) + 1)]
    marks[0].record()
    for p in range(passes):
        for f in range(len(frames)):
            load(f)
            graph.replay()
            marks[1 + p * len(frames) + f].record()
    torch.cuda.synchronize()
    lat = np.array([marks[i].elapsed_time(marks[i + 1]) for i in range(len(marks) - 1)])
    total_ms = marks[0].elapsed_time(marks[-1])
    npts = passes * sum(f.n for f in frames)
    r = fgbd.read_results(res_s)[0]
    ctx.close()
    return {"workload": f"{len(frames)} frames of a rigidly moving body (~1M points each, "
                        f"{min(f.n for f in frames)}-{cap}), noise sigma 20, one captured HIP graph replayed "
                        f"per frame, frame size in device memory",
            "frames": int(lat.size), "frames_per_s": lat.size / (total_ms / 1e3),
            "points_per_s": npts / (total_ms / 1e3), "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "max_ms": float(lat.max()),
            "latency_includes": "device copy of the frame into the graph's input buffers + graph replay",
            "last_q": r["q"]}


def bench_streaming_periodic(frames, prm, dev, fgbd, torch, np, period=10) -> dict:
    """The paper's real-time mode (Sec. 4): noise estimation and filter
    selection on every period-th frame (the captured full per-frame graph),
    the frames in between filtered with the last selected q (a second
    captured graph of the fixed-q call, captured again whenever q changes).
    After each full frame the host reads its q, which drains the queue once
    per period; those waits are inside the timed region."""
    cap = max(f.n for f in frames)
    dxyz = [torch.as_tensor(f.xyz, device=dev) for f in frames]
    drgb = [torch.as_tensor(f.noisy, device=dev) for f in frames]
    doff = [torch.tensor([0, f.n], dtype=torch.int64, device=dev) for f in frames]
    ctx = fgbd.Context(dev)
    ctx.reserve(prm, cap, 1)
    xyz_s = torch.zeros((cap, 3), dtype=torch.int32, device=dev)
    rgb_s = torch.zeros((cap, 3), dtype=torch.float32, device=dev)
    off_s = torch.zeros(2, dtype=torch.int64, device=dev)
    out_s = torch.zeros((cap, 3), dtype=torch.float32, device=dev)
    res_s = fgbd.new_result(dev, 1)

    def load(f):
        n = frames[f].n
        xyz_s[:n].copy_(dxyz[f])
        rgb_s[:n].copy_(drgb[f])
        off_s.copy_(doff[f])

    def capture(call):
        side = torch.cuda.Stream(dev)
        side.wait_stream(torch.cuda.current_stream(dev))
        with torch.cuda.stream(side):
            call()
        torch.cuda.current_stream(dev).wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            call()
        torch.cuda.synchronize()
        return g

    load(0)
    full = capture(lambda: fgbd.denoise_batched(xyz_s, rgb_s, off_s, prm, ctx=ctx, out=out_s, res=res_s))
    full.replay()
    torch.cuda.synchronize()
    q = fgbd.read_results(res_s)[0]["q"]
    fixed_q, fixed = q, capture(lambda: fgbd.denoise_batched_fixed_q(xyz_s, rgb_s, off_s, q, prm, ctx=ctx,
                                                                    out=out_s, res=res_s))
    for f in range(min(3, len(frames))):  # warm replays
        load(f)
        fixed.replay()
    torch.cuda.synchronize()
    passes, recaptures, qs = 3, 0, []
    n_frames = passes * len(frames)
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(n_frames + 1)]
    marks[0].record()
    k = 0
    for p in range(passes):
        for f in range(len(frames)):
            load(f)
            if k % period == 0:
                full.replay()
                marks[1 + k].record()
                marks[1 + k].synchronize()
                q = fgbd.read_results(res_s)[0]["q"]
                qs.append(q)
                if q != fixed_q:
                    fixed_q = q
                    fixed = capture(lambda: fgbd.denoise_batched_fixed_q(xyz_s, rgb_s, off_s, fixed_q, prm, ctx=ctx,
                                                                         out=out_s, res=res_s))
                    recaptures += 1
            else:
                fixed.replay()
                marks[1 + k].record()
            k += 1
    torch.cuda.synchronize()
    lat = np.array([marks[i].elapsed_time(marks[i + 1]) for i in range(len(marks) - 1)])
    total_ms = marks[0].elapsed_time(marks[-1])
    npts = passes * sum(f.n for f in frames)
    ctx.close()
    return {"workload": f"{len(frames)} frames of a rigidly moving body (~1M points each), noise sigma 20; "
                        f"noise estimate and selection every {period} frames, the frames in between filtered "
                        f"with the last selected q (two captured HIP graphs)",
            "frames": int(lat.size), "frames_per_s": lat.size / (total_ms / 1e3),
            "points_per_s": npts / (total_ms / 1e3), "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "max_ms": float(lat.max()),
            "selected_q": qs, "recaptures": recaptures,
            "latency_includes": "device copy of the frame + graph replay; full frames also the host read of q"}


def bench_shuffled(cloud, prm, dev, args, fgbd, torch, np) -> dict:
    """The headline frame with its points in a fixed random order (a capture
    that is not in raster order): the same K timed fgbd_denoise steps, next to
    the frame in its raster order."""
    perm = np.random.default_rng(20240117).permutation(cloud.n)
    stream = torch.cuda.current_stream(dev)
    ctx = fgbd.Context(dev)
    ctx.reserve(prm, cloud.n)
    out = {}
    for name, idx in (("raster", None), ("shuffled", perm)):
        xyz = torch.as_tensor(cloud.xyz if idx is None else cloud.xyz[idx], device=dev)
        rgb = torch.as_tensor(cloud.noisy if idx is None else cloud.noisy[idx], device=dev)
        o = torch.empty_like(rgb)
        res = fgbd.new_result(dev)
        for _ in range(args.warmup):
            fgbd.denoise(xyz, rgb, prm, ctx=ctx, out=o, res=res)
        torch.cuda.synchronize()
        e0, e1 = _events(torch)
        e0.record(stream)
        for _ in range(args.steps):
            fgbd.denoise(xyz, rgb, prm, ctx=ctx, out=o, res=res)
        e1.record(stream)
        torch.cuda.synchronize()
        r = fgbd.read_result(res)
        out[name] = {"ms_per_frame": e0.elapsed_time(e1) / args.steps, "q": r["q"], "sigma_est": r["sigma_est"]}
    ctx.close()
    out["slowdown"] = out["shuffled"]["ms_per_frame"] / out["raster"]["ms_per_frame"]
    out["workload"] = f"the headline frame ({cloud.n} points) in its raster order and in a fixed random order"
    return out


def bench_io(cloud, prm, dev, fgbd, torch, np, reps: int = 20) -> dict:
    """The steps on either side of the path on the headline frame: its voxel
    coordinates as float32 (voxel centres) quantised onto the 2^b grid, the
    denoised colours rounded to uint8, and geometry smoothing (the graph and
    four eq. 5 sweeps on the coordinates).  HIP events on the launch stream."""
    n = cloud.n
    stream = torch.cuda.current_stream(dev)
    xf = torch.as_tensor(cloud.xyz.astype(np.float32) + np.float32(0.5), device=dev)
    rgb = torch.as_tensor(cloud.noisy, device=dev)
    xyz = torch.as_tensor(cloud.xyz, device=dev)
    ctx = fgbd.Context(dev)
    ctx.reserve(prm, n)
    g = torch.empty((n, 3), dtype=torch.int32, device=dev)
    frame = torch.empty(4, dtype=torch.float64, device=dev)
    u8 = torch.empty((n, 3), dtype=torch.uint8, device=dev)
    gout = torch.empty((n, 3), dtype=torch.float32, device=dev)
    gres = fgbd.new_result(dev)
    calls = {
        "quantize": (lambda: fgbd.quantize(xf, prm.bits, ctx=ctx, out=g, frame=frame), 36 * n),
        "round_u8": (lambda: fgbd.round_u8(rgb, ctx=ctx, out=u8), 15 * n),
        "smooth_geometry_q4": (lambda: fgbd.smooth_geometry(xyz, 4, prm, ctx=ctx, out=gout, res=gres), None),
    }
    out = {"workload": f"the headline frame ({n} points)"}
    for name, (fn, nbytes) in calls.items():
        fn()
        torch.cuda.synchronize()
        e0, e1 = _events(torch)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        us = 1e3 * e0.elapsed_time(e1) / reps
        row = {"us": us}
        if nbytes:
            row["algorithmic_bytes"] = nbytes
            row["GB_per_s"] = nbytes / us / 1e3
        out[name] = row
    ctx.close()
    return out


def bench_fwd_bwd(clouds, dev, args, fgbd, torch) -> dict:
    """Polynomial filter (8 coefficients, trained bandwidth) forward and
    hand-written adjoint on 4 x 500k points, inside Adam steps fitting the
    coefficients and the bandwidth to the clean colours (MSE)."""
    import numpy as np

    prm = fgbd.default_params()
    ctx = fgbd.Context(dev)
    graphs = []
    for c in clouds:
        ctx.reserve(prm, c.n)
        graphs.append(fgbd.build_slg(torch.as_tensor(c.xyz, device=dev), prm, ctx=ctx))
    offs = np.concatenate([[0], np.cumsum([c.n for c in clouds])])
    col = torch.cat([torch.where(g.col >= 0, g.col + int(o), g.col) for g, o in zip(graphs, offs[:-1])])
    g = fgbd.SLGraph(col.contiguous(), torch.cat([g.dist2 for g in graphs]).contiguous(),
                     torch.cat([g.p for g in graphs]).contiguous(), graphs[0].result)
    sg0 = float(np.mean([fgbd.read_result(gr.result)["sigma_g"] for gr in graphs]))
    x = torch.as_tensor(np.concatenate([c.noisy for c in clouds]), device=dev)
    clean = torch.as_tensor(np.concatenate([c.clean for c in clouds]).astype(np.float32), device=dev)
    n = int(x.shape[0])
    ctx.reserve(prm, n)
    coef = torch.zeros(8, dtype=torch.float32, device=dev)
    coef[2] = 1.0  # start from two sweeps of eq. 5
    coef.requires_grad_(True)
    sigma_g = torch.tensor(sg0, dtype=torch.float64, device=dev, requires_grad=True)
    opt = torch.optim.Adam([coef, sigma_g], lr=1e-2)

    def step():
        out = fgbd.poly_filter_autograd(x, coef, sigma_g, g, ctx=ctx)
        loss = torch.mean((out - clean) ** 2)
        opt.zero_grad(set_to_none=True)
        loss.backward()
        opt.step()
        return loss.detach()

    mse_noisy = float(torch.mean((x - clean) ** 2))
    mse0 = float(step())  # also the warm-up
    torch.cuda.synchronize()
    e0, e1 = _events(torch)
    e0.record()
    loss = None
    for _ in range(args.adam_steps):
        loss = step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.adam_steps
    # the filter's own forward+backward, without the optimiser and loss
    out, saved = fgbd.poly_filter(g, x, coef.detach(), sigma_g.detach(), ctx=ctx)
    go = torch.ones_like(out)
    e0.record()
    for _ in range(args.adam_steps):
        out, saved = fgbd.poly_filter(g, x, coef.detach(), sigma_g.detach(), ctx=ctx)
        fgbd.poly_filter_backward(g, saved, coef.detach(), sigma_g.detach(), go, ctx=ctx)
    e1.record()
    torch.cuda.synchronize()
    ms_f = e0.elapsed_time(e1) / args.adam_steps
    ctx.close()
    return {"workload": "4 body clouds x 500k points, noise sigma 25, polynomial filter with 8 coefficients "
                        "and trained bandwidth, MSE to the clean colours, Adam (lr 1e-2)",
            "n_points": n, "adam_steps": args.adam_steps, "ms_per_adam_step": ms,
            "points_per_s": n / (ms_f / 1e3), "ms_fwd_bwd": ms_f,
            "points_per_s_with_optimizer": n / (ms / 1e3),
            "mse_noisy": mse_noisy, "mse_start": mse0, "mse_end": float(loss),
            "coef": [round(v, 4) for v in coef.detach().cpu().tolist()], "sigma_g": float(sigma_g)}


# ---------------------------------------------------------------- CPU baseline
_CPU_JOB = None  # (xyz, rgb, params) inherited by the forked workers


def oracle_params(args) -> dict:
    """The library's default parameters (fgbd_default_params) for the oracle;
    main() checks them against the library's own."""
    return dict(bits=10, num_dirs=args.num_dirs, window=4, k=8, patch=0, q_max=32, fslr_kappa=2.0, sigma_g=0.0,
                patch_order=0)


def _oracle_stages(_=None):
    """The oracle's per-frame path on the shared frame, its three stages timed
    as the paper's Table 1 splits them: graph construction (scan-line graph,
    bandwidth, eq. 4 weights), noise estimation (NE-GBP and the FSLR spreads),
    low-pass filter (FSLR subset, eq. 6 selection and the eq. 5 sweeps).  The
    calls are the oracle's own, in the order its denoise() makes them."""
    import numpy as np

    import oracle

    xyz, rgb, prm = _CPU_JOB
    g = np.asarray(xyz, np.int64)
    y = np.asarray(rgb, np.float64)
    t0 = time.perf_counter()
    col, dist2 = oracle.slg_graph(g, prm["bits"], prm["num_dirs"], prm["window"], prm["k"])
    sg = prm["sigma_g"] if prm["sigma_g"] > 0 else oracle.bandwidth(col, dist2)
    p = oracle.edge_weights(col, dist2, sg)
    t1 = time.perf_counter()
    ne = oracle.estimate_noise(col, y, prm["patch"], prm["patch_order"])
    spread = oracle.patch_spread(col, y, prm["patch"])
    t2 = time.perf_counter()
    S = oracle.fslr_subset(spread, ne["sigma_est"], prm["fslr_kappa"])
    sel = oracle.select_filter(col, p, y, ne["sigma_est"], S, prm["q_max"])
    t3 = time.perf_counter()
    return {"GC": t1 - t0, "NE": t2 - t1, "LF": t3 - t2, "q": int(sel["q"])}


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cloud, prm: dict) -> dict:
    """The FP64 oracle on the host: one thread on the headline frame (stage
    split as in Table 1), then all the host cores this process may use (at
    most 16), one forked worker per core, each running the same frame, for the
    aggregate points/s."""
    import multiprocessing as mp

    global _CPU_JOB
    _CPU_JOB = (cloud.xyz, cloud.noisy, prm)
    n = cloud.n
    c0 = os.times()
    w0 = time.perf_counter()
    one = _oracle_stages()
    wall1 = time.perf_counter() - w0
    c1 = os.times()
    busy = (c1.user - c0.user) + (c1.system - c0.system)
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    procs = max(1, min(16, cores))
    w0 = time.perf_counter()
    pool = mp.get_context("fork").Pool(procs)  # closed, not terminated, as in make_inputs
    try:
        runs = pool.map(_oracle_stages, range(procs), chunksize=1)
    finally:
        pool.close()
        pool.join()
    wall_all = time.perf_counter() - w0
    _CPU_JOB = None
    stages = {k: one[k] for k in ("GC", "NE", "LF")}
    return {"value": procs * n / wall_all, "unit": "points/s", "cores": procs, "kind": "oracle",
            "sample": f"{procs} forked processes, each the FP64 numpy oracle on the full headline frame "
                      f"({n} points); {wall_all:.1f} s wall",
            "single_thread": {"value": n / wall1, "unit": "points/s", "s_per_frame": wall1,
                              "cpu_s": busy, "stages_s": stages, "q": one["q"]},
            "all_cores_s_per_frame_mean": sum(sum(r[k] for k in ("GC", "NE", "LF")) for r in runs) / len(runs),
            "host": {"nproc": os.cpu_count(), "usable_cores": cores, "cpu_model": _cpu_model()}}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--sigma", type=float, default=20.0)
    ap.add_argument("--num-dirs", type=int, default=8)
    ap.add_argument("--points", type=int, default=1_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="skip the per-kernel profiled pass")
    ap.add_argument("--autotune", action="store_true",
                    help="let the library's autotuner pick the launch schedule of the headline frame first")
    ap.add_argument("--no-patterns", action="store_true",
                    help="skip the batched, streaming and forward+backward measurements")
    ap.add_argument("--patterns", default="batched,streaming,streaming_periodic,fwd_bwd,io,shuffled",
                    help="comma-separated patterns to run beside the headline (with --no-patterns: none)")
    ap.add_argument("--stream-frames", type=int, default=30)
    ap.add_argument("--adam-steps", type=int, default=50)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (reference for hardware byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the FGBD path runs on a single device and this build has no "
              "multi-GPU path (use --gpus 1).", file=sys.stderr)
        return 2

    from paper_2401_09721_amd import synth

    # Inputs are generated on the host before the GPU is touched, in worker
    # processes (the generator is pure numpy).
    t0 = time.time()
    inputs = make_inputs(args, synth)
    gen_s = time.time() - t0
    cloud = inputs["frame"]
    # the CPU oracle on the host, also before the GPU is touched (its worker
    # processes are forked): a reported baseline, not a target
    cpu = None if args.no_cpu_baseline else cpu_baseline(cloud, oracle_params(args))

    import numpy as np
    import torch

    from paper_2401_09721_amd import fgbd

    n = cloud.n
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    xyz = torch.as_tensor(cloud.xyz, device=dev)
    rgb = torch.as_tensor(cloud.noisy, device=dev)
    prm = fgbd.default_params(num_dirs=args.num_dirs)
    if dict(prm.as_dict()) != oracle_params(args):
        raise RuntimeError("the CPU baseline's parameters differ from the library defaults")
    P = prm.patch if prm.patch > 0 else prm.k
    ctx = fgbd.Context(dev)
    ctx.reserve(prm, n)
    out = torch.empty_like(rgb)
    res = fgbd.new_result(dev)
    stream = torch.cuda.current_stream(dev)

    for _ in range(args.warmup):
        fgbd.denoise(xyz, rgb, prm, ctx=ctx, out=out, res=res)
    torch.cuda.synchronize()
    if args.autotune:  # the library's own tuner picks the launch schedule for this frame
        one = torch.tensor([0, n], dtype=torch.int64, device=dev)
        ctx.autotune(xyz, rgb, one, prm, reps=3, out=out, res=res)
        for _ in range(args.warmup):
            fgbd.denoise(xyz, rgb, prm, ctx=ctx, out=out, res=res)
        torch.cuda.synchronize()
    print(f"# warmup done ({args.warmup} steps), n={n}, generation {gen_s:.1f}s", file=sys.stderr, flush=True)

    # ---- timed region (headline): K steps, no per-kernel events
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        fgbd.denoise(xyz, rgb, prm, ctx=ctx, out=out, res=res)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms_total = ev0.elapsed_time(ev1)
    ms_step = ms_total / args.steps
    r = fgbd.read_result(res)
    print(f"# timed: {ms_step:.3f} ms/step (host wall {1e3 * wall / args.steps:.3f} ms/step), q={r['q']} "
          f"sweeps={r['sweeps']} sigma_est={r['sigma_est']:.3f}", file=sys.stderr, flush=True)

    line = {
        "metric": METRIC,
        "value": n * args.steps / (ms_total / 1e3),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"single frame, {n} points, 2^10 voxel grid, 6 ellipsoid + 2 plane shells, "
                        f"colour noise sigma {args.sigma:g}",
            "n_points": n,
            "num_dirs": prm.num_dirs, "window": prm.window, "k": prm.k, "patch": P, "q_max": prm.q_max,
            "fslr_kappa": prm.fslr_kappa,
        },
        "frames_per_s": 1e3 / ms_step,
        "schedule": ctx.schedule(),
        "result": {k: r[k] for k in ("sigma_est", "sigma_g", "q", "sweeps", "n_fslr", "n_eff", "m")},
    }

    # ---- profiled pass over the same K steps: per-kernel HIP events
    if not args.no_profile:
        ctx.profile(True)
        ctx.profile_read()
        for _ in range(args.steps):
            fgbd.denoise(xyz, rgb, prm, ctx=ctx, out=out, res=res)
        torch.cuda.synchronize()
        prof = ctx.profile_read()
        ctx.profile(False)
        kernels = {}
        for kind, (ms, launches) in prof.items():
            if launches == 0:
                continue
            per_launch = ms / launches
            b = algorithmic_bytes(kind, n, prm.num_dirs, prm.k, P)
            kernels[kind] = {"ms_per_step": ms / args.steps, "launches_per_step": launches / args.steps,
                             "us_per_launch": 1e3 * per_launch,
                             "algo_GBs": (b / (per_launch / 1e3) / 1e9) if b else None}
        line["kernels"] = kernels
        line["profiled_ms_per_step"] = sum(v["ms_per_step"] for v in kernels.values())
        # Bytes each kind moves per step: its algorithmic bytes per launch for
        # every launch that computes (the sweep kind: sweep_kind_bytes).
        def step_bytes(kind):
            if kind == "sweep":
                return sweep_kind_bytes(n, r["sweeps"], prm.num_dirs, prm.k, P, "finalize" not in kernels)
            return algorithmic_bytes(kind, n, prm.num_dirs, prm.k, P) * kernels[kind]["launches_per_step"]

        tcfg = {"n_points": n, "num_dirs": prm.num_dirs, "window": prm.window, "k": prm.k, "patch": P,
                "sigma": args.sigma}

        # Counter-measured HBM bytes of the same launches per step (None while
        # a kernel's sources differ from the ones the record was taken on).
        def step_traffic(kind):
            if kind == "sweep":
                return sweep_kind_sum(r["sweeps"], prm.k, "finalize" not in kernels,
                                      lambda k: measured_traffic(k, tcfg))
            t = measured_traffic(kind, tcfg)
            return t * kernels[kind]["launches_per_step"] if t is not None else None

        dom = max((k for k in kernels if algorithmic_bytes(k, n, prm.num_dirs, prm.k, P) > 0),
                  key=lambda k: kernels[k]["ms_per_step"])
        line["roofline"] = roofline_object(dom, kernels[dom], step_bytes(dom), step_traffic(dom),
                                           measured_valu(dom, tcfg, kernels[dom]["us_per_launch"]))
        print(f"# kernels: {json.dumps(kernels)}", file=sys.stderr, flush=True)

        # Active sweeps alone, the kernel the bandwidth target is set on: the
        # filter at a fixed q computes a sweep in every launch; one event pair
        # around q = 32 and one around q = 0 (same setup and final copy), so
        # the difference is 32 sweeps with no per-launch event in between.
        g = fgbd.build_slg(xyz, prm, ctx=ctx)
        qf = 32
        fgbd.filter(g, rgb, prm, q_fixed=qf, ctx=ctx)
        torch.cuda.synchronize()
        times = {}
        for q in (qf, 0):
            e0, e1 = _events(torch)
            e0.record(stream)
            for _ in range(args.steps):
                fgbd.filter(g, rgb, prm, q_fixed=q, ctx=ctx)
            e1.record(stream)
            torch.cuda.synchronize()
            times[q] = e0.elapsed_time(e1) / args.steps
        per_launch = (times[qf] - times[0]) / qf
        b = algorithmic_bytes("sweep", n, prm.num_dirs, prm.k, P)
        line["roofline_sweep"] = {"kernel": "sweep (fixed q, every launch active)", "bound": "hbm",
                                  "achieved": b / (per_launch / 1e3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                  "frac": b / (per_launch / 1e3) / 1e9 / HBM_PEAK_GBS,
                                  "traffic": measured_traffic("sweep", tcfg),
                                  "bytes_per_launch": b, "us_per_launch": 1e3 * per_launch,
                                  "timing": f"(filter at q={qf} - filter at q=0) / {qf}, one event pair each"}

    pats = selected_patterns(args)
    runs = [
        ("batched", lambda: bench_batched(inputs["batch"], prm, dev, args, fgbd, torch)),
        ("streaming", lambda: bench_streaming(inputs["stream"], prm, dev, fgbd, torch, np)),
        ("streaming_periodic", lambda: bench_streaming_periodic(inputs["stream"], prm, dev, fgbd, torch, np)),
        ("fwd_bwd", lambda: bench_fwd_bwd(inputs["diff"], dev, args, fgbd, torch)),
        ("io", lambda: bench_io(cloud, prm, dev, fgbd, torch, np)),
        ("shuffled", lambda: bench_shuffled(cloud, prm, dev, args, fgbd, torch, np)),
    ]
    for name, fn in runs:
        if name in pats:
            line[name] = fn()
            print(f"# {name}: {json.dumps(line[name])}", file=sys.stderr, flush=True)

    if args.copy_calibration:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device=dev)  # 256 MiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        line["copy_calibration_bytes"] = {"read": src.numel() * 4, "written": dst.numel() * 4, "launches": 3}

    if cpu is not None:
        line["cpu_baseline"] = cpu
    ctx.close()
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
