#!/usr/bin/env python3
"""Benchmark of the FX correlator hot path on one MI355X.

Workload (default): the precision form of the GMRT-scale correlator --
64 signals (32 antennas x 2 polarisations), 4096-point FFT (2048 channels),
32768 spectra per step (one 2.01 s block at 66.67 MS/s), F-engine ->
X-engine -> integrate, all inputs resident in HBM.  The headline value is the
int8-MFMA path's correlated bandwidth; the FP32 path at the same shape is
timed beside it.  One step = F-engine (held requantisation scales, set once
on a calibration pass like the paper's gain table) + X-engine + integrate
with dump, over one block of all 64 signals.

--streamed also times the blocks streamed, the F-engine of block i + 1
running beside the X-engine of block i (two streams, two spectra buffers),
and reports that rate as the value; the per-kernel times are always those of
the one-stream step.

Prints one JSON line.  Options: --steps K --warmup W --gpus 1
[--config c2|c3|c4|c5] [--no-fp32] [--no-cpu-baseline] [--streamed].  c4 is the batched
form (six uneven sub-arrays in one graph launch); c5 the flagged path with the
learned RFI flagger (64 signals, 8192-pt FFT, 8192 spectra).
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

FS = 66.666666e6
CONFIGS = {
    # name: (S, N, T, description)
    "c3": (64, 4096, 32768, "precision form: 64 signals, 4096-pt FFT (2048 ch), 32768 spectra"),
    "c2": (64, 1024, 16384, "GMRT scale: 64 signals with 8 point sources, 1024-pt FFT (512 ch), 16384 spectra, FP32"),
}
HBM_PEAK = 8.0e12           # B/s
INT8_PEAK = 5.0e15          # dense int8 MFMA OP/s
FP32_MFMA_PEAK = 157.3e12   # dense FP32 matrix FLOP/s
FP16_MFMA_PEAK = 2.5e15     # dense FP16 matrix FLOP/s
CNN_FLOP_PER_CELL = 2 * (16 * 9 + 16 * 16 * 9 + 16 * 9)  # 2592 MACs of the three 3x3 layers
# FP32 vector peak without packed-FP32 instructions (which this library never
# emits): 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz.  The 157.3
# TFLOP/s datasheet figure assumes two FP32 FMAs per lane per cycle (packed).
FP32_VALU_PEAK = 256 * 4 * 16 * 2 * 2.4e9
FP32_PUBLISHED_PEAK = 157.3e12  # the datasheet's FP32 vector figure (packed FP32)

# HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE (scaled by the
# calibration copy, see profiles/), valid only for the kernel source they were
# taken from: reported as `traffic` when the source hash still matches.
MEASURED_TRAFFIC = {
    # profiles/fx_int8_64sig_4096pt_32768spec.md: FETCH_SIZE 4468485 KiB x 2.000, WRITE_SIZE 8388932 KiB x 1.000
    # (medians of 7 dispatches, with the source's instruction-level-parallelism schedule)
    "fengine_int8_c3": {"source": "paper_0910_1517_amd/csrc/fengine4.hip",
                        "sha256": "59ba376590687bfeb9bf11ebeabfc7cccdfdcc610893e4b27ca29d0f09025fda",
                        "flags": ["-mllvm", "-amdgpu-mfma-vgpr-form", "-mllvm", "-amdgpu-sched-strategy=max-ilp"],
                        "read": 9.151e9, "write": 8.590e9},
    # profiles/fx_fp32_64sig_1024pt_16384spec_pointsources.md: FETCH_SIZE 537802 KiB x 2.000, WRITE_SIZE 4194304 KiB
    # (medians of 6 dispatches)
    "fengine_fp32_c2": {"source": "paper_0910_1517_amd/csrc/fengine.hip",
                        "sha256": "752cc90ed275dea5e3ee47a0f95cb1472859c15dff0c235504cf6068a8a8039a",
                        "flags": [],
                        "read": 1.101e9, "write": 4.295e9},
    # profiles/cnn_flagged_64sig_8192pt_8192spec.md (FP16 power, column guard, max-ilp schedule): FETCH_SIZE
    # 2097368 KiB x 2.000, WRITE_SIZE 2097152 KiB
    "cnn_infer_c5": {"source": "paper_0910_1517_amd/csrc/cnn.hip",
                     "sha256": "262fd32417682dd772bc249c879504260bc82e884cae8115691124ba211a5e03",
                     "flags": ["-mllvm", "-amdgpu-sched-strategy=max-ilp"],
                     "read": 4.295e9, "write": 2.147e9},
    # profiles/fx_int8_64sig_4096pt_32768spec.md: FETCH_SIZE 4197483 KiB x 2.000, WRITE_SIZE 1572864 KiB x 1.000
    "beam_int8_c3": {"source": "paper_0910_1517_amd/csrc/beam.hip",
                     "sha256": "fdea2c6b6d608a65e64c732609303dc9d4f9377b18ad830e8b407f4c35843b4f",
                     "read": 8.597e9, "write": 1.611e9},
    # profiles/blank_int8_64sig_134Msamples.md: out of place FETCH_SIZE 4211175 KiB x 2.000, WRITE_SIZE 9624595 KiB
    "blank_out_c3": {"source": "paper_0910_1517_amd/csrc/blank.hip",
                     "sha256": "3d7db02ee39e54f695df0e2e89e58bb8292bdfc262d90a9c60d3e880341b0b8b",
                     "read": 8.624e9, "write": 9.856e9},
    # same profile, in place: FETCH_SIZE 4211023 KiB x 2.000, WRITE_SIZE 900710 KiB.  (Both blank.hip records
    # follow host-side and comment changes whose device code compiles to the same instructions.)
    "blank_in_c3": {"source": "paper_0910_1517_amd/csrc/blank.hip",
                    "sha256": "3d7db02ee39e54f695df0e2e89e58bb8292bdfc262d90a9c60d3e880341b0b8b",
                    "read": 8.624e9, "write": 0.922e9},
}


def measured_traffic(key):
    """The record's bytes while its source (and, when the record names them,
    the source's per-file compiler flags) are those the counters were taken on."""
    import hashlib
    rec = MEASURED_TRAFFIC.get(key)
    if not rec or not rec["sha256"]:
        return None
    try:
        h = hashlib.sha256(open(os.path.join(ROOT, rec["source"]), "rb").read()).hexdigest()
    except OSError:
        return None
    if "flags" in rec:
        from paper_0910_1517_amd import build as hipbuild
        if hipbuild.EXTRA.get(os.path.basename(rec["source"]), []) != rec["flags"]:
            return None
    return rec["read"] + rec["write"] if h == rec["sha256"] else None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def f_algorithmic(S, N, T, out_bytes_per_ch):
    """F-engine algorithmic flops and bytes per launch.
    flops/spectrum: real FFT 2.5 N log2 N + phase rotation 6 per channel;
    bytes/spectrum: N int8 samples in + N/2 channels x out_bytes_per_ch out."""
    C = N // 2
    flops = S * T * (2.5 * N * np.log2(N) + 6.0 * C)
    nbytes = S * T * (N + C * out_bytes_per_ch)
    return flops, nbytes


def x_algorithmic(S, N, T, in_bytes_per_ch):
    """X-engine algorithmic ops (8 per complex MAC over all S(S+1)/2 pairs) and input bytes."""
    C, P = N // 2, S * (S + 1) // 2
    return 8.0 * P * C * T, float(S * C * T * in_bytes_per_ch)


def run_path(corr, torch, prec, S, N, T, x_dev, rs, g_dev, steps, warmup, scale=None, graph=True):
    """One step = F-engine + X-engine + integrate (dump and reset) on one stream.

    Per-kernel times: HIP events around each launch of `steps` eager steps
    after `warmup` ones, median over the steps.  Step time: the same three
    calls captured once into a HIP graph, `warmup` replays, then the median of
    `steps` replays bracketed by events on the replay stream; the graph's dumped
    visibilities must equal the eager run's bit for bit."""
    plan = corr.Plan(S, N, T, precision=prec, max_delay=16, scale_mode=corr.SCALE_HOLD)
    spec = plan.alloc("spectra", zero=False)
    acc, state, vis = plan.alloc("acc"), plan.alloc("state"), plan.alloc("vis")
    st = torch.cuda.Stream()
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]

    def step(e=None):
        if e: e[0].record(st)
        plan.fengine(x_dev, g_dev, spec, scale, row_stride=rs, stream=st)
        if e: e[1].record(st)
        plan.xengine(spec, acc, stream=st)
        if e: e[2].record(st)
        plan.integrate(acc, state, vis, scale, flags=corr.DUMP | corr.RESET, stream=st)
        if e: e[3].record(st)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        step(ev[i])
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    med = lambda a, b: float(np.median([e[a].elapsed_time(e[b]) for e in ev])) * 1e-3
    out = dict(t_f=med(0, 1), t_x=med(1, 2), t_int=med(2, 3), t_eager_step=med(0, 3), wall=wall,
               splits=plan.splits, fkernel=plan.fengine_kernel)
    out["t_step"] = out["t_eager_step"]
    plan.check_device_errors()
    if graph:
        eager_vis = vis.clone()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=st):
            step()
        vis.zero_()
        ge = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        with torch.cuda.stream(st):
            for _ in range(warmup):
                g.replay()
            st.synchronize()
            ok = bool(torch.equal(vis, eager_vis))  # a replay reproduces the eager step
            for e0, e1 in ge:
                e0.record(st)
                g.replay()
                e1.record(st)
        torch.cuda.synchronize()
        ok = ok and bool(torch.equal(vis, eager_vis))
        if not ok:
            raise RuntimeError("graph replay of the step differs from the eager step")
        out["t_step"] = float(np.median([a.elapsed_time(b) for a, b in ge])) * 1e-3
        out["graph_matches_eager"] = ok
        del g, eager_vis
    del spec, acc, state, vis
    return out


def run_pipelined(corr, torch, prec, S, N, T, x_dev, rs, g_dev, steps, warmup, scale=None):
    """The same passes streamed: the F-engine of block i + 1 (one stream) runs
    while the X-engine and integrator of block i (a second stream) consume the
    other of two spectra buffers; events order each buffer's reuse.  Returns
    the steady-state time per block from HIP events around all `steps`."""
    fplan = corr.Plan(S, N, T, precision=prec, max_delay=16, scale_mode=corr.SCALE_HOLD)
    xplan = corr.Plan(S, N, T, precision=prec, max_delay=16, scale_mode=corr.SCALE_HOLD)
    specs = [fplan.alloc("spectra", zero=False) for _ in range(2)]
    acc, state, vis = xplan.alloc("acc"), xplan.alloc("state"), xplan.alloc("vis")
    sf, sx = torch.cuda.current_stream(), torch.cuda.Stream()
    f_done = [torch.cuda.Event() for _ in range(2)]
    x_done = [torch.cuda.Event() for _ in range(2)]

    def step(i):
        b = i & 1
        if i >= 2:
            sf.wait_event(x_done[b])  # spectra buffer b has been consumed
        fplan.fengine(x_dev, g_dev, specs[b], scale, row_stride=rs, stream=sf)
        f_done[b].record(sf)
        sx.wait_event(f_done[b])
        xplan.xengine(specs[b], acc, stream=sx)
        xplan.integrate(acc, state, vis, scale, flags=corr.DUMP | corr.RESET, stream=sx)
        x_done[b].record(sx)

    for i in range(warmup):
        step(i)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(sf)
    sx.wait_event(e0)
    for i in range(steps):
        step(warmup + i)
    sf.wait_stream(sx)
    e1.record(sf)
    torch.cuda.synchronize()
    fplan.check_device_errors()
    t = e0.elapsed_time(e1) * 1e-3 / steps
    del specs, acc, state, vis
    return t


def calibrate_scales(corr, torch, S, N, T, x_dev, rs, g_dev, prec=None):
    prec = corr.INT8 if prec is None else prec
    plan = corr.Plan(S, N, T, precision=prec, max_delay=16, scale_mode=corr.SCALE_COMPUTE)
    spec = plan.alloc("spectra", zero=False)
    scale = torch.zeros(S * plan.C, dtype=torch.float32, device="cuda")
    plan.fengine(x_dev, g_dev, spec, scale, row_stride=rs)
    torch.cuda.synchronize()
    del spec, plan
    torch.cuda.empty_cache()
    return scale


def _omp_set_threads(n):
    """Set the OpenMP thread count of the oracle's runtime (libgomp) for the calls
    that follow; returns the count it reports."""
    import ctypes
    gomp = ctypes.CDLL("libgomp.so.1")
    gomp.omp_set_num_threads(int(n))
    return int(gomp.omp_get_max_threads())


def cpu_model():
    import subprocess
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
    except (OSError, subprocess.SubprocessError):
        return None
    for line in txt.splitlines():
        if line.startswith("Model name:"):
            return line.split(":", 1)[1].strip()
    return None


def cpu_baseline(S, N, T_sample, threads, prec="int8", chunk=128):
    """The CPU oracle as it stands, on T_sample spectra of the workload's shape,
    with `threads` OpenMP threads: F-engine (FP64 DFT, phase) and X-engine
    (int8 requantisation, int64 products, FP64 scaling; or the FP64 products of
    the FP32 path) timed apart.  Returns a dict (MHz = N T / (2 t))."""
    import oracle
    import synth
    geo = synth.make_geometry(S // 2, seed=synth.BASE_SEED + 2)
    og = oracle.Geometry(geo.D, geo.f, geo.psi0, geo.rate)
    x = synth.voltages(S, N * T_sample + 64, geo, FS, mode="bulk", seed=synth.BASE_SEED + 2,
                       tone_bin=37, tone_N=N)
    oracle.build()
    used = _omp_set_threads(threads)
    tf = tx = 0.0
    A = V = scale = None
    for m0 in range(0, T_sample, chunk):
        n = min(chunk, T_sample - m0)
        xs = np.ascontiguousarray(x[:, m0 * N:])
        t0 = time.perf_counter()
        Y = oracle.fengine(xs, N, n, og, FS, spectrum0=m0)
        t1 = time.perf_counter()
        if prec == "int8":
            if scale is None:
                scale = oracle.int8_scale(oracle.sigma(Y)).astype(np.float64)
            A = oracle.xengine_int(oracle.quantize_int8(Y, scale), A)
        else:
            V = oracle.xengine(Y, V)
        tx += time.perf_counter() - t1
        tf += t1 - t0
    t1 = time.perf_counter()
    if prec == "int8":
        V = oracle.scale_visibilities(A, scale)
    tx += time.perf_counter() - t1
    assert np.isfinite(V).all()
    bw = lambda t: N * T_sample / (2 * t) / 1e6
    return {"value": bw(tf + tx), "threads": used, "t_s": tf + tx, "f_engine_mhz": bw(tf), "x_engine_mhz": bw(tx),
            "f_s": tf, "x_s": tx, "spectra": T_sample}


def cpu_baseline_record(S, N, prec, sample_all, sample_one):
    """cpu_baseline at every host core (the reported value) and at one thread."""
    ncores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    allc = cpu_baseline(S, N, sample_all, ncores, prec)
    one = cpu_baseline(S, N, sample_one, 1, prec)
    _omp_set_threads(ncores)
    desc = ("%s path of the oracle (FP64 F-engine: DFT and Eq. 2 phase; %s), %d signals, N = %d"
            % (prec, "int8 requantisation + int64 X-engine + FP64 scaling" if prec == "int8" else
               "FP64 X-engine", S, N))
    return {"value": round(allc["value"], 4), "unit": "MHz", "cores": allc["threads"], "kind": "oracle",
            "sample": "%d spectra (%.1f s) of the workload's shape; %s" % (allc["spectra"], allc["t_s"], desc),
            "cpu_model": cpu_model(),
            "f_engine_mhz": round(allc["f_engine_mhz"], 4), "x_engine_mhz": round(allc["x_engine_mhz"], 4),
            "f_s": round(allc["f_s"], 3), "x_s": round(allc["x_s"], 3),
            "single_thread": {"value": round(one["value"], 5), "cores": one["threads"],
                              "sample": "%d spectra (%.1f s)" % (one["spectra"], one["t_s"]),
                              "f_engine_mhz": round(one["f_engine_mhz"], 5),
                              "x_engine_mhz": round(one["x_engine_mhz"], 5)}}


BATCH_SHAPES = [  # (signals, channels, spectra) of the six uneven sub-arrays
    (8, 256, 65536), (16, 512, 32768), (30, 1024, 16384), (48, 2048, 8192), (60, 4096, 2048), (64, 8192, 1024)]


def bench_batch(args):
    """Batched form: six sub-arrays in one captured HIP-graph launch (int8, held scales,
    autotuned X-engine splits).  Prints one JSON line."""
    import torch
    import paper_0910_1517_amd as corr
    import synth
    torch.cuda.set_device(0)
    shapes, inputs = [], []
    for i, (S, C, T) in enumerate(BATCH_SHAPES):
        N = 2 * C
        split, ms = corr.autotune_x_split(S, N, T)
        log("sub-array %d: S=%d C=%d T=%d autotuned split %d (%.3f ms X)" % (i, S, C, T, split, ms))
        shapes.append(dict(n_signals=S, fft_len=N, n_spectra=T, x_split=split))
    b = corr.Batch(shapes)
    bufs = []
    for i, sh in enumerate(shapes):
        S, N, T = sh["n_signals"], sh["fft_len"], sh["n_spectra"]
        geo = synth.make_geometry((S + 1) // 2, seed=synth.BASE_SEED + 10 + i).subset(np.arange(S))
        rs = (N * T + 16 + 255) // 256 * 256
        x = synth.voltages_device(S, N * T + 16, geo, seed=synth.BASE_SEED + 10 + i, row_stride=rs)
        g = corr.geom_to_device(corr.geom_array(geo.D, geo.f, geo.psi0, geo.rate))
        p = b.plans[i]
        # scales from a calibration pass of the sub-array itself
        cal = corr.Plan(S, N, T, precision=corr.INT8, scale_mode=corr.SCALE_COMPUTE)
        scale = torch.zeros(S * p.C, dtype=torch.float32, device="cuda")
        tmp = cal.alloc("spectra", zero=False)
        cal.fengine(x, g, tmp, scale, row_stride=rs)
        torch.cuda.synchronize()
        del tmp, cal
        spec = p.alloc("spectra", zero=False)
        acc, state, vis = p.alloc("acc"), p.alloc("state"), p.alloc("vis")
        b.set_io(i, x=x, row_stride=rs, geom=g, spec=spec, scale=scale, acc=acc, state=state, vis=vis,
                 flags=corr.DUMP | corr.RESET)
        bufs.append((x, g, scale, spec, acc, state, vis))
    stream = torch.cuda.Stream()
    b.capture(stream)
    for _ in range(args.warmup):
        b.launch(stream)
    stream.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    for e0, e1 in ev:
        e0.record(stream)
        b.launch(stream)
        e1.record(stream)
    stream.synchronize()
    t = float(np.median([e0.elapsed_time(e1) for e0, e1 in ev])) * 1e-3
    per = []
    tot_bw = tot_ops = 0.0
    for (S, C, T) in BATCH_SHAPES:
        bw = 2 * C * T / (2 * t) / 1e6
        ops = 8.0 * S * (S + 1) / 2 * C * T
        tot_bw += bw
        tot_ops += ops
        per.append({"signals": S, "channels": C, "spectra": T, "correlated_bandwidth_mhz": round(bw, 3)})
    out = {
        "metric": "correlated bandwidth (MHz) & X-engine TOP/s: batched uneven sub-arrays, one graph launch",
        "value": round(tot_bw, 3), "unit": "MHz", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(t * 1e3, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int8", "data": "synthetic (seeded Gaussian + common source, generated on the GPU)",
        "config": {"workload": "6 sub-arrays, 8-64 signals, 256-8192 channels, 1024-65536 spectra",
                   "sub_arrays": per, "parallelism": "single GPU"},
        "aggregate_tops": round(tot_ops / t / 1e12, 3),
    }
    b.close()
    print(json.dumps(out), flush=True)


def bench_rfi(args):
    """Flagged int8 path with the learned flagger: F-engine (held scales, power
    output) -> CNN inference (fused FP16 MFMA kernel) -> keep bits from the
    flags -> X-engine with the keep bits applied as it stages the spectra, and
    the exact per-pair unflagged counts, in one corr_xengine call -> integrate.
    Prints one JSON line."""
    import torch
    import paper_0910_1517_amd as corr
    import synth
    from paper_0910_1517_amd.flagger import init_params
    S, N, T = 64, 8192, 8192
    C = N // 2
    torch.cuda.set_device(0)
    geo = synth.make_geometry(S // 2, seed=synth.BASE_SEED + 5)
    rs = (N * T + 16 + 255) // 256 * 256
    log("generating %d x %d int8 samples on the GPU" % (S, rs))
    x = synth.voltages_device(S, N * T + 16, geo, seed=synth.BASE_SEED + 5, tone_bin=37, tone_N=N, row_stride=rs)
    g = corr.geom_to_device(corr.geom_array(geo.D, geo.f, geo.psi0, geo.rate))
    # the 1 GiB read + 1 GiB write copy that scales a profiled run's HBM byte counters
    src = x.view(-1)[: 1 << 30].view(torch.int32)
    torch.neg(src, out=torch.empty_like(src))
    del src
    scale = calibrate_scales(corr, torch, S, N, T, x, rs, g)
    # power cells in FP16 (|X|^2 / N^2): half the bytes of FP32 for the F-engine to write and the CNN to read
    plan = corr.Plan(S, N, T, precision=corr.INT8, scale_mode=corr.SCALE_HOLD, power_fp16=1)
    spec = plan.alloc("spectra", zero=False)
    power = plan.alloc("power", zero=False).view(S, T, C)
    flags = plan.alloc("flags", zero=False).view(S, T, C)
    keep = plan.alloc("keep", zero=False)
    acc, state, vis = plan.alloc("acc"), plan.alloc("state"), plan.alloc("vis")
    counts = torch.zeros(C * plan.P, dtype=torch.int32, device="cuda")
    params = torch.from_numpy(init_params(1)).cuda()
    st = torch.cuda.current_stream()
    names = ["fengine", "cnn_infer", "keep_bits", "xengine_masked_with_counts", "integrate"]

    def step(e=None):
        if e: e[0].record(st)
        plan.fengine(x, g, spec, scale, power=power, row_stride=rs, stream=st)
        if e: e[1].record(st)
        corr.cnn_infer(params, power, flags, threshold=0.5, guard=3.0, stream=st)
        if e: e[2].record(st)
        plan.apply_flags(flags, None, keep, stream=st)  # keep words only: the X-engine applies them
        if e: e[3].record(st)
        plan.xengine(spec, acc, keep=keep, counts=counts, stream=st)
        if e: e[4].record(st)
        plan.integrate(acc, state, vis, scale, flags=corr.DUMP | corr.RESET, stream=st)
        if e: e[5].record(st)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(args.steps)]
    for e in ev:
        step(e)
    torch.cuda.synchronize()
    plan.check_device_errors()
    t = {n: float(np.median([e[i].elapsed_time(e[i + 1]) for e in ev])) * 1e-3 for i, n in enumerate(names)}
    # the MAD flagger on the same power (the fallback and the network's teacher), timed apart
    mad = plan.alloc("flags", zero=False)
    em = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(3)]
    plan.mad_flag(power, mad, 3.0, stream=st)
    for e0, e1 in em:
        e0.record(st)
        plan.mad_flag(power, mad, 3.0, stream=st)
        e1.record(st)
    torch.cuda.synchronize()
    t_mad = float(np.median([e0.elapsed_time(e1) for e0, e1 in em])) * 1e-3
    t_step = float(np.median([e[0].elapsed_time(e[5]) for e in ev])) * 1e-3
    cells = S * T * C
    cnn_flops = float(cells) * CNN_FLOP_PER_CELL
    ach = cnn_flops / t["cnn_infer"] / 1e12
    xops, _ = x_algorithmic(S, N, T, 2)
    out = {
        "metric": "correlated bandwidth (MHz) with learned RFI flagging, 64 signals",
        "value": round(N * T / (2 * t_step) / 1e6, 3), "unit": "MHz", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(t_step * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int8 (X) / fp16 (CNN)",
        "data": "synthetic (seeded Gaussian + common source + tone, generated on the GPU); "
                "CNN weights He-normal random (the kernel's time does not depend on them)",
        "config": {"workload": "64 signals, 8192-pt FFT (4096 ch), 8192 spectra, int8 X-engine, "
                               "learned flagger with the MAD column guard on %d FP16 power cells (%d tiles of 64 x 256)"
                               % (cells, cells // 16384),
                   "parallelism": "single GPU"},
        "ms": {n: round(v * 1e3, 4) for n, v in t.items()},
        "mad_flag_ms": round(t_mad * 1e3, 4),
        "x_engine_tops_with_counts": round(xops / t["xengine_masked_with_counts"] / 1e12, 3),
        "roofline": {"kernel": "cnn_infer_kernel<_Float16> (fused 3-layer conv, FP16 MFMA, column guard)", "bound": "mfma",
                     "achieved": round(ach, 3), "peak": FP16_MFMA_PEAK / 1e12, "unit": "TFLOP/s",
                     "frac": round(ach * 1e12 / FP16_MFMA_PEAK, 4), "traffic": measured_traffic("cnn_infer_c5"),
                     "algorithmic_flop_per_cell": CNN_FLOP_PER_CELL},
    }
    print(json.dumps(out), flush=True)


def bench_beamformer(corr, torch, S, N, T, x_dev, rs, g_dev, scale, steps, warmup):
    """B-engine on the int8 spectra of one F-engine call: one incoherent beam and
    one full-polar coherent beam at the raw FFT time resolution (the paper's
    beamformer outputs).  Returns (ms per call, algorithmic bytes per call)."""
    C = N // 2
    plan = corr.Plan(S, N, T, precision=corr.INT8, scale_mode=corr.SCALE_HOLD)
    spec = plan.alloc("spectra", zero=False)
    plan.fengine(x_dev, g_dev, spec, scale, row_stride=rs)
    w = torch.ones(S, device="cuda")
    ph = torch.rand(S, device="cuda", generator=torch.Generator(device="cuda").manual_seed(7)) * 6.283185
    c = torch.stack([torch.cos(ph), torch.sin(ph)], -1).view(1, S, 2).contiguous()
    inc = torch.empty(2, T, C, device="cuda")
    coh = torch.empty(1, 4, T, C, device="cuda")
    f = lambda: plan.beamform(spec, scale, w, inc, c, coh, mode=corr.BEAM_FULLPOL, tint=1)
    for _ in range(warmup):
        f()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        f()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    nbytes = S * C * T * 2 + S * C * 4 + (2 + 4) * T * C * 4
    del spec, inc, coh, plan
    torch.cuda.empty_cache()
    return ms, nbytes


def bench_blanker(corr, torch, synth, S, n, x_dev, geo, steps, warmup, block=16384, M=3.0, table_len=1 << 16):
    """Time-domain MAD voltage blanker on the F-engine's input rows (S rows of
    n samples) after adding impulsive bursts to about 2.5 % of the samples
    (on a copy; x_dev is left as it is).  Out of place (reads and writes every
    sample: 2 bytes per sample) back to back; in place (reads every sample,
    writes back only the 16-byte chunks holding a blanked one) on a fresh copy
    per call, the copy outside the timed events.  Returns a dict."""
    x_rfi = x_dev.clone()
    synth.add_impulses(x_rfi, geo, n, seed=synth.BASE_SEED + 3)
    table = torch.empty(S, table_len, device="cuda")
    corr.blank_noise_table(0x5EED, table)
    nb = -(-n // block)
    counts = torch.zeros(S, nb, dtype=torch.int32, device="cuda")
    y = torch.empty_like(x_rfi)
    f = lambda: corr.blank_voltages(x_rfi, table, block=block, M=M, out=y, n=n)
    for _ in range(warmup):
        f()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        f()
    e1.record()
    torch.cuda.synchronize()
    ms_out = e0.elapsed_time(e1) / steps
    ms_in = []
    for i in range(max(2, steps // 4)):
        y.copy_(x_rfi)
        e0.record()
        corr.blank_voltages(y, table, block=block, M=M, counts=counts, n=n)
        e1.record()
        torch.cuda.synchronize()
        ms_in.append(e0.elapsed_time(e1))
    frac = counts.sum().item() / (S * n)
    del x_rfi, y, table, counts
    torch.cuda.empty_cache()
    return {"ms_out_of_place": ms_out, "ms_in_place": float(np.median(ms_in[1:])), "blanked_fraction": frac,
            "bytes_out_of_place": 2.0 * S * n, "bytes_read": 1.0 * S * n}


def bench_gated(corr, torch, S, N, T, x_dev, rs, g_dev, scale, steps, warmup, period=1.5578e-3):
    """Gated int8 X-engine on the spectra of one F-engine call: two gates (the
    on and off halves of a pulsar period of 1.5578 ms, about 25 spectra), one
    launch.  Each timed call is bracketed by its own events; both gates are
    integrated (and their accumulators zeroed) outside them.  Returns ms per
    call."""
    plan = corr.Plan(S, N, T, precision=corr.INT8, scale_mode=corr.SCALE_HOLD)
    spec = plan.alloc("spectra", zero=False)
    plan.fengine(x_dev, g_dev, spec, scale, row_stride=rs)
    gate, _ = corr.pulsar_gates(0, T, N, FS, 0.0, period, 2)
    gate_d = torch.from_numpy(gate).cuda()
    words = plan.acc_bytes // 4
    acc = torch.zeros(2 * words, dtype=torch.int32, device="cuda")
    states = [plan.alloc("state") for _ in range(2)]
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for i in range(warmup + steps):
        if i >= warmup:
            ev[i - warmup][0].record()
        plan.xengine_gated(spec, gate_d, 2, acc)
        if i >= warmup:
            ev[i - warmup][1].record()
        for b in range(2):
            plan.integrate(acc[b * words:(b + 1) * words], states[b], None, scale, flags=0)
    torch.cuda.synchronize()
    ms = float(np.median([a.elapsed_time(b) for a, b in ev]))
    del spec, acc, states, plan
    torch.cuda.empty_cache()
    return ms


def bench_table_phase(corr, torch, S, N, T, x_dev, rs, g_dev, scale, steps, warmup):
    """The int8 F-engine with the phase from the 1440-step table of section
    2.3.2 instead of direct sincos, same input and scales.  Returns ms per
    call."""
    plan = corr.Plan(S, N, T, precision=corr.INT8, scale_mode=corr.SCALE_HOLD, phase_lut=1)
    spec = plan.alloc("spectra", zero=False)
    f = lambda: plan.fengine(x_dev, g_dev, spec, scale, row_stride=rs)
    for _ in range(warmup):
        f()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        f()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    name = plan.fengine_kernel
    del spec, plan
    torch.cuda.empty_cache()
    return ms, name


def bench_dedisperse(corr, torch, N, T, steps, warmup, dm=71.0, nu0=325e6, n_int=1024):
    """Coherent dedispersion of one beam's two polarisations of channel
    voltages, the shape of one block of the step (T spectra x N/2 channels:
    L = T N/2 complex samples per polarisation, T N / FS seconds): DM 71 pc
    cm^-3 at 325 MHz, as for the paper's B1937+21, whose sweep across the band
    fits in the block.  Random voltages (the cost does not depend on them).
    Returns (ms per call, HBM bytes of its passes, block seconds, valid
    fraction)."""
    import math
    C = N // 2
    L = T * C
    g = torch.Generator(device="cuda").manual_seed(5)
    v = torch.randn(2, T, C, dtype=torch.complex64, device="cuda", generator=g)
    work = torch.empty(2, L, dtype=torch.complex64, device="cuda")
    out = torch.empty(L // n_int, dtype=torch.float32, device="cuda")
    f = lambda: corr.dedisperse(v, sample_rate=FS, nu0=nu0, dm=dm, n_int=n_int, work=work, out=out)
    for _ in range(warmup):
        f()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        f()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    npass = math.ceil(math.log2(L) / 8)
    # read + write each: the inverse DFT per spectrum, the forward passes but
    # the last, the last forward pass fused with the chirp and the first
    # inverse pass, the other inverse passes; the detection reads once
    nbytes = 2.0 * L * 8 * (2 * (1 + (npass - 1) + 1 + (npass - 1)) + 1)
    sweep = 4.148808e15 * dm * (nu0 ** -2 - (nu0 + FS / 2) ** -2) * FS / 2
    del v, work, out
    torch.cuda.empty_cache()
    return ms, nbytes, L / (FS / 2), 1.0 - sweep / L


def bench_adc(corr, torch, S, n, steps, warmup):
    """Demultiplex and unpack S / 4 acquisition-card streams of n time samples
    into the F-engine's S int8 rows, in the 4-bit (33 MHz) and the 8-bit
    (16 MHz) mode.  Returns {bits: (ms per call, algorithmic bytes)}."""
    cards = S // 4
    rs = (n + 255) // 256 * 256
    x = torch.empty(S, rs, dtype=torch.int8, device="cuda")
    out = {}
    for bits in (4, 8):
        rrs = (n * bits // 2 + 255) // 256 * 256
        g = torch.Generator(device="cuda").manual_seed(bits)
        raw = torch.randint(0, 256, (cards, rrs), dtype=torch.uint8, device="cuda", generator=g)
        f = lambda: corr.adc_unpack(raw, x, bits=bits, n=n)
        for _ in range(warmup):
            f()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            f()
        e1.record()
        torch.cuda.synchronize()
        out[bits] = (e0.elapsed_time(e1) / steps, float(cards) * n * bits / 2 + float(S) * n)
        del raw
    del x
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c3", choices=sorted(CONFIGS) + ["c4", "c5"])
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-fp8", action="store_true")
    ap.add_argument("--no-legs", action="store_true", help="skip the legs beside the step (beams, blanker, ...)")
    ap.add_argument("--streamed", action="store_true",
                    help="also time blocks streamed (F of block i+1 beside X of block i) and report that as the value")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=None,
                    help="spectra in the all-core CPU-oracle sample (default 2048 for c3, 8192 for c2)")
    ap.add_argument("--cpu-sample-1t", type=int, default=None,
                    help="spectra in the one-thread CPU-oracle sample (default 128 for c3, 512 for c2)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    if args.config == "c4":
        return bench_batch(args)
    if args.config == "c5":
        return bench_rfi(args)
    import torch
    import paper_0910_1517_amd as corr
    import synth

    S, N, T, desc = CONFIGS[args.config]
    gmrt = args.config == "c2"  # FP32 form with 8 point sources; c3 is the int8 precision form
    C = N // 2
    torch.cuda.set_device(0)
    geo = synth.make_geometry(S // 2, seed=synth.BASE_SEED + 2)
    rs = (N * T + 16 + 255) // 256 * 256
    log("generating %d x %d int8 samples on the GPU" % (S, rs))
    if gmrt:
        src = synth.point_sources(S, 8, 0.3, seed=synth.BASE_SEED + 2)
        x_dev = synth.voltages_device_physical(S, N * T + 16, geo, FS, seed=synth.BASE_SEED + 2, sources=src,
                                               tone_bin=37, tone_N=N, row_stride=rs)
    else:
        x_dev = synth.voltages_device(S, N * T + 16, geo, seed=synth.BASE_SEED + 2, tone_bin=37, tone_N=N,
                                      row_stride=rs)
    g_dev = corr.geom_to_device(corr.geom_array(geo.D, geo.f, geo.psi0, geo.rate))
    # a plain elementwise copy of known size (reads 1 GiB, writes 1 GiB; its kernel
    # is named neg_kernel), outside the timed region: the reference that scales
    # the HBM byte counters of a profiled run
    src_c = x_dev.view(-1)[: 1 << 30].view(torch.int32)
    torch.neg(src_c, out=torch.empty_like(src_c))
    del src_c
    torch.cuda.synchronize()

    log("calibrating int8 scales")
    scale = calibrate_scales(corr, torch, S, N, T, x_dev, rs, g_dev)
    log("timing int8 path: %d warmup + %d steps (eager, then graph replays)" % (args.warmup, args.steps))
    r8 = run_path(corr, torch, corr.INT8, S, N, T, x_dev, rs, g_dev, args.steps, args.warmup, scale)
    log("int8: step %.3f ms (F %.3f, X %.3f, int %.3f; eager step %.3f)" % (
        r8["t_step"] * 1e3, r8["t_f"] * 1e3, r8["t_x"] * 1e3, r8["t_int"] * 1e3, r8["t_eager_step"] * 1e3))
    t8 = r8["t_step"]
    if args.streamed:
        torch.cuda.empty_cache()
        t8 = run_pipelined(corr, torch, corr.INT8, S, N, T, x_dev, rs, g_dev, args.steps, args.warmup, scale)
        log("int8 streamed (F of block i+1 beside X of block i): %.3f ms per block" % (t8 * 1e3))
    legs = not (args.no_legs or gmrt)
    if legs:
        torch.cuda.empty_cache()
        log("timing the beamformer (one incoherent + one full-polar coherent beam)")
        tb_ms, tb_bytes = bench_beamformer(corr, torch, S, N, T, x_dev, rs, g_dev, scale, args.steps, args.warmup)
        log("beamformer: %.3f ms per call" % tb_ms)
        torch.cuda.empty_cache()
        log("timing the voltage blanker (blocks of 16384 samples, M = 3, impulsive bursts on a copy of the input)")
        rb = bench_blanker(corr, torch, synth, S, N * T + 16, x_dev, geo, args.steps, args.warmup)
        log("blanker: %.3f ms out of place, %.3f ms in place, %.4f of the samples blanked"
            % (rb["ms_out_of_place"], rb["ms_in_place"], rb["blanked_fraction"]))
        log("timing the gated X-engine (two pulse-phase gates)")
        tg_ms = bench_gated(corr, torch, S, N, T, x_dev, rs, g_dev, scale, args.steps, args.warmup)
        log("gated X-engine: %.3f ms per call (ungated %.3f ms)" % (tg_ms, r8["t_x"] * 1e3))
        log("timing the int8 F-engine with the 1440-step phase table")
        tt_ms, tt_name = bench_table_phase(corr, torch, S, N, T, x_dev, rs, g_dev, scale, args.steps, args.warmup)
        log("table-phase F-engine: %.3f ms (direct sincos %.3f ms)" % (tt_ms, r8["t_f"] * 1e3))
        log("timing coherent dedispersion of one beam (DM 71 at 325 MHz)")
        rd = bench_dedisperse(corr, torch, N, T, max(2, args.steps // 2), min(1, args.warmup))
        log("dedispersion: %.3f ms per %.2f s block (%.0fx real time)" % (rd[0], rd[2], rd[2] / (rd[0] * 1e-3)))
        log("timing the ADC demultiplexing and unpacking (4-bit and 8-bit card streams)")
        ra = bench_adc(corr, torch, S, N * T + 16, args.steps, args.warmup)
        log("adc unpack: %.3f ms (4-bit), %.3f ms (8-bit)" % (ra[4][0], ra[8][0]))
    r8f = None
    if not args.no_fp8 and not gmrt:
        torch.cuda.empty_cache()
        log("timing fp8 (e4m3) path")
        scale8 = calibrate_scales(corr, torch, S, N, T, x_dev, rs, g_dev, corr.FP8_E4M3)
        r8f = run_path(corr, torch, corr.FP8_E4M3, S, N, T, x_dev, rs, g_dev, max(3, args.steps // 2),
                       min(2, args.warmup), scale8)
        log("fp8: step %.3f ms (F %.3f, X %.3f, int %.3f)" % (r8f["t_step"] * 1e3, r8f["t_f"] * 1e3,
                                                             r8f["t_x"] * 1e3, r8f["t_int"] * 1e3))
        del scale8
    r32 = None
    t32 = None
    if gmrt or not args.no_fp32:
        torch.cuda.empty_cache()
        n32 = args.steps if gmrt else max(3, args.steps // 4)
        log("timing fp32 path")
        r32 = run_path(corr, torch, corr.FP32, S, N, T, x_dev, rs, g_dev, n32, args.warmup)
        log("fp32: step %.3f ms (F %.3f, X %.3f, int %.3f)" % (r32["t_step"] * 1e3, r32["t_f"] * 1e3,
                                                              r32["t_x"] * 1e3, r32["t_int"] * 1e3))
        t32 = r32["t_step"]
        if args.streamed:
            torch.cuda.empty_cache()
            t32 = run_pipelined(corr, torch, corr.FP32, S, N, T, x_dev, rs, g_dev, max(3, args.steps // 4),
                                min(2, args.warmup))
            log("fp32 streamed: %.3f ms per block" % (t32 * 1e3))

    bw = lambda t: N * T / (2.0 * t) / 1e6  # correlated bandwidth, MHz
    xops8, xin8 = x_algorithmic(S, N, T, 2)
    xops32, xin32 = x_algorithmic(S, N, T, 8)
    ff8, fb8 = f_algorithmic(S, N, T, 2)
    ff32, fb32 = f_algorithmic(S, N, T, 8)
    head, t_head = (r32, t32) if gmrt else (r8, t8)
    out = {
        "metric": "correlated bandwidth (MHz) & X-engine TOP/s, 64 signals: int8-MFMA vs FP32",
        "value": round(bw(t_head), 3),
        "unit": "MHz",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_head * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if gmrt else "int8",
        "data": ("synthetic (seeded physical recipe on the GPU: fractional delays, fringe rotation, 8 point "
                 "sources + noise + tone)" if gmrt else
                 "synthetic (seeded Gaussian + common source + tone, generated on the GPU)"),
        "config": {"workload": desc, "signals": S, "fft_len": N, "channels": C, "spectra": T,
                   "pairs": S * (S + 1) // 2, "sample_rate_hz": FS, "parallelism": "single GPU"},
        "step_mode": ("streamed: F-engine of block i+1 beside X-engine + integrate of block i (two streams, "
                      "two spectra buffers)" if args.streamed else
                      "one HIP graph replay of F-engine, X-engine, integrate (median of the timed replays; "
                      "per-kernel times: median of eager steps)"),
        "int8": {"correlated_bandwidth_mhz": round(bw(t8), 3),
                 "x_engine_tops": round(xops8 / r8["t_x"] / 1e12, 3),
                 "ms": {k: round(v * 1e3, 4) for k, v in r8.items() if k.startswith("t_")},
                 "x_splits": r8["splits"], "graph_matches_eager": r8.get("graph_matches_eager")},
    }

    def f_roof(tf, fflops, fbytes, kernel):
        # HBM-bound by the algorithmic bytes (N int8 in, C channels x code size out per spectrum);
        # the FP32 vector fraction beside it against both the non-packed issue rate (this library
        # never emits packed FP32) and the published 157.3 TF
        return {"kernel": kernel, "bound": "hbm", "achieved": round(fbytes / tf / 1e9, 1), "peak": HBM_PEAK / 1e9,
                "unit": "GB/s", "frac": round(fbytes / tf / HBM_PEAK, 4), "algorithmic_bytes": fbytes,
                "valu_tflops": round(fflops / tf / 1e12, 3),
                "valu_frac_nonpacked_78.6TF": round(fflops / tf / FP32_VALU_PEAK, 4),
                "valu_frac_published_157.3TF": round(fflops / tf / FP32_PUBLISHED_PEAK, 4)}

    if gmrt:
        tf, tx = r32["t_f"], r32["t_x"]
        f_part = f_roof(tf, ff32, fb32, "%s (FP32 F-engine)" % r32["fkernel"])
        x_part = {"kernel": "xengine_kernel<2, 0> (FP32 MFMA X-engine)", "bound": "mfma",
                  "achieved": round(xops32 / tx / 1e12, 3), "peak": FP32_MFMA_PEAK / 1e12, "unit": "TFLOP/s",
                  "frac": round(xops32 / tx / FP32_MFMA_PEAK, 4), "hbm_gbs": round(xin32 / tx / 1e9, 1)}
        dom = f_part if tf >= tx else x_part
        traffic = measured_traffic("fengine_fp32_c2") if tf >= tx else None
    else:
        tf, tx = r8["t_f"], r8["t_x"]
        f_part = f_roof(tf, ff8, fb8, "%s (int8 F-engine)" % r8["fkernel"])
        x_part = {"kernel": "xengine_kernel<2, 1> (int8 MFMA X-engine)", "bound": "hbm",
                  "achieved": round(xin8 / tx / 1e9, 1), "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                  "frac": round(xin8 / tx / HBM_PEAK, 4), "mfma_frac_algorithmic": round(xops8 / tx / INT8_PEAK, 4)}
        dom = f_part if tf >= tx else x_part
        traffic = measured_traffic("fengine_int8_%s" % args.config) if tf >= tx else None
    out["roofline"] = {k: dom[k] for k in ("kernel", "bound", "achieved", "peak", "unit", "frac")}
    out["roofline"]["traffic"] = traffic
    out["roofline"]["f_engine"] = f_part
    out["roofline"]["x_engine"] = x_part
    if legs:
        out["beamformer"] = {"kernel": "beam_kernel<int8, 1 beam> (B-engine)", "bound": "hbm",
                             "beams": "1 incoherent (2 pol) + 1 coherent full-polar (4 products), tint 1",
                             "ms": round(tb_ms, 4), "achieved_gbs": round(tb_bytes / tb_ms / 1e6, 1),
                             "hbm_frac": round(tb_bytes / tb_ms / 1e6 / (HBM_PEAK / 1e9), 4),
                             "algorithmic_bytes": tb_bytes,
                             "traffic": measured_traffic("beam_int8_%s" % args.config)}
        gbs = rb["bytes_out_of_place"] / rb["ms_out_of_place"] / 1e6
        out["voltage_blanker"] = {
            "kernel": "blank_kernel<4> (MAD blanker, blocks of 16384 samples)", "bound": "hbm",
            "input": "the int8 input rows with impulsive bursts added to about 2.5 % of the samples",
            "blanked_fraction": round(rb["blanked_fraction"], 5),
            "ms_out_of_place": round(rb["ms_out_of_place"], 4), "achieved_gbs": round(gbs, 1),
            "hbm_frac": round(gbs / (HBM_PEAK / 1e9), 4), "algorithmic_bytes": rb["bytes_out_of_place"],
            "traffic": measured_traffic("blank_out_%s" % args.config),
            "ms_in_place": round(rb["ms_in_place"], 4),
            "in_place_read_gbs": round(rb["bytes_read"] / rb["ms_in_place"] / 1e6, 1),
            "traffic_in_place": measured_traffic("blank_in_%s" % args.config),
            "share_of_step": round(rb["ms_in_place"] / (t8 * 1e3), 4)}
        out["gated_xengine"] = {
            "kernel": "xengine_gated_kernel<2, int8> (two pulse-phase gates, one launch)", "bound": "hbm",
            "ms": round(tg_ms, 4), "ungated_ms": round(r8["t_x"] * 1e3, 4),
            "achieved_gbs": round(xin8 / (tg_ms * 1e-3) / 1e9, 1),
            "hbm_frac": round(xin8 / (tg_ms * 1e-3) / HBM_PEAK, 4),
            "mfma_frac_issued": round(2 * xops8 / (tg_ms * 1e-3) / INT8_PEAK, 4)}
        out["table_phase_fengine"] = {
            "kernel": "%s (int8, phase from the 1440-step table)" % tt_name, "bound": "hbm",
            "ms": round(tt_ms, 4), "direct_sincos_ms": round(r8["t_f"] * 1e3, 4),
            "hbm_frac": round(fb8 / (tt_ms * 1e-3) / HBM_PEAK, 4)}
        out["coherent_dedispersion"] = {
            "kernel": "dd_fft_kernel<log2R> passes + chirp + detection (one beam, two polarisations)", "bound": "hbm",
            "block": "%d spectra x %d channels = 2^%d complex samples per polarisation" % (T, N // 2, int(np.log2(T * N // 2))),
            "dm": 71.0, "nu0_hz": 325e6, "ms": round(rd[0], 4), "block_seconds": round(rd[2], 4),
            "real_time_factor": round(rd[2] / (rd[0] * 1e-3), 1), "valid_fraction": round(rd[3], 4),
            "pass_bytes": rd[1], "achieved_gbs": round(rd[1] / rd[0] / 1e6, 1),
            "hbm_frac": round(rd[1] / rd[0] / 1e6 / (HBM_PEAK / 1e9), 4)}
        out["adc_unpack"] = {
            "kernel": "adc_unpack_kernel<bits> (4-input demultiplexing, 4-bit to 8-bit)", "bound": "hbm",
            "cards": S // 4,
            **{"bits%d" % b: {"ms": round(ra[b][0], 4), "algorithmic_bytes": ra[b][1],
                               "achieved_gbs": round(ra[b][1] / ra[b][0] / 1e6, 1),
                               "hbm_frac": round(ra[b][1] / ra[b][0] / 1e6 / (HBM_PEAK / 1e9), 4)} for b in (4, 8)}}
    if r32:
        out["fp32"] = {"correlated_bandwidth_mhz": round(bw(t32), 3), "ms_per_step": round(t32 * 1e3, 4),
                       "x_engine_tops": round(xops32 / r32["t_x"] / 1e12, 3),
                       "ms": {k: round(v * 1e3, 4) for k, v in r32.items() if k.startswith("t_")},
                       "x_mfma_frac_algorithmic": round(xops32 / r32["t_x"] / FP32_MFMA_PEAK, 4),
                       "x_splits": r32["splits"], "graph_matches_eager": r32.get("graph_matches_eager")}
        out["int8_vs_fp32_speedup"] = round(t32 / t8, 3)
    if r8f:
        out["fp8_e4m3"] = {"correlated_bandwidth_mhz": round(bw(r8f["t_step"]), 3),
                           "ms_per_step": round(r8f["t_step"] * 1e3, 4),
                           "x_engine_tops": round(xops8 / r8f["t_x"] / 1e12, 3),
                           "ms": {k: round(v * 1e3, 4) for k, v in r8f.items() if k.startswith("t_")},
                           "x_hbm_frac": round(xin8 / r8f["t_x"] / HBM_PEAK, 4),
                           "x_splits": r8f["splits"]}
    if not args.no_cpu_baseline:
        prec = "fp32" if gmrt else "int8"
        args.cpu_sample = args.cpu_sample or (8192 if gmrt else 2048)
        args.cpu_sample_1t = args.cpu_sample_1t or (512 if gmrt else 128)
        log("cpu baseline: oracle (%s path) on %d spectra at all cores and %d at one thread"
            % (prec, args.cpu_sample, args.cpu_sample_1t))
        out["cpu_baseline"] = cpu_baseline_record(S, N, prec, args.cpu_sample, args.cpu_sample_1t)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
