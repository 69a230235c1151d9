"""Parity at the full benchmark sizes, in the launch configurations bench.py
times, on outputs the oracle can compute one by one: a few sampled channels
(direct DFT per channel in FP64, then the pair products) or a few sampled
flagging tiles.  Inputs come from the seeded generators only (generated on the
GPU where they are many GB, and copied back for the oracle).
"""
import numpy as np
import pytest

import oracle
import paper_0910_1517_amd as corr
import synth
from gpu_util import FS, beam_bounds, check_beams, near_threshold_cells

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def ogeom(g):
    return oracle.Geometry(g.D, g.f, g.psi0, g.rate)


def workload(S, N, T, seed):
    """The benchmark's input: bulk recipe on the GPU, tone at bin 37."""
    geo = synth.make_geometry(S // 2, seed=seed)
    rs = (N * T + 16 + 255) // 256 * 256
    x = synth.voltages_device(S, N * T + 16, geo, seed=seed, tone_bin=37, tone_N=N, row_stride=rs)
    g = corr.geom_to_device(corr.geom_array(geo.D, geo.f, geo.psi0, geo.rate))
    return geo, x, rs, g


def state_channels(state, C, P, chans):
    st = state.view(C, P, 2)[list(chans)].cpu().numpy()
    return st[..., 0] + 1j * st[..., 1]


def int8_channels(spec, S, C, T, chans):
    """[S][T][len(chans)][2] int8 codes of the listed channels, read from the X layout on the device."""
    import torch
    v = spec.view(T // 8, C // 8, S, 8, 2, 8)
    out = [v[:, k // 8, :, k % 8].permute(1, 0, 3, 2).reshape(S, T, 2) for k in chans]
    return torch.stack(out, 2).cpu().numpy().view(np.int8)


def test_gmrt_scale_fp32_sampled_channels():
    """64 signals, 1024-pt, 16384 spectra, FP32 F + X + integrate: e_max <= 1e-5."""
    S, N, T = 64, 1024, 16384
    C = N // 2
    geo, x, rs, g = workload(S, N, T, synth.BASE_SEED + 1)
    plan = corr.Plan(S, N, T, precision=corr.FP32)
    spec = plan.alloc("spectra", zero=False)
    acc, state, vis = plan.alloc("acc"), plan.alloc("state"), plan.alloc("vis")
    plan.fengine(x, g, spec, row_stride=rs)
    plan.xengine(spec, acc)
    plan.integrate(acc, state, vis, flags=corr.DUMP)
    plan.check_device_errors()
    chans = [0, 37, 300, 511]
    V = state_channels(state, C, plan.P, chans)
    xh = x.cpu().numpy()
    V64 = oracle.xengine(oracle.fengine_channels(xh, N, T, ogeom(geo), FS, chans))
    e_max, e_fro = oracle.normalized_error(V, V64, S)
    print("c2 sampled channels: e_max %.3g e_fro %.3g" % (e_max, e_fro))
    assert e_max <= 1e-5


def test_gmrt_scale_point_sources_fp32_sampled_channels():
    """The GMRT-scale form as specified: 64 signals drawn from the physical recipe
    (fractional delays, fringe rotation) with 8 random coherent point sources --
    source 0 at the phase centre, the others with extra per-antenna delays and
    fringe rates -- 1024-pt FFT, 16384 spectra, FP32 F + X + integrate: sampled
    channels against the FP64 oracle at e_max <= 1e-5."""
    S, N, T = 64, 1024, 16384
    C = N // 2
    seed = synth.BASE_SEED + 1
    geo = synth.make_geometry(S // 2, seed=seed)
    src = synth.point_sources(S, 8, 0.3, seed=seed)
    rs = (N * T + 16 + 255) // 256 * 256
    x = synth.voltages_device_physical(S, N * T + 16, geo, FS, seed=seed, sources=src, tone_bin=37, tone_N=N,
                                       row_stride=rs)
    g = corr.geom_to_device(corr.geom_array(geo.D, geo.f, geo.psi0, geo.rate))
    plan = corr.Plan(S, N, T, precision=corr.FP32)
    spec = plan.alloc("spectra", zero=False)
    acc, state, vis = plan.alloc("acc"), plan.alloc("state"), plan.alloc("vis")
    plan.fengine(x, g, spec, row_stride=rs)
    plan.xengine(spec, acc)
    plan.integrate(acc, state, vis, flags=corr.DUMP)
    plan.check_device_errors()
    chans = [1, 37, 260, 510]
    V = state_channels(state, C, plan.P, chans)
    xh = x.cpu().numpy()
    V64 = oracle.xengine(oracle.fengine_channels(xh, N, T, ogeom(geo), FS, chans))
    e_max, e_fro = oracle.normalized_error(V, V64, S)
    print("c2 with 8 point sources, sampled channels: e_max %.3g e_fro %.3g" % (e_max, e_fro))
    assert e_max <= 1e-5
    # the sources are there: same-polarisation cross coherence well above the noise
    # level sqrt(1/T) ~ 0.008 on average, cross-polarisation coherence at it (channel 37,
    # where the tone common to both polarisations dominates, left out)
    sel = [0, 2, 3]
    auto = lambda i: V64[sel, oracle.pair_index(i, i)].real
    coh = lambda i, j: np.abs(V64[sel, oracle.pair_index(i, j)]) / np.sqrt(auto(i) * auto(j))
    same = np.mean([coh(i, j) for i in range(0, 16, 2) for j in range(i + 2, 16, 2)])
    cross = np.mean([coh(i, i + 1) for i in range(0, 16, 2)])
    print("c2 mean coherence: same pol %.4f, cross pol %.4f" % (same, cross))
    assert same > 0.03 and cross < 0.02


def test_precision_form_int8_sampled_channels():
    """64 signals, 4096-pt, 32768 spectra, int8 with held scales (calibration
    pass first, as the benchmark does): quantiser codes and visibilities of
    sampled channels against the FP64 oracle; then the FP8 (e4m3) variant's
    visibilities."""
    import torch
    S, N, T = 64, 4096, 32768
    C = N // 2
    geo, x, rs, g = workload(S, N, T, synth.BASE_SEED + 2)
    chans = [37, 1500]
    xh = x.cpu().numpy()
    Y = oracle.fengine_channels(xh, N, T, ogeom(geo), FS, chans)
    del xh
    oscale = oracle.int8_scale(oracle.sigma(Y))  # [S][len(chans)]
    # calibration pass on the GPU, then the oracle's scales for the sampled channels
    cal = corr.Plan(S, N, T, precision=corr.INT8, scale_mode=corr.SCALE_COMPUTE)
    scale = torch.zeros(S * C, dtype=torch.float32, device="cuda")
    tmp = cal.alloc("spectra", zero=False)
    cal.fengine(x, g, tmp, scale, row_stride=rs)
    torch.cuda.synchronize()
    del tmp, cal
    sg = scale.view(S, C)
    assert np.max(np.abs(sg[:, chans].cpu().numpy() / oscale - 1)) < 1e-5
    sg[:, chans] = torch.from_numpy(oscale.astype(np.float32)).cuda()
    plan = corr.Plan(S, N, T, precision=corr.INT8, scale_mode=corr.SCALE_HOLD)
    spec = plan.alloc("spectra", zero=False)
    acc, state, vis = plan.alloc("acc"), plan.alloc("state"), plan.alloc("vis")
    plan.fengine(x, g, spec, scale, row_stride=rs)
    plan.xengine(spec, acc)
    plan.integrate(acc, state, vis, scale, flags=corr.DUMP)
    plan.check_device_errors()
    qg = int8_channels(spec, S, C, T, chans).astype(np.int64)
    qo = oracle.quantize_int8(Y, oscale.astype(np.float64)).astype(np.int64)
    u = np.stack([Y.real, Y.imag], -1) / oscale.astype(np.float64)[:, None, :, None]
    frac = np.abs(np.abs(u - np.floor(u)) - 0.5)
    diff = qg - qo
    bad = diff != 0
    print("c3 quantiser mismatches: %d of %d" % (bad.sum(), bad.size))
    assert np.abs(diff).max() <= 1 and np.all(frac[bad] < 1e-3) and bad.mean() <= 1e-4
    V = state_channels(state, C, plan.P, chans)
    V64 = oracle.xengine(Y)
    e_max, e_fro = oracle.normalized_error(V, V64, S)
    print("c3 int8 sampled channels: e_max %.3g e_fro %.3g" % (e_max, e_fro))
    assert e_fro <= 1e-3
    # the FP8 (OCP e4m3) variant of the same form: its own calibration (4 sigma -> 448)
    del spec, acc, state, vis, plan
    torch.cuda.empty_cache()
    cal = corr.Plan(S, N, T, precision=corr.FP8_E4M3, scale_mode=corr.SCALE_COMPUTE)
    scale8 = torch.zeros(S * C, dtype=torch.float32, device="cuda")
    tmp = cal.alloc("spectra", zero=False)
    cal.fengine(x, g, tmp, scale8, row_stride=rs)
    torch.cuda.synchronize()
    del tmp, cal
    plan = corr.Plan(S, N, T, precision=corr.FP8_E4M3, scale_mode=corr.SCALE_HOLD)
    spec = plan.alloc("spectra", zero=False)
    acc, state, vis = plan.alloc("acc"), plan.alloc("state"), plan.alloc("vis")
    plan.fengine(x, g, spec, scale8, row_stride=rs)
    plan.xengine(spec, acc)
    plan.integrate(acc, state, vis, scale8, flags=corr.DUMP)
    plan.check_device_errors()
    e_max8, e_fro8 = oracle.normalized_error(state_channels(state, C, plan.P, chans), V64, S)
    print("c3 fp8 sampled channels: e_max %.3g e_fro %.3g" % (e_max8, e_fro8))
    assert e_fro8 <= 5e-3


def test_beamformer_at_the_precision_form_sampled_channels():
    """Array beams at the precision form's shape (64 signals, 4096-pt, 32768
    spectra, int8 from the F-engine with computed scales) in bench.py's
    configuration: one incoherent beam and one full-polar coherent beam at the
    raw FFT time resolution.  Sampled channels against the oracle on the same
    int8 codes and scales."""
    import torch
    S, N, T = 64, 4096, 32768
    C = N // 2
    geo, x, rs, g = workload(S, N, T, synth.BASE_SEED + 2)
    plan = corr.Plan(S, N, T, precision=corr.INT8, scale_mode=corr.SCALE_COMPUTE)
    scale = torch.zeros(S * C, dtype=torch.float32, device="cuda")
    spec = plan.alloc("spectra", zero=False)
    plan.fengine(x, g, spec, scale, row_stride=rs)
    del x
    rng = np.random.default_rng(5)
    w = rng.uniform(0.5, 1.5, S).astype(np.float32)
    w[9] = 0.0  # one signal left out of the incoherent sum
    c = np.exp(2j * np.pi * rng.uniform(size=S)).astype(np.complex64)  # antenna phases
    inc = torch.empty(2, T, C, device="cuda")
    coh = torch.empty(1, 4, T, C, device="cuda")
    cw = torch.from_numpy(np.stack([c.real, c.imag], -1)[None].copy()).cuda()
    plan.beamform(spec, scale, torch.from_numpy(w).cuda(), inc, cw, coh, mode=corr.BEAM_FULLPOL, tint=1)
    torch.cuda.synchronize()
    chans = [37, 1500]
    q = int8_channels(spec, S, C, T, chans).astype(np.float64)  # [S][T][2 ch][2]
    sc = scale.view(S, C)[:, chans].cpu().numpy().astype(np.float64)
    Y = (q[..., 0] + 1j * q[..., 1]) * sc[:, None, :]
    w64, c64 = w.astype(np.float64), c.astype(np.complex128)[None]
    ref_inc, ref_coh = oracle.beamform(Y, w=w64, c=c64, mode=oracle.BEAM_FULLPOL)
    inc_b, coh_b = beam_bounds(Y, w64, c64, 1)
    got_inc = inc[:, :, chans].cpu().numpy()
    got_coh = coh[:, :, :, chans].cpu().numpy()
    check_beams(got_inc, got_coh, ref_inc, ref_coh, inc_b, coh_b, corr.BEAM_FULLPOL, 1)


def test_voltage_blanker_at_the_fx_input_sampled_blocks():
    """The time-domain blanker on the precision form's input (64 signals x
    (4096 x 32768 + 16) samples) with impulsive bursts on about 2.5 % of the
    samples, in bench.py's configuration (blocks of 16384, M = 3, a 2^16-entry
    table per signal).  Out of place over the whole input, then in place:
    the two results are identical.  Sampled blocks (first, middle, the ragged
    last one) of three rows, their counts and statistics equal the oracle's,
    each block computed on its own."""
    import torch
    S, N, T = 64, 4096, 32768
    B, M, L, seed = 16384, 3.0, 1 << 16, 0x5EED
    geo, x, rs, _ = workload(S, N, T, synth.BASE_SEED + 2)
    n = N * T + 16
    synth.add_impulses(x, geo, n, seed=synth.BASE_SEED + 3)
    nb = -(-n // B)
    rows, blocks = [0, 33, 63], [0, nb // 2, nb - 1]
    before = {(s, b): x[s, b * B:min(n, (b + 1) * B)].cpu().numpy() for s in rows for b in blocks}
    table = torch.empty(S, L, device="cuda")
    corr.blank_noise_table(seed, table)
    y = torch.empty_like(x)
    counts = torch.empty(S, nb, dtype=torch.int32, device="cuda")
    stats = torch.empty(S, nb, 2, dtype=torch.int32, device="cuda")
    corr.blank_voltages(x, table, block=B, M=M, out=y, n=n)
    corr.blank_voltages(x, table, block=B, M=M, counts=counts, stats=stats, n=n)
    torch.cuda.synchronize()
    assert torch.equal(x[:, :n], y[:, :n])
    frac = counts.sum().item() / (S * n)
    print("blanked fraction %.4f" % frac)
    assert 0.01 < frac < 0.05
    ref_table = oracle.blank_noise_table(seed, S, L)
    assert np.array_equal(table.cpu().numpy(), ref_table)
    for s in rows:
        trow = ref_table[s:s + 1]
        for b in blocks:
            xb = before[(s, b)]
            ref, rc, rst = oracle.mad_blank(xb[None], B, M, trow, sample0=b * B)
            got = x[s, b * B:b * B + xb.size].cpu().numpy()
            assert np.array_equal(got, ref[0]), (s, b)
            assert counts[s, b].item() == rc[0, 0] and stats[s, b].tolist() == rst[0, 0].tolist(), (s, b)


def test_adc_unpack_at_the_fx_input_sampled_ranges():
    """4-bit, 33 MHz-mode card streams for the precision form's input: 16
    cards x 4 inputs = 64 rows of 4096 x 32768 + 16 samples, in bench.py's
    configuration.  Sampled ranges of three cards (first, middle, last with
    the row's end) equal the oracle's unpacking of the same raw bytes."""
    import torch
    cards, n = 16, 4096 * 32768 + 16
    rrs = (2 * n + 255) // 256 * 256
    rs = (n + 255) // 256 * 256
    g = torch.Generator(device="cuda").manual_seed(11)
    raw = torch.randint(0, 256, (cards, rrs), dtype=torch.uint8, device="cuda", generator=g)
    x = torch.empty(4 * cards, rs, dtype=torch.int8, device="cuda")
    corr.adc_unpack(raw, x, bits=4, n=n)
    torch.cuda.synchronize()
    for c in (0, 7, 15):
        for t0, t1 in ((0, 4096), (n // 2 - 33, n // 2 + 4000), (n - 4100, n)):
            ref = oracle.adc_unpack(raw[c:c + 1, 2 * t0:2 * t1].cpu().numpy(), t1 - t0, 4)
            assert np.array_equal(x[4 * c:4 * c + 4, t0:t1].cpu().numpy(), ref), (c, t0)


def test_precision_form_int8_xengine_bit_exact_sampled_channels():
    """The int8 X-engine at 64 x 2048 x 32768 in the benchmark's split, on
    seeded int8 codes: sampled channels equal the int64 triple loop exactly."""
    import torch
    S, N, T = 64, 4096, 32768
    C = N // 2
    gen = torch.Generator(device="cuda")
    gen.manual_seed(synth.BASE_SEED + 77)
    q = torch.randint(-127, 128, (S, T, C, 2), generator=gen, device="cuda", dtype=torch.int16).to(torch.int8)
    plan = corr.Plan(S, N, T, precision=corr.INT8)
    spec = plan.alloc("spectra", zero=False)
    plan.xpack(q, spec)
    acc = plan.alloc("acc")
    plan.xengine(spec, acc)
    torch.cuda.synchronize()
    chans = [0, 1027, 2047]
    qh = q[:, :, chans].cpu().numpy()
    a = acc.view(plan.splits, C, plan.P, 2)[:, chans].cpu().numpy().astype(np.int64).sum(0)
    assert np.array_equal(a, oracle.xengine_int(qh))


def test_gated_int8_xengine_bit_exact_sampled_channels():
    """The gated X-engine at 64 x 2048 x 32768 in bench.py's configuration
    (two gates: the halves of a 1.5578 ms pulsar period), on seeded int8
    codes: sampled channels of both gates equal the int64 triple loop over
    each gate's spectra exactly."""
    import torch
    S, N, T = 64, 4096, 32768
    C = N // 2
    gen = torch.Generator(device="cuda")
    gen.manual_seed(synth.BASE_SEED + 78)
    q = torch.randint(-127, 128, (S, T, C, 2), generator=gen, device="cuda", dtype=torch.int16).to(torch.int8)
    plan = corr.Plan(S, N, T, precision=corr.INT8)
    spec = plan.alloc("spectra", zero=False)
    plan.xpack(q, spec)
    gate, counts = corr.pulsar_gates(0, T, N, FS, 0.0, 1.5578e-3, 2)
    acc = torch.zeros(2 * plan.acc_bytes // 4, dtype=torch.int32, device="cuda")
    plan.xengine_gated(spec, torch.from_numpy(gate).cuda(), 2, acc)
    torch.cuda.synchronize()
    chans = [5, 1100, 2046]
    qh = q[:, :, chans].cpu().numpy()
    ref = oracle.xengine_int_gated(qh, gate, 2)
    a = acc.view(2, plan.splits, C, plan.P, 2)[:, :, chans].cpu().numpy().astype(np.int64).sum(1)
    assert np.array_equal(a, ref)
    assert counts.min() > 0.45 * T


def test_coherent_dedispersion_at_the_bench_block():
    """Coherent dedispersion in bench.py's configuration: two polarisations of
    32768 spectra x 2048 channels (2^26 complex samples each, a four-pass
    transform), DM 71 at 325 MHz, 1024 samples per output.  Every output
    against the oracle's FP64 transforms."""
    import torch
    T, C, dm, n_int = 32768, 2048, 71.0, 1024
    g = torch.Generator(device="cuda").manual_seed(5)
    v = torch.randn(2, T, C, dtype=torch.complex64, device="cuda", generator=g)
    out, _ = corr.dedisperse(v, sample_rate=FS, nu0=325e6, dm=dm, n_int=n_int)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    ref = oracle.dedisperse(v.cpu().numpy().astype(np.complex128), FS, 325e6, dm, n_int)
    rms = np.sqrt(np.mean(ref ** 2))
    err = np.abs(got - ref)
    print("dedispersion 2^26: max err %.3g, rms err %.3g of rms" % (err.max() / rms, np.sqrt(np.mean(err ** 2)) / rms))
    assert np.sqrt(np.mean(err ** 2)) <= 2e-5 * rms and err.max() <= 2e-4 * rms


def test_batched_form_sampled_channels():
    """The six uneven sub-arrays in one captured graph (autotuned splits, held
    scales).  For every sub-array's sampled channels the oracle runs its own
    int8 path (its scales, RNE quantisation, int64 products, FP64 scaling):
    the GPU must reproduce those visibilities, and its error against FP64 must
    be the quantisation's own.  int8 requantisation noise averages down as
    T^(-1/2), so the short integrations of this form (1024-2048 spectra) sit
    above the 1e-3 reached at 32768 spectra."""
    import torch
    sub_arrays = [(8, 256, 65536), (16, 512, 32768), (30, 1024, 16384), (48, 2048, 8192), (60, 4096, 2048),
                  (64, 8192, 1024)]
    shapes, data = [], []
    for i, (S, C, T) in enumerate(sub_arrays):
        split, _ = corr.autotune_x_split(S, 2 * C, T, cache=False)
        shapes.append(dict(n_signals=S, fft_len=2 * C, n_spectra=T, x_split=split))
    b = corr.Batch(shapes)
    for i, sh in enumerate(shapes):
        S, N, T = sh["n_signals"], sh["fft_len"], sh["n_spectra"]
        C = N // 2
        geo = synth.make_geometry((S + 1) // 2, seed=synth.BASE_SEED + 10 + i).subset(np.arange(S))
        rs = (N * T + 16 + 255) // 256 * 256
        x = synth.voltages_device(S, N * T + 16, geo, seed=synth.BASE_SEED + 10 + i, row_stride=rs)
        g = corr.geom_to_device(corr.geom_array(geo.D, geo.f, geo.psi0, geo.rate))
        chans = [37, C - 1]
        Y = oracle.fengine_channels(x.cpu().numpy(), N, T, ogeom(geo), FS, chans)
        oscale = oracle.int8_scale(oracle.sigma(Y))
        cal = corr.Plan(S, N, T, precision=corr.INT8, scale_mode=corr.SCALE_COMPUTE)
        scale = torch.zeros(S * C, dtype=torch.float32, device="cuda")
        tmp = cal.alloc("spectra", zero=False)
        cal.fengine(x, g, tmp, scale, row_stride=rs)
        torch.cuda.synchronize()
        del tmp, cal
        scale.view(S, C)[:, chans] = torch.from_numpy(oscale.astype(np.float32)).cuda()
        p = b.plans[i]
        spec = p.alloc("spectra", zero=False)
        acc, state, vis = p.alloc("acc"), p.alloc("state"), p.alloc("vis")
        b.set_io(i, x=x, row_stride=rs, geom=g, spec=spec, scale=scale, acc=acc, state=state, vis=vis,
                 flags=corr.DUMP | corr.RESET)
        V64 = oracle.xengine(Y)
        q = oracle.quantize_int8(Y, oscale.astype(np.float64))
        vq = oracle.scale_visibilities(oracle.xengine_int(q), oscale.astype(np.float64))
        Vq = vq[..., 0] + 1j * vq[..., 1]
        data.append((chans, V64, Vq, vis))
    stream = torch.cuda.Stream()
    b.capture(stream)
    b.launch(stream)
    stream.synchronize()
    for i, sh in enumerate(shapes):
        S, N, T = sh["n_signals"], sh["fft_len"], sh["n_spectra"]
        C, P = N // 2, S * (S + 1) // 2
        chans, V64, Vq, vis = data[i]
        vv = vis.view(C, P, 2)[chans].cpu().numpy().astype(np.float64)
        V = vv[..., 0] + 1j * vv[..., 1]
        _, e_gpu = oracle.normalized_error(V, V64, S)
        _, e_q = oracle.normalized_error(Vq, V64, S)
        _, e_rep = oracle.normalized_error(V, Vq, S)
        print("c4 sub-array %d (S=%d C=%d T=%d): e_fro vs FP64 %.3g (oracle int8 path %.3g), vs oracle int8 %.3g"
              % (i, S, C, T, e_gpu, e_q, e_rep))
        assert e_rep <= 1e-4                        # the GPU reproduces the int8 path
        assert e_gpu <= 1.05 * e_q + 1e-5           # and its error is the quantisation's own
        if T >= 8192:
            assert e_gpu <= 1e-3
    b.close()


def test_rfi_form_flaggers_sampled_tiles():
    """Learned-flagger inference and MAD flags over all 131072 tiles of
    64 x 8192 x 4096 power (the flagged benchmark's shape): sampled tiles
    against the oracle, including the last tile."""
    import torch
    S, T, C = 64, 8192, 4096
    gen = torch.Generator(device="cuda")
    gen.manual_seed(synth.BASE_SEED + 88)
    power = torch.empty(S, T, C, device="cuda").exponential_(1.0, generator=gen)
    # a persistent tone column and a burst row in the sampled tiles, so both flaggers have work
    power[3, :, 1000] *= 40.0
    power[3, 130, :] *= 25.0
    from paper_0910_1517_amd.flagger import init_params
    params = init_params(3)
    pd = torch.from_numpy(params).cuda()
    flags = torch.empty(S, T, C, dtype=torch.uint8, device="cuda")
    logits = torch.empty(S, T, C, device="cuda")
    corr.cnn_infer(pd, power, flags, logits=logits)
    plan = corr.Plan(S, 2 * C, T, precision=corr.INT8)
    mad = plan.alloc("flags").view(S, T, C)
    plan.mad_flag(power, mad, 3.0)
    torch.cuda.synchronize()
    ntm, ntk = T // 64, C // 256
    for (s, mt, kt) in [(0, 0, 0), (3, 2, 3), (3, 15, 3), (41, 77, 9), (S - 1, ntm - 1, ntk - 1)]:
        sl = (s, slice(mt * 64, mt * 64 + 64), slice(kt * 256, kt * 256 + 256))
        P = power[sl].cpu().numpy().astype(np.float64)
        z64, _ = oracle.cnn_forward(params.astype(np.float64), oracle.cnn_tile_input(P)[None, None])
        z = logits[sl].cpu().numpy().astype(np.float64)
        scale = 1.0 + np.abs(z64).max()
        assert np.abs(z - z64[0, 0]).max() < 2e-3 * scale, (s, mt, kt)
        f = flags[sl].cpu().numpy()
        clear = np.abs(z64[0, 0]) > 2e-3 * scale
        assert np.array_equal(f[clear], (z64[0, 0][clear] > 0).astype(np.uint8))
        mo = oracle.mad_tile_flags(P[None], 3.0)[0]
        mg = mad[sl].cpu().numpy()
        # FP32 statistics vs FP64: a decision may only differ at the threshold
        assert not np.any((mg != mo) & ~near_threshold_cells(P[None])[0]), (s, mt, kt)
        if (s, mt, kt) == (3, 2, 3):
            assert mo[:, 1000 - 768].all() and mo[130 - 128].all()  # the tone column and the burst row
