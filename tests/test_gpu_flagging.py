"""GPU parity of the flagging path (power output, MAD tile flags, zeroing,
pair counts) against the CPU oracle."""
import numpy as np
import pytest

import oracle
import paper_0910_1517_amd as corr
import synth
from gpu_util import FS, acc_sum, geom_dev, near_threshold_cells, pack_input, run_fengine, upload_streams

pytestmark = pytest.mark.gpu


def ogeom(g):
    return oracle.Geometry(g.D, g.f, g.psi0, g.rate)


def rfi_case(S=4, N=512, T=128, seed=7):
    geo = synth.make_geometry(S // 2, seed=seed)
    x = synth.voltages(S, N * T + 64, geo, FS, seed=seed + 1, rfi=synth.RFI(N, seed=seed + 2))
    return geo, x


@pytest.mark.parametrize("prec", [corr.FP32, corr.INT8])
def test_power_output_matches_oracle(prec):
    import torch
    S, N, T = 4, 1024, 64
    geo, x = rfi_case(S, N, T, seed=11)
    plan = corr.Plan(S, N, T, precision=prec)
    x_dev, rs = upload_streams(x, N, T, 16)
    pw = plan.alloc("power", zero=False)
    spec = plan.alloc("spectra", zero=False)
    scale = torch.full((S * plan.C,), 1000.0, device="cuda")
    plan.fengine(x_dev, geom_dev(geo), spec, scale if prec else None, power=pw, row_stride=rs)
    torch.cuda.synchronize()
    P64 = oracle.power(oracle.fengine(x, N, T, ogeom(geo), FS))
    pg = pw.cpu().numpy().reshape(S, T, plan.C)
    # FP32 FFT error is relative to the cell's own amplitude (tone cells carry up to
    # ~200x the mean power), so normalise by the larger of the cell and the mean power
    ref = np.maximum(P64, P64.mean(axis=-1, keepdims=True))
    assert np.max(np.abs(pg - P64) / ref) < 1e-5


@pytest.mark.parametrize("N", [1024, 2048, 8192])
def test_power_fp16_output_matches_oracle(N):
    # FP16 power cells |X|^2 / N^2 from both F-engine kernels (1024 and 8192 points on the
    # LDS-radix one, 2048 on the four-step one): within the FP16 rounding (half a unit in the
    # last place, 2^-11 relative; 2^-25 absolute in the subnormal range) plus the FP32 FFT error
    # of the FP32 power test, against the FP64 oracle's |X|^2 scaled by the same power of two
    import torch
    S, T = 4, 64
    geo, x = rfi_case(S, N, T, seed=12)
    plan = corr.Plan(S, N, T, precision=corr.INT8, power_fp16=1)
    assert plan.alloc("power").dtype == torch.float16 and plan.alloc("power").numel() == S * T * plan.C
    x_dev, rs = upload_streams(x, N, T, 16)
    pw = plan.alloc("power", zero=False)
    spec = plan.alloc("spectra", zero=False)
    scale = torch.full((S * plan.C,), 1000.0, device="cuda")
    plan.fengine(x_dev, geom_dev(geo), spec, scale, power=pw, row_stride=rs)
    torch.cuda.synchronize()
    P64 = oracle.power(oracle.fengine(x, N, T, ogeom(geo), FS)) / float(N) ** 2
    pg = pw.cpu().numpy().astype(np.float64).reshape(S, T, plan.C)
    ref = np.maximum(P64, P64.mean(axis=-1, keepdims=True))
    bound = np.maximum(2.0 ** -11 * P64, 2.0 ** -25) + 1e-5 * ref
    print("FP16 power, N %d: max error / bound %.3g, %s" % (N, np.max(np.abs(pg - P64) / bound), plan.fengine_kernel))
    assert np.all(np.abs(pg - P64) <= bound)


def test_mad_flags_fp16_power_match_oracle():
    # the MAD flagger reading FP16 power (synthetic cells rounded to FP16 on the host, at the
    # scale |X|^2 / N^2 puts them): the same flags as the FP64 oracle on the same FP16 values,
    # except where a statistic lies at the threshold
    import torch
    S, T, C = 4, 256, 512
    p16 = (synth.power_spectra(S, T, C, seed=23) * np.float32(2.0 ** -20)).astype(np.float16)
    plan = corr.Plan(S, 2 * C, T, precision=corr.FP32, power_fp16=1)
    flags = plan.alloc("flags", zero=False)
    plan.mad_flag(torch.from_numpy(p16).cuda(), flags, 3.0)
    torch.cuda.synchronize()
    P64 = p16.astype(np.float64)
    fo = oracle.mad_tile_flags(P64, 3.0)
    fg = flags.cpu().numpy().reshape(S, T, C)
    assert not np.any((fg != fo) & ~near_threshold_cells(P64))
    assert fo.mean() > 0.01


def test_mad_flags_match_oracle():
    import torch
    S, N, T = 4, 1024, 256
    geo, x = rfi_case(S, N, T, seed=21)
    plan = corr.Plan(S, N, T, precision=corr.FP32)
    x_dev, rs = upload_streams(x, N, T, 16)
    pw = plan.alloc("power", zero=False)
    spec = plan.alloc("spectra", zero=False)
    plan.fengine(x_dev, geom_dev(geo), spec, power=pw, row_stride=rs)
    flags = plan.alloc("flags", zero=False)
    plan.mad_flag(pw, flags, 3.0)
    torch.cuda.synchronize()
    fg = flags.cpu().numpy().reshape(S, T, plan.C)
    P64 = oracle.power(oracle.fengine(x, N, T, ogeom(geo), FS))
    fo = oracle.mad_tile_flags(P64, 3.0)
    diff = fg != fo
    assert fg.max() <= 1
    # FP32 power and statistics vs FP64: a decision may only differ at the threshold
    assert not np.any(diff & ~near_threshold_cells(P64))
    assert fo.mean() > 0.01  # the injected RFI is found


@pytest.mark.parametrize("prec,S", [(corr.INT8, 16), (corr.FP32, 16), (corr.INT8, 30)])
def test_apply_flags_and_pair_counts_bit_exact(prec, S):
    import torch
    T = 256
    plan = corr.Plan(S, 512, T, precision=prec)
    g = synth.rng(31, prec)
    fl = (g.random((S, T, plan.C)) < 0.1).astype(np.uint8)
    fl[3] = 1  # one signal fully flagged
    fl[5] *= g.integers(1, 256, fl[5].shape, dtype=np.uint8)  # any nonzero byte flags
    flags = torch.from_numpy(fl).cuda()
    if prec == corr.INT8:
        q = synth.random_spectra_int8(S, T, plan.C, seed=32)
        spec = pack_input(plan, q)
    else:
        y = synth.random_spectra_f32(S, T, plan.C, seed=32)
        spec = pack_input(plan, np.stack([y.real, y.imag], -1).astype(np.float32))
    keep, keep_only = plan.alloc("keep"), plan.alloc("keep")
    plan.apply_flags(flags, spec, keep)
    plan.apply_flags(flags, None, keep_only)  # the keep-words-only kernel
    counts = torch.zeros(plan.C * plan.P, dtype=torch.int32, device="cuda")
    plan.pair_counts(keep, counts)
    # flags not 8-byte aligned: the keep-only call falls back to the zeroing kernel's keep mode
    fbuf = torch.zeros(flags.numel() + 1, dtype=torch.uint8, device="cuda")
    fbuf[1:] = flags.reshape(-1)
    keep_odd = plan.alloc("keep")
    plan.apply_flags(fbuf[1:], None, keep_odd)
    torch.cuda.synchronize()
    assert torch.equal(keep_only, keep)
    assert torch.equal(keep_odd, keep)
    # zeroed spectra, read back through the layout
    back = corr.unpack_spectra(spec, prec, S, plan.C, T)
    if prec == corr.INT8:
        assert np.array_equal(back, np.where(fl[..., None] != 0, 0, q))
    else:
        ref = np.where(fl != 0, 0, y)
        assert np.array_equal(back[..., 0], ref.real.astype(np.float32))
        assert np.array_equal(back[..., 1], ref.imag.astype(np.float32))
    assert np.array_equal(counts.cpu().numpy().reshape(plan.C, plan.P), oracle.pair_counts(fl))
    # keep masks: bit i of word w = spectrum 32 w + i kept
    # layout [C/8][T/32][S][8]
    kb = keep.cpu().numpy().view(np.uint32).reshape(plan.C // 8, T // 32, S, 8).transpose(0, 3, 2, 1).reshape(plan.C, S, T // 32)
    bits = ((kb[..., None] >> np.arange(32, dtype=np.uint32)) & 1).reshape(plan.C, S, T)
    assert np.array_equal(bits.transpose(1, 2, 0), (fl == 0).astype(np.uint32))


@pytest.mark.parametrize("S,T", [(1, 96), (33, 96), (64, 32), (40, 288)])
def test_pair_counts_edge_shapes(S, T):
    """Pair counts (the keep bits' Gram matrix on the matrix cores) at one
    signal, one past a 32-signal tile, a single span of 32 spectra, and span
    counts that leave a partial staging batch; counts accumulate (+=)."""
    import torch
    print("pair counts", S, T, flush=True)
    plan = corr.Plan(S, 512, T, precision=corr.INT8)
    g = synth.rng(61, S, T)
    fl = (g.random((S, T, plan.C)) < 0.2).astype(np.uint8)
    keep = plan.alloc("keep")
    plan.apply_flags(torch.from_numpy(fl).cuda(), None, keep)
    counts = torch.full((plan.C * plan.P,), 7, dtype=torch.int32, device="cuda")
    plan.pair_counts(keep, counts)
    torch.cuda.synchronize()
    assert np.array_equal(counts.cpu().numpy().reshape(plan.C, plan.P), oracle.pair_counts(fl) + 7)


def test_flagged_int8_visibilities_bit_exact():
    import torch
    S, T = 8, 512
    plan = corr.Plan(S, 512, T, precision=corr.INT8)
    g = synth.rng(41, 1)
    fl = (g.random((S, T, plan.C)) < 0.05).astype(np.uint8)
    q = synth.random_spectra_int8(S, T, plan.C, seed=42)
    spec = pack_input(plan, q)
    plan.apply_flags(torch.from_numpy(fl).cuda(), spec)
    acc = plan.alloc("acc")
    plan.xengine(spec, acc)
    torch.cuda.synchronize()
    A = oracle.xengine_int(np.where(fl[..., None] != 0, 0, q).astype(np.int8))
    assert np.array_equal(acc_sum(acc.cpu().numpy(), plan), A)


@pytest.mark.parametrize("prec,S,T,split", [(corr.INT8, 8, 1024, 2), (corr.INT8, 48, 512, 1),
                                             (corr.FP8_E4M3, 40, 512, 2), (corr.FP32, 8, 256, 4),
                                             (corr.FP32, 64, 128, 1)])
def test_masked_xengine_equals_zeroing_then_xengine(prec, S, T, split):
    """corr_xengine with keep words (the flag mask applied as the spectra are
    staged) against corr_apply_flags' zeroing followed by the unmasked
    X-engine: the same accumulators bit for bit, the spectra untouched, and
    the counts of the same call equal to the oracle's pair counts."""
    import torch
    print("masked X", prec, S, T, split, flush=True)
    plan = corr.Plan(S, 512, T, precision=prec, x_split=split)
    g = synth.rng(51, prec, S)
    fl = (g.random((S, T, plan.C)) < 0.07).astype(np.uint8)
    fl[S // 2, :, 5] = 1            # a flagged channel
    fl[1, T // 3: T // 3 + 9] = 1   # a flagged burst
    if prec == corr.INT8:
        arr = synth.random_spectra_int8(S, T, plan.C, seed=52)
    elif prec == corr.FP8_E4M3:
        y = g.standard_normal((S, T, plan.C)) * 112 + 1j * g.standard_normal((S, T, plan.C)) * 112
        arr = oracle.quantize_fp8(y, np.ones((S, plan.C)))
    else:
        y = synth.random_spectra_f32(S, T, plan.C, seed=52)
        arr = np.stack([y.real, y.imag], -1).astype(np.float32)
    spec = pack_input(plan, arr)
    zeroed = spec.clone()
    flags = torch.from_numpy(fl).cuda()
    keep = plan.alloc("keep")
    plan.apply_flags(flags, None, keep)            # keep words only
    plan.apply_flags(flags, zeroed)                # zeroing only
    acc_m, acc_z = plan.alloc("acc"), plan.alloc("acc")
    counts = torch.zeros(plan.C * plan.P, dtype=torch.int32, device="cuda")
    before = spec.clone()
    plan.xengine(spec, acc_m, keep=keep, counts=counts)
    plan.xengine(zeroed, acc_z)
    torch.cuda.synchronize()
    assert torch.equal(spec, before)
    assert torch.equal(acc_m.view(torch.int32), acc_z.view(torch.int32))
    assert np.array_equal(counts.cpu().numpy().reshape(plan.C, plan.P), oracle.pair_counts(fl))
    if prec == corr.INT8:  # and against the oracle's integer X-engine on zeroed codes
        A = oracle.xengine_int(np.where(fl[..., None] != 0, 0, arr).astype(np.int8))
        assert np.array_equal(acc_sum(acc_m.cpu().numpy(), plan), A)


def test_mad_flag_rejects_ragged_time():
    plan = corr.Plan(4, 512, 96, precision=corr.FP32)
    pw = plan.alloc("power")
    flags = plan.alloc("flags")
    with pytest.raises(corr.CorrError) as e:
        plan.mad_flag(pw, flags)
    assert e.value.status == -1
