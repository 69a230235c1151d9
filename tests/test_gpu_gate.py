"""Gated correlator (section 5: visibilities per pulse-phase gate) through
the C ABI against the oracle: int8 bit-exact for every bin (the sum over bins
also equals the ungated X-engine exactly), FP32 and FP8 to the X-engine's
tolerances, spectra outside every bin left out, several K-splits and both
signal-tile sizes."""
import numpy as np
import pytest

import oracle
import paper_0910_1517_amd as corr
import synth
from gpu_util import acc_sum, pack_input

pytestmark = pytest.mark.gpu


def run_gated(plan, spec, gate, n_bins):
    import torch
    acc = torch.zeros(n_bins * plan.acc_bytes // 4, dtype=torch.int32 if plan.precision == corr.INT8
                      else torch.float32, device="cuda")
    plan.xengine_gated(spec, torch.from_numpy(np.ascontiguousarray(gate)).cuda(), n_bins, acc)
    torch.cuda.synchronize()
    a = acc.cpu().numpy().reshape(n_bins, -1)
    return [acc_sum(a[b], plan) for b in range(n_bins)]


def gates(T, n_bins, seed, outside=True):
    g = synth.rng(seed, 60).integers(0, n_bins + (1 if outside else 0), size=T).astype(np.uint8)
    if outside:
        g[g == n_bins] = 255  # left out of every bin
    return g


@pytest.mark.parametrize("S,T,split,n_bins", [(64, 512, 0, 2), (8, 256, 1, 3), (33, 256, 2, 5), (64, 1024, 4, 1),
                                              (30, 64, 1, 16)])
def test_gated_int8_bit_exact(S, T, split, n_bins):
    import torch
    print("gated int8", S, T, split, n_bins, flush=True)
    plan = corr.Plan(S, 512, T, precision=corr.INT8, x_split=split)
    q = synth.random_spectra_int8(S, T, plan.C, seed=700 + S)
    spec = pack_input(plan, q)
    gate = gates(T, n_bins, S + T)
    got = run_gated(plan, spec, gate, n_bins)
    ref = oracle.xengine_int_gated(q, gate, n_bins)
    for b in range(n_bins):
        assert np.array_equal(got[b], ref[b]), b
    # all bins together = the ungated X-engine on the gated-in spectra; with
    # nothing left out, = the plain X-engine
    full = np.zeros(T, np.uint8) if n_bins == 1 else np.minimum(gate, n_bins - 1)
    got_all = run_gated(plan, spec, full, n_bins)
    acc = plan.alloc("acc")
    plan.xengine(spec, acc)
    torch.cuda.synchronize()
    assert np.array_equal(sum(got_all), acc_sum(acc.cpu().numpy(), plan))


@pytest.mark.parametrize("S,T,n_bins", [(64, 512, 2), (8, 128, 3)])
def test_gated_fp32(S, T, n_bins):
    plan = corr.Plan(S, 512, T, precision=corr.FP32)
    y = synth.random_spectra_f32(S, T, plan.C, seed=800 + S)
    spec = pack_input(plan, np.stack([y.real, y.imag], axis=-1).astype(np.float32))
    gate = gates(T, n_bins, 5 + S)
    got = run_gated(plan, spec, gate, n_bins)
    ref = oracle.xengine_gated(y.astype(np.complex128), gate, n_bins)
    for b in range(n_bins):
        g = got[b]
        e_max, e_fro = oracle.normalized_error(g[..., 0] + 1j * g[..., 1], ref[b], S)
        assert e_max < 1e-6 and e_fro < 1e-6, (b, e_max, e_fro)


def test_gated_fp8_exact_on_narrow_codes():
    S, T, n_bins = 64, 128, 2
    plan = corr.Plan(S, 512, T, precision=corr.FP8_E4M3)
    g = synth.rng(901, S)
    codes = ((g.integers(0, 256, size=(S, T, plan.C, 2)) & 0x87) | 0x38).astype(np.uint8)  # +-[1, 2)
    spec = pack_input(plan, codes)
    gate = gates(T, n_bins, 77)
    got = run_gated(plan, spec, gate, n_bins)
    vals = oracle.e4m3_decode_table()[codes]
    ref = oracle.xengine_gated(vals[..., 0] + 1j * vals[..., 1], gate, n_bins)
    for b in range(n_bins):
        assert np.array_equal(got[b][..., 0] + 1j * got[b][..., 1], ref[b]), b


def test_pulsar_gates_drive_the_gated_correlator():
    """Gates from a pulsar period (on / off halves of a 1.5578 ms period at
    4096-point spectra) on int8 spectra: bit-exact per gate."""
    S, T = 16, 2048
    plan = corr.Plan(S, 4096, T, precision=corr.INT8)
    gate, counts = corr.pulsar_gates(1000, T, 4096, 66.666666e6, 0.0, 1.5578e-3, 2)
    assert counts.sum() == T and counts.min() > 0.4 * T
    q = synth.random_spectra_int8(S, T, plan.C, seed=902)
    spec = pack_input(plan, q)
    got = run_gated(plan, spec, gate, 2)
    ref = oracle.xengine_int_gated(q, gate, 2)
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
