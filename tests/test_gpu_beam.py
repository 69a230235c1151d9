"""B-engine (array beams, section 2.2) through the C ABI against the oracle.

Spectra are packed by the library's corner turn from host values the oracle
sees too: FP32 values, INT8 codes or finite e4m3 codes with per-(signal,
channel) scales.  Every coherent mode, 0..4 beams, time sums tint = 1..8, with
and without the incoherent beam, at the largest signal count, an odd one and
a single antenna.

Tolerance: gpu_util.check_beams.
"""
import numpy as np
import pytest

import oracle
import paper_0910_1517_amd as corr
from gpu_util import beam_bounds, check_beams, pack_input

pytestmark = pytest.mark.gpu


def spectra(prec, S, T, C, seed):
    """Host spectra [S][T][C][2] of the precision, the scales, and the values
    the oracle uses (complex [S][T][C], scale applied)."""
    rng = np.random.default_rng(seed)
    if prec == corr.FP32:
        a = rng.normal(size=(S, T, C, 2)).astype(np.float32)
        return a, None, a[..., 0].astype(np.float64) + 1j * a[..., 1]
    scale = rng.uniform(0.25, 2.0, size=(S, C)).astype(np.float32)
    if prec == corr.INT8:
        q = rng.integers(-127, 128, size=(S, T, C, 2)).astype(np.int8)
        v = q.astype(np.float64)
    else:
        q = rng.integers(0, 256, size=(S, T, C, 2)).astype(np.uint8)
        q[(q & 0x7F) == 0x7F] = 0x38  # 0x7F / 0xFF are NaN in e4m3: use 1.0
        v = oracle.e4m3_decode_table()[q]
    Y = (v[..., 0] + 1j * v[..., 1]) * scale.astype(np.float64)[:, None, :]
    return q, scale, Y


def run_beams(prec, S, N, T, seed, nb, mode, tint, with_inc):
    import torch
    C = N // 2
    q, scale, Y = spectra(prec, S, T, C, seed)
    plan = corr.Plan(S, N, T, precision=prec)
    spec = pack_input(plan, q)
    rng = np.random.default_rng(seed + 100)
    w = rng.uniform(0.0, 2.0, size=S) if with_inc else None
    if w is not None:
        w[rng.integers(0, S)] = 0.0  # one signal left out
    c = (rng.normal(size=(nb, S)) + 1j * rng.normal(size=(nb, S))) if nb else None
    To = T // tint
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    inc = torch.full((2, To, C), float("nan"), device="cuda") if with_inc else None
    coh = None
    if nb:
        coh = (torch.full((nb, 2, T, C), float("nan"), dtype=torch.complex64, device="cuda")
               if mode == corr.BEAM_VOLTAGE else
               torch.full((nb, 4 if mode == corr.BEAM_FULLPOL else 2, To, C), float("nan"), device="cuda"))
    cw = dev(np.stack([c.real, c.imag], axis=-1).astype(np.float32)) if nb else None
    # the GPU rounds the weights to FP32: the oracle takes the same values
    w32 = None if w is None else w.astype(np.float32).astype(np.float64)
    c32 = None if c is None else (c.real.astype(np.float32) + 1j * c.imag.astype(np.float32)).astype(np.complex128)
    plan.beamform(spec, None if scale is None else dev(scale), None if w is None else dev(w.astype(np.float32)),
                  inc, cw, coh, mode=mode, tint=tint)
    torch.cuda.synchronize()
    ref_inc, ref_coh = oracle.beamform(Y, w=w32, c=c32, mode=mode, tint=tint)
    inc_b, coh_b = beam_bounds(Y, w32, c32, tint)
    return (None if inc is None else inc.cpu().numpy(), None if coh is None else coh.cpu().numpy(),
            ref_inc, ref_coh, inc_b, coh_b)


CASES = [  # (n_beams, mode, tint, incoherent)
    (1, corr.BEAM_FULLPOL, 1, True),
    (4, corr.BEAM_INTENSITY, 2, True),
    (3, corr.BEAM_VOLTAGE, 1, False),
    (2, corr.BEAM_FULLPOL, 8, False),
    (0, corr.BEAM_FULLPOL, 4, True),
]


@pytest.mark.parametrize("prec", [corr.FP32, corr.INT8, corr.FP8_E4M3])
@pytest.mark.parametrize("case", CASES)
def test_beams_match_oracle(prec, case):
    nb, mode, tint, with_inc = case
    for (S, N, T) in [(64, 512, 32), (7, 1024, 64), (2, 512, 32)]:
        print("prec %d S %d N %d T %d beams %d mode %d tint %d inc %s" % (prec, S, N, T, nb, mode, tint, with_inc),
              flush=True)
        out = run_beams(prec, S, N, T, 10 * S + prec, nb, mode, tint, with_inc)
        check_beams(*out, mode, tint)


def test_single_antenna_beam_equals_its_correlator_products():
    """A unit-weight coherent beam of one antenna, summed over the call, is the
    GPU X-engine's RR*, LL*, RL* of that antenna (int8 path, exact codes)."""
    import torch
    S, N, T, a = 8, 512, 64, 3
    C = N // 2
    q, scale, _ = spectra(corr.INT8, S, T, C, 77)
    scale[:] = 1.0
    plan = corr.Plan(S, N, T, precision=corr.INT8)
    spec = pack_input(plan, q)
    c = np.zeros((1, S, 2), np.float32)
    c[0, 2 * a, 0] = c[0, 2 * a + 1, 0] = 1.0
    coh = torch.empty(1, 4, T // 8, C, device="cuda")
    plan.beamform(spec, torch.from_numpy(scale).cuda(), None, None, torch.from_numpy(c).cuda(), coh,
                  mode=corr.BEAM_FULLPOL, tint=8)
    acc = plan.alloc("acc")
    plan.xengine(spec, acc)
    torch.cuda.synchronize()
    A = acc.cpu().numpy().reshape(plan.splits, C, plan.P, 2).astype(np.int64).sum(0)
    beam = coh.cpu().numpy()[0].sum(axis=1)  # [4][C]
    pij = lambda i, j: oracle.pair_index(i, j)
    assert np.array_equal(beam[0], A[:, pij(2 * a, 2 * a), 0].astype(np.float32))
    assert np.array_equal(beam[1], A[:, pij(2 * a + 1, 2 * a + 1), 0].astype(np.float32))
    assert np.array_equal(beam[2], A[:, pij(2 * a, 2 * a + 1), 0].astype(np.float32))
    assert np.array_equal(beam[3], A[:, pij(2 * a, 2 * a + 1), 1].astype(np.float32))
