"""The F-engines' requantisation encoders (section 4.1's fixed point ahead of
the MAC, at 8 bits) through corr_requantize against the oracle's encoders:
OCP e4m3 on every code value, every tie between neighbouring codes and the
floats on either side of it, the flush tie below the smallest subnormal, the
saturation at 448, and 2^21 random values over 22 binades; int8 on every tie
k + 1/2 and its neighbours, the rails and infinities.  NaN maps to the
documented codes."""
import numpy as np
import pytest

import oracle
import paper_0910_1517_amd as corr
import synth

pytestmark = pytest.mark.gpu


def _run(prec, vals):
    """vals: float32 [n] -> GPU codes [n] (uint8) and the plan's shape."""
    import torch
    S, C = 1, 256
    n2 = (len(vals) + 1) // 2
    T = max(32, -(-n2 // C) // 32 * 32 + (32 if (-(-n2 // C)) % 32 else 0))
    buf = np.zeros(S * T * C * 2, dtype=np.float32)
    buf[:len(vals)] = vals
    plan = corr.Plan(S, 2 * C, T, precision=prec)
    out = torch.full((S * T * C * 2,), 0x55, dtype=torch.uint8, device="cuda")
    plan.requantize(torch.from_numpy(buf).cuda(), torch.ones(S * C, device="cuda"), out)
    torch.cuda.synchronize()
    R = buf.reshape(S, T, C, 2).astype(np.float64)
    Y = np.empty((S, T, C), dtype=np.complex128)  # set component-wise: 1j * inf would put a NaN in the real part
    Y.real, Y.imag = R[..., 0], R[..., 1]
    return out.cpu().numpy()[:len(vals)], Y, np.ones((S, C))


def _e4m3_boundaries():
    f32 = np.float32
    table = oracle.e4m3_decode_table()[:0x7F]
    v = np.unique(table[np.isfinite(table)]).astype(np.float64)  # 0 and every positive code value
    mids = ((v[:-1] + v[1:]) / 2).astype(f32)                      # ties (exact in FP32)
    up, dn = np.nextafter(mids, f32(np.inf)), np.nextafter(mids, f32(0))
    extra = np.array([2.0 ** -10, 448.0, 464.0, 480.0, 500.0, 1e6, 3.4e38, 2.0 ** -20, 1e-30], dtype=f32)
    extra = np.concatenate([extra, np.nextafter(extra, f32(np.inf)), np.nextafter(extra, f32(0))])
    pos = np.concatenate([v.astype(f32), mids, up, dn, extra])
    g = synth.rng(71, 8)
    rnd = (2.0 ** g.uniform(-12, 10, 1 << 21) * np.where(g.random(1 << 21) < 0.5, -1, 1)).astype(f32)
    return np.concatenate([pos, -pos, rnd, np.array([np.inf, -np.inf, 0.0, -0.0], dtype=f32)])


def test_e4m3_encoder_matches_the_oracle_on_every_boundary():
    vals = _e4m3_boundaries()
    q, Y, sc = _run(corr.FP8_E4M3, vals)
    qo = oracle.quantize_fp8(Y, sc).reshape(-1)[:len(vals)]
    bad = np.nonzero(q != qo)[0]
    print("e4m3: %d values, %d mismatches" % (len(vals), len(bad)))
    assert len(bad) == 0, [(float(vals[i]), hex(q[i]), hex(qo[i])) for i in bad[:10]]
    # +0 for values that round to zero, whatever their sign
    neg_tie = np.nonzero(vals == np.float32(-(2.0 ** -10)))[0]
    assert len(neg_tie) > 0 and np.all(q[neg_tie] == 0)
    assert np.all(q[np.nonzero((vals == 0) & np.signbit(vals))[0]] == 0)


def test_int8_encoder_matches_the_oracle_on_every_tie():
    f32 = np.float32
    k = np.arange(-130, 130, dtype=np.float64)
    ties = (k + 0.5).astype(f32)
    vals = np.concatenate([ties, np.nextafter(ties, f32(np.inf)), np.nextafter(ties, f32(-np.inf)),
                           k.astype(f32), np.array([1e9, -1e9, np.inf, -np.inf, 0.0, -0.0], dtype=f32)])
    q, Y, sc = _run(corr.INT8, vals)
    qo = oracle.quantize_int8(Y, sc).reshape(-1)[:len(vals)].view(np.uint8)
    assert np.array_equal(q, qo)


def test_nan_codes_are_the_documented_ones():
    nan = np.array([np.nan, 1.0, -np.nan, 2.0], dtype=np.float32)
    q8, _, _ = _run(corr.INT8, nan)
    q4, _, _ = _run(corr.FP8_E4M3, nan)
    assert q8[0] == q8[2] == np.uint8(0x81)  # -127
    assert q4[0] == q4[2] == np.uint8(0xFE)  # -448
