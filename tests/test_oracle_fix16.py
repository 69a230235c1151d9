"""Pins of the oracle's 16-bit fixed-point numerics (sections 3.1 and 4.1: the
16-bit fixed-point FFT output, the integer fringe table scaled into 16 bits,
32-bit products): closed forms of the Q14 table, exact identities of the
integer rotation, its error bound, unbiased rounding (a planted truncation
fails), saturation, ties to even, and the 16-bit X oracle against the int8 one
and a brute-force sum."""
import numpy as np
import pytest

import oracle

FS = 66.666666e6


def _geom(S, f=0.0, psi0=0.0, rate=0.0):
    return oracle.Geometry(np.zeros(S, np.int32), np.full(S, f), np.full(S, psi0), np.full(S, rate))


def test_table_closed_forms():
    w = oracle.fix16_table()
    assert w.shape == (1440, 2)
    assert tuple(w[0]) == (16384, 0) and tuple(w[360]) == (0, 16384)
    assert tuple(w[720]) == (-16384, 0) and tuple(w[1080]) == (0, -16384)
    assert tuple(w[180]) == (11585, 11585)  # 2^14 / sqrt(2) = 11585.24
    j = np.arange(1, 1440)
    assert np.array_equal(w[1440 - j, 0], w[j, 0]) and np.array_equal(w[1440 - j, 1], -w[j, 1])
    th = 2 * np.pi * np.arange(1440) / 1440
    assert np.max(np.abs(w[:, 0] - 16384 * np.cos(th))) <= 0.5 and np.max(np.abs(w[:, 1] - 16384 * np.sin(th))) <= 0.5


def _random_spectra(S, T, C, seed, sigma=4000.0):
    g = np.random.default_rng(seed)
    return g.normal(0, sigma, (S, T, C)) + 1j * g.normal(0, sigma, (S, T, C))


def test_zero_phase_is_the_identity_and_a_quarter_cycle_is_i():
    S, T, C = 3, 4, 64
    X = _random_spectra(S, T, C, 1)
    scale = np.ones((S, C))
    q, y = oracle.fix16_spectra(X, _geom(S), FS, scale)
    assert np.array_equal(q, y)
    assert np.array_equal(q[..., 0], np.clip(np.rint(X.real), -32767, 32767).astype(np.int16))
    # psi0 = 1/4 cycle, no delay terms: every channel takes entry 360, exactly i
    q, y = oracle.fix16_spectra(X, _geom(S, psi0=0.25), FS, scale)
    assert np.array_equal(y[..., 0], -q[..., 1]) and np.array_equal(y[..., 1], q[..., 0])


def test_rotation_error_bound_and_no_bias():
    # |y - q e^(i theta_j)| per component <= 1/2 (the rounding) + |q| 2^-14 / sqrt(2) (the table's
    # own rounding, <= 1/2 per Q14 component); rounding, not truncation, keeps the mean error ~0
    S, T, C = 2, 64, 256
    X = _random_spectra(S, T, C, 2)
    geom = _geom(S, f=0.37, psi0=0.123, rate=3.1)
    q, y = oracle.fix16_spectra(X, geom, FS, np.ones((S, C)))
    qc = q[..., 0].astype(float) + 1j * q[..., 1]
    yc = y[..., 0].astype(float) + 1j * y[..., 1]
    # the table entry of each channel and spectrum, from the same phase as the table-mode F-engine
    N = 2 * C
    tm = (np.arange(T) + 0.5) * N / FS
    c = (geom.psi0[0] + geom.rate[0] * tm) % 1.0
    phi = c[:, None] + np.arange(C)[None, :] * (geom.f[0] / N)
    j = np.rint(phi * 1440).astype(np.int64) % 1440
    exact = qc * np.exp(2j * np.pi * j / 1440)[None]
    err = yc - exact
    bound = 0.5 + np.abs(qc) * 2.0 ** -14 / np.sqrt(2) + 1e-9
    assert np.all(np.abs(err.real) <= bound) and np.all(np.abs(err.imag) <= bound)
    assert abs(err.real.mean()) < 0.02 and abs(err.imag.mean()) < 0.02
    # a planted truncating shift (floor without the half) is biased by -1/2
    w = oracle.fix16_table()[j]
    qr, qi = q[..., 0].astype(np.int64), q[..., 1].astype(np.int64)
    trunc = np.floor_divide(qr * w[None, ..., 0] - qi * w[None, ..., 1], 16384)
    assert abs((trunc - exact.real).mean()) > 0.3


def test_saturation_and_ties_to_even():
    S, T, C = 1, 1, 8
    X = np.array([2.5, 3.5, -2.5, -3.5, 1e9, -1e9, 0.5, 32767.4]).reshape(S, T, C) + 0j
    q, y = oracle.fix16_spectra(X, _geom(S), FS, np.ones((S, C)))
    assert list(q[0, 0, :, 0]) == [2, 4, -2, -4, 32767, -32767, 0, 32767]
    # 45 degrees of (32767, 32767) is (0, 46340): the imaginary part saturates
    X = np.full((1, 1, 1), 32767 + 32767j)
    q, y = oracle.fix16_spectra(X, _geom(1, psi0=0.125), FS, np.ones((1, 1)))
    assert y[0, 0, 0, 1] == 32767 and abs(int(y[0, 0, 0, 0])) <= 1


def test_scale_divides_before_rounding():
    # FP32 spectra and levels, the division in FP32 (numpy's float32 division is IEEE)
    X = _random_spectra(2, 3, 16, 3, sigma=100.0)
    X = X.real.astype(np.float32) + 1j * X.imag.astype(np.float32)
    sc = np.random.default_rng(4).uniform(0.1, 2.0, (2, 16)).astype(np.float32)
    q, _ = oracle.fix16_spectra(X, _geom(2), FS, sc)
    for part, comp in ((X.real, 0), (X.imag, 1)):
        u = part.astype(np.float32) / sc[:, None, :]
        assert u.dtype == np.float32
        assert np.array_equal(q[..., comp], np.clip(np.rint(u.astype(np.float64)), -32767, 32767).astype(np.int16))
    # a quotient that FP64 would round the other way: fl32(3.5 x 1.3f) / 1.3f is 3.5 exactly in
    # FP32 (code 4, ties to even) and 3.4999999 in FP64 (code 3)
    lv = np.float32(1.3)
    x = np.float32(np.float32(3.5) * lv)
    assert np.float32(x) / lv == np.float32(3.5) and float(x) / float(lv) < 3.5
    q, _ = oracle.fix16_spectra(np.full((1, 1, 1), complex(float(x), -float(x))), _geom(1), FS, np.full((1, 1), lv))
    assert tuple(q[0, 0, 0]) == (4, -4)


def test_i16_xengine_matches_the_int8_one_and_brute_force():
    g = np.random.default_rng(5)
    q8 = g.integers(-127, 128, (5, 7, 3, 2)).astype(np.int8)
    assert np.array_equal(oracle.xengine_i16(q8.astype(np.int16)), oracle.xengine_int(q8))
    q = g.integers(-32767, 32768, (4, 9, 2, 2)).astype(np.int16)
    A = oracle.xengine_i16(q)
    z = q[..., 0].astype(object) + 0 * 1j  # exact integer arithmetic below
    qr, qi = q[..., 0].astype(np.int64), q[..., 1].astype(np.int64)
    for j in range(4):
        for i in range(j + 1):
            p = oracle.pair_index(i, j)
            re = (qr[i] * qr[j] + qi[i] * qi[j]).sum(0)
            im = (qi[i] * qr[j] - qr[i] * qi[j]).sum(0)
            assert np.array_equal(A[:, p, 0], re) and np.array_equal(A[:, p, 1], im)
    # the largest products: 2 x 32767^2 per spectrum fits int32, the sums do not need to
    big = np.full((2, 4, 1, 2), 32767, dtype=np.int16)
    big[1, ..., 1] = -32767
    A = oracle.xengine_i16(big)
    assert A[0, oracle.pair_index(0, 0), 0] == 4 * 2 * 32767 ** 2
