"""Pins of the CPU oracle against things other than itself (CPU only).

Every check here is fixed by mathematics, a library routine used as a special
case, brute force on tiny inputs, or a closed form that follows from the
paper's definitions -- never by re-typing the oracle's own formula.
"""
import math

import numpy as np
import pytest

import oracle
import synth

FS = 66.666666e6  # 33.33 MHz band, the paper's 33 MHz mode (section 2.3.1)


def geom_of(g):
    return oracle.Geometry(g.D, g.f, g.psi0, g.rate)


# ---------------------------------------------------------------- transforms
@pytest.mark.parametrize("n", [1, 2, 4, 8, 64, 512, 4096, 16384])
def test_fft_matches_numpy(n):
    g = np.random.default_rng(n)
    z = g.standard_normal(n) + 1j * g.standard_normal(n)
    ref = np.fft.fft(z)  # library special case of the same definition
    assert np.max(np.abs(oracle.fft(z) - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("n", [1, 3, 8, 12, 256, 1024])
def test_dft_matches_numpy_and_fft(n):
    g = np.random.default_rng(100 + n)
    z = g.standard_normal(n) + 1j * g.standard_normal(n)
    d = oracle.dft(z)
    ref = np.fft.fft(z)
    assert np.max(np.abs(d - ref)) <= 1e-11 * max(1.0, np.max(np.abs(ref)))
    if n & (n - 1) == 0:
        assert np.max(np.abs(d - oracle.fft(z))) <= 1e-11 * max(1.0, np.max(np.abs(ref)))


def test_fft_rejects_non_power_of_two():
    with pytest.raises(ValueError):
        oracle.fft(np.ones(12))


@pytest.mark.parametrize("N,k0,phi", [(512, 37, 0.3), (1024, 1, -1.2), (4096, 2047, 2.0)])
def test_tone_lands_in_one_bin(N, k0, phi):
    # A cos(2 pi k0 n / N + phi) -> X[k0] = (A N / 2) e^{i phi}, all other bins < N/2 zero.
    A = 4.0
    n = np.arange(N)
    X = oracle.fft(A * np.cos(2 * np.pi * k0 * n / N + phi))
    assert abs(X[k0] - A * N / 2 * np.exp(1j * phi)) < 1e-9 * N
    others = np.delete(np.abs(X[:N // 2]), k0)
    assert np.max(others) < 1e-9 * N


def test_parseval_and_real_symmetry():
    g = np.random.default_rng(7)
    x = g.integers(-127, 128, 2048).astype(float)
    X = oracle.fft(x)
    assert abs(np.sum(np.abs(X) ** 2) / x.size - np.sum(x ** 2)) < 1e-9 * np.sum(x ** 2)
    k = np.arange(1, x.size)
    assert np.max(np.abs(X[x.size - k] - np.conj(X[k]))) < 1e-9 * np.max(np.abs(X))


# ------------------------------------------------------------------ F-engine
def small_input(S=4, N=64, T=8, pad=24, seed=5):
    g = np.random.default_rng(seed)
    x = g.integers(-127, 128, size=(S, N * T + pad)).astype(np.int8)
    geo = oracle.Geometry(g.integers(0, pad + 1, S), g.random(S), g.random(S), g.uniform(-5, 5, S))
    return x, geo


def test_fengine_zero_geometry_is_plain_rfft():
    # With no delay, fraction or fringe the F-engine is the first N/2 bins of the DFT of
    # contiguous windows (section 2.1); numpy.fft.rfft is the library special case.
    S, N, T = 3, 128, 5
    g = np.random.default_rng(11)
    x = g.integers(-127, 128, size=(S, N * T)).astype(np.int8)
    z = oracle.Geometry(np.zeros(S), np.zeros(S), np.zeros(S), np.zeros(S))
    Y = oracle.fengine(x, N, T, z, FS)
    ref = np.fft.rfft(x.reshape(S, T, N).astype(float), axis=-1)[..., :N // 2]
    assert np.max(np.abs(Y - ref)) < 1e-9 * np.max(np.abs(ref))


def test_fengine_fft_equals_dft_and_channel_path():
    x, geo = small_input()
    N, T = 64, 8
    a = oracle.fengine(x, N, T, geo, FS, method="fft")
    b = oracle.fengine(x, N, T, geo, FS, method="dft")
    ks = [0, 1, 17, 31]
    c = oracle.fengine_channels(x, N, T, geo, FS, ks)
    scale = np.max(np.abs(a))
    assert np.max(np.abs(a - b)) < 1e-11 * scale
    assert np.max(np.abs(a[:, :, ks] - c)) < 1e-11 * scale


def test_integer_delay_is_a_read_pointer_shift():
    # Brute force: delaying the row by d samples and reading with D = d gives
    # bit-identical spectra to reading the undelayed row with D = 0.
    S, N, T = 2, 64, 6
    g = np.random.default_rng(3)
    base = g.integers(-127, 128, size=(S, N * T)).astype(np.int8)
    f, psi, r = g.random(S), g.random(S), g.uniform(-5, 5, S)
    y0 = oracle.fengine(base, N, T, oracle.Geometry([0, 0], f, psi, r), FS)
    for d in (1, 7, 16):
        shifted = np.zeros((S, N * T + d), dtype=np.int8)
        shifted[:, d:] = base
        yd = oracle.fengine(shifted, N, T, oracle.Geometry([d, d], f, psi, r), FS)
        assert np.array_equal(yd, y0)


def test_fengine_rejects_window_past_row():
    x, geo = small_input(pad=4)
    geo.D[:] = 5
    with pytest.raises(ValueError):
        oracle.fengine(x, 64, 8, geo, FS)


def test_spectrum0_continuity():
    # Splitting one call into two with spectrum0 advanced gives the same spectra.
    x, geo = small_input(T=8)
    N = 64
    a = oracle.fengine(x, N, 8, geo, FS)
    b = oracle.fengine(np.ascontiguousarray(x[:, 4 * N:]), N, 4, geo, FS, spectrum0=4)
    assert np.array_equal(a[:, 4:], b)


def test_fractional_delay_phase_is_linear_in_channel():
    # A pure delay of f samples of the same tone content rotates bin k by 2 pi k f / N:
    # feeding the same stream to two signals, one with fraction f, gives
    # arg(Y_1 / Y_0) = 2 pi k f / N exactly (no fringe).
    N, T = 256, 2
    g = np.random.default_rng(9)
    row = g.integers(-127, 128, N * T).astype(np.int8)
    x = np.stack([row, row])
    geo = oracle.Geometry([0, 0], [0.0, 0.37], [0, 0], [0, 0])
    Y = oracle.fengine(x, N, T, geo, FS)
    k = np.arange(N // 2)
    ratio = Y[1] / Y[0]
    assert np.allclose(ratio, np.exp(2j * np.pi * k * 0.37 / N)[None, :], atol=1e-12)


# ----------------------------------------------------- sky-model pins (phase)
def _zero_phase_case(sideband_gen=1, sideband_corr=1, flip_f=False, tone_only=False, T=64):
    S, N = 8, 256
    geo = synth.make_geometry(S // 2, seed=21)
    n = N * T + 32
    if tone_only:
        x = synth.voltages(S, n, geo, FS, seed=22, rho=0.0, sigma_t=0.0, noise=False,
                           tone_bin=37, tone_N=N, tone_amp=100.0, sideband=sideband_gen)
    else:
        x = synth.voltages(S, n, geo, FS, seed=22, rho=1.0, sigma_t=12.0, noise=False,
                           sideband=sideband_gen)
    f = -geo.f if flip_f else geo.f
    Y = oracle.fengine(x, N, T, oracle.Geometry(geo.D, f, geo.psi0, geo.rate), FS,
                       sideband=sideband_corr)
    V = oracle.xengine(Y)
    return V, S, N, T, geo


def _same_pol_pairs(S):
    return [(i, j) for i in range(S) for j in range(i + 1, S) if (i - j) % 2 == 0]


def _max_same_pol_phase(V, S, ks):
    return max(float(np.max(np.abs(np.angle(V[ks, oracle.pair_index(i, j)]))))
               for i, j in _same_pol_pairs(S))


def test_zero_phase_after_correction_broadband():
    # rho = 1 delayed, fringe-rotated copies of one sky signal: after the integer delay,
    # FSTC and fringe stop of Eq. 2 every same-polarisation baseline has zero phase up to
    # (a) the random phase of the decorrelated part -- the |f_i - f_j| samples at the edge
    # of each window that the other window does not hold, and ADC rounding (variance 1/12
    # against sigma_t^2 = 144 per signal) -- whose per-channel std is sqrt(eps / 2T), and
    # (b) leakage of the mirror-image (negative-frequency) half of the real signal through
    # the rectangular window's sidelobes, which post-FFT fringe stopping rotates the wrong
    # way; its relative power into bin k is about 1/(pi^2 k) + 1/(pi^2 (N/2 - k)).
    V, S, N, T, geo = _zero_phase_case(T=512)
    ks = np.arange(8, N // 2 - 8)
    leak = 1 / (math.pi ** 2 * ks) + 1 / (math.pi ** 2 * (N // 2 - ks))
    for i, j in _same_pol_pairs(S):
        eps = 2 * abs(geo.f[i] - geo.f[j]) / N + 2 * (1 / 12) / 144
        sd = math.sqrt(eps / (2 * T))
        ph = np.angle(V[ks, oracle.pair_index(i, j)])
        assert np.all(np.abs(ph) < 6 * sd + leak), (i, j)
        # a wrong fractional-delay term would give a phase of order 2 pi k f / N here
        assert abs(np.mean(ph)) < 6 * sd / math.sqrt(len(ks)) + np.mean(leak), (i, j)


def test_zero_phase_after_correction_tone():
    # A bin-centred tone has no leakage, so only ADC rounding of the int8 samples moves its
    # phase: rounding noise of variance 1/12 per sample puts sqrt(N/12) into the bin against
    # the tone's A N / 2, so per signal the phase std is at most sqrt(N/12) / (A N / 2).
    V, S, N, T, _ = _zero_phase_case(tone_only=True)
    bound = 4 * math.sqrt(2) * math.sqrt(N / 12) / (100.0 * N / 2)
    assert _max_same_pol_phase(V, S, [37]) < bound


def test_zero_phase_fails_with_wrong_sideband_or_fraction_sign():
    ks = np.arange(4, 124)
    V, S, *_ = _zero_phase_case(sideband_corr=-1)
    assert _max_same_pol_phase(V, S, ks) > 0.1
    V, S, *_ = _zero_phase_case(flip_f=True)
    assert _max_same_pol_phase(V, S, ks) > 0.1


def test_coherence_matches_analytic_value():
    # Common component of power fraction rho: expected same-pol cross coherence
    # rho * (1 - |f_i - f_j| / N) * sigma_t^2 / (sigma_t^2 + 1/12) (window offset of the
    # residual fraction, ADC rounding noise); cross-pol coherence 0 (independent pols).
    S, N, T, rho, st = 8, 512, 512, 0.3, 12.0
    geo = synth.make_geometry(S // 2, seed=31)
    x = synth.voltages(S, N * T + 32, geo, FS, seed=32, rho=rho, sigma_t=st)
    Y = oracle.fengine(x, N, T, geom_of(geo), FS)
    V = oracle.xengine(Y)
    ks = np.arange(4, N // 2 - 2)
    tol = 5 * (1 - rho ** 2) / math.sqrt(len(ks) * T)
    for i in range(S):
        for j in range(i + 1, S):
            p = oracle.pair_index(i, j)
            r = V[ks, p] / np.sqrt(V[ks, oracle.pair_index(i, i)].real * V[ks, oracle.pair_index(j, j)].real)
            if (i - j) % 2 == 0:
                expect = rho * (1 - abs(geo.f[i] - geo.f[j]) / N) * st ** 2 / (st ** 2 + 1 / 12)
            else:
                expect = 0.0
            assert abs(np.mean(r.real) - expect) < tol, (i, j)
            assert abs(np.mean(r.imag)) < tol, (i, j)


# ------------------------------------------------------------------ X-engine
def _full_matrix(Vk, S):
    M = np.zeros((S, S), dtype=complex)
    for j in range(S):
        for i in range(j + 1):
            M[i, j] = Vk[oracle.pair_index(i, j)]
            M[j, i] = np.conj(M[i, j])
    return M


def test_xengine_hermitian_psd_cauchy_schwarz():
    S, T, C = 6, 40, 5
    Y = synth.random_spectra_f32(S, T, C, seed=3).astype(np.complex128)
    V = oracle.xengine(Y)
    for k in range(C):
        M = _full_matrix(V[k], S)
        assert np.all(np.diag(M).imag == 0)
        ev = np.linalg.eigvalsh(M)
        assert ev.min() > -1e-9 * ev.max()
        d = np.real(np.diag(M))
        assert np.all(np.abs(M) ** 2 <= np.outer(d, d) * (1 + 1e-12))


def test_xengine_brute_force_tiny():
    # Two signals, two spectra, one channel, by hand.
    Y = np.array([[[1 + 2j], [3 - 1j]], [[-2 + 1j], [0.5 + 0.5j]]])  # [S=2][T=2][C=1]
    V = oracle.xengine(Y)
    y0, y1 = Y[0, :, 0], Y[1, :, 0]
    assert V[0, 0] == pytest.approx(np.sum(np.abs(y0) ** 2))
    assert V[0, 2] == pytest.approx(np.sum(np.abs(y1) ** 2))
    assert V[0, 1] == pytest.approx((1 + 2j) * (-2 - 1j) + (3 - 1j) * (0.5 - 0.5j))


def test_int_xengine_constant_input_closed_form():
    # q = (127, -127) everywhere: A = T * 2 * 127^2 for every pair, imaginary part 0.
    S, T, C = 5, 33, 3
    q = np.zeros((S, T, C, 2), dtype=np.int8)
    q[..., 0], q[..., 1] = 127, -127
    A = oracle.xengine_int(q)
    assert np.all(A[..., 0] == T * 2 * 127 * 127)
    assert np.all(A[..., 1] == 0)


def test_int_xengine_equals_float_xengine_on_integers():
    S, T, C = 7, 50, 4
    q = synth.random_spectra_int8(S, T, C, seed=4)
    A = oracle.xengine_int(q)
    V = oracle.xengine(q[..., 0].astype(float) + 1j * q[..., 1].astype(float))
    assert np.array_equal(A[..., 0].astype(float), V.real)
    assert np.array_equal(A[..., 1].astype(float), V.imag)
    for k in range(C):
        assert np.all(A[k, [oracle.pair_index(s, s) for s in range(S)], 1] == 0)


def test_integration_split_invariance():
    S, T, C = 4, 64, 3
    q = synth.random_spectra_int8(S, T, C, seed=8)
    A = oracle.xengine_int(q)
    B = oracle.xengine_int(np.ascontiguousarray(q[:, :T // 2]))
    oracle.xengine_int(np.ascontiguousarray(q[:, T // 2:]), B)
    assert np.array_equal(A, B)


# ---------------------------------------------------------------- requantise
def test_quantize_round_half_even_and_clamp():
    vals = np.array([0.5, 1.5, 2.5, -0.5, -1.5, -2.5, 126.5, 127.5, 200.0, -200.0, 0.49999, -3.2])
    Y = (vals + 1j * vals[::-1]).reshape(1, 1, -1)
    q = oracle.quantize_int8(Y, np.ones((1, vals.size)))
    expect = np.array([0, 2, 2, 0, -2, -2, 126, 127, 127, -127, 0, -3])
    assert np.array_equal(q[0, 0, :, 0], expect)
    assert np.array_equal(q[0, 0, :, 1], expect[::-1])
    assert q.min() >= -127


def test_sigma_closed_form():
    # |Y| = a everywhere -> sigma = a / sqrt(2)
    a = 3.0
    Y = a * np.exp(1j * np.linspace(0, 6, 24)).reshape(2, 4, 3)
    assert np.allclose(oracle.sigma(Y), a / np.sqrt(2), rtol=1e-14)
    assert np.allclose(oracle.int8_scale(oracle.sigma(Y)), np.float32(4 * a / np.sqrt(2) / 127))


def test_e4m3_table_matches_ocp_definition():
    # OCP FP8 E4M3: max finite 448 (0x7E), 1.0 = 0x38, min normal 2^-6 (0x08),
    # min subnormal 2^-9 (0x01), NaN at 0x7F/0xFF, no infinities, symmetric sign.
    t = oracle.e4m3_decode_table()
    assert t[0x7E] == 448.0 and t[0x38] == 1.0 and t[0x08] == 2.0 ** -6 and t[0x01] == 2.0 ** -9
    assert math.isnan(t[0x7F]) and math.isnan(t[0xFF])
    pos = t[:0x7F]
    assert np.all(np.diff(pos) > 0)  # strictly increasing codes 0..0x7E
    assert np.array_equal(t[0x80:0xFF], -pos)
    assert t[0x3F] == 1.875 and t[0x40] == 2.0


def test_e4m3_encode_rounding():
    enc = oracle.e4m3_encode
    assert enc(1.0) == 0x38 and enc(448.0) == 0x7E and enc(1e9) == 0x7E and enc(-1e9) == 0xFE
    assert enc(1.0625) == 0x38   # tie 1.0 / 1.125 -> even code
    assert enc(1.1875) == 0x3A   # tie 1.125 / 1.25 -> even code
    assert enc(2.0 ** -10) == 0  # tie 0 / 2^-9 -> 0
    assert enc(3 * 2.0 ** -10) == 0x02  # tie 2^-9 / 2^-8 -> even code 0x02
    assert enc(-1.3) == 0x80 | enc(1.3)
    g = np.random.default_rng(1)
    t = oracle.e4m3_decode_table()[:0x7F]
    for v in g.uniform(-500, 500, 300):
        c = enc(v)
        dv = oracle.e4m3_decode([c])[0]
        # nearest representable value (saturated)
        best = np.min(np.abs(t - min(abs(v), 448.0)))
        assert abs(abs(dv) - min(abs(v), 448.0)) == pytest.approx(best, abs=1e-12)


def test_scale_visibilities():
    A = np.array([[[10, -2], [4, 0], [7, 1]]], dtype=np.int64)  # C=1, P=3 (S=2)
    sc = np.array([[0.5], [2.0]])
    V = oracle.scale_visibilities(A, sc)
    assert np.allclose(V[0, 0], [2.5, -0.5]) and np.allclose(V[0, 1], [4.0, 0.0])
    assert np.allclose(V[0, 2], [28.0, 4.0])


# ----------------------------------------------------------------------- MAD
def test_median_matches_numpy():
    g = np.random.default_rng(2)
    for n in (1, 2, 5, 64, 257):
        v = g.standard_normal(n)
        assert oracle.median(v) == np.median(v)


def test_mad_worked_example():
    # Eq. 3 / Eq. 4 by hand: x = 1,2,3,4,100 -> median 3, deviations 2,1,0,1,97 -> MAD 1;
    # threshold M*MAD/0.6745 = 4.448 for M = 3: only 100 is flagged.
    fl, med, mad = oracle.mad_flags([1, 2, 3, 4, 100], 3.0)
    assert med == 3 and mad == 1
    assert list(fl) == [0, 0, 0, 0, 1]


@pytest.mark.parametrize("M", [2.5, 3.0])
def test_mad_false_flag_rate_on_gaussian(M):
    # For Gaussian data MAD/0.6745 estimates sigma, so the false-flag rate is 2(1 - Phi(M)).
    n = 200_000
    x = np.random.default_rng(int(M * 10)).standard_normal(n)
    fl, _, _ = oracle.mad_flags(x, M)
    p = math.erfc(M / math.sqrt(2))
    assert abs(fl.mean() - p) < 3 * math.sqrt(p * (1 - p) / n) + 2e-4


def test_error_metric_properties():
    S, T, C = 4, 20, 3
    Y = synth.random_spectra_f32(S, T, C, seed=12).astype(np.complex128)
    V = oracle.xengine(Y)
    assert oracle.normalized_error(V, V, S) == (0.0, 0.0)
    e_max, e_fro = oracle.normalized_error(V * (1 + 1e-6), V, S)
    assert 0.9e-6 < e_max <= 1.01e-6 and abs(e_fro - 1e-6) < 1e-9


# ---------------------------------------------------------------- MAD tiles
def test_mad_tile_flags_worked_example():
    # constant power with one loud spectrum (row 5) and one loud channel (col 17):
    # every other row mean and column mean is identical, so MAD = 0 and exactly
    # row 5 and column 17 exceed Eq. 4's threshold (strict >).
    pw = np.ones((1, 64, 256))
    pw[0, 5, :] *= 10
    pw[0, :, 17] *= 10
    fl = oracle.mad_tile_flags(pw)
    expect = np.zeros((64, 256), dtype=np.uint8)
    expect[5, :] = 1
    expect[:, 17] = 1
    assert np.array_equal(fl[0], expect)


def test_mad_tile_flags_outliers_in_noise_and_tiling():
    g = np.random.default_rng(3)
    pw = g.exponential(1.0, size=(2, 128, 512))
    pw[1, 70:72, 256:512] += 50.0       # a 2-spectrum burst in the lower-right tile of signal 1
    pw[0, :64, 300] += 40.0             # a tone in the upper-right tile of signal 0
    fl = oracle.mad_tile_flags(pw)
    assert fl[1, 70:72, 256:].all() and fl[0, :64, 300].all()
    assert not fl[1, 70:72, :256].all()  # the burst's other tile is unaffected
    assert not fl[0, 64:, 300].all()      # the tone only lives in the first tile


def test_mad_tile_statistics_apart():
    # the worked example with one statistic at a time: the loud spectrum alone, the loud
    # channel alone, and a cell of a noisy tile flagged by both is the union of the two
    pw = np.ones((1, 64, 256))
    pw[0, 5, :] *= 10
    pw[0, :, 17] *= 10
    rows = oracle.mad_tile_flags(pw, stats="rows")[0]
    cols = oracle.mad_tile_flags(pw, stats="columns")[0]
    assert rows[5].all() and rows.sum() == 256
    assert cols[:, 17].all() and cols.sum() == 64
    g = np.random.default_rng(6)
    pw = g.exponential(1.0, size=(2, 128, 512))
    pw[0, 10:12, :] += 30.0
    pw[1, :, 40] += 25.0
    both = oracle.mad_tile_flags(pw)
    r, c = oracle.mad_tile_flags(pw, stats="rows"), oracle.mad_tile_flags(pw, stats="columns")
    assert np.array_equal(both, r | c)
    assert r[0, 10:12].all() and not c[0, 10:12].all()
    assert c[1, :, 40].all() and not r[1, :, 40].all()


def test_guarded_flags_are_the_network_or_the_column_statistic():
    # the guard adds the tile columns that the column statistic flags and nothing else;
    # guard_m = 0 is the network alone
    g = np.random.default_rng(7)
    pw = g.exponential(1.0, size=(1, 64, 256))
    pw[0, :, 99] += 6.0  # a weak tone: a column outlier the network's 7 x 7 view may not see
    params = g.normal(0, 0.1, oracle.cnn_param_count())
    f0, z = oracle.cnn_guarded_flags(params, pw, 0.5, 0.0)
    f3, z3 = oracle.cnn_guarded_flags(params, pw, 0.5, 3.0)
    assert np.array_equal(z, z3) and np.array_equal(f0, (z > 0).astype(np.uint8))
    cols = oracle.mad_tile_flags(pw, 3.0, stats="columns")
    assert np.array_equal(f3, f0 | cols) and f3[0, :, 99].all()


def test_mad_tile_false_flag_rate_on_clean_power():
    # Clean per-cell power is exponential; a row statistic averages 256 cells and a column
    # statistic 64, both close to Gaussian, so each is flagged with probability close to
    # 2(1 - Phi(3)) = 0.27% (skew of the means makes the upper tail a little heavier).
    g = np.random.default_rng(4)
    pw = g.exponential(1.0, size=(4, 64 * 40, 256))
    fl = oracle.mad_tile_flags(pw)
    rows = fl.all(axis=2).mean()     # a flagged row flags its whole tile width
    p = math.erfc(3 / math.sqrt(2))
    assert 0.3 * p < rows < 3 * p
    cols = fl.reshape(4, 40, 64, 256).all(axis=2).mean()
    assert 0.3 * p < cols < 4 * p


def test_pair_counts_brute_force():
    g = np.random.default_rng(5)
    fl = (g.random((3, 40, 4)) < 0.3).astype(np.uint8)
    n = oracle.pair_counts(fl)
    for k in range(4):
        for j in range(3):
            for i in range(j + 1):
                assert n[k, oracle.pair_index(i, j)] == sum(
                    1 for m in range(40) if fl[i, m, k] == 0 and fl[j, m, k] == 0)
