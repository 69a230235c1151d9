"""Pins of the oracle voltage blanker (section 5, Eq. 3 and 4: per block of
samples, MAD = median |x - median|, outliers beyond M MAD / 0.6745 replaced by
precomputed Gaussian noise independent per antenna) and of its noise table.

The pins come from outside the oracle's own loops: the generator's published
known-answer vectors, numpy's median, hand-worked blocks, the Irwin-Hall
moments, the normal false-alarm rate 2(1 - Phi(M)), and statistical facts
about the blanked streams (spikes removed, noise scale, independence of the
replacements between antennas)."""
import math
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def test_philox_known_answer_vectors():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(w, 16) for w in r]
        assert list(oracle.philox4x32_10(v[0:4], v[4:6])) == v[6:10]


def test_noise_table_moments_and_grid():
    """Irwin-Hall of 12 uniforms: mean 0, variance 1, excess kurtosis -0.1,
    support (-6, 6), values on the 2^-16 grid; rows of different signals
    uncorrelated; different seeds give different tables."""
    S, L = 4, 1 << 16
    t = oracle.blank_noise_table(7, S, L).astype(np.float64)
    n = t.size
    assert np.all(np.abs(t) < 6.0)
    assert np.array_equal(t * 65536.0, np.round(t * 65536.0))
    assert abs(t.mean()) < 4.0 / math.sqrt(n)
    assert abs(t.var() - 1.0) < 4.0 * math.sqrt(2.0 / n)
    kurt = ((t - t.mean()) ** 4).mean() / t.var() ** 2 - 3.0
    assert abs(kurt - (-0.1)) < 4.0 * math.sqrt(24.0 / n)
    for a in range(S):
        for b in range(a + 1, S):
            assert abs(np.corrcoef(t[a], t[b])[0, 1]) < 4.0 / math.sqrt(L)
    t2 = oracle.blank_noise_table(8, S, L)
    assert abs(np.corrcoef(t[0], t2[0])[0, 1]) < 4.0 / math.sqrt(L)


def test_noise_table_entries_come_from_their_counters():
    """Entry (s, j) is the 12-uniform sum of the Philox blocks at counters
    (j, 0, s, 0) and (j, 0, s, 1) under the seed's two key words."""
    seed = 0x0123456789ABCDEF
    t = oracle.blank_noise_table(seed, 3, 8)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for s, j in [(0, 0), (2, 5), (1, 7)]:
        a = oracle.philox4x32_10([j, 0, s, 0], key)
        b = oracle.philox4x32_10([j, 0, s, 1], key)
        halves = [int(w) & 0xFFFF for w in list(a) + list(b[:2])] + [int(w) >> 16 for w in list(a) + list(b[:2])]
        assert t[s, j] == (sum(halves) + 6 - 6 * 65536) / 65536.0


def test_hand_worked_blocks():
    """Odd block [1, 2, 3, 4, 100]: median 3, deviations 2 1 0 1 97, MAD 1,
    M = 3 threshold 4.448, only 100 is blanked; with a zero table it becomes
    the median.  Even block [-3, -1, 0, 2, 7, 40]: median 1, deviations
    4 2 1 1 6 39, MAD 3, threshold 13.34: only 40 is blanked; with z = 0.5
    it becomes rint(1 + 0.5 * 3 / 0.6745) = rint(3.224) = 3."""
    x = np.array([[1, 2, 3, 4, 100]], np.int8)
    out, cnt, st = oracle.mad_blank(x, 5, 3.0, np.zeros((1, 8), np.float32))
    assert out.tolist() == [[1, 2, 3, 4, 3]] and cnt.tolist() == [[1]] and st.tolist() == [[[6, 4]]]
    x = np.array([[-3, -1, 0, 2, 7, 40]], np.int8)
    out, cnt, st = oracle.mad_blank(x, 6, 3.0, np.full((1, 8), 0.5, np.float32))
    assert out.tolist() == [[-3, -1, 0, 2, 7, 3]] and cnt.tolist() == [[1]] and st.tolist() == [[[2, 12]]]
    # M = 1 lowers the threshold to 4.448: 7 (deviation 6) goes too
    out, cnt, _ = oracle.mad_blank(x, 6, 1.0, np.full((1, 8), 0.5, np.float32))
    assert out.tolist() == [[-3, -1, 0, 2, 3, 3]] and cnt.tolist() == [[2]]


def test_rounding_ties_to_even_and_clamping():
    """A half-integer median with z = 0 rounds to even (rint); a replacement
    beyond the int8 range is clamped."""
    x = np.array([[0, 2, 3, 5, 90, -90]], np.int8)  # median 2.5, MAD 2.5
    out, cnt, _ = oracle.mad_blank(x, 6, 3.0, np.zeros((1, 8), np.float32))
    assert out.tolist() == [[0, 2, 3, 5, 2, 2]] and cnt.tolist() == [[2]]
    x = np.array([[120, 100, 126, 127, 110, -128, 118]], np.int8)  # median 118, MAD 8
    out, _, _ = oracle.mad_blank(x, 7, 3.0, np.full((1, 8), 5.0, np.float32))
    assert out[0, 5] == 127                      # 118 + 5 * 8 / 0.6745 = 177.3
    out, _, _ = oracle.mad_blank(x, 7, 3.0, np.full((1, 8), -5.9, np.float32))
    assert out[0, 5] == 48                       # 118 - 5.9 * 11.861 = 48.02


@pytest.mark.parametrize("B", [6, 7, 64, 255])
def test_block_statistics_and_flags_follow_eq3_eq4(B):
    """Per block (ragged tail included): 2 median and 4 MAD equal numpy's;
    blanked samples are exactly Eq. 4's outliers (the count, and every
    sample outside them untouched)."""
    rng = np.random.default_rng(B)
    S, n, M = 3, 4 * B + B // 2 + 1, 2.5
    x = np.clip(np.round(rng.standard_t(3, size=(S, n)) * 6), -128, 127).astype(np.int8)
    out, cnt, st = oracle.mad_blank(x, B, M, oracle.blank_noise_table(1, S, 64))
    for s in range(S):
        for b in range(cnt.shape[1]):
            blk = x[s, b * B:(b + 1) * B].astype(np.float64)
            med = np.median(blk)
            mad = np.median(np.abs(blk - med))
            assert st[s, b].tolist() == [2 * med, 4 * mad]
            out_blk = out[s, b * B:(b + 1) * B]
            outl = np.abs(blk - med) > M * mad / 0.6745 if mad > 0 else np.zeros(blk.size, bool)
            assert cnt[s, b] == outl.sum()
            assert np.array_equal(out_blk[~outl], blk[~outl].astype(np.int8))


def test_zero_mad_block_is_unchanged():
    """Over half the samples equal: MAD = 0, no scale estimate, nothing
    blanked."""
    x = np.array([[5, 5, 5, 5, 5, -100, 100, 7, 5]], np.int8)
    out, cnt, st = oracle.mad_blank(x, 9, 3.0, np.ones((1, 4), np.float32))
    assert np.array_equal(out, x) and cnt[0, 0] == 0 and st[0, 0].tolist() == [10, 0]


@pytest.mark.parametrize("M", [2.5, 3.0])
def test_false_blank_rate_on_gaussian_noise(M):
    """Clean Gaussian voltages (sigma 20 levels): the blanked fraction is
    close to the normal two-sided tail 2 (1 - Phi(M)) that the 0.6745
    normalisation of Eq. 4 is built on."""
    rng = np.random.default_rng(int(M * 10))
    S, n, B = 2, 1 << 18, 4096
    x = np.clip(np.round(rng.normal(0, 20, size=(S, n))), -128, 127).astype(np.int8)
    _, cnt, _ = oracle.mad_blank(x, B, M, oracle.blank_noise_table(2, S, 1 << 12))
    rate = cnt.sum() / x.size
    expect = math.erfc(M / math.sqrt(2))
    assert 0.8 * expect < rate < 1.2 * expect


def test_spikes_are_removed_and_replacements_have_the_robust_scale():
    """Impulsive RFI (2 % of samples, amplitude 60-120 levels over sigma = 8)
    is blanked completely; the replacements, normalised by each block's
    median and MAD / 0.6745, have mean 0 and variance 1 (plus the rounding's
    1/12 level^2); the blanked stream has the clean stream's variance."""
    rng = np.random.default_rng(5)
    S, n, B, sig = 2, 1 << 17, 2048, 8.0
    clean = np.round(rng.normal(0, sig, size=(S, n)))
    spikes = rng.random((S, n)) < 0.02
    amp = rng.uniform(60, 120, size=(S, n)) * rng.choice([-1, 1], size=(S, n))
    x = np.clip(np.where(spikes, amp, clean), -128, 127).astype(np.int8)
    out, cnt, st = oracle.mad_blank(x, B, 3.0, oracle.blank_noise_table(3, S, 1 << 16))
    assert np.all(np.abs(out[spikes].astype(np.float64)) < 6 * 1.2 * sig)
    z = []
    for s in range(S):
        for b in range(n // B):
            sl = slice(b * B, (b + 1) * B)
            med, sg = st[s, b, 0] / 2.0, st[s, b, 1] / 4.0 / 0.6745
            z.append((out[s, sl][spikes[s, sl]] - med) / sg)
    z = np.concatenate(z)
    assert abs(z.mean()) < 4.0 / math.sqrt(z.size)
    assert abs(z.var() - 1.0) < 0.1
    assert abs(out.astype(np.float64).var() / clean.var() - 1.0) < 0.05
    assert cnt.sum() >= spikes.sum()


def test_replacements_are_independent_between_antennas():
    """Common-mode RFI (the same spikes in two antennas' streams, the usual
    case for terrestrial RFI) correlates the raw streams; the blanked
    streams' correlation is back at the clean level because each antenna's
    replacements come from its own noise table."""
    rng = np.random.default_rng(9)
    n, B, sig = 1 << 18, 4096, 10.0
    clean = np.round(rng.normal(0, sig, size=(4, n)))
    spikes = rng.random(n) < 0.02
    amp = rng.uniform(50, 120, size=n) * rng.choice([-1, 1], size=n)
    x = np.clip(np.where(spikes[None], amp[None], clean), -128, 127).astype(np.int8)
    out, _, _ = oracle.mad_blank(x, B, 3.0, oracle.blank_noise_table(11, 4, 1 << 16))
    raw = np.corrcoef(x[0].astype(np.float64), x[2].astype(np.float64))[0, 1]
    fixed = np.corrcoef(out[0].astype(np.float64), out[2].astype(np.float64))[0, 1]
    rep = np.corrcoef(out[0, spikes].astype(np.float64), out[2, spikes].astype(np.float64))[0, 1]
    assert raw > 0.5
    assert abs(fixed) < 4.0 / math.sqrt(n)
    assert abs(rep) < 4.0 / math.sqrt(spikes.sum())


def test_blocks_are_local_and_the_table_follows_the_absolute_sample():
    """Blanking a row in two calls split on a block edge, the second with
    sample0 at the split, equals one call over the whole row."""
    rng = np.random.default_rng(4)
    S, B = 2, 256
    x = np.clip(np.round(rng.standard_t(2, size=(S, 10 * B)) * 5), -128, 127).astype(np.int8)
    table = oracle.blank_noise_table(6, S, 1 << 10)
    whole, cw, _ = oracle.mad_blank(x, B, 2.5, table)
    a, ca, _ = oracle.mad_blank(x[:, :3 * B], B, 2.5, table)   # 3 B is not a multiple of L
    b, cb, _ = oracle.mad_blank(x[:, 3 * B:], B, 2.5, table, sample0=3 * B)
    assert np.array_equal(whole, np.concatenate([a, b], axis=1))
    assert np.array_equal(cw, np.concatenate([ca, cb], axis=1))
    assert cw.sum() > 0
