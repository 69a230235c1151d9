"""Voltage blanker (section 5, Eq. 3 and 4) and its noise table through the C
ABI against the oracle.

Everything here is integer or exactly representable, so the bar is
bit-exactness: the noise table, the blanked bytes (in place and out of place),
the per-block counts and the per-block (2 median, 4 MAD).  The cases cover
every register-tile size of the kernel (blocks of 16 to 65536 samples), ragged
last blocks and rows shorter than a chunk, blocks whose MAD is 0, replacements
that clamp, tables shorter than a block, blocks with more outliers than the
kernel's queue holds (small M), and the row padding, which must never be
written.
"""
import numpy as np
import pytest

import oracle
import paper_0910_1517_amd as corr
import synth

pytestmark = pytest.mark.gpu


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def gpu_table(seed, S, L):
    import torch
    t = torch.full((S, L), float("nan"), device="cuda")
    corr.blank_noise_table(seed, t)
    torch.cuda.synchronize()
    return t


def run_blank(x, B, M, table, *, sample0=0, in_place=True, pad=0):
    """x int8 [S][n] host; returns (out [S][n], padding after the call,
    counts, stats) from the GPU, rows padded by `pad` bytes (a multiple of
    16 after rounding n up) that hold a marker."""
    import torch
    S, n = x.shape
    rs = (n + 15) // 16 * 16 + pad
    buf = np.full((S, rs), 0x5A, np.int8)
    buf[:, :n] = x
    xd = dev(buf)
    out = xd if in_place else torch.full_like(xd, 0x33)
    nb = -(-n // B) if n else 0
    counts = torch.full((S, max(nb, 1)), -1, dtype=torch.int32, device="cuda")
    stats = torch.full((S, max(nb, 1), 2), -7, dtype=torch.int32, device="cuda")
    corr.blank_voltages(xd, table, block=B, M=M, out=out, counts=counts, stats=stats, sample0=sample0, n=n)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    if not in_place:
        assert np.array_equal(xd.cpu().numpy(), buf), "the input changed out of place"
    return o[:, :n], o[:, n:], counts.cpu().numpy()[:, :nb], stats.cpu().numpy()[:, :nb]


def data(kind, S, n, seed):
    g = synth.rng(seed, 40, S, n)
    if kind == "impulses":
        geo = synth.make_geometry(max(1, S // 2))
        x = synth.voltages(S, n, geo.subset(np.arange(S)) if geo.S != S else geo, 66.666666e6, mode="bulk",
                           seed=seed)
        synth.add_impulses(x, geo.subset(np.arange(S)) if geo.S != S else geo, n, seed=seed)
        return x
    if kind == "heavy":   # Student-t 2: many outliers of every size
        return np.clip(np.rint(g.standard_t(2, size=(S, n)) * 6), -128, 127).astype(np.int8)
    if kind == "low":     # a level or two of noise: MAD = 0 and half-integer medians
        v = np.rint(g.normal(0, 0.6, size=(S, n)))
        v[g.random((S, n)) < 0.01] = 90
        return np.clip(v, -128, 127).astype(np.int8)
    if kind == "extreme":  # wide noise with rails: replacements clamp
        v = np.rint(g.normal(60, 50, size=(S, n)))
        v[g.random((S, n)) < 0.03] = -128
        return np.clip(v, -128, 127).astype(np.int8)
    raise ValueError(kind)


CASES = [  # (kind, S, n, block, M, table length, sample0, in place, pad)
    ("impulses", 4, 3 * 16384 + 1000 + 5, 16384, 3.0, 1 << 16, 0, True, 16),
    ("impulses", 2, 5 * 4096, 4096, 2.5, 1 << 12, 12345, False, 0),
    ("heavy", 3, 2 * 65536 + 17, 65536, 3.0, 1 << 10, 7, True, 32),
    ("heavy", 2, 3 * 32768 - 48, 32768, 2.75, 1 << 15, 0, False, 16),
    ("heavy", 2, 2 * 8192 + 16, 8192, 3.0, 1 << 13, 99, True, 0),
    ("heavy", 5, 1000, 16, 2.5, 64, 3, True, 16),
    ("low", 3, 4 * 1024 + 9, 1024, 3.0, 256, 0, False, 0),
    ("low", 2, 3000, 48, 2.5, 32, 1, True, 0),
    ("extreme", 3, 20000, 2048, 2.5, 1 << 11, 5, True, 0),
    ("extreme", 1, 70000, 65536, 3.0, 1, 0, False, 48),
    ("heavy", 2, 70000, 65536, 0.5, 1 << 12, 11, True, 0),     # more blanked than the queue holds
    ("heavy", 2, 2 * 32768, 32768, 1.0, 1 << 12, 0, False, 16),
    ("heavy", 3, 1, 256, 3.0, 16, 0, True, 16),
    ("heavy", 3, 15, 256, 3.0, 16, 0, False, 0),
    ("heavy", 3, 17, 16, 3.0, 16, 0, True, 0),
]


@pytest.mark.parametrize("case", CASES, ids=["%s-S%d-n%d-B%d" % (c[0], c[1], c[2], c[3]) for c in CASES])
def test_blanker_matches_oracle(case):
    kind, S, n, B, M, L, sample0, in_place, pad = case
    print("blank", case, flush=True)
    x = data(kind, S, n, seed=n + S)
    seed = 1000 + n
    table = gpu_table(seed, S, L)
    ref_table = oracle.blank_noise_table(seed, S, L)
    assert np.array_equal(table.cpu().numpy(), ref_table)
    out, tail, cnt, st = run_blank(x, B, M, table, sample0=sample0, in_place=in_place, pad=pad)
    ref, rcnt, rst = oracle.mad_blank(x, B, M, ref_table, sample0=sample0)
    assert np.array_equal(st, rst), "block statistics"
    assert np.array_equal(cnt, rcnt), "blanked counts"
    bad = np.argwhere(out != ref)
    assert bad.size == 0, "first mismatches %s" % bad[:5].tolist()
    assert np.all(tail == (0x5A if in_place else 0x33)), "row padding written"
    if kind in ("impulses", "heavy", "extreme") and n >= 4096:
        assert rcnt.sum() > 0


def test_empty_rows_enqueue_nothing():
    import torch
    xd = torch.full((2, 64), 7, dtype=torch.int8, device="cuda")
    out = torch.full_like(xd, 3)
    t = gpu_table(1, 2, 16)
    corr.blank_voltages(xd, t, block=16, out=out, n=0)
    torch.cuda.synchronize()
    assert torch.all(out == 3)


@pytest.mark.parametrize("seed,S,L", [(1, 3, 4096), (0xFFFFFFFF00000001, 2, 1), ((1 << 64) - 1, 5, 256),
                                      (0x0910151709101517, 64, 1 << 14)])
def test_noise_table_matches_oracle(seed, S, L):
    print("table", seed, S, L, flush=True)
    assert np.array_equal(gpu_table(seed, S, L).cpu().numpy(), oracle.blank_noise_table(seed, S, L))


def test_noise_table_of_the_largest_rows_sampled():
    """2 x 2^26 entries (the grid strides over them): sampled entries,
    the last ones included, equal the oracle's entry-by-entry values."""
    seed, S, L = 77, 2, 1 << 26
    t = gpu_table(seed, S, L)
    g = np.random.default_rng(3)
    js = np.concatenate([[0, 1, L - 2, L - 1], g.integers(0, L, 60)])
    host = t.cpu().numpy()
    for s in range(S):
        for j in js:
            assert host[s, j] == oracle.blank_noise_entry(seed, s, int(j)), (s, j)
    del t


def test_blanking_versus_zeroing_on_impulsive_rfi():
    """Section 5's outcome on synthetic data: impulsive bursts common to every
    antenna (about 2.5 % of the samples) bias the cross visibilities.
    Blanking the voltages removes most of the bias.  The spectral flagger
    with zeroing and per-pair counts (the library's other RFI path) is shown
    beside it.  The reference is the same pipeline (FP32 F-engine, X-engine,
    integrate) on the inputs without bursts.  The errors are printed; the
    test asserts that blanking cuts the error at least fourfold and preserves
    the autocorrelation power."""
    import torch
    from gpu_util import run_fengine, run_x_integrate
    S, N, T = 8, 1024, 4096
    n = N * T + 16
    rs = (n + 255) // 256 * 256
    geo = synth.make_geometry(S // 2, seed=synth.BASE_SEED + 50)
    z = np.zeros(S)
    g = corr.geom_to_device(corr.geom_array(geo.D, z, z, z))  # the bulk recipe has integer delays only
    x_clean = synth.voltages_device(S, n, geo, seed=synth.BASE_SEED + 51, row_stride=rs)
    x_rfi = x_clean.clone()
    synth.add_impulses(x_rfi, geo, n, seed=synth.BASE_SEED + 52)
    x_blk = x_rfi.clone()
    table = gpu_table(9, S, 1 << 16)
    counts = torch.zeros(S, -(-n // 16384), dtype=torch.int32, device="cuda")
    corr.blank_voltages(x_blk, table, block=16384, M=3.0, counts=counts, n=n)
    plan = corr.Plan(S, N, T, precision=corr.FP32)

    def vis(x):
        spec = run_fengine(plan, x, rs, g)
        return run_x_integrate(plan, spec)[1]

    V0, Vr, Vb = vis(x_clean), vis(x_rfi), vis(x_blk)
    # spectral MAD flags, zeroing and the flag-corrected mean (times T)
    spec = plan.alloc("spectra", zero=False)
    pw = plan.alloc("power", zero=False)
    plan.fengine(x_rfi, g, spec, power=pw, row_stride=rs)
    flags = plan.alloc("flags", zero=False)
    plan.mad_flag(pw, flags, 3.0)
    keep = plan.alloc("keep")
    plan.apply_flags(flags, spec, keep)
    pc = torch.zeros(plan.C * plan.P, dtype=torch.int32, device="cuda")
    plan.pair_counts(keep, pc)
    Vz = run_x_integrate(plan, spec)[1]
    nij = pc.cpu().numpy().reshape(plan.C, plan.P).astype(np.float64)
    Vz = np.where(nij > 0, Vz * T / np.maximum(nij, 1), 0)
    cross = np.array([oracle.pair_index(i, j) for j in range(S) for i in range(j) if i // 2 != j // 2])
    auto = np.array([oracle.pair_index(i, i) for i in range(S)])
    err = lambda V: np.linalg.norm(V[:, cross] - V0[:, cross]) / np.linalg.norm(V0[:, cross])
    e_raw, e_blank, e_zero = err(Vr), err(Vb), err(Vz)
    p_auto = lambda V: V[:, auto].real.sum()
    frac_blanked = counts.sum().item() / (S * n)
    frac_flagged = float(flags.float().mean().item())
    print("impulsive RFI, cross-visibility error vs the burst-free run: raw %.4f, blanked %.4f "
          "(%.4f of the samples replaced), zeroed + counts %.4f (%.4f of the cells flagged); "
          "auto power / clean: raw %.4f, blanked %.4f"
          % (e_raw, e_blank, frac_blanked, e_zero, frac_flagged, p_auto(Vr) / p_auto(V0), p_auto(Vb) / p_auto(V0)))
    assert e_blank < 0.25 * e_raw
    assert abs(p_auto(Vb) / p_auto(V0) - 1.0) < 0.05
    assert 0.01 < frac_blanked < 0.05
