"""The 16-bit fixed-point path (sections 3.1 and 4.1: the 16-bit FFT output,
the integer fringe stop and FSTC from the Q14 phase table, exact 32-bit
correlation products) through the C ABI against the oracle: every 16-bit code
and every rotated value bit-exact on seeded FP32 spectra (levels that are
powers of two and levels that are not, exact halves, saturation, both
sidebands, spectrum offsets), the integer sums of the X-engine bit-exact on
seeded int16 spectra (the largest products included) and its FP64 scaling."""
import numpy as np
import pytest

import oracle
import paper_0910_1517_amd as corr
import synth
from gpu_util import FS, pack_input

pytestmark = pytest.mark.gpu


def _levels(S, C, seed, pow2):
    g = synth.rng(seed, 1)
    if pow2:
        return np.ldexp(np.ones((S, C), np.float32), g.integers(-3, 5, (S, C))).astype(np.float32)
    return g.uniform(0.3, 3.0, (S, C)).astype(np.float32)


def _spectra(S, T, C, sc, seed):
    # ~4000 levels of spread, a few values past the 16-bit range, a few exact halves
    X = synth.random_spectra_f32(S, T, C, seed=seed, sigma=1.0)
    re = (X.real * 4000.0 * sc[:, None, :]).astype(np.float32)
    im = (X.imag * 4000.0 * sc[:, None, :]).astype(np.float32)
    g = synth.rng(seed, 2)
    n = re.size // 500
    i = g.integers(0, re.size, n)
    re.reshape(-1)[i] = (g.integers(-40000, 40000, n) + 0.5).astype(np.float32) * np.broadcast_to(
        sc[:, None, :], re.shape).reshape(-1)[i]
    i = g.integers(0, im.size, n)
    im.reshape(-1)[i] = np.where(g.random(n) < 0.5, -1e6, 1e6).astype(np.float32)
    return re, im


@pytest.mark.parametrize("N,T,sideband,spectrum0,nu_bb,pow2", [
    (512, 64, 1, 0, 0.0, True), (1024, 32, -1, 123457, 150e6, True),
    (2048, 32, 1, 77, 1.4e9, False), (4096, 32, -1, 5, 0.0, False)])
def test_fix16_spectra_bit_exact(N, T, sideband, spectrum0, nu_bb, pow2):
    import torch
    S, C = 6, N // 2
    sc = _levels(S, C, 10 + N, pow2)
    re, im = _spectra(S, T, C, sc, 20 + N)
    g = synth.rng(30 + N)
    f = g.random(S).astype(np.float32).astype(np.float64)
    psi0, rate = g.random(S), g.uniform(-5, 5, S)
    plan = corr.Plan(S, N, T, precision=corr.FP32, sideband=sideband, nu_bb=nu_bb)
    spec = pack_input(plan, np.stack([re, im], -1))
    gd = corr.geom_to_device(corr.geom_array(np.zeros(S, np.int32), f, psi0, rate))
    sc_dev = torch.from_numpy(sc.ravel()).cuda()
    q16 = torch.empty((S, T, C, 2), dtype=torch.int16, device="cuda")
    y16 = torch.empty_like(q16)
    plan.fix16_spectra(spec, gd, sc_dev, y16, q16=q16, spectrum0=spectrum0)
    torch.cuda.synchronize()
    qo, yo = oracle.fix16_spectra(re.astype(np.float64) + 1j * im.astype(np.float64),
                                  oracle.Geometry(np.zeros(S, np.int32), f, psi0, rate), FS, sc.astype(np.float64),
                                  nu_bb=nu_bb, sideband=sideband, spectrum0=spectrum0)
    qg, yg = q16.cpu().numpy(), y16.cpu().numpy()
    print("N %d: %d saturated codes, %d of %d rotated values differ" %
          (N, int((np.abs(qo) == 32767).sum()), int((yg != yo).sum()), yo.size))
    assert (np.abs(qo) == 32767).any()
    assert np.array_equal(qg, qo)
    assert np.array_equal(yg, yo)
    # the output without the optional codes is the same
    y2 = torch.empty_like(y16)
    plan.fix16_spectra(spec, gd, sc_dev, y2, spectrum0=spectrum0)
    assert torch.equal(y2, y16)


@pytest.mark.parametrize("S,T,C", [(8, 64, 512), (5, 96, 256), (16, 320, 256)])
def test_fix16_xengine_bit_exact(S, T, C):
    import torch
    q = synth.random_spectra_int16(S, T, C, seed=S * 1000 + T)
    if S == 16:  # every value at the limit: the largest products, both signs
        q[:] = 32767
        q[1::2, ..., 1] = -32767
    sc = _levels(S, C, 7, False)
    plan = corr.Plan(S, 2 * C, T, precision=corr.FP32)
    y = torch.from_numpy(q).cuda()
    acc = torch.empty(C * plan.P * 2, dtype=torch.int64, device="cuda")
    vis = torch.empty(C * plan.P * 2, dtype=torch.float64, device="cuda")
    plan.fix16_xengine(y, acc, scale=torch.from_numpy(sc.ravel()).cuda(), vis=vis)
    torch.cuda.synchronize()
    A = oracle.xengine_i16(q)
    Ag = acc.cpu().numpy().reshape(C, plan.P, 2)
    assert np.array_equal(Ag, A)
    ii, jj = oracle.pair_table(S)
    f = sc[ii].T.astype(np.float64) * sc[jj].T.astype(np.float64)  # [C][P], exact in FP64
    assert np.array_equal(vis.cpu().numpy().reshape(C, plan.P, 2), A * f[..., None])
    # without the visibilities the sums are the same
    acc2 = torch.empty_like(acc)
    plan.fix16_xengine(y, acc2)
    assert torch.equal(acc2, acc)


def test_fix16_requires_an_fp32_plan():
    import torch
    plan = corr.Plan(4, 512, 32, precision=corr.INT8)
    spec = plan.alloc("spectra")
    gd = corr.geom_to_device(corr.geom_array(np.zeros(4, np.int32), np.zeros(4), np.zeros(4), np.zeros(4)))
    y = torch.empty((4, 32, 256, 2), dtype=torch.int16, device="cuda")
    with pytest.raises(corr.CorrError):
        plan.fix16_spectra(spec, gd, torch.ones(4 * 256, device="cuda"), y)
