"""F-engine in table mode (the 1440-step sin/cos look-up table of section
2.3.2) through the C ABI against the table-mode oracle, which decides every
table index with the same FP64 operations: FP32 spectra at several lengths,
sidebands, baseband offsets and spectrum offsets, the whole FX chain at the
FP32 gate, and the int8 codes.  Also the precision diagnostics of section 4.1
(mean-to-rms ratio of auto spectra, spread of visibility ratios), comparing
the table, 16-bit fixed-point, int8 and e4m3 paths with the FP32 path."""
import numpy as np
import pytest

import oracle
import paper_0910_1517_amd as corr
import synth
from gpu_util import FS, geom_dev, run_fengine, run_x_integrate, upload_streams

pytestmark = pytest.mark.gpu


def ogeom(g):
    return oracle.Geometry(g.D, g.f, g.psi0, g.rate)


def case(S, N, T, seed):
    geo = synth.make_geometry(S // 2, seed=seed)
    x = synth.voltages(S, N * T + 32, geo, FS, seed=seed + 1, tone_bin=37, tone_N=N)
    return geo, x


@pytest.mark.parametrize("N,T,nu_bb,sb,s0", [(512, 64, 0.0, 1, 5), (2048, 32, 150e6, -1, 123457),
                                             (4096, 32, 0.0, 1, 0), (16384, 32, 1.4e9, 1, 77)])
def test_table_mode_fp32_spectra(N, T, nu_bb, sb, s0):
    S = 4
    print("lut fp32", N, T, nu_bb, sb, s0, flush=True)
    geo, x = case(S, N, T, seed=N + 1)
    plan = corr.Plan(S, N, T, precision=corr.FP32, max_delay=16, phase_lut=1, nu_bb=nu_bb, sideband=sb)
    x_dev, rs = upload_streams(x, N, T, 16)
    spec = run_fengine(plan, x_dev, rs, geom_dev(geo), spectrum0=s0)
    Yg = corr.unpack_spectra(spec, corr.FP32, S, plan.C, T)
    Yg = Yg[..., 0].astype(np.float64) + 1j * Yg[..., 1]
    Y = oracle.fengine_lut(x, N, T, ogeom(geo), FS, nu_bb=nu_bb, sideband=sb, spectrum0=s0)
    rms = np.sqrt(np.mean(np.abs(Y) ** 2, axis=-1, keepdims=True))
    err = np.abs(Yg - Y) / rms
    # same bound as the direct phase; one table index decided differently
    # would put a 4e-3 relative error on its cell
    assert err.max() < 2e-5, err.max()
    assert np.sqrt(np.mean(err ** 2)) < 2e-6
    # and the table is really used: the direct phase differs by up to half a step
    Yd = oracle.fengine(x, N, T, ogeom(geo), FS, nu_bb=nu_bb, sideband=sb, spectrum0=s0)
    assert (np.abs(Yg - Yd) / rms).max() > 1e-4


def test_table_mode_fx_fp32_e_max():
    S, N, T = 8, 512, 1024
    geo, x = case(S, N, T, seed=5)
    plan = corr.Plan(S, N, T, precision=corr.FP32, phase_lut=1)
    x_dev, rs = upload_streams(x, N, T, 16)
    spec = run_fengine(plan, x_dev, rs, geom_dev(geo))
    _, state, _ = run_x_integrate(plan, spec)
    V64 = oracle.xengine(oracle.fengine_lut(x, N, T, ogeom(geo), FS))
    e_max, _ = oracle.normalized_error(state, V64, S)
    assert e_max <= 1e-5, e_max


def test_table_mode_int8_codes():
    import torch
    S, N, T = 8, 1024, 256
    geo, x = case(S, N, T, seed=21)
    Y = oracle.fengine_lut(x, N, T, ogeom(geo), FS)
    scale = oracle.int8_scale(oracle.sigma(Y))
    plan = corr.Plan(S, N, T, precision=corr.INT8, phase_lut=1)
    x_dev, rs = upload_streams(x, N, T, 16)
    spec = run_fengine(plan, x_dev, rs, geom_dev(geo), torch.from_numpy(scale.ravel()).cuda())
    qg = corr.unpack_spectra(spec, corr.INT8, S, plan.C, T).astype(np.int64)
    qo = oracle.quantize_int8(Y, scale.astype(np.float64)).astype(np.int64)
    u = np.stack([Y.real, Y.imag], -1) / scale.astype(np.float64)[:, None, :, None]
    frac = np.abs(np.abs(u - np.floor(u)) - 0.5)
    diff = qg - qo
    assert np.abs(diff).max() <= 1
    bad = diff != 0
    assert np.all(frac[bad] < 1e-3) and bad.mean() <= 1e-4


def _diagnostics(out, S):
    """Section 4.1's two figures for every path of out (name -> [nsub][C][P]
    complex visibilities per sub-integration, "fp32" the reference): the
    change of the mean-to-rms ratio of the auto spectra over the
    sub-integrations, and the rms of V_path / V_fp32 - 1 over the
    cross-antenna visibilities of the whole observation (channel 0 left out).
    The ratio is taken on the same-polarisation pairs, where the common source
    makes the visibility large: the cross-polarisation pairs of this
    unpolarised sky hold noise only, and a ratio to noise has no scale (a few
    near-zero channels would set the figure)."""
    auto = [oracle.pair_index(i, i) for i in range(S)]
    cross = [oracle.pair_index(i, j) for j in range(S) for i in range(j) if i // 2 != j // 2 and i % 2 == j % 2]
    mr = {k: (v[:, 1:, auto].real.mean(0) / v[:, 1:, auto].real.std(0)) for k, v in out.items()}
    total = {k: v.sum(0) for k, v in out.items()}
    res = {}
    for k in out:
        if k == "fp32":
            continue
        deg = 1.0 - np.mean(mr[k]) / np.mean(mr["fp32"])
        ratio = total[k][1:, cross] / total["fp32"][1:, cross] - 1.0
        res[k] = (deg, float(np.sqrt(np.mean(np.abs(ratio) ** 2))))
    return res


def _oracle_paths(x, geo, S, N, Tsub, nsub):
    """The same observation through the oracle: FP32 reference (FP64 here), the
    table phase, int8 and e4m3 with scales from the first sub-integration, and
    the 16-bit fixed-point path from the bare FFT (its FP32 values) at 8 sigma /
    32767; per sub-integration visibilities as in _diagnostics."""
    T = Tsub * nsub
    g = ogeom(geo)
    z = np.zeros(S)
    Y = oracle.fengine(x, N, T, g, FS)
    Yl = oracle.fengine_lut(x, N, T, g, FS)
    sig = oracle.sigma(Y[:, :Tsub])
    s8, s4 = oracle.int8_scale(sig), oracle.fp8_scale(sig)
    q8 = oracle.quantize_int8(Y, s8)
    d4 = oracle.e4m3_decode_table()[oracle.quantize_fp8(Y, s4)]
    Y4 = (d4[..., 0] + 1j * d4[..., 1]) * s4[:, None, :].astype(np.float64)
    Xb = oracle.fengine(x, N, T, oracle.Geometry(geo.D, z, z, z), FS).astype(np.complex64)
    s16 = s8 * np.float32(2 * 127.0 / 32767.0)
    _, y16 = oracle.fix16_spectra(Xb, g, FS, s16)
    out = {k: [] for k in ("fp32", "table", "int8", "e4m3", "fix16")}
    for i in range(nsub):
        sl = slice(i * Tsub, (i + 1) * Tsub)
        out["fp32"].append(oracle.xengine(Y[:, sl]))
        out["table"].append(oracle.xengine(Yl[:, sl]))
        out["e4m3"].append(oracle.xengine(Y4[:, sl]))
        for k, A, sc in (("int8", oracle.xengine_int(q8[:, sl]), s8),
                         ("fix16", oracle.xengine_i16(y16[:, sl]), s16)):
            v = oracle.scale_visibilities(A, sc)
            out[k].append(v[..., 0] + 1j * v[..., 1])
    return {k: np.stack(v) for k, v in out.items()}


def test_precision_diagnostics():
    """Section 4.1's two diagnostics on one synthetic observation: for each
    path (FP32 with the table phase, the 16-bit fixed-point path, int8,
    e4m3), the mean-to-rms ratio of every auto spectrum over 32
    sub-integrations relative to the FP32 path's, and the rms spread of
    V_path / V_fp32 - 1 over the cross visibilities.  The paper reports 1.5%
    and 2% for its 16-bit fixed-point path.  Both figures of every path are
    pinned to the oracle's, computed from the same samples with the same
    definitions (its paths are pinned on their own: the table's phase error
    to half a step, the quantisers to their rounding rules, the integer
    X-engines to brute force): the GPU's figures must agree with them, the
    spread to 0.1% of itself and the mean/rms change to 0.5% of itself
    (2e-8 where it is zero).  Measured: the spreads agree to 5e-5 of
    themselves, the changes to 6e-5 (int8) and 9e-4 (e4m3, whose coarse steps
    turn the FP32-against-FP64 differences of the spectra into a few
    whole-step code flips) of themselves."""
    import torch
    S, N, Tsub, nsub = 8, 1024, 256, 32
    geo = synth.make_geometry(S // 2, seed=41)
    x = synth.voltages(S, N * Tsub * nsub + 32, geo, FS, seed=42, rho=0.5)
    x_dev, rs = upload_streams(x, N, Tsub * nsub, 16)
    g_dev = geom_dev(geo)
    paths = {"fp32": dict(precision=corr.FP32), "table": dict(precision=corr.FP32, phase_lut=1),
             "int8": dict(precision=corr.INT8), "e4m3": dict(precision=corr.FP8_E4M3)}
    out = {}
    for name, kw in paths.items():
        plan = corr.Plan(S, N, Tsub, **kw)
        scale = None
        if kw["precision"] != corr.FP32:  # scales held from a calibration call, as in the benchmark
            cal = corr.Plan(S, N, Tsub, precision=kw["precision"], scale_mode=corr.SCALE_COMPUTE)
            scale = torch.zeros(S * plan.C, dtype=torch.float32, device="cuda")
            tmp = cal.alloc("spectra", zero=False)
            cal.fengine(x_dev, g_dev, tmp, scale, row_stride=rs)
        vis = []
        for i in range(nsub):
            spec = plan.alloc("spectra", zero=False)
            # sub-integration i starts at sample i Tsub N of the rows
            plan.fengine(x_dev[:, i * Tsub * N:], g_dev, spec, scale, row_stride=rs, spectrum0=i * Tsub)
            _, state, _ = run_x_integrate(plan, spec, scale)
            vis.append(state)
        out[name] = np.stack(vis)  # [nsub][C][P]
    # the 16-bit fixed-point path: the FP32 F-engine without the fractional-delay and fringe
    # terms (the bare FFT of the integer-delayed samples), 16-bit codes at a level of
    # 8 sigma / 32767 (the int8 calibration's 4 sigma / 127, rescaled: codes of rms 4096 that
    # never clip; at 4 sigma the clipped tails alone move the mean/rms ratio by ~0.13%), the
    # integer rotation by the Q14 table, exact integer sums
    plan = corr.Plan(S, N, Tsub, precision=corr.FP32)
    cal = corr.Plan(S, N, Tsub, precision=corr.INT8, scale_mode=corr.SCALE_COMPUTE)
    s8 = torch.zeros(S * plan.C, dtype=torch.float32, device="cuda")
    cal.fengine(x_dev, g_dev, cal.alloc("spectra", zero=False), s8, row_stride=rs)
    sc16 = s8 * np.float32(2 * 127.0 / 32767.0)
    bare = corr.geom_to_device(corr.geom_array(geo.D, np.zeros(S), np.zeros(S), np.zeros(S)))
    spec = plan.alloc("spectra", zero=False)
    y16 = torch.empty((S, Tsub, plan.C, 2), dtype=torch.int16, device="cuda")
    acc = torch.empty(plan.C * plan.P * 2, dtype=torch.int64, device="cuda")
    v16 = torch.empty(plan.C * plan.P * 2, dtype=torch.float64, device="cuda")
    vis = []
    for i in range(nsub):
        plan.fengine(x_dev[:, i * Tsub * N:], bare, spec, None, row_stride=rs, spectrum0=i * Tsub)
        plan.fix16_spectra(spec, g_dev, sc16, y16, spectrum0=i * Tsub)
        plan.fix16_xengine(y16, acc, scale=sc16, vis=v16)
        v = v16.cpu().numpy().reshape(plan.C, plan.P, 2)
        vis.append(v[..., 0] + 1j * v[..., 1])
    out["fix16"] = np.stack(vis)
    gpu = _diagnostics(out, S)
    ref = _diagnostics(_oracle_paths(x, geo, S, N, Tsub, nsub), S)
    for k in ("table", "fix16", "int8", "e4m3"):
        (dg, sg), (do, so) = gpu[k], ref[k]
        print("precision diagnostics %s: mean/rms change %.6g%% (oracle %.6g%%), visibility ratio spread %.6g "
              "(oracle %.6g)" % (k, 100 * dg, 100 * do, sg, so), flush=True)
        assert abs(dg - do) <= 5e-3 * abs(do) + 2e-8, k
        assert abs(sg / so - 1.0) < 1e-3, k
