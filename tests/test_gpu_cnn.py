"""Learned flagger on the GPU against the FP64 oracle: FP32 training-path
forward, loss and parameter gradient, the Adam update, and the fused FP16
inference kernel (logits and flags), with its edge cases."""
import numpy as np
import pytest

import oracle
import paper_0910_1517_amd as corr
import synth

pytestmark = pytest.mark.gpu

TH, TW = 64, 256


def he_params(seed, scale=1.0):
    """float32 parameters: He-normal weights (std sqrt(2 / fan_in)), small biases."""
    g = synth.rng(seed, 30)
    parts = []
    for co, ci in oracle.CNN_SHAPES:
        parts.append(g.standard_normal(co * ci * 9) * np.sqrt(2.0 / (ci * 9)) * scale)
        parts.append(g.uniform(-0.1, 0.1, co))
    return np.concatenate(parts).astype(np.float32)


def tile_slice(power, tile):
    S, T, C = power.shape
    ntm, ntk = T // TH, C // TW
    s, mt, kt = tile // (ntm * ntk), (tile // ntk) % ntm, tile % ntk
    return power[s, mt * TH:(mt + 1) * TH, kt * TW:(kt + 1) * TW]


def oracle_inputs(power, tiles, labels=None):
    P = power.astype(np.float64)
    x = np.stack([oracle.cnn_tile_input(tile_slice(P, t)) for t in tiles])[:, None]
    if labels is None:
        return x
    y = np.stack([tile_slice(labels, t) for t in tiles]).astype(np.float64)[:, None]
    return x, y


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_forward_fp32_matches_oracle():
    import torch
    S, T, C = 2, 128, 512
    power = synth.power_spectra(S, T, C, seed=11)
    params = he_params(1)
    tiles = np.array([5, 0, 3, 7, 2], dtype=np.int32)
    cnn = corr.CNN(max_tiles=8)
    logits = torch.empty(len(tiles), TH, TW, device="cuda")
    cnn.forward(dev(params), dev(power), dev(tiles), logits)
    z = logits.cpu().numpy().astype(np.float64)
    z64, _ = oracle.cnn_forward(params.astype(np.float64), oracle_inputs(power, tiles))
    err = np.abs(z - z64[:, 0]).max() / (1.0 + np.abs(z64).max())
    print("FP32 forward: max |dz| / (1 + max |z|) = %.3g" % err)
    assert err < 1e-5


def test_loss_and_gradient_match_oracle():
    import torch
    S, T, C = 2, 128, 512
    power = synth.power_spectra(S, T, C, seed=12)
    labels = oracle.mad_tile_flags(power.astype(np.float64), 3.0)
    params = he_params(2, scale=0.7)
    tiles = np.array([1, 6, 4], dtype=np.int32)
    cnn = corr.CNN(max_tiles=4)
    loss = torch.zeros(1, device="cuda")
    grad = torch.zeros(corr.CNN_PARAMS, device="cuda")
    cnn.loss_grad(dev(params), dev(power), dev(labels), dev(tiles), loss, grad)
    x, y = oracle_inputs(power, tiles, labels)
    loss64, g64 = oracle.cnn_loss_and_grad(params.astype(np.float64), x, y)
    g = grad.cpu().numpy().astype(np.float64)
    lerr = abs(loss.item() - loss64) / loss64
    gerr = np.abs(g - g64).max() / np.abs(g64).max()
    print("loss %.6f vs %.6f (rel %.3g); gradient max err / max |g| = %.3g" % (loss.item(), loss64, lerr, gerr))
    assert lerr < 1e-5
    # every layer's block of the gradient, not only the largest entries
    for lo, hi in [(0, 160), (160, 2480), (2480, 2625)]:
        assert np.abs(g[lo:hi] - g64[lo:hi]).max() <= 1e-4 * np.abs(g64[lo:hi]).max(), (lo, hi)
    assert gerr < 1e-5


def test_adam_update_matches_oracle():
    import torch
    g = synth.rng(3, 31)
    p, m, gr = [g.standard_normal(corr.CNN_PARAMS).astype(np.float32) for _ in range(3)]
    v = np.abs(g.standard_normal(corr.CNN_PARAMS)).astype(np.float32)
    cnn = corr.CNN(max_tiles=1, lr=3e-3, beta1=0.8, beta2=0.99, eps=1e-6)
    pd, md, vd = dev(p), dev(m), dev(v)
    cnn.adam(pd, md, vd, step=3, grad=dev(gr))
    torch.cuda.synchronize()
    p64, m64, v64 = oracle.adam_step(p, m, v, gr, 3, 3e-3, 0.8, 0.99, 1e-6)
    assert np.allclose(md.cpu().numpy(), m64, rtol=1e-6, atol=1e-7)
    assert np.allclose(vd.cpu().numpy(), v64, rtol=1e-6, atol=1e-7)
    assert np.abs(pd.cpu().numpy() - p64).max() < 1e-6


# Inference: FP16 operands (relative rounding 2^-11 on x, a1, a2 and the
# weights), FP32 accumulation.  Each layer adds about 2^-11 of its output's
# scale to the logit, so 2e-3 of (1 + max |z|) bounds the error with margin.
INFER_TOL = 2e-3


def _infer(params, power, threshold=0.5):
    import torch
    S, T, C = power.shape
    flags = torch.full((S, T, C), 7, dtype=torch.uint8, device="cuda")
    logits = torch.full((S, T, C), float("nan"), device="cuda")
    corr.cnn_infer(dev(params), dev(power), flags, threshold=threshold, logits=logits)
    torch.cuda.synchronize()
    return flags.cpu().numpy(), logits.cpu().numpy().astype(np.float64)


def _check_infer(params, power, threshold=0.5):
    flags, z = _infer(params, power, threshold)
    z64 = oracle.cnn_tile_logits(params.astype(np.float64), power.astype(np.float64))
    scale = 1.0 + np.abs(z64).max()
    err = np.abs(z - z64).max() / scale
    print("FP16 inference: max |dz| / (1 + max |z|) = %.3g" % err)
    assert err < INFER_TOL
    # flags: identical wherever the FP64 logit is clear of the threshold by the bound
    thr = np.log(threshold / (1 - threshold))
    clear = np.abs(z64 - thr) > INFER_TOL * scale
    assert np.array_equal(flags[clear], (z64[clear] > thr).astype(np.uint8))
    assert set(np.unique(flags)) <= {0, 1}
    return flags, z64


def test_infer_matches_oracle_over_several_tiles():
    power = synth.power_spectra(2, 192, 768, seed=13)  # 2 x 3 x 3 tiles
    _check_infer(he_params(4), power)


def test_infer_fp16_power_matches_oracle():
    # FP16 power cells (the F-engine's power_fp16 output: |X|^2 / N^2, here synthetic cells
    # rounded on the host, some in the FP16 subnormal range): the oracle on the same values,
    # and the FP32-input kernel on the same values gives bit-identical logits and flags
    power = synth.power_spectra(2, 128, 512, seed=16) * np.float32(2.0 ** -20)
    power[1, :, 256:512] *= np.float32(2.0 ** -12)  # cells of ~2^-22: subnormal in FP16
    p16 = power.astype(np.float16)
    params = he_params(8)
    f16, z16 = _infer(params, p16)
    _check_infer(params, p16)
    f32, z32 = _infer(params, p16.astype(np.float32))
    assert np.array_equal(z16, z32) and np.array_equal(f16, f32)


@pytest.mark.parametrize("f16", [False, True])
def test_guarded_inference_matches_the_oracle(f16):
    # the network's flags OR the MAD column statistic's (M = 3): weak tone columns that the
    # network's 7 x 7 view misses are flagged whole; the logits are those of the plain kernel
    import torch
    from gpu_util import near_threshold_cells
    power = synth.power_spectra(2, 128, 768, seed=17, tone_k=(0.3, 2.0))  # weak persistent tones
    if f16:
        power = (power * np.float32(2.0 ** -20)).astype(np.float16)
    params = he_params(9)
    S, T, C = power.shape
    flags = torch.empty((S, T, C), dtype=torch.uint8, device="cuda")
    logits = torch.empty((S, T, C), device="cuda")
    corr.cnn_infer(dev(params), dev(power), flags, logits=logits, guard=3.0)
    torch.cuda.synchronize()
    f0, z0 = _infer(params, power)
    z = logits.cpu().numpy().astype(np.float64)
    assert np.array_equal(z, z0)  # the guard does not touch the logits
    P = power.astype(np.float64)
    fo, z64 = oracle.cnn_guarded_flags(params.astype(np.float64), P, 0.5, 3.0)
    scale = 1.0 + np.abs(z64).max()
    clear = (np.abs(z64) > INFER_TOL * scale) & ~near_threshold_cells(P)
    fg = flags.cpu().numpy()
    cols = oracle.mad_tile_flags(P, 3.0, stats="columns")
    print("guarded inference: %d guard columns, %d cells added by the guard, %d not clear"
          % (cols[:, 0, :].sum(), int(((fg != 0) & (f0 == 0)).sum()), int((~clear).sum())))
    assert cols.any() and ((fg != 0) & (f0 == 0)).any()
    assert np.array_equal(fg[clear], fo[clear])
    assert np.all(fg >= f0)  # the guard only adds flags
    # guard = 0 is the plain kernel
    g0 = torch.empty_like(flags)
    corr.cnn_infer(dev(params), dev(power), g0, guard=0.0)
    torch.cuda.synchronize()
    assert np.array_equal(g0.cpu().numpy(), f0)


def test_infer_many_tiles_per_workgroup():
    """1280 tiles, several per workgroup (one workgroup per compute unit, each
    walking its tiles as one stream): sampled tiles against the oracle, and
    every sampled tile bit-identical to the same tile inferred on its own (a
    tile's result may not depend on its neighbours in the stream)."""
    import torch
    S, T, C = 2, 4096, 2560
    gen = torch.Generator(device="cuda")
    gen.manual_seed(synth.BASE_SEED + 31)
    power = torch.empty(S, T, C, device="cuda").exponential_(1.0, generator=gen)
    power[1, :, 777] *= 30.0  # a tone column crossing many tiles of one stream
    params = he_params(7)
    pd = dev(params)
    flags = torch.empty(S, T, C, dtype=torch.uint8, device="cuda")
    logits = torch.empty(S, T, C, device="cuda")
    corr.cnn_infer(pd, power, flags, logits=logits)
    torch.cuda.synchronize()
    ntm, ntk = T // TH, C // TW
    n = S * ntm * ntk
    rng = np.random.default_rng(3)
    sample = sorted(set([0, 1, 255, 256, 257, n - 1] + rng.integers(0, n, 34).tolist()))
    for k, tile in enumerate(sample):
        s, rest = divmod(tile, ntm * ntk)
        mt, kt = divmod(rest, ntk)
        sl = (s, slice(mt * TH, mt * TH + TH), slice(kt * TW, kt * TW + TW))
        one = power[sl].contiguous().view(1, TH, TW)
        f1 = torch.empty(1, TH, TW, dtype=torch.uint8, device="cuda")
        z1 = torch.empty(1, TH, TW, device="cuda")
        corr.cnn_infer(pd, one, f1, logits=z1)
        torch.cuda.synchronize()
        assert torch.equal(z1[0], logits[sl]) and torch.equal(f1[0], flags[sl]), tile
        if k % 5 == 0 or tile in (0, n - 1):
            P = one[0].cpu().numpy().astype(np.float64)
            z64, _ = oracle.cnn_forward(params.astype(np.float64), oracle.cnn_tile_input(P)[None, None])
            scale = 1.0 + np.abs(z64).max()
            assert np.abs(logits[sl].cpu().numpy() - z64[0, 0]).max() < INFER_TOL * scale, tile


def test_infer_single_tile_and_thresholds():
    power = synth.power_spectra(1, 64, 256, seed=14)
    params = he_params(5)
    for thr in (0.1, 0.5, 0.93):
        _check_infer(params, power, thr)


def test_infer_edge_tiles():
    """An all-zero tile (no reference level: input 0 everywhere), a tile of one
    huge value, and a constant tile."""
    power = synth.power_spectra(1, 64, 1024, seed=15)
    power[0, :, 0:256] = 0.0
    power[0, 17, 300] = 3e30
    power[0, :, 768:1024] = 5.0
    _check_infer(he_params(6), power)


def test_training_forward_agrees_with_inference():
    """The FP32 training forward and the FP16 fused kernel compute the same logits."""
    import torch
    power = synth.power_spectra(1, 128, 512, seed=16)
    params = he_params(7)
    tiles = np.arange(4, dtype=np.int32)
    cnn = corr.CNN(max_tiles=4)
    logits = torch.empty(4, TH, TW, device="cuda")
    cnn.forward(dev(params), dev(power), dev(tiles), logits)
    _, z16 = _infer(params, power)
    z32 = logits.cpu().numpy()
    for t in tiles:
        a, b = z32[t], tile_slice(z16, t)
        assert np.abs(a - b).max() < INFER_TOL * (1 + np.abs(a).max())


def test_bad_tile_number_is_reported():
    import torch
    power = synth.power_spectra(1, 64, 256, seed=17)
    cnn = corr.CNN(max_tiles=2)
    logits = torch.empty(2, TH, TW, device="cuda")
    cnn.forward(dev(he_params(8)), dev(power), dev(np.array([0, 99], dtype=np.int32)), logits)
    with pytest.raises(corr.CorrError) as e:
        cnn.check_device_errors()
    assert e.value.status == -10
    cnn.check_device_errors()  # cleared


def test_save_load_round_trip(tmp_path):
    import torch
    p, m, v = (dev(he_params(k)) for k in (9, 10, 11))
    path = str(tmp_path / "flagger.bin")
    corr.cnn_save(path, p, m, v, step=123)
    q, mq, vq = (torch.zeros(corr.CNN_PARAMS, device="cuda") for _ in range(3))
    assert corr.cnn_load(path, q, mq, vq) == 123
    assert torch.equal(p, q) and torch.equal(m, mq) and torch.equal(v, vq)
