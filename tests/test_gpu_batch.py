"""Batched sub-arrays (one X-engine launch over every sub-array, HIP-graph
replay) and the X-engine split autotuner.  The integer path makes every
comparison exact: a batched run must reproduce the separately run plans bit for
bit, whatever split the autotuner picks."""
import numpy as np
import pytest

import paper_0910_1517_amd as corr
import synth
from gpu_util import FS, acc_sum, geom_dev, upload_streams

pytestmark = pytest.mark.gpu

SHAPES = [dict(n_signals=8, fft_len=512, n_spectra=256),
          dict(n_signals=30, fft_len=1024, n_spectra=128),
          dict(n_signals=64, fft_len=2048, n_spectra=64, x_split=2)]


def make_inputs(sh, seed):
    import torch
    S, N, T = sh["n_signals"], sh["fft_len"], sh["n_spectra"]
    geo = synth.make_geometry((S + 1) // 2, seed=seed)
    geo = geo.subset(np.arange(S))
    x = synth.voltages(S, N * T + 64, geo, FS, seed=seed + 1, mode="bulk", tone_bin=5, tone_N=N)
    x_dev, rs = upload_streams(x, N, T, 16)
    scale = torch.from_numpy(synth.rng(seed, 99).uniform(20, 40, S * N // 2).astype(np.float32)).cuda()
    return x_dev, rs, geom_dev(geo), scale


def run_single(sh, x_dev, rs, g_dev, scale):
    import torch
    plan = corr.Plan(sh["n_signals"], sh["fft_len"], sh["n_spectra"], precision=corr.INT8,
                     x_split=sh.get("x_split", 0))
    spec = plan.alloc("spectra", zero=False)
    acc, state, vis = plan.alloc("acc"), plan.alloc("state"), plan.alloc("vis")
    plan.fengine(x_dev, g_dev, spec, scale, row_stride=rs)
    plan.xengine(spec, acc)
    acc_h = acc.cpu().numpy().copy()
    plan.integrate(acc, state, vis, scale, flags=corr.DUMP)
    torch.cuda.synchronize()
    return acc_sum(acc_h, plan), state.cpu().numpy(), vis.cpu().numpy()


def setup_batch(inputs):
    b = corr.Batch(SHAPES)
    bufs = []
    for i, (sh, (x_dev, rs, g_dev, scale)) in enumerate(zip(SHAPES, inputs)):
        p = b.plans[i]
        spec = p.alloc("spectra", zero=False)
        acc, state, vis = p.alloc("acc"), p.alloc("state"), p.alloc("vis")
        b.set_io(i, x=x_dev, row_stride=rs, geom=g_dev, spec=spec, scale=scale, acc=acc, state=state,
                 vis=vis, flags=corr.DUMP | corr.RESET)
        bufs.append((spec, acc, state, vis))
    return b, bufs


def test_batch_equals_separate_plans_bit_exact():
    import torch
    inputs = [make_inputs(sh, 100 + 10 * i) for i, sh in enumerate(SHAPES)]
    ref = [run_single(sh, *inp) for sh, inp in zip(SHAPES, inputs)]
    b, bufs = setup_batch(inputs)
    b.run()
    torch.cuda.synchronize()
    for i, (spec, acc, state, vis) in enumerate(bufs):
        assert np.array_equal(vis.cpu().numpy(), ref[i][2]), i
        assert not acc.any().item()  # integrate zeroed it
    b.close()


def test_batch_graph_replays_follow_new_data():
    import torch
    inputs = [make_inputs(sh, 200 + 10 * i) for i, sh in enumerate(SHAPES)]
    b, bufs = setup_batch(inputs)
    stream = torch.cuda.Stream()
    b.capture(stream)
    for rep in range(3):
        # new data and geometry in place between replays (eager work on the default stream)
        for i, (x_dev, rs, g_dev, scale) in enumerate(inputs):
            x_dev.copy_(torch.roll(x_dev, shifts=7 * (rep + 1), dims=1))
            scale.mul_(1.25)
        torch.cuda.synchronize()
        refs = [run_single(sh, *inp) for sh, inp in zip(SHAPES, inputs)]
        b.launch(stream)
        stream.synchronize()
        for i, (spec, acc, state, vis) in enumerate(bufs):
            assert np.array_equal(vis.cpu().numpy(), refs[i][2]), (rep, i)
    b.close()


def test_autotuned_split_gives_identical_int_results():
    import torch
    S, N, T = 64, 1024, 512
    split, ms = corr.autotune_x_split(S, N, T, cache=False)
    assert split >= 1 and (T // 32) % split == 0 and ms > 0
    q = synth.random_spectra_int8(S, T, N // 2, seed=7)
    out = []
    for sp in (1, split):
        plan = corr.Plan(S, N, T, precision=corr.INT8, x_split=sp)
        assert plan.splits == sp
        spec = plan.alloc("spectra", zero=False)
        plan.xpack(torch.from_numpy(q).cuda(), spec)
        acc = plan.alloc("acc")
        plan.xengine(spec, acc)
        torch.cuda.synchronize()
        out.append(acc_sum(acc.cpu().numpy(), plan))
    assert np.array_equal(out[0], out[1])


def test_batch_rejects_non_int8():
    with pytest.raises(corr.CorrError) as e:
        corr.Batch([dict(n_signals=8, fft_len=512, n_spectra=64)], precision=corr.FP32)
    assert e.value.status == -4
