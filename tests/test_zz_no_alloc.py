"""The no-allocation entry point (corr_dedisperse_noalloc, for callers that
cannot allocate device memory) against corr_dedisperse, which takes a
caller-allocated workspace: two calls in a row on the same GPU, the second
with a smaller input, both equal to the workspace entry point's output bit for
bit (the same kernels on the same data); sizes beyond the scratch limit are
rejected on the host."""
import numpy as np
import pytest

import paper_0910_1517_amd as corr

pytestmark = pytest.mark.gpu

FS = 66.666666e6


def _voltages(npol, T, C, seed):
    import torch
    g = torch.Generator(device="cuda").manual_seed(seed)
    return torch.randn(npol, T, C, dtype=torch.complex64, device="cuda", generator=g)


@pytest.mark.parametrize("first,second", [((2, 2048, 1024, 64), (1, 256, 64, 16))])
def test_noalloc_dedisperse_equals_workspace_entry_point(first, second):
    import torch
    for (npol, T, C, n_int), seed in ((first, 1), (second, 2)):
        print("no-alloc dedispersion: npol %d T %d C %d n_int %d" % (npol, T, C, n_int), flush=True)
        v = _voltages(npol, T, C, seed)
        ref, _ = corr.dedisperse(v, sample_rate=FS, nu0=325e6, dm=0.5, n_int=n_int)
        out = torch.full((T * C // n_int,), float("nan"), device="cuda")
        corr.dedisperse_noalloc(v, out, sample_rate=FS, nu0=325e6, dm=0.5, n_int=n_int)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), float((out - ref).abs().max())
        assert np.isfinite(out.cpu().numpy()).all()


def test_noalloc_dedisperse_rejects_sizes_beyond_its_scratch():
    import torch
    npol, T, C = 2, 4096, 1024  # 2^23 samples > 2^22
    v = torch.zeros(npol, T, C, dtype=torch.complex64, device="cuda")
    out = torch.empty(T * C, device="cuda")
    with pytest.raises(corr.CorrError) as e:
        corr.dedisperse_noalloc(v, out, sample_rate=FS, nu0=325e6, dm=0.5, n_int=1)
    assert e.value.status == -1 and "no-allocation limit" in str(e.value)
