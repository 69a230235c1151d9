"""The Python binding rejects undersized, host-resident or mistyped buffers
before any launch (the C-ABI receives raw pointers and cannot see sizes):
each call below raises in the binding, and the device is still usable after
them."""
import pytest

import paper_0910_1517_amd as corr

pytestmark = pytest.mark.gpu


def test_plan_calls_reject_small_buffers():
    import torch
    plan = corr.Plan(8, 512, 64, precision=corr.INT8)
    spec = plan.alloc("spectra")
    acc = plan.alloc("acc")
    with pytest.raises(ValueError, match="acc holds"):
        plan.xengine(spec, acc[:-1])
    with pytest.raises(ValueError, match="spec holds"):
        plan.xengine(spec[:-16], acc)
    with pytest.raises(ValueError, match="device tensor"):
        plan.xengine(spec.cpu(), acc)
    rs = 512 * 64 + 256
    x = torch.zeros(8, rs, dtype=torch.int8, device="cuda")
    g = torch.zeros(24 * 8, dtype=torch.uint8, device="cuda")
    scale = torch.ones(8, 256, device="cuda")
    with pytest.raises(ValueError, match="x holds"):
        plan.fengine(x[:7].reshape(-1), g, spec, scale, row_stride=rs)
    with pytest.raises(ValueError, match="geom holds"):
        plan.fengine(x, g[:-1], spec, scale)
    with pytest.raises(ValueError, match="scale is required"):
        plan.fengine(x, g, spec, None)
    with pytest.raises(ValueError, match="acc holds"):
        plan.xengine_gated(spec, torch.zeros(64, dtype=torch.uint8, device="cuda"), 2, acc)
    with pytest.raises(TypeError):
        plan.integrate(acc, torch.zeros(plan.state_bytes // 4, dtype=torch.float32, device="cuda"))
    plan.close()


def test_module_calls_reject_small_buffers():
    import torch
    v = torch.zeros(2, 64, 64, dtype=torch.complex64, device="cuda")
    with pytest.raises(ValueError, match="out holds"):
        corr.dedisperse(v, sample_rate=1e6, nu0=3e8, dm=1.0, n_int=4,
                        out=torch.empty(64 * 64 // 4 - 1, device="cuda"))
    with pytest.raises(TypeError):
        corr.dedisperse(v.real.contiguous(), sample_rate=1e6, nu0=3e8, dm=1.0, n_int=4)
    x = torch.zeros(4, 4096, dtype=torch.int8, device="cuda")
    table = torch.zeros(4, 1024, device="cuda")
    with pytest.raises(ValueError, match="row stride"):
        corr.blank_voltages(x, table, block=256, out=torch.zeros(4, 4112, dtype=torch.int8, device="cuda")[:, :4096])
    with pytest.raises(ValueError, match="counts holds"):
        corr.blank_voltages(x, table, block=256, counts=torch.zeros(4 * 16 - 1, dtype=torch.int32, device="cuda"))
    raw = torch.zeros(2, 4096, dtype=torch.uint8, device="cuda")
    with pytest.raises(ValueError, match="4 per card"):
        corr.adc_unpack(raw, torch.zeros(7, 1024, dtype=torch.int8, device="cuda"), bits=8)
    with pytest.raises(ValueError, match="raw holds"):  # 1024 8-bit samples need 4096 bytes per card
        corr.adc_unpack(torch.zeros(2, 2048, dtype=torch.uint8, device="cuda"),
                        torch.zeros(8, 1024, dtype=torch.int8, device="cuda"), bits=8)
    # nothing was launched: the device is idle and usable
    y = torch.ones(16, device="cuda") * 2
    torch.cuda.synchronize()
    assert float(y.sum()) == 32.0
