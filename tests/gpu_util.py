"""Helpers shared by the GPU tests: run the HIP path through the C ABI on
seeded synthetic inputs and return host arrays for comparison with the oracle.
Every buffer is sized from the plan's own size queries before any launch."""
from __future__ import annotations

import numpy as np

import oracle
import paper_0910_1517_amd as corr

FS = 66.666666e6


def row_stride_for(N: int, T: int, max_delay: int) -> int:
    need = N * T + max_delay
    return (need + 255) // 256 * 256


def upload_streams(x_host: np.ndarray, N: int, T: int, max_delay: int):
    """int8 [S][n] host streams -> device tensor with a 256-aligned row stride."""
    import torch
    S, n = x_host.shape
    rs = row_stride_for(N, T, max_delay)
    assert n >= N * T + max_delay
    buf = np.zeros((S, rs), dtype=np.int8)
    buf[:, :min(n, rs)] = x_host[:, :min(n, rs)]
    return torch.from_numpy(buf).cuda(), rs


def geom_dev(geom):
    return corr.geom_to_device(corr.geom_array(geom.D, geom.f, geom.psi0, geom.rate))


def run_fengine(plan: corr.Plan, x_dev, rs: int, g_dev, scale_dev=None, spectrum0: int = 0):
    spec = plan.alloc("spectra", zero=False)
    plan.fengine(x_dev, g_dev, spec, scale_dev, row_stride=rs, spectrum0=spectrum0)
    return spec


def run_x_integrate(plan: corr.Plan, spec, scale_dev=None):
    import torch
    acc = plan.alloc("acc")
    state = plan.alloc("state")
    vis = plan.alloc("vis")
    plan.xengine(spec, acc)
    acc_host = acc.cpu().numpy().copy()
    plan.integrate(acc, state, vis, scale_dev, flags=corr.DUMP)
    torch.cuda.synchronize()
    st = state.cpu().numpy().reshape(plan.C, plan.P, 2)
    return acc_host, st[..., 0] + 1j * st[..., 1], corr.vis_complex(vis, plan.C, plan.P)


def acc_sum(acc_host: np.ndarray, plan: corr.Plan) -> np.ndarray:
    """[splits][C][P][2] -> summed over splits (int64 or float64) [C][P][2]."""
    a = acc_host.reshape(plan.splits, plan.C, plan.P, 2)
    return a.astype(np.int64).sum(0) if a.dtype == np.int32 else a.astype(np.float64).sum(0)


def pack_input(plan: corr.Plan, arr: np.ndarray):
    """[S][T][C][2] host array -> device X layout via the library's corner turn."""
    import torch
    inp = torch.from_numpy(np.ascontiguousarray(arr)).cuda()
    spec = plan.alloc("spectra", zero=False)
    plan.xpack(inp, spec)
    return spec


def near_threshold_cells(P64, M=3.0):
    """Cells whose row or column statistic lies within 1e-4 (relative) of Eq. 4's threshold."""
    S, T, C = P64.shape
    near = np.zeros(P64.shape, dtype=bool)
    for s in range(S):
        for m0 in range(0, T, 64):
            for k0 in range(0, C, 256):
                t = P64[s, m0:m0 + 64, k0:k0 + 256]
                for axis, sl in ((1, "row"), (0, "col")):
                    v = t.mean(axis=axis)
                    med = oracle.median(v)
                    mad = oracle.median(np.abs(v - med))
                    d = np.abs(np.abs(v - med) - M * mad / 0.6745)
                    close = d <= 1e-4 * max(M * mad / 0.6745, 1e-30)
                    if sl == "row":
                        near[s, m0:m0 + 64, k0:k0 + 256] |= close[:, None]
                    else:
                        near[s, m0:m0 + 64, k0:k0 + 256] |= close[None, :]
    return near


# Beamformer tolerance (FP32 accumulation of at most 64 terms, the scale folded
# into the weights in FP32): per cell, |error| <= 1e-5 of the sum of the
# magnitudes of the terms -- sum_s w_s |Y_s|^2 for the incoherent beam,
# B_p = sum_s |c_s| |Y_s| per polarisation for a voltage, B_p^2 for |V_p|^2 and
# B_0 B_1 for V_0 conj(V_1).
BEAM_TOL = 1e-5


def beam_bounds(Y, w, c, tint):
    """Per-cell error scales: incoherent sum_s w |Y|^2 [2][T/tint][C]; coherent
    B [nb][2][T][C] = sum over the signals of each polarisation of |c| |Y|."""
    S, T, C = Y.shape
    pol = np.arange(S) % 2
    A = np.abs(Y)
    inc_b = None
    if w is not None:
        inc_b = np.stack([np.tensordot(w * (pol == p), A ** 2, axes=1) for p in (0, 1)])
        inc_b = inc_b.reshape(2, T // tint, tint, C).sum(axis=2)
    coh_b = None
    if c is not None:
        coh_b = np.stack([np.stack([np.tensordot(np.abs(cb) * (pol == p), A, axes=1) for p in (0, 1)])
                          for cb in c])
    return inc_b, coh_b


def check_beams(got_inc, got_coh, ref_inc, ref_coh, inc_b, coh_b, mode, tint):
    if ref_inc is not None:
        assert np.all(np.isfinite(got_inc))
        err = np.abs(got_inc - ref_inc)
        assert np.all(err <= BEAM_TOL * inc_b + 1e-30), err.max()
    if ref_coh is None:
        return
    assert np.all(np.isfinite(got_coh))
    nb = ref_coh.shape[0]
    B = coh_b  # [nb][2][T][C]
    if mode == corr.BEAM_VOLTAGE:
        err = np.abs(got_coh - ref_coh)
        assert np.all(err <= BEAM_TOL * B + 1e-30), err.max()
        return
    T, C = B.shape[2], B.shape[3]
    fold = lambda x: x.reshape(nb, T // tint, tint, C).sum(axis=2)
    bounds = [fold(B[:, 0] ** 2), fold(B[:, 1] ** 2)]
    if mode == corr.BEAM_FULLPOL:
        bounds += [fold(B[:, 0] * B[:, 1])] * 2
    for q, bq in enumerate(bounds):
        err = np.abs(got_coh[:, q] - ref_coh[:, q])
        assert np.all(err <= BEAM_TOL * bq + 1e-30), (q, err.max())
