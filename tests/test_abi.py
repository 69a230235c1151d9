"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and validates plan descriptions on the host."""
import ctypes
import os
import re

import pytest

import paper_0910_1517_amd as corr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "corr.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(corr_[a-z_0-9]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert header_functions() == sorted(corr.SYMBOLS)


def test_library_exports_every_declared_symbol():
    L = corr.lib()
    for name in header_functions():
        assert hasattr(L, name), name
        assert ctypes.cast(getattr(L, name), ctypes.c_void_p).value


def test_status_strings():
    L = corr.lib()
    for code in corr.STATUS:
        assert L.corr_status_string(code)
    assert L.corr_status_string(0) == b"ok"


def create(**kw):
    args = dict(n_signals=64, fft_len=4096, n_spectra=32768, precision=corr.INT8)
    args.update(kw)
    n, N, T = args.pop("n_signals"), args.pop("fft_len"), args.pop("n_spectra")
    d = corr.make_desc(n, N, T, **args)
    h = ctypes.c_void_p()
    rc = corr.lib().corr_plan_create(ctypes.byref(d), ctypes.byref(h))
    return rc, h


@pytest.mark.parametrize("kw,code", [
    (dict(n_signals=0), -1), (dict(n_signals=65), -1), (dict(fft_len=1000), -1),
    (dict(fft_len=256), -1), (dict(fft_len=32768), -1), (dict(n_spectra=48), -1),
    (dict(n_spectra=0), -1), (dict(max_delay=-1), -1), (dict(precision=7), -1),
    (dict(sideband=0), -1), (dict(scale_mode=3), -1), (dict(sample_rate=0.0), -1),
    (dict(sample_rate=float("nan")), -1), (dict(x_split=-2), -1), (dict(phase_lut=2), -1),
    (dict(power_fp16=2), -1), (dict(power_fp16=-1), -1),
])
def test_plan_create_rejects_bad_descriptions(kw, code):
    rc, h = create(**kw)
    assert rc == code and not h.value
    assert corr.lib().corr_last_error(None)


def test_plan_create_rejects_reserved_and_null():
    d = corr.make_desc(8, 512, 1024)
    d.reserved[3] = 1
    h = ctypes.c_void_p()
    assert corr.lib().corr_plan_create(ctypes.byref(d), ctypes.byref(h)) == -1
    assert corr.lib().corr_plan_create(None, ctypes.byref(h)) == -2


def test_plan_sizes_and_calls_without_workspace():
    L = corr.lib()
    rc, h = create(n_signals=64, fft_len=4096, n_spectra=32768, precision=corr.INT8)
    assert rc == 0
    try:
        C, P = 2048, 64 * 65 // 2
        assert L.corr_plan_spectra_bytes(h) == 2 * C * 32768 * 64
        assert L.corr_plan_state_bytes(h) == C * P * 16
        assert L.corr_plan_vis_bytes(h) == C * P * 8
        sp = L.corr_plan_x_splits(h)
        assert sp >= 1 and (32768 // 32) % sp == 0
        assert L.corr_plan_acc_bytes(h) == sp * C * P * 8
        assert L.corr_plan_workspace_bytes(h) >= 2 * 8 * C
        # data-path calls before a workspace is bound are rejected on the host, before
        # any launch (the placeholder pointer is never dereferenced)
        fake = ctypes.c_void_p(1 << 20)
        assert L.corr_fengine(h, fake, 32768 * 4096 + 64, fake, 0, fake, fake, None, None) == -5
        assert L.corr_integrate(h, fake, fake, fake, None, 0, None) == -5
        assert L.corr_fengine(h, None, 0, fake, 0, fake, fake, None, None) == -2
    finally:
        L.corr_plan_destroy(h)


def test_power_cells_are_half_the_bytes_in_fp16():
    L = corr.lib()
    rc1, h1 = create(n_signals=8, fft_len=1024, n_spectra=64)
    rc2, h2 = create(n_signals=8, fft_len=1024, n_spectra=64, power_fp16=1)
    assert rc1 == 0 and rc2 == 0
    try:
        assert L.corr_plan_power_bytes(h1) == 4 * 8 * 64 * 512
        assert L.corr_plan_power_bytes(h2) == 2 * 8 * 64 * 512
    finally:
        L.corr_plan_destroy(h1)
        L.corr_plan_destroy(h2)


def test_workspace_grows_with_compute_scale_mode():
    L = corr.lib()
    rc1, h1 = create(scale_mode=corr.SCALE_HOLD)
    rc2, h2 = create(scale_mode=corr.SCALE_COMPUTE)
    assert rc1 == 0 and rc2 == 0
    try:
        assert L.corr_plan_workspace_bytes(h2) > L.corr_plan_workspace_bytes(h1)
    finally:
        L.corr_plan_destroy(h1)
        L.corr_plan_destroy(h2)


def test_fp32_split_choice_bounds_running_sums():
    L = corr.lib()
    rc, h = create(n_signals=64, fft_len=1024, n_spectra=16384, precision=corr.FP32)
    assert rc == 0
    try:
        sp = L.corr_plan_x_splits(h)
        assert 16384 // sp <= 1024
    finally:
        L.corr_plan_destroy(h)


# ----------------------------------------------------------- learned flagger

def _cnn_desc(**kw):
    d = corr.CnnDesc()
    d.max_tiles, d.lr, d.beta1, d.beta2, d.eps = 4, 1e-3, 0.9, 0.999, 1e-8
    for k, v in kw.items():
        setattr(d, k, v)
    return d


@pytest.mark.parametrize("kw", [dict(max_tiles=0), dict(max_tiles=5000), dict(lr=0.0), dict(lr=float("nan")),
                                dict(beta1=1.0), dict(beta2=-0.1), dict(eps=0.0)])
def test_cnn_create_rejects_bad_descriptions(kw):
    L = corr.lib()
    h = ctypes.c_void_p()
    assert L.corr_cnn_create(ctypes.byref(_cnn_desc(**kw)), ctypes.byref(h)) == -1
    assert L.corr_cnn_last_error(None)


def test_cnn_workspace_and_unbound_calls():
    L = corr.lib()
    h = ctypes.c_void_p()
    assert L.corr_cnn_create(ctypes.byref(_cnn_desc()), ctypes.byref(h)) == 0
    try:
        n = L.corr_cnn_workspace_bytes(h)
        # activations of 4 tiles: 68 planes of 64 x 256 floats each, plus the gradient partials
        assert n >= 4 * 68 * 64 * 256 * 4
        fake = ctypes.c_void_p(1 << 20)  # never dereferenced: every call below fails its checks first
        assert L.corr_cnn_forward(h, fake, fake, 1, 64, 256, fake, 1, fake, None) == -5  # no workspace
        assert L.corr_cnn_adam(h, fake, fake, fake, None, 1, None) == -5
        assert L.corr_cnn_adam(h, fake, fake, fake, fake, 0, None) == -1                # step 0
        assert L.corr_cnn_bind_workspace(h, ctypes.c_void_p(1 << 20 | 16), n) == -3
        assert L.corr_cnn_bind_workspace(h, fake, n - 1) == -5
    finally:
        L.corr_cnn_destroy(h)


@pytest.mark.parametrize("shape,thr,code", [((1, 64, 256), 0.0, -1), ((1, 64, 256), 1.0, -1),
                                            ((1, 100, 256), 0.5, -1), ((1, 64, 300), 0.5, -1),
                                            ((0, 64, 256), 0.5, -1), ((1, 64, (1 << 22) + 256), 0.5, -1)])
def test_cnn_infer_rejects_bad_arguments(shape, thr, code):
    L = corr.lib()
    fake = ctypes.c_void_p(1 << 20)
    assert L.corr_cnn_infer(fake, fake, *shape, thr, fake, None, None) == code
    assert L.corr_cnn_infer(None, fake, 1, 64, 256, 0.5, fake, None, None) == -2
    assert L.corr_cnn_infer_f16(fake, fake, *shape, thr, fake, None, None) == code
    for f16 in (0, 1):
        assert L.corr_cnn_infer_guarded(fake, fake, f16, *shape, thr, 3.0, fake, None, None) == code
    assert L.corr_cnn_last_error(None)


def test_cnn_infer_guarded_rejects_bad_guard_and_cell_type():
    L = corr.lib()
    fake = ctypes.c_void_p(1 << 20)
    assert L.corr_cnn_infer_guarded(fake, fake, 0, 1, 64, 256, 0.5, -1.0, fake, None, None) == -1
    assert L.corr_cnn_infer_guarded(fake, fake, 0, 1, 64, 256, 0.5, float("nan"), fake, None, None) == -1
    assert L.corr_cnn_infer_guarded(fake, fake, 2, 1, 64, 256, 0.5, 3.0, fake, None, None) == -1
    assert L.corr_cnn_infer_guarded(None, fake, 0, 1, 64, 256, 0.5, 3.0, fake, None, None) == -2


def test_cnn_load_rejects_missing_and_foreign_files(tmp_path):
    L = corr.lib()
    fake = ctypes.c_void_p(1 << 20)
    st = ctypes.c_int64()
    assert L.corr_cnn_load(str(tmp_path / "none.bin").encode(), fake, None, None, ctypes.byref(st)) == -11
    bad = tmp_path / "bad.bin"
    bad.write_bytes(b"NOTACNN!" + bytes(64))
    assert L.corr_cnn_load(str(bad).encode(), fake, None, None, ctypes.byref(st)) == -1


def test_beamform_rejects_bad_arguments():
    """Every call below fails a host-side check before any launch (the
    placeholder pointers are never dereferenced)."""
    L = corr.lib()
    rc, h = create(n_signals=8, fft_len=512, n_spectra=32, precision=corr.INT8)
    assert rc == 0
    try:
        f = ctypes.c_void_p(1 << 20)  # 256-byte aligned placeholder

        def bf(spec=f, scale=f, w=f, inc=f, c=f, nb=1, mode=corr.BEAM_FULLPOL, coh=f, tint=1):
            return L.corr_beamform(h, spec, scale, w, inc, c, nb, mode, coh, tint, None)

        assert bf(nb=5) == -1 and bf(nb=-1) == -1
        assert bf(mode=7) == -1
        assert bf(tint=3) == -1 and bf(tint=16) == -1 and bf(tint=0) == -1
        assert bf(mode=corr.BEAM_VOLTAGE, tint=2) == -1  # voltages are not summed over time
        assert bf(inc=None, nb=0) == -1                   # no beam requested
        assert bf(spec=None) == -2
        assert bf(w=None) == -2                           # incoherent beam without weights
        assert bf(c=None) == -2 and bf(coh=None) == -2
        assert bf(scale=None) == -2                       # INT8 spectra need their scales
        assert bf(spec=ctypes.c_void_p((1 << 20) + 16)) == -3
        assert bf(coh=ctypes.c_void_p((1 << 20) + 2)) == -3
        assert bf(mode=corr.BEAM_VOLTAGE, coh=ctypes.c_void_p((1 << 20) + 4)) == -3
        assert L.corr_beamform(None, f, f, f, f, f, 1, 0, f, 1, None) == -2
        assert L.corr_last_error(h)
    finally:
        L.corr_plan_destroy(h)


def test_blanker_rejects_bad_arguments():
    """Host-side checks of the voltage blanker and its noise table; every call
    returns before any launch (placeholder pointers, never dereferenced)."""
    L = corr.lib()
    f = ctypes.c_void_p(1 << 20)

    def bv(x=f, rs=1024, S=4, n=1000, block=256, M=3.0, table=f, tl=1024, s0=0, out=f, counts=f, stats=f):
        return L.corr_blank_voltages(x, rs, S, n, block, M, table, tl, s0, out, counts, stats, None)

    assert bv(x=None) == -2 and bv(table=None) == -2 and bv(out=None) == -2
    assert bv(x=ctypes.c_void_p((1 << 20) + 8)) == -3 and bv(out=ctypes.c_void_p((1 << 20) + 4)) == -3
    assert bv(table=ctypes.c_void_p((1 << 20) + 2)) == -3 and bv(stats=ctypes.c_void_p((1 << 20) + 1)) == -3
    assert bv(S=0) == -1 and bv(S=65536) == -1
    assert bv(n=-1) == -1 and bv(rs=1000) == -1 and bv(rs=992) == -1      # not a multiple of 16 / below n
    assert bv(block=8) == -1 and bv(block=100) == -1 and bv(block=65552) == -1
    assert bv(M=0.0) == -1 and bv(M=-1.0) == -1 and bv(M=float("inf")) == -1 and bv(M=float("nan")) == -1
    assert bv(tl=0) == -1 and bv(tl=1000) == -1 and bv(tl=1 << 32) == -1
    assert bv(s0=-1) == -1 and bv(s0=(1 << 63) - 1000) == -1             # sample0 + n would overflow
    assert bv(n=1 << 40, rs=1 << 40, block=16) == -1                     # 2^36 blocks per row
    assert L.corr_blank_last_error()
    assert bv(n=0, counts=None, stats=None) == 0                         # nothing to do, nothing launched
    assert L.corr_blank_last_error() == b""

    def nt(seed=1, S=4, n=1024, t=f):
        return L.corr_blank_noise_table(seed, S, n, t, None)

    assert nt(t=None) == -2 and nt(t=ctypes.c_void_p((1 << 20) + 2)) == -3
    assert nt(S=0) == -1 and nt(n=0) == -1 and nt(n=3) == -1 and nt(n=1 << 32) == -1


def test_adc_unpack_rejects_bad_arguments():
    L = corr.lib()
    f = ctypes.c_void_p(1 << 20)

    def au(raw=f, rrs=2048, cards=2, n=512, bits=4, x=f, rs=512):
        return L.corr_adc_unpack(raw, rrs, cards, n, bits, x, rs, None)

    assert au(raw=None) == -2 and au(x=None) == -2
    assert au(raw=ctypes.c_void_p((1 << 20) + 8)) == -3 and au(x=ctypes.c_void_p((1 << 20) + 4)) == -3
    assert au(bits=2) == -1 and au(bits=16) == -1
    assert au(cards=0) == -1 and au(cards=16384) == -1
    assert au(n=-1) == -1 and au(n=(1 << 40) + 1, rrs=1 << 44, rs=1 << 44) == -1
    assert au(rrs=1008) == -1 and au(rrs=1000) == -1               # below n*bits/2, not a multiple of 16
    assert au(bits=8, rrs=2032) == -1                              # 8-bit needs 4 n bytes
    assert au(rs=496) == -1 and au(rs=520) == -1
    assert L.corr_adc_last_error()
    assert au(n=0) == 0 and L.corr_adc_last_error() == b""


def test_gated_xengine_and_gates_reject_bad_arguments():
    L = corr.lib()
    rc, h = create(n_signals=8, fft_len=512, n_spectra=32, precision=corr.INT8)
    assert rc == 0
    try:
        f = ctypes.c_void_p(1 << 20)
        gx = lambda spec=f, gate=f, nb=2, acc=f: L.corr_xengine_gated(h, spec, gate, nb, acc, None)
        assert gx(spec=None) == -2 and gx(gate=None) == -2 and gx(acc=None) == -2
        assert gx(spec=ctypes.c_void_p((1 << 20) + 16)) == -3 and gx(gate=ctypes.c_void_p((1 << 20) + 8)) == -3
        assert gx(nb=0) == -1 and gx(nb=256) == -1
        assert L.corr_xengine_gated(None, f, f, 1, f, None) == -2
    finally:
        L.corr_plan_destroy(h)
    g = (ctypes.c_uint8 * 8)()
    pg = lambda s0=0, n=8, N=512, fs=1e6, t0=0.0, P=1e-3, nb=2, gate=g: \
        L.corr_pulsar_gates(s0, n, N, fs, t0, P, nb, gate, None)
    assert pg() == 0
    assert pg(gate=None) == -2
    assert pg(n=-1) == -1 and pg(s0=-1) == -1 and pg(N=0) == -1 and pg(fs=0.0) == -1 and pg(fs=float("inf")) == -1
    assert pg(P=0.0) == -1 and pg(P=float("nan")) == -1 and pg(t0=float("nan")) == -1
    assert pg(nb=0) == -1 and pg(nb=256) == -1


def test_dedisperse_rejects_bad_arguments():
    L = corr.lib()
    f = ctypes.c_void_p(1 << 20)

    def dd(v=f, npol=2, T=1024, C=64, fs=33e6, nu0=325e6, dm=1.0, n=16, work=ctypes.c_void_p(1 << 21), out=f):
        return L.corr_dedisperse(v, npol, T, C, fs, nu0, dm, n, work, out, None)

    assert dd(v=None) == -2 and dd(work=None) == -2 and dd(out=None) == -2
    assert dd(v=ctypes.c_void_p((1 << 20) + 4)) == -3 and dd(out=ctypes.c_void_p((1 << 20) + 2)) == -3
    assert dd(npol=0) == -1 and dd(npol=3) == -1
    assert dd(C=8) == -1 and dd(C=100) == -1 and dd(C=16384) == -1
    assert dd(T=1000) == -1 and dd(T=16) == -1 and dd(T=1 << 22, C=128) == -1  # T C below 4096 / above 2^28
    assert dd(n=3) == -1 and dd(n=0) == -1
    assert dd(fs=0.0) == -1 and dd(nu0=-1.0) == -1 and dd(dm=-0.5) == -1 and dd(dm=float("nan")) == -1
    assert dd(work=f) == -1  # the input must not be the workspace
    assert L.corr_dedisperse_last_error()
    assert L.corr_dedisperse_workspace_bytes(2, 1024, 64) == 2 * 1024 * 64 * 8


# ------------------------------------------------------ int32 accumulator bound
def test_xengine_rejects_a_call_past_the_int32_bound():
    # 66592 spectra (the first multiple of 32 above 66572) in one INT8 call: rejected on the
    # host before any launch, so the placeholder pointers are never dereferenced
    L = corr.lib()
    rc, h = create(n_signals=8, fft_len=512, n_spectra=66592, precision=corr.INT8)
    assert rc == 0
    try:
        fake = ctypes.c_void_p(1 << 20)
        assert L.corr_xengine(h, fake, None, fake, None, None) == -6
        assert b"int32" in L.corr_last_error(h)
        # FP32 has no such bound: the same shape is not rejected for it (not called here)
    finally:
        L.corr_plan_destroy(h)


def test_batch_rejects_an_entry_past_the_int32_bound():
    # one batch run sums each entry's whole call in int32 before integrating it
    descs = (corr.CorrDesc * 2)(corr.make_desc(8, 512, 1024, precision=corr.INT8),
                                corr.make_desc(16, 1024, 66592, precision=corr.INT8))
    h = ctypes.c_void_p()
    assert corr.lib().corr_batch_create(descs, 2, ctypes.byref(h)) == -6 and not h.value
    assert b"entry 1" in corr.lib().corr_last_error(None)


# --------------------------------------------------- X-engine keep masks and counts
def test_xengine_mask_and_count_arguments_are_checked_on_the_host():
    # rejected before any launch: the placeholder pointers are never dereferenced
    L = corr.lib()
    rc, h = create(n_signals=8, fft_len=512, n_spectra=64, precision=corr.INT8)
    assert rc == 0
    try:
        fake = ctypes.c_void_p(1 << 20)
        assert L.corr_xengine(h, fake, None, fake, fake, None) == -2       # counts without keep
        assert L.corr_xengine(h, fake, ctypes.c_void_p((1 << 20) + 2), fake, None, None) == -3  # keep misaligned
        assert L.corr_xengine(h, fake, fake, fake, ctypes.c_void_p((1 << 20) + 1), None) == -3  # counts misaligned
        assert L.corr_xengine(h, fake, fake, fake, fake, None) == -5       # counts need the workspace
        assert b"workspace" in L.corr_last_error(h)
        assert L.corr_apply_flags(h, fake, None, None, None) == -2         # neither spectra nor keep
    finally:
        L.corr_plan_destroy(h)
