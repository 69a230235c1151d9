"""Plain CPU oracle for the FX correlator hot path (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never does, and the two
share no code.  The arithmetic lives in ``oracle.c`` (FP64 / int64, built with
gcc); this module only marshals numpy arrays into it and adds the few
definitions that are clearer in numpy (pair indexing, error metrics).

Each wrapper names the passage of Roy et al. (arXiv:0910.1517) it follows; the
C source restates the definition.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (no fast-math, no contraction into FMA) into
    liboracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-shared", "-fPIC", "-std=c11",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build()
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    i64, i32, dbl = ctypes.c_int64, ctypes.c_int, ctypes.c_double
    lib.orc_dft.argtypes = [P, P, i64]
    lib.orc_fft.argtypes = [P, i64]
    lib.orc_fft.restype = i32
    lib.orc_fengine.argtypes = [P, i64, i32, i64, i64, i64, P, P, P, P, dbl, dbl, i32, i32, P]
    lib.orc_fengine_lut.argtypes = [P, i64, i32, i64, i64, i64, P, P, P, P, dbl, dbl, i32, P]
    lib.orc_fengine.restype = i32
    lib.orc_fengine_channels.argtypes = [P, i64, i32, i64, i64, i64, P, P, P, P, dbl, dbl, i32,
                                         P, i32, P]
    lib.orc_fengine_channels.restype = i32
    lib.orc_xengine_f64.argtypes = [P, i32, i64, i64, P]
    lib.orc_xengine_int.argtypes = [P, i32, i64, i64, P]
    lib.orc_xengine_i16.argtypes = [P, i32, i64, i64, P]
    lib.orc_fix16_table.argtypes = [P]
    lib.orc_fix16_spectra.argtypes = [P, i32, i64, i64, i64, P, P, P, dbl, dbl, i32, P, P, P]
    lib.orc_beamform.argtypes = [P, i32, i64, i64, P, P, i32, i32, i32, P, P]
    lib.orc_sigma.argtypes = [P, i32, i64, i64, P]
    lib.orc_quantize_int8.argtypes = [P, P, i32, i64, i64, P]
    lib.orc_quantize_fp8.argtypes = [P, P, i32, i64, i64, P]
    lib.orc_e4m3_decode.argtypes = [ctypes.c_uint8]
    lib.orc_e4m3_decode.restype = dbl
    lib.orc_e4m3_encode.argtypes = [dbl]
    lib.orc_e4m3_encode.restype = ctypes.c_uint8
    lib.orc_scale_visibilities.argtypes = [P, P, i32, i64, P]
    lib.orc_median.argtypes = [P, i64]
    lib.orc_median.restype = dbl
    lib.orc_mad_flags.argtypes = [P, i64, dbl, P, P, P]
    lib.orc_mad_flags.restype = i64
    lib.orc_mad_tile_flags.argtypes = [P, i32, i64, i64, i32, i32, dbl, P]
    lib.orc_mad_tile_flags.restype = i32
    lib.orc_mad_tile_flags_which.argtypes = [P, i32, i64, i64, i32, i32, dbl, i32, P]
    lib.orc_mad_tile_flags_which.restype = i32
    lib.orc_pair_counts.argtypes = [P, i32, i64, i64, P]
    lib.orc_adc_unpack.argtypes = [P, i64, i32, i64, i32, P, i64]
    lib.orc_philox4x32_10.argtypes = [P, P, P]
    lib.orc_blank_noise_table.argtypes = [ctypes.c_uint64, i32, i64, P]
    lib.orc_blank_noise_entry.argtypes = [ctypes.c_uint64, i32, i64]
    lib.orc_blank_noise_entry.restype = ctypes.c_float
    lib.orc_mad_blank.argtypes = [P, i64, i32, i64, i64, dbl, P, i64, i64, P, P, P]
    lib.orc_conv3x3_fwd.argtypes = [P, P, P, i32, i32, i32, i32, i32, P]
    lib.orc_conv3x3_bwd.argtypes = [P, P, P, i32, i32, i32, i32, i32, P, P, P]
    _lib = lib
    return lib


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


# ---------------------------------------------------------------------------
# Transforms (section 2.1: FX correlator -- channelise by FFT first)
# ---------------------------------------------------------------------------
def dft(z: np.ndarray) -> np.ndarray:
    """Direct DFT X[k] = sum_n z[n] exp(-2 pi i k n / N), FP64."""
    z = np.ascontiguousarray(z, dtype=np.complex128)
    out = np.empty_like(z)
    _load().orc_dft(_p(z), _p(out), z.size)
    return out


def fft(z: np.ndarray) -> np.ndarray:
    """Radix-2 FFT with the same definition as :func:`dft`, FP64."""
    z = np.array(z, dtype=np.complex128, order="C", copy=True)
    if _load().orc_fft(_p(z), z.size) != 0:
        raise ValueError("length must be a power of two")
    return z


class Geometry:
    """Per-signal delay/fringe parameters of one call (section 2.1, Eq. 2).

    D: integer delay in samples (read-pointer advance), f: fractional delay in
    samples in [0, 1), psi0: fringe phase in cycles at the call's reference
    epoch, rate: fringe rate in Hz.
    """

    def __init__(self, D, f, psi0, rate):
        self.D = np.ascontiguousarray(D, dtype=np.int32)
        self.f = np.ascontiguousarray(f, dtype=np.float64)
        self.psi0 = np.ascontiguousarray(psi0, dtype=np.float64)
        self.rate = np.ascontiguousarray(rate, dtype=np.float64)


def geom_from_model(tau0, taudot, fs: float, nu_lo: float, t0: float = 0.0, t_delay: float = 0.0) -> Geometry:
    """Per-call geometry from an antenna-based delay model (section 2.1, Eq. 1-2).

    tau_s(t) = tau0[s] + taudot[s] (t - t0) seconds at stream time t.  The
    integer delay and the fractional sample-time correction are taken at
    t_delay: D + f = tau_s(t_delay) fs, D = floor, f in [0, 1) (f kept as the
    nearest float32, a fraction that rounds to 1 carried into D).  The fringe
    term of Eq. 2, nu_lo tau_tot(t), is taken when the samples of a spectrum
    arrived: at its aligned time stamp t_m plus the delay tau_c = tau_s(t_delay)
    that the read pointer skips, so psi0 + rate t_m = nu_lo tau_s(t_m + tau_c):
    rate = nu_lo taudot[s], psi0 = nu_lo (tau_s(0) + taudot[s] tau_c) mod 1
    (the sideband sign is the F-engine's).

    Evaluated in exact rational arithmetic on the binary values of the inputs
    (fractions.Fraction), each result rounded once at the end.
    """
    from fractions import Fraction as Fr
    tau0 = np.atleast_1d(np.asarray(tau0, dtype=np.float64))
    taudot = np.atleast_1d(np.asarray(taudot, dtype=np.float64))
    S = tau0.size
    D = np.zeros(S, dtype=np.int32)
    f = np.zeros(S)
    psi0 = np.zeros(S)
    rate = np.zeros(S)
    for s in range(S):
        a, b = Fr(float(tau0[s])), Fr(float(taudot[s]))
        x = (a + b * (Fr(float(t_delay)) - Fr(float(t0)))) * Fr(float(fs))
        d = x.numerator // x.denominator                # floor of the exact value
        fr = float(np.float32(float(x - d)))            # the fraction, nearest float32
        if fr >= 1.0:
            d, fr = d + 1, 0.0
        c = Fr(float(nu_lo)) * (a - b * Fr(float(t0)) + b * x / Fr(float(fs)))  # cycles at t_m = 0
        c -= c.numerator // c.denominator               # mod 1, exactly
        D[s], f[s], psi0[s] = d, fr, float(c)
        if psi0[s] >= 1.0:
            psi0[s] = 0.0
        rate[s] = float(Fr(float(nu_lo)) * b)
    return Geometry(D, f, psi0, rate)


def fengine(x: np.ndarray, N: int, T: int, geom: Geometry, fs: float, nu_bb: float = 0.0,
            sideband: int = 1, spectrum0: int = 0, method: str = "fft") -> np.ndarray:
    """F-engine of section 2.1 / 2.3.2 with Eq. 2 phase; returns Y[S][T][C] complex128.

    x: int8 [S][row_stride]; row s must hold at least T*N + D_s samples.
    """
    x = np.ascontiguousarray(x, dtype=np.int8)
    S, stride = x.shape
    if np.any(geom.D < 0) or np.any(T * N + geom.D > stride):
        raise ValueError("delay window runs past the row")
    C = N // 2
    Y = np.empty((S, T, C), dtype=np.complex128)
    rc = _load().orc_fengine(_p(x), stride, S, N, T, spectrum0, _p(geom.D), _p(geom.f),
                             _p(geom.psi0), _p(geom.rate), fs, nu_bb, sideband,
                             1 if method == "dft" else 0, _p(Y))
    if rc != 0:
        raise ValueError("orc_fengine failed (%d)" % rc)
    return Y


def fengine_lut(x: np.ndarray, N: int, T: int, geom: Geometry, fs: float, nu_bb: float = 0.0,
                sideband: int = 1, spectrum0: int = 0) -> np.ndarray:
    """F-engine with the phase from the 1440-step sin/cos table of section
    2.3.2 (each channel's Eq. 2 phase rounded to the nearest 0.25 degree
    step); returns Y[S][T][C] complex128."""
    x = np.ascontiguousarray(x, dtype=np.int8)
    S, stride = x.shape
    if np.any(geom.D < 0) or np.any(T * N + geom.D > stride):
        raise ValueError("delay window runs past the row")
    Y = np.empty((S, T, N // 2), dtype=np.complex128)
    rc = _load().orc_fengine_lut(_p(x), stride, S, N, T, spectrum0, _p(geom.D), _p(geom.f), _p(geom.psi0),
                                 _p(geom.rate), fs, nu_bb, sideband, _p(Y))
    if rc != 0:
        raise ValueError("orc_fengine_lut failed (%d)" % rc)
    return Y


def fengine_channels(x: np.ndarray, N: int, T: int, geom: Geometry, fs: float, channels,
                     nu_bb: float = 0.0, sideband: int = 1, spectrum0: int = 0) -> np.ndarray:
    """Direct-DFT F-engine for selected channels; returns Y[S][T][len(channels)]."""
    x = np.ascontiguousarray(x, dtype=np.int8)
    S, stride = x.shape
    if np.any(geom.D < 0) or np.any(T * N + geom.D > stride):
        raise ValueError("delay window runs past the row")
    kk = np.ascontiguousarray(channels, dtype=np.int64)
    Y = np.empty((S, T, kk.size), dtype=np.complex128)
    rc = _load().orc_fengine_channels(_p(x), stride, S, N, T, spectrum0, _p(geom.D), _p(geom.f),
                                      _p(geom.psi0), _p(geom.rate), fs, nu_bb, sideband,
                                      _p(kk), kk.size, _p(Y))
    if rc != 0:
        raise ValueError("orc_fengine_channels failed (%d)" % rc)
    return Y


# ---------------------------------------------------------------------------
# X-engine (section 2.1: cross-multiply every pair, integrate over time)
# ---------------------------------------------------------------------------
def n_pairs(S: int) -> int:
    return S * (S + 1) // 2


def pair_index(i: int, j: int) -> int:
    """Pair (i <= j) -> p = j(j+1)/2 + i."""
    if i > j:
        raise ValueError("pair index needs i <= j")
    return j * (j + 1) // 2 + i


def pair_table(S: int):
    """Arrays (i, j) indexed by p."""
    ii = np.empty(n_pairs(S), dtype=np.int64)
    jj = np.empty(n_pairs(S), dtype=np.int64)
    for j in range(S):
        for i in range(j + 1):
            ii[pair_index(i, j)] = i
            jj[pair_index(i, j)] = j
    return ii, jj


def xengine(Y: np.ndarray, V: np.ndarray | None = None) -> np.ndarray:
    """V[C][P] += sum_m Y_i conj(Y_j) (FP64 triple loop).  Y: complex [S][T][C]."""
    Y = np.ascontiguousarray(Y, dtype=np.complex128)
    S, T, C = Y.shape
    if V is None:
        V = np.zeros((C, n_pairs(S)), dtype=np.complex128)
    _load().orc_xengine_f64(_p(Y), S, T, C, _p(V))
    return V


def xengine_int(q: np.ndarray, A: np.ndarray | None = None) -> np.ndarray:
    """A[C][P][2] += sum_m q_i conj(q_j) in int64.  q: int8 [S][T][C][2]."""
    q = np.ascontiguousarray(q, dtype=np.int8)
    S, T, C, two = q.shape
    assert two == 2
    if A is None:
        A = np.zeros((C, n_pairs(S), 2), dtype=np.int64)
    _load().orc_xengine_int(_p(q), S, T, C, _p(A))
    return A


def xengine_i16(q: np.ndarray, A: np.ndarray | None = None) -> np.ndarray:
    """A[C][P][2] += sum_m q_i conj(q_j) in int64 on 16-bit integer spectra
    (sections 3.1 and 4.1: 16-bit data, exact 32-bit products).  q: int16 [S][T][C][2]."""
    q = np.ascontiguousarray(q, dtype=np.int16)
    S, T, C, two = q.shape
    assert two == 2
    if A is None:
        A = np.zeros((C, n_pairs(S), 2), dtype=np.int64)
    _load().orc_xengine_i16(_p(q), S, T, C, _p(A))
    return A


def fix16_table() -> np.ndarray:
    """The 1440-step phase table as Q14 integers (cos, sin) [1440][2] (section 4.1)."""
    w = np.zeros((1440, 2), dtype=np.int32)
    _load().orc_fix16_table(_p(w))
    return w


def fix16_spectra(X: np.ndarray, geom: Geometry, fs: float, scale: np.ndarray, nu_bb: float = 0.0,
                  sideband: int = 1, spectrum0: int = 0):
    """The 16-bit fixed-point spectra of the real-time pipeline (sections 3.1
    and 4.1) from the unrotated FFT output X [S][T][C] (complex): the 16-bit
    fixed-point FFT output q = sat16(rne(X / scale)) (X and scale FP32 values,
    the division in FP32), then the integer fringe
    stop and FSTC y = sat16(round((q w_j) / 2^14)) with the Q14 table entry j of
    the Eq. 2 phase.  Returns (q, y), int16 [S][T][C][2] each."""
    X = np.ascontiguousarray(np.stack([X.real, X.imag], -1), dtype=np.float64)
    S, T, C, _ = X.shape
    scale = np.ascontiguousarray(scale, dtype=np.float64).reshape(S, C)
    q = np.zeros((S, T, C, 2), dtype=np.int16)
    y = np.zeros((S, T, C, 2), dtype=np.int16)
    _load().orc_fix16_spectra(_p(X), S, T, C, spectrum0, _p(geom.f), _p(geom.psi0), _p(geom.rate), fs, nu_bb,
                              sideband, _p(scale), _p(q), _p(y))
    return q, y


# ---------------------------------------------------------------------------
# Array beams (section 2.2)
# ---------------------------------------------------------------------------
BEAM_INTENSITY, BEAM_FULLPOL, BEAM_VOLTAGE = 0, 1, 2


def beamform(Y: np.ndarray, w=None, c=None, mode: int = BEAM_FULLPOL, tint: int = 1):
    """Incoherent beam (detected intensities of the selected signals added,
    weights w [S]) and coherent beams (voltages added with complex weights
    c [nb][S], then detected: |V_0|^2, |V_1|^2 and, full-polar, V_0 conj(V_1);
    or the voltages), the two beamformer modes of section 2.2.  Y: complex
    [S][T][C]; signal s = 2a + pol.  Returns (inc [2][T/tint][C] or None,
    coh [nb][planes][T/tint][C] or None), sums over tint spectra."""
    Y = np.ascontiguousarray(Y, dtype=np.complex128)
    S, T, C = Y.shape
    To = T // tint
    inc = np.zeros((2, To, C)) if w is not None else None
    nb = 0 if c is None else len(c)
    coh = None
    if nb:
        c = np.ascontiguousarray(c, dtype=np.complex128).reshape(nb, S)
        coh = (np.zeros((nb, 2, T, C), dtype=np.complex128) if mode == BEAM_VOLTAGE
               else np.zeros((nb, 4 if mode == BEAM_FULLPOL else 2, To, C)))
    wv = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
    _load().orc_beamform(_p(Y), S, T, C, _p(wv) if wv is not None else None,
                         _p(c) if nb else None, nb, mode, tint,
                         _p(inc) if inc is not None else None, _p(coh) if coh is not None else None)
    return inc, coh


# ---------------------------------------------------------------------------
# Coherent dedispersion of phased-array voltages (section 4.3)
# ---------------------------------------------------------------------------
K_DM = 4.148808e15  # dispersion constant, Hz^2 s / (pc cm^-3): delay = K_DM DM / nu^2


def baseband_series(V: np.ndarray) -> np.ndarray:
    """Broadband complex time series of channel voltages V [..][T][C]: per
    spectrum the inverse DFT over the channels, z[m C + n] = sum_k
    V[m, k] exp(+2 pi i k n / C) (unnormalised); the channels k fs/N of the
    band become a complex baseband signal at fs/2 samples per second."""
    V = np.asarray(V, dtype=np.complex128)
    C = V.shape[-1]
    z = np.fft.ifft(V, axis=-1) * C
    return z.reshape(V.shape[:-2] + (V.shape[-2] * C,))


def dispersion_phase_cycles(f: np.ndarray, nu0: float, dm: float) -> np.ndarray:
    """Phase (cycles) of the cold-plasma transfer function at sky frequency
    nu0 + f, referenced to nu0: K_DM DM (1/nu - 1/nu0 + (nu - nu0)/nu0^2) =
    K_DM DM f^2 / (nu0^2 (nu0 + f)).  Its group delay is K_DM DM (nu^-2 -
    nu0^-2), the dispersion delay relative to nu0 (a pure delay and a
    constant phase dropped)."""
    f = np.asarray(f, dtype=np.float64)
    return K_DM * dm * f * f / (nu0 * nu0 * (nu0 + f))


def dedisperse(V: np.ndarray, fs: float, nu0: float, dm: float, n_int: int) -> np.ndarray:
    """Coherent dedispersion of phased-array voltages V [npol][T][C] (upper
    sideband, channel k at sky frequency nu0 + k fs/N, N = 2C) as in section
    4.3: the broadband series of each polarisation (inverse FFT of its
    spectra), its Fourier transform multiplied by the inverse dispersion
    transfer function exp(-2 pi i phase(f)), f = q fs / (2 L) for bin q of L =
    T C, the inverse transform (divided by L), intensities |z|^2 added over
    polarisations and summed over n_int samples: I [L / n_int].  The
    transform is circular: the first K_DM DM (nu0^-2 - (nu0 + fs/2)^-2) fs/2
    samples wrap around and are not valid."""
    V = np.asarray(V, dtype=np.complex128)
    npol, T, C = V.shape
    L = T * C
    z = baseband_series(V)
    f = np.arange(L, dtype=np.float64) * (fs / (2.0 * L))
    ph = dispersion_phase_cycles(f, nu0, dm)
    ph = ph - np.floor(ph)
    H = np.exp(-2j * np.pi * ph)
    zd = np.fft.ifft(np.fft.fft(z, axis=-1) * H, axis=-1)
    I = (np.abs(zd) ** 2).sum(0)
    return I.reshape(L // n_int, n_int).sum(1)


def smear_samples(fs: float, nu0: float, dm: float) -> int:
    """Dispersion sweep across the band [nu0, nu0 + fs/2] in complex samples
    at fs/2."""
    return int(np.ceil(K_DM * dm * (1.0 / nu0 ** 2 - 1.0 / (nu0 + fs / 2) ** 2) * fs / 2))


# ---------------------------------------------------------------------------
# Gated correlator (section 5)
# ---------------------------------------------------------------------------
def pulsar_gates(spectrum0: int, n: int, N: int, fs: float, t0: float, period: float, n_bins: int) -> np.ndarray:
    """Gate bin of spectra spectrum0 .. spectrum0 + n - 1: the pulse phase
    frac((t - t0) / P) at the window centre t = (m + 1/2) N / fs, in n_bins
    equal bins (FP64, each operation rounded on its own)."""
    out = np.empty(n, dtype=np.uint8)
    t_spec = float(N) / float(fs)
    for i in range(n):
        t = (float(spectrum0 + i) + 0.5) * t_spec
        x = (t - t0) / period
        phase = x - np.floor(x)
        b = int(np.floor(phase * float(n_bins)))
        out[i] = min(max(b, 0), n_bins - 1)
    return out


def xengine_gated(Y: np.ndarray, gate, n_bins: int) -> np.ndarray:
    """V_b = sum over the spectra with gate == b of Y_i conj(Y_j): the X
    oracle on each bin's spectra ([n_bins][C][P] complex128)."""
    gate = np.asarray(gate)
    return np.stack([xengine(np.ascontiguousarray(Y[:, gate == b, :])) for b in range(n_bins)])


def xengine_int_gated(q: np.ndarray, gate, n_bins: int) -> np.ndarray:
    """The int64 X oracle on each bin's int8 spectra ([n_bins][C][P][2])."""
    gate = np.asarray(gate)
    return np.stack([xengine_int(np.ascontiguousarray(q[:, gate == b])) for b in range(n_bins)])


# ---------------------------------------------------------------------------
# ADC input formats (sections 2.3.2 and 3.3)
# ---------------------------------------------------------------------------
def adc_unpack(raw: np.ndarray, n: int, bits: int) -> np.ndarray:
    """Demultiplex and unpack the raw streams of acquisition cards (uint8
    [cards][bytes], time-major, 4 inputs per time sample, 8-bit bytes or
    4-bit nibbles low first, two's complement) into int8 rows [4 cards][n]
    (row 4 c + i = input i of card c)."""
    raw = np.ascontiguousarray(raw, dtype=np.uint8)
    cards = raw.shape[0]
    assert bits in (4, 8) and raw.shape[1] >= n * 4 * bits // 8
    x = np.zeros((4 * cards, n), dtype=np.int8)
    _load().orc_adc_unpack(_p(raw), raw.shape[1], cards, n, bits, _p(x), n)
    return x


# ---------------------------------------------------------------------------
# Time-domain MAD voltage blanker (section 5, Eq. 3 and 4)
# ---------------------------------------------------------------------------
def philox4x32_10(ctr, key) -> np.ndarray:
    """One Philox4x32-10 block (Salmon et al., SC'11): 4 counter words and 2
    key words in, 4 words out."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(4)
    k = np.ascontiguousarray(key, dtype=np.uint32).reshape(2)
    out = np.zeros(4, dtype=np.uint32)
    _load().orc_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def blank_noise_table(seed: int, S: int, L: int) -> np.ndarray:
    """Precomputed replacement noise [S][L] (float32, mean 0, variance 1):
    Irwin-Hall sums of twelve 16-bit uniforms from Philox4x32-10, one
    independent row per signal."""
    t = np.zeros((S, L), dtype=np.float32)
    _load().orc_blank_noise_table(int(seed) & 0xFFFFFFFFFFFFFFFF, S, L, _p(t))
    return t


def blank_noise_entry(seed: int, s: int, j: int) -> float:
    """Entry j of signal s's noise-table row, computed on its own."""
    return float(_load().orc_blank_noise_entry(int(seed) & 0xFFFFFFFFFFFFFFFF, s, j))


def mad_blank(x: np.ndarray, B: int, M: float, table: np.ndarray, sample0: int = 0):
    """Blank voltage outliers per block of B samples of each row of x (int8
    [S][n]): samples with |x - median| > M MAD / 0.6745 become
    rint(median + MAD / 0.6745 * z) clamped to int8, z from the signal's row
    of the noise table at (sample0 + i) mod L.  Returns (out, counts
    [S][nblocks], stats [S][nblocks][2] = (2 median, 4 MAD))."""
    x = np.ascontiguousarray(x, dtype=np.int8)
    S, n = x.shape
    table = np.ascontiguousarray(table, dtype=np.float32)
    assert table.shape[0] == S
    L = table.shape[1]
    assert L > 0 and L & (L - 1) == 0
    nb = (n + B - 1) // B
    out = np.empty_like(x)
    counts = np.zeros((S, nb), dtype=np.int32)
    stats = np.zeros((S, nb, 2), dtype=np.int32)
    _load().orc_mad_blank(_p(x), n, S, n, B, float(M), _p(table), L, sample0, _p(out), _p(counts), _p(stats))
    return out, counts, stats


# ---------------------------------------------------------------------------
# Requantisation (section 4.1) and FP8 encoding
# ---------------------------------------------------------------------------
def sigma(Y: np.ndarray) -> np.ndarray:
    """sigma[s][k] = sqrt(sum_m |Y|^2 / (2T)): RMS of one component."""
    Y = np.ascontiguousarray(Y, dtype=np.complex128)
    S, T, C = Y.shape
    out = np.empty((S, C), dtype=np.float64)
    _load().orc_sigma(_p(Y), S, T, C, _p(out))
    return out


def int8_scale(sig: np.ndarray) -> np.ndarray:
    """Recorded int8 scale 4 sigma / 127 (1 where sigma is 0), as float32."""
    s = (4.0 * np.asarray(sig, dtype=np.float64) / 127.0).astype(np.float32)
    s[s == 0] = 1.0
    return s


def fp8_scale(sig: np.ndarray) -> np.ndarray:
    """Recorded e4m3 scale 4 sigma / 448 (1 where sigma is 0), as float32."""
    s = (4.0 * np.asarray(sig, dtype=np.float64) / 448.0).astype(np.float32)
    s[s == 0] = 1.0
    return s


def quantize_int8(Y: np.ndarray, scale: np.ndarray) -> np.ndarray:
    """q = clamp(rne(Y/scale), +-127) per component -> int8 [S][T][C][2]."""
    Y = np.ascontiguousarray(Y, dtype=np.complex128)
    S, T, C = Y.shape
    sc = np.ascontiguousarray(scale, dtype=np.float64)
    q = np.empty((S, T, C, 2), dtype=np.int8)
    _load().orc_quantize_int8(_p(Y), _p(sc), S, T, C, _p(q))
    return q


def quantize_fp8(Y: np.ndarray, scale: np.ndarray) -> np.ndarray:
    """b = e4m3(Y/scale) per component -> uint8 codes [S][T][C][2]."""
    Y = np.ascontiguousarray(Y, dtype=np.complex128)
    S, T, C = Y.shape
    sc = np.ascontiguousarray(scale, dtype=np.float64)
    q = np.empty((S, T, C, 2), dtype=np.uint8)
    _load().orc_quantize_fp8(_p(Y), _p(sc), S, T, C, _p(q))
    return q


def e4m3_decode(codes) -> np.ndarray:
    lib = _load()
    c = np.asarray(codes, dtype=np.uint8)
    return np.array([lib.orc_e4m3_decode(int(b)) for b in c.ravel()]).reshape(c.shape)


def e4m3_decode_table() -> np.ndarray:
    """All 256 code values (NaN for 0x7F / 0xFF)."""
    return e4m3_decode(np.arange(256, dtype=np.uint8))


def e4m3_encode(v: float) -> int:
    return int(_load().orc_e4m3_encode(float(v)))


def scale_visibilities(A: np.ndarray, scale: np.ndarray, V: np.ndarray | None = None):
    """V += scale_i scale_j A (FP64).  A: [C][P][2] int64/float; scale [S][C]."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    C, P, _ = A.shape
    S = int(round((np.sqrt(8 * P + 1) - 1) / 2))
    sc = np.ascontiguousarray(scale, dtype=np.float64)
    out = np.zeros((C, P, 2), dtype=np.float64) if V is None else V
    _load().orc_scale_visibilities(_p(A), _p(sc), S, C, _p(out))
    return out


# ---------------------------------------------------------------------------
# MAD (section 5, Eq. 3 and Eq. 4)
# ---------------------------------------------------------------------------
def median(v) -> float:
    v = np.ascontiguousarray(v, dtype=np.float64).ravel()
    return float(_load().orc_median(_p(v), v.size))


def mad_flags(x, M: float = 3.0):
    """Flags of Eq. 4 on the block x; returns (flags uint8, median, MAD)."""
    x = np.ascontiguousarray(x, dtype=np.float64).ravel()
    fl = np.empty(x.size, dtype=np.uint8)
    med = ctypes.c_double()
    mad = ctypes.c_double()
    _load().orc_mad_flags(_p(x), x.size, M, _p(fl), ctypes.byref(med), ctypes.byref(mad))
    return fl, med.value, mad.value


def power(Y: np.ndarray) -> np.ndarray:
    """|Y|^2 of F-engine spectra [S][T][C] (FP64)."""
    return np.abs(np.asarray(Y)) ** 2


def mad_tile_flags(pw: np.ndarray, M: float = 3.0, TT: int = 64, KT: int = 256, stats: str = "both") -> np.ndarray:
    """Eq. 3 / Eq. 4 on TT x KT power tiles; flags [S][T][C] uint8.  stats:
    "both" (a cell is flagged when its row or its column is), "rows" or
    "columns" (one statistic only)."""
    pw = np.ascontiguousarray(pw, dtype=np.float64)
    S, T, C = pw.shape
    fl = np.empty((S, T, C), dtype=np.uint8)
    which = {"rows": 1, "columns": 2, "both": 3}[stats]
    if _load().orc_mad_tile_flags_which(_p(pw), S, T, C, TT, KT, M, which, _p(fl)) != 0:
        raise ValueError("T must be a multiple of %d and C of %d" % (TT, KT))
    return fl


def pair_counts(flags: np.ndarray) -> np.ndarray:
    """n_ij[k] = number of spectra where neither signal is flagged; int64 [C][P]."""
    fl = np.ascontiguousarray(flags, dtype=np.uint8)
    S, T, C = fl.shape
    n = np.zeros((C, n_pairs(S)), dtype=np.int64)
    _load().orc_pair_counts(_p(fl), S, T, C, _p(n))
    return n


def apply_flags(Y: np.ndarray, flags: np.ndarray) -> np.ndarray:
    """Zero the flagged cells of the spectra: a flagged sample contributes nothing."""
    return np.where(np.asarray(flags) != 0, 0, Y)


# ---------------------------------------------------------------------------
# Learned flagger: conv3x3(1->16)-ReLU-conv3x3(16->16)-ReLU-conv3x3(16->1),
# sigmoid, binary cross-entropy against MAD labels (FP64 reference)
# ---------------------------------------------------------------------------
CNN_SHAPES = [(16, 1), (16, 16), (1, 16)]  # (Cout, Cin) per layer


def cnn_param_count() -> int:
    return sum(o * i * 9 + o for o, i in CNN_SHAPES)


def cnn_unpack(params):
    """Flat parameter vector -> [(w [Cout][Cin][3][3], bias [Cout]) per layer]
    (layout: layer by layer, weights then biases)."""
    params = np.asarray(params, dtype=np.float64)
    out, o0 = [], 0
    for co, ci in CNN_SHAPES:
        w = params[o0:o0 + co * ci * 9].reshape(co, ci, 3, 3)
        o0 += co * ci * 9
        b = params[o0:o0 + co]
        o0 += co
        out.append((np.ascontiguousarray(w), np.ascontiguousarray(b)))
    return out


def conv3x3(x, w, b):
    x = np.ascontiguousarray(x, dtype=np.float64)
    B, Ci, H, W = x.shape
    Co = w.shape[0]
    y = np.empty((B, Co, H, W))
    _load().orc_conv3x3_fwd(_p(x), _p(np.ascontiguousarray(w, dtype=np.float64)),
                            _p(np.ascontiguousarray(b, dtype=np.float64)), B, Ci, Co, H, W, _p(y))
    return y


def conv3x3_bwd(x, w, dy, need_dx=True):
    x = np.ascontiguousarray(x, dtype=np.float64)
    dy = np.ascontiguousarray(dy, dtype=np.float64)
    B, Ci, H, W = x.shape
    Co = w.shape[0]
    dx = np.empty_like(x) if need_dx else None
    dw = np.empty((Co, Ci, 3, 3))
    db = np.empty(Co)
    _load().orc_conv3x3_bwd(_p(x), _p(np.ascontiguousarray(w, dtype=np.float64)), _p(dy), B, Ci, Co, H, W,
                            _p(dx) if need_dx else None, _p(dw), _p(db))
    return dx, dw, db


def cnn_forward(params, x):
    """x [B][1][H][W] -> logits [B][1][H][W] and the intermediate values."""
    (w1, b1), (w2, b2), (w3, b3) = cnn_unpack(params)
    z1 = conv3x3(x, w1, b1)
    a1 = np.maximum(z1, 0)
    z2 = conv3x3(a1, w2, b2)
    a2 = np.maximum(z2, 0)
    z3 = conv3x3(a2, w3, b3)
    return z3, (x, z1, a1, z2, a2)


def bce_with_logits(z, y):
    """Mean binary cross-entropy of sigmoid(z) against labels y, in the stable
    form max(z, 0) - z y + log(1 + exp(-|z|))."""
    z = np.asarray(z, dtype=np.float64)
    return float(np.mean(np.maximum(z, 0) - z * y + np.log1p(np.exp(-np.abs(z)))))


def cnn_loss_and_grad(params, x, y):
    """Loss and its gradient with respect to the flat parameter vector (chain rule
    through the three convolutions and the ReLUs)."""
    z3, (x0, z1, a1, z2, a2) = cnn_forward(params, x)
    loss = bce_with_logits(z3, y)
    dz3 = (1.0 / (1.0 + np.exp(-z3)) - y) / z3.size
    (w1, _), (w2, _), (w3, _) = cnn_unpack(params)
    da2, dw3, db3 = conv3x3_bwd(a2, w3, dz3)
    dz2 = da2 * (z2 > 0)
    da1, dw2, db2 = conv3x3_bwd(a1, w2, dz2)
    dz1 = da1 * (z1 > 0)
    _, dw1, db1 = conv3x3_bwd(x0, w1, dz1, need_dx=False)
    g = np.concatenate([dw1.ravel(), db1, dw2.ravel(), db2, dw3.ravel(), db3])
    return loss, g


def cnn_tile_input(power_tile):
    """Network input of one 64 x 256 power tile: log(1 + P / m), m = median over the
    tile's channels of the channel's mean power over the tile's spectra; a tile
    whose median is not positive (all zero) has no reference level and takes
    m = 1, so its input is log(1 + P)."""
    P = np.asarray(power_tile, dtype=np.float64)
    m = median(P.mean(axis=0))
    if not m > 0:
        m = 1.0
    return np.log1p(P / m)


def adam_step(params, m, v, g, t: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update (Kingma & Ba 2015, Algorithm 1) at step t >= 1: biased
    moments m, v, their bias corrections 1 - beta^t, and the step
    lr * m_hat / (sqrt(v_hat) + eps).  Returns new (params, m, v)."""
    g = np.asarray(g, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1 - beta2) * g * g
    m_hat = m / (1 - beta1 ** t)
    v_hat = v / (1 - beta2 ** t)
    return np.asarray(params, dtype=np.float64) - lr * m_hat / (np.sqrt(v_hat) + eps), m, v


def cnn_tile_logits(params, power, TT: int = 64, KT: int = 256):
    """Logits of the network on every TT x KT tile of power [S][T][C] (each tile
    its own zero-padded image), same layout as power."""
    P = np.asarray(power, dtype=np.float64)
    S, T, C = P.shape
    out = np.empty_like(P)
    tiles = []
    for s in range(S):
        for mt in range(T // TT):
            for kt in range(C // KT):
                tiles.append(cnn_tile_input(P[s, mt * TT:(mt + 1) * TT, kt * KT:(kt + 1) * KT]))
    z, _ = cnn_forward(params, np.stack(tiles)[:, None])
    i = 0
    for s in range(S):
        for mt in range(T // TT):
            for kt in range(C // KT):
                out[s, mt * TT:(mt + 1) * TT, kt * KT:(kt + 1) * KT] = z[i, 0]
                i += 1
    return out


def cnn_guarded_flags(params, power, threshold: float = 0.5, guard_m: float = 3.0, TT: int = 64, KT: int = 256):
    """Flags of the learned flagger with the column guard: a cell is flagged
    when sigmoid(its logit) > threshold, or when its tile column is an outlier
    of the MAD column statistic (Eq. 3 and Eq. 4 with M = guard_m on the
    tile's channel means over its spectra).  guard_m <= 0: the network alone.
    Returns (flags uint8, logits), both [S][T][C]."""
    z = cnn_tile_logits(params, power, TT, KT)
    f = (z > np.log(threshold / (1.0 - threshold))).astype(np.uint8)
    if guard_m > 0:
        f |= mad_tile_flags(power, guard_m, TT, KT, stats="columns")
    return f, z


# ---------------------------------------------------------------------------
# Error metrics (the paper's tolerance is not stated; these are the build's)
# ---------------------------------------------------------------------------
def normalized_error(V: np.ndarray, V64: np.ndarray, S: int):
    """(e_max, e_fro): e_max = max |V - V64| / sqrt(V64_ii V64_jj) over all
    channels and pairs; e_fro = ||V - V64||_F / ||V64||_F."""
    V = np.asarray(V, dtype=np.complex128)
    V64 = np.asarray(V64, dtype=np.complex128)
    ii, jj = pair_table(S)
    auto = np.real(V64[:, [pair_index(s, s) for s in range(S)]])  # [C][S]
    denom = np.sqrt(np.abs(auto[:, ii] * auto[:, jj]))
    denom = np.where(denom > 0, denom, 1.0)
    err = np.abs(V - V64)
    e_max = float(np.max(err / denom))
    e_fro = float(np.linalg.norm(V - V64) / max(np.linalg.norm(V64), 1e-300))
    return e_max, e_fro
