"""Seeded synthetic GMRT-shaped inputs for the FX correlator.

This module is the only code that both the GPU tests/benchmark and the CPU
oracle consume.  It generates input samples and geometry; it holds none of the
correlator's arithmetic (no channelisation, phase correction, cross-multiply or
requantisation).

Recipe (stand-in for recorded GMRT baseband, which is not available):

* signal s = 2a + pol for antenna a and polarisation pol;
* per antenna: integer delay D ~ U{0..16} samples, fractional delay
  f ~ U[0, 1) samples, fringe phase psi0 ~ U[0, 1) cycles, fringe rate
  r ~ U[-5, 5] Hz; both polarisations share them;
* a common sky component per polarisation (independent for the two
  polarisations): white Gaussian noise, band-limited to (0, fs/2), delayed
  by D + f samples and fringe-rotated by exp(-2 pi i sigma (psi0 + r t)) --
  the forward model whose inverse the correlator applies;
* independent receiver noise per signal;
* optional CW tone at the centre of one channel, delayed and rotated like
  the sky component;
* x = clip(rint(sigma_t (sqrt(rho) c + sqrt(1 - rho) n) + tone), -127, 127).

``mode="physical"`` synthesises the delayed, fringe-rotated analytic signal in
the frequency domain with numpy's FFT, in circular blocks of ``block`` samples.
``mode="bulk"`` (large inputs where only the shape, rate and distribution
matter) uses the integer part of the delay only and no fringe rotation; it is
cheap and multi-threaded.

Random numbers come from numpy's Philox counter-based generator keyed by
(seed, purpose, signal, block), so any slice can be regenerated.
"""
from __future__ import annotations

import concurrent.futures as _cf
import os

import numpy as np

BASE_SEED = 0x09101517


def rng(seed: int, *key: int) -> np.random.Generator:
    """Philox-4x32-10 stream keyed by (seed, *key)."""
    ss = np.random.SeedSequence([int(seed) & 0xFFFFFFFF, *[int(k) & 0xFFFFFFFF for k in key]])
    return np.random.Generator(np.random.Philox(ss))


class Geom:
    """Per-signal geometry: D (int32), f, psi0, rate (float64) arrays."""

    def __init__(self, D, f, psi0, rate):
        self.D = np.asarray(D, dtype=np.int32)
        self.f = np.asarray(f, dtype=np.float64)
        self.psi0 = np.asarray(psi0, dtype=np.float64)
        self.rate = np.asarray(rate, dtype=np.float64)

    @property
    def S(self):
        return self.D.size

    def subset(self, idx):
        return Geom(self.D[idx], self.f[idx], self.psi0[idx], self.rate[idx])


def make_geometry(n_ant: int, n_pol: int = 2, seed: int = BASE_SEED, max_delay: int = 16,
                  rate_max: float = 5.0, frac: bool = True, fringe: bool = True) -> Geom:
    """Antenna-based delays/fringes, repeated for each polarisation (s = n_pol*a + pol)."""
    g = rng(seed, 1)
    D = g.integers(0, max_delay + 1, size=n_ant)
    # fractions are float32-representable: the device geometry holds them as float
    f = (g.random(n_ant).astype(np.float32).astype(np.float64)) if frac else np.zeros(n_ant)
    psi0 = g.random(n_ant) if fringe else np.zeros(n_ant)
    rate = g.uniform(-rate_max, rate_max, size=n_ant) if fringe else np.zeros(n_ant)
    rep = lambda a: np.repeat(a, n_pol)
    return Geom(rep(D), rep(f), rep(psi0), rep(rate))


def _analytic_block(g: np.random.Generator, B: int) -> np.ndarray:
    """One-sided white spectrum Z[nu], nu = 0..B-1 (only 1..B/2-1 non-zero),
    scaled so that Re of the analytic signal has unit variance."""
    nb = B // 2 - 1
    Z = np.zeros(B, dtype=np.complex128)
    amp = np.sqrt(2.0 / nb) / np.sqrt(2.0)
    Z[1:B // 2] = amp * (g.standard_normal(nb) + 1j * g.standard_normal(nb))
    return Z


class RFI:
    """Injected radio-frequency interference (added before rounding and clipping).

    * narrowband persistent tones in a fraction ``tone_frac`` of the channels of
      an N-point channelisation, at a random frequency inside the channel, each
      with excess power k * mu in its channel (k ~ U[tone_k]), where
      mu = N sigma_t^2 is the mean per-cell noise power; the same channels for
      every signal, random phase per signal;
    * broadband bursts per antenna (both polarisations): a burst starts in a
      spectrum with probability ``burst_p``, lasts U{burst_len} spectra and adds
      Gaussian noise of variance k * sigma_t^2 (k ~ U[burst_k]); a fraction
      ``bl_frac`` of them is band-limited to a random contiguous band of
      U[bl_width] of the channels (same excess power per cell inside it);
    * intermittent narrowband lines per antenna: a line starts in a spectrum
      with probability ``nb_p``, lasts U{nb_len} spectra, at a random frequency
      with excess power k * mu in its channel (k ~ U[nb_k]).
    The last two are off by default.
    """

    def __init__(self, N: int, seed: int = BASE_SEED, tone_frac: float = 0.05, tone_k=(20.0, 200.0),
                 burst_p: float = 0.002, burst_k=(10.0, 100.0), burst_len=(1, 8),
                 bl_frac: float = 0.0, bl_width=(0.05, 0.3), nb_p: float = 0.0, nb_k=(20.0, 200.0),
                 nb_len=(4, 32)):
        self.N, self.seed = N, seed
        self.tone_frac, self.tone_k = tone_frac, tone_k
        self.burst_p, self.burst_k, self.burst_len = burst_p, burst_k, burst_len
        self.bl_frac, self.bl_width = bl_frac, bl_width
        self.nb_p, self.nb_k, self.nb_len = nb_p, nb_k, nb_len

    def tones(self):
        """(channel, frequency in cycles/sample, excess power factor k) of every tone."""
        g = rng(self.seed, 9, self.N)
        C = self.N // 2
        n = max(1, int(round(self.tone_frac * C)))
        ch = np.sort(g.choice(np.arange(2, C - 1), size=n, replace=False))
        freq = (ch + g.uniform(-0.5, 0.5, n)) / self.N
        k = g.uniform(*self.tone_k, n)
        return ch, freq, k

    def bursts(self, n_ant: int, n_spec: int):
        """list per antenna of (start spectrum, length, variance factor, band):
        band = None (broadband) or (first, last) frequency bin of an N-point FFT."""
        out = []
        C = self.N // 2
        for a in range(n_ant):
            g = rng(self.seed, 10, a)
            starts = np.nonzero(g.random(n_spec) < self.burst_p)[0]
            lens = g.integers(self.burst_len[0], self.burst_len[1] + 1, starts.size)
            ks = g.uniform(*self.burst_k, starts.size)
            gb = rng(self.seed, 13, a)
            bands = []
            for _ in range(starts.size):
                if gb.random() < self.bl_frac:
                    w = max(1, int(round(gb.uniform(*self.bl_width) * C)))
                    lo = int(gb.integers(0, C - w + 1))
                    bands.append((lo, lo + w - 1))
                else:
                    bands.append(None)
            out.append(list(zip(starts.tolist(), lens.tolist(), ks.tolist(), bands)))
        return out

    def lines(self, n_ant: int, n_spec: int):
        """list per antenna of intermittent narrowband lines
        (start spectrum, length, frequency in cycles/sample, excess factor k)."""
        out = []
        C = self.N // 2
        for a in range(n_ant):
            g = rng(self.seed, 14, a)
            starts = np.nonzero(g.random(n_spec) < self.nb_p)[0]
            lens = g.integers(self.nb_len[0], self.nb_len[1] + 1, starts.size)
            freq = (g.integers(2, C - 1, starts.size) + g.uniform(-0.5, 0.5, starts.size)) / self.N
            ks = g.uniform(*self.nb_k, starts.size)
            out.append(list(zip(starts.tolist(), lens.tolist(), freq.tolist(), ks.tolist())))
        return out

    def signal(self, S: int, n_samples: int, sigma_t: float, n_pol: int = 2) -> np.ndarray:
        """The RFI-only float signal [S][n_samples] (the last one is cached)."""
        key = (S, n_samples, float(sigma_t), n_pol)
        if getattr(self, "_cache_key", None) == key:
            return self._cache
        self._cache_key, self._cache = key, self._signal(S, n_samples, sigma_t, n_pol)
        return self._cache

    def _signal(self, S: int, n_samples: int, sigma_t: float, n_pol: int) -> np.ndarray:
        N = self.N
        out = np.zeros((S, n_samples))
        n = np.arange(n_samples)
        ch, freq, k = self.tones()
        amp = 2.0 * sigma_t * np.sqrt(k / N)  # (A N / 2)^2 = k N sigma_t^2
        phs = [rng(self.seed, 11, s).uniform(0, 2 * np.pi, ch.size) for s in range(S)]

        def tone_job(job):  # every sample's tones are summed in the same order in any job
            s, lo, hi = job
            for c in range(ch.size):
                out[s, lo:hi] += amp[c] * np.cos(2 * np.pi * freq[c] * n[lo:hi] + phs[s][c])

        span = 1 << 20
        jobs = [(s, lo, min(n_samples, lo + span)) for s in range(S) for lo in range(0, n_samples, span)]
        with _cf.ThreadPoolExecutor(min(16, os.cpu_count() or 1)) as ex:
            list(ex.map(tone_job, jobs))
        for a, bl in enumerate(self.bursts(S // n_pol, n_samples // N)):
            for (m0, ln, kk, band) in bl:
                lo, hi = m0 * N, min(n_samples, (m0 + ln) * N)
                for pol in range(n_pol):
                    s = a * n_pol + pol
                    z = sigma_t * np.sqrt(kk) * rng(self.seed, 12, s, m0).standard_normal(hi - lo)
                    if band is not None:  # keep the bins of [band] at the resolution of N-point spectra
                        Z = np.fft.rfft(z)
                        f = np.arange(Z.size) * N / (hi - lo)
                        Z[(f < band[0] - 0.5) | (f > band[1] + 0.5)] = 0
                        z = np.fft.irfft(Z, hi - lo)
                    out[s, lo:hi] += z
        for a, ll in enumerate(self.lines(S // n_pol, n_samples // N)):
            for (m0, ln, fr, kk) in ll:
                lo, hi = m0 * N, min(n_samples, (m0 + ln) * N)
                ph = rng(self.seed, 15, a, m0).uniform(0, 2 * np.pi, n_pol)
                for pol in range(n_pol):
                    out[a * n_pol + pol, lo:hi] += 2.0 * sigma_t * np.sqrt(kk / N) * np.cos(
                        2 * np.pi * fr * np.arange(lo, hi) + ph[pol])
        return out


def voltages(S: int, n_samples: int, geom: Geom, fs: float, *, seed: int = BASE_SEED,
             rho: float = 0.3, sigma_t: float = 12.0, sideband: int = 1, n_pol: int = 2,
             tone_bin: int | None = None, tone_N: int | None = None, tone_amp: float = 4.0,
             sources: list | None = None, noise: bool = True, block: int = 1 << 20,
             mode: str = "physical", threads: int | None = None, rfi: RFI | None = None) -> np.ndarray:
    """int8 [S][n_samples] streams (see module docstring).

    sources: list of dicts {"power": p, "dD": per-signal extra delay (samples),
    "drate": per-signal extra fringe rate (Hz)}; default one source of power
    rho at the phase centre.  rfi: interference added before rounding (physical
    mode only).
    """
    if sources is None:
        sources = [{"power": rho}]
    if mode == "bulk":
        return _voltages_bulk(S, n_samples, geom, seed=seed, rho=rho, sigma_t=sigma_t,
                              n_pol=n_pol, tone_bin=tone_bin, tone_N=tone_N, tone_amp=tone_amp,
                              noise=noise, threads=threads)
    tot_src = float(sum(s["power"] for s in sources))
    out = np.empty((S, n_samples), dtype=np.int8)
    n_blocks = -(-n_samples // block)
    nu = np.fft.fftfreq(block) * block  # integer frequencies (cycles per block)
    rfi_sig = rfi.signal(S, n_samples, sigma_t, n_pol) if rfi is not None else None

    def work(b):  # blocks are independent (their random streams are keyed by b)
        n0 = b * block
        nb = min(block, n_samples - n0)
        t = (n0 + np.arange(nb)) / fs
        acc = np.zeros((S, nb), dtype=np.float64)
        for si, src in enumerate(sources):
            amp_src = np.sqrt(src["power"])
            dD = np.asarray(src.get("dD", np.zeros(S)), dtype=np.float64)
            drate = np.asarray(src.get("drate", np.zeros(S)), dtype=np.float64)
            for pol in range(n_pol):
                Z = _analytic_block(rng(seed, 2, si, pol, b), block)
                for s in range(pol, S, n_pol):
                    tau = geom.D[s] + geom.f[s] + dD[s]
                    u = np.fft.ifft(Z * np.exp(-2j * np.pi * nu * tau / block)) * block
                    ph = np.exp(-2j * np.pi * sideband * (geom.psi0[s] + (geom.rate[s] + drate[s]) * t))
                    acc[s] += amp_src * np.real(u[:nb] * ph)
        if noise:
            for s in range(S):
                acc[s] += np.sqrt(max(0.0, 1.0 - tot_src)) * rng(seed, 3, s, b).standard_normal(nb)
        acc *= sigma_t
        if tone_bin is not None:
            n = n0 + np.arange(nb)
            for s in range(S):
                tau = geom.D[s] + geom.f[s]
                ph = 2 * np.pi * (tone_bin / tone_N) * (n - tau) \
                    - 2 * np.pi * sideband * (geom.psi0[s] + geom.rate[s] * t)
                acc[s] += tone_amp * np.cos(ph)
        if rfi_sig is not None:
            acc += rfi_sig[:, n0:n0 + nb]
        out[:, n0:n0 + nb] = np.clip(np.rint(acc), -127, 127).astype(np.int8)

    threads = threads or min(16, os.cpu_count() or 1)
    if n_blocks == 1 or threads == 1:
        for b in range(n_blocks):
            work(b)
    else:
        with _cf.ThreadPoolExecutor(min(threads, n_blocks)) as ex:
            list(ex.map(work, range(n_blocks)))
    return out


def _voltages_bulk(S, n_samples, geom, *, seed, rho, sigma_t, n_pol, tone_bin, tone_N, tone_amp,
                   noise, threads):
    """Integer-delayed common component + noise (+ undelayed tone), multi-threaded."""
    out = np.empty((S, n_samples), dtype=np.int8)
    chunk = 1 << 22
    maxD = int(geom.D.max()) if geom.S else 0
    threads = threads or min(16, os.cpu_count() or 1)
    a, bn = np.float32(sigma_t * np.sqrt(rho)), np.float32(sigma_t * np.sqrt(max(0.0, 1.0 - rho)))

    def work(job):
        pol, c0 = job
        nb = min(chunk, n_samples - c0)
        # common component for samples [c0 - maxD, c0 + nb)
        g = rng(seed, 4, pol, c0 // chunk)
        common = g.standard_normal(nb + maxD, dtype=np.float32)
        for s in range(pol, S, n_pol):
            d = int(geom.D[s])
            v = a * common[maxD - d:maxD - d + nb]
            if noise:
                v = v + bn * rng(seed, 5, s, c0 // chunk).standard_normal(nb, dtype=np.float32)
            if tone_bin is not None:
                n = np.arange(c0, c0 + nb, dtype=np.float64)
                v = v + (tone_amp * np.cos(2 * np.pi * (tone_bin / tone_N) * (n - d))).astype(np.float32)
            np.clip(np.rint(v), -127, 127, out=v)
            out[s, c0:c0 + nb] = v.astype(np.int8)

    jobs = [(pol, c0) for pol in range(n_pol) for c0 in range(0, n_samples, chunk)]
    with _cf.ThreadPoolExecutor(threads) as ex:
        list(ex.map(work, jobs))
    return out


def voltages_device(S: int, n_samples: int, geom: Geom, *, seed: int = BASE_SEED, rho: float = 0.3,
                    sigma_t: float = 12.0, n_pol: int = 2, tone_bin: int | None = None,
                    tone_N: int | None = None, tone_amp: float = 4.0, row_stride: int | None = None,
                    device="cuda"):
    """The ``bulk`` recipe generated on the GPU with torch's seeded Philox generator
    (for inputs of many GB).  Returns an int8 device tensor [S][row_stride] whose
    first n_samples columns hold the streams (the rest is zero)."""
    import torch
    rs = row_stride or n_samples
    out = torch.zeros((S, rs), dtype=torch.int8, device=device)
    maxD = int(geom.D.max()) if geom.S else 0
    a, bn = float(sigma_t * np.sqrt(rho)), float(sigma_t * np.sqrt(max(0.0, 1.0 - rho)))
    gen = torch.Generator(device=device)
    if tone_bin is not None:
        n = torch.arange(n_samples, device=device, dtype=torch.float64)
    for pol in range(n_pol):
        gen.manual_seed((int(seed) * 1000003 + 17 * pol + 1) & 0x7FFFFFFFFFFFFFFF)
        common = torch.randn(n_samples + maxD, generator=gen, device=device, dtype=torch.float32)
        for s in range(pol, S, n_pol):
            d = int(geom.D[s])
            gen.manual_seed((int(seed) * 1000003 + 7919 * (s + 1) + 2) & 0x7FFFFFFFFFFFFFFF)
            v = torch.randn(n_samples, generator=gen, device=device, dtype=torch.float32).mul_(bn)
            v.add_(common[maxD - d:maxD - d + n_samples], alpha=a)
            if tone_bin is not None:
                v.add_((tone_amp * torch.cos(2 * np.pi * (tone_bin / tone_N) * (n - d))).float())
            out[s, :n_samples] = v.round_().clamp_(-127, 127).to(torch.int8)
            del v
        del common
    return out


def voltages_device_physical(S: int, n_samples: int, geom: Geom, fs: float, *, seed: int = BASE_SEED,
                             rho: float = 0.3, sigma_t: float = 12.0, sideband: int = 1, n_pol: int = 2,
                             sources: list | None = None, tone_bin: int | None = None, tone_N: int | None = None,
                             tone_amp: float = 4.0, block: int = 1 << 20, row_stride: int | None = None,
                             device="cuda"):
    """The ``physical`` recipe of :func:`voltages` (fractional delays, fringe
    rotation, point sources, tone) generated on the GPU with torch's FFT and
    seeded generator, for full-size inputs.  Same model as the numpy version,
    other random numbers.  Returns an int8 device tensor [S][row_stride] whose
    first n_samples columns hold the streams (the rest is zero)."""
    import torch
    if sources is None:
        sources = [{"power": rho}]
    tot_src = float(sum(src["power"] for src in sources))
    rs = row_stride or n_samples
    out = torch.zeros((S, rs), dtype=torch.int8, device=device)
    gen = torch.Generator(device=device)
    nu = torch.fft.fftfreq(block, d=1.0 / block, device=device, dtype=torch.float64)  # cycles per block
    nb_half = block // 2 - 1
    amp = np.sqrt(2.0 / nb_half) / np.sqrt(2.0)
    for b in range(-(-n_samples // block)):
        n0 = b * block
        nb = min(block, n_samples - n0)
        t = (n0 + torch.arange(nb, device=device, dtype=torch.float64)) / fs
        acc = torch.zeros((S, nb), dtype=torch.float64, device=device)
        for si, src in enumerate(sources):
            amp_src = float(np.sqrt(src["power"]))
            dD = np.asarray(src.get("dD", np.zeros(S)), dtype=np.float64)
            drate = np.asarray(src.get("drate", np.zeros(S)), dtype=np.float64)
            for pol in range(n_pol):
                gen.manual_seed((int(seed) * 7919 + 104729 * b + 1009 * si + 31 * pol + 3) & 0x7FFFFFFFFFFFFFFF)
                Z = torch.zeros(block, dtype=torch.complex128, device=device)
                Z[1:block // 2] = amp * torch.complex(
                    torch.randn(nb_half, generator=gen, device=device, dtype=torch.float64),
                    torch.randn(nb_half, generator=gen, device=device, dtype=torch.float64))
                for s in range(pol, S, n_pol):
                    tau = float(geom.D[s] + geom.f[s] + dD[s])
                    u = torch.fft.ifft(Z * torch.exp(-2j * np.pi * nu * (tau / block))) * block
                    ph = torch.exp(-2j * np.pi * sideband * (float(geom.psi0[s]) + (float(geom.rate[s]) + drate[s]) * t))
                    acc[s] += amp_src * (u[:nb] * ph).real
                    del u, ph
                del Z
        for s in range(S):
            gen.manual_seed((int(seed) * 15485863 + 7 * b + 1000003 * (s + 1)) & 0x7FFFFFFFFFFFFFFF)
            acc[s] += np.sqrt(max(0.0, 1.0 - tot_src)) * torch.randn(nb, generator=gen, device=device,
                                                                      dtype=torch.float64)
        acc *= sigma_t
        if tone_bin is not None:
            n = n0 + torch.arange(nb, device=device, dtype=torch.float64)
            for s in range(S):
                tau = float(geom.D[s] + geom.f[s])
                ph = 2 * np.pi * (tone_bin / tone_N) * (n - tau) \
                    - 2 * np.pi * sideband * (float(geom.psi0[s]) + float(geom.rate[s]) * t)
                acc[s] += tone_amp * torch.cos(ph)
        out[:, n0:n0 + nb] = acc.round_().clamp_(-127, 127).to(torch.int8)
        del acc
    return out


def random_spectra_int8(S: int, T: int, C: int, seed: int = BASE_SEED, sigma: float = 32.0,
                        extremes: bool = True) -> np.ndarray:
    """Requantised-spectrum-like int8 [S][T][C][2] in [-127, 127] for X-engine tests.

    Gaussian of the given sigma, clipped; with ``extremes`` a few entries are
    forced to +-127 so that the largest products are exercised."""
    g = rng(seed, 6, S, T, C)
    q = np.clip(np.rint(g.standard_normal((S, T, C, 2), dtype=np.float32) * sigma), -127, 127)
    q = q.astype(np.int8)
    if extremes and q.size:
        idx = g.integers(0, q.size, size=max(1, q.size // 1000))
        q.reshape(-1)[idx] = np.where(g.random(idx.size) < 0.5, -127, 127).astype(np.int8)
    return q


def random_spectra_f32(S: int, T: int, C: int, seed: int = BASE_SEED, sigma: float = 100.0):
    """complex64 [S][T][C] Gaussian spectra for FP32 X-engine tests."""
    g = rng(seed, 7, S, T, C)
    re = g.standard_normal((S, T, C), dtype=np.float32) * sigma
    im = g.standard_normal((S, T, C), dtype=np.float32) * sigma
    return (re + 1j * im).astype(np.complex64)


def random_spectra_int16(S: int, T: int, C: int, seed: int = BASE_SEED, sigma: float = 8000.0,
                         extremes: bool = True) -> np.ndarray:
    """int16 [S][T][C][2] in [-32767, 32767] (Gaussian of the given sigma,
    clipped) for tests of the 16-bit X-engine; with ``extremes`` a few entries
    are forced to +-32767 so that the largest products are exercised."""
    g = rng(seed, 8, S, T, C)
    q = np.clip(np.rint(g.standard_normal((S, T, C, 2), dtype=np.float32) * sigma), -32767, 32767)
    q = q.astype(np.int16)
    if extremes and q.size:
        idx = g.integers(0, q.size, size=max(1, q.size // 1000))
        q.reshape(-1)[idx] = np.where(g.random(idx.size) < 0.5, -32767, 32767).astype(np.int16)
    return q


def point_sources(S: int, n_src: int, power: float, seed: int = BASE_SEED, n_pol: int = 2):
    """n_src sources sharing total power; source 0 at the phase centre, the others
    with per-antenna extra delay U[-2, 2] samples and rate U[-0.5, 0.5] Hz."""
    g = rng(seed, 8)
    n_ant = S // n_pol
    out = []
    for k in range(n_src):
        if k == 0:
            dD = np.zeros(S)
            dr = np.zeros(S)
        else:
            dD = np.repeat(g.uniform(-2, 2, n_ant), n_pol)
            dr = np.repeat(g.uniform(-0.5, 0.5, n_ant), n_pol)
        out.append({"power": power / n_src, "dD": dD, "drate": dr})
    return out


def power_spectra(S: int, T: int, C: int, seed: int = BASE_SEED, *, tone_frac: float = 0.05,
                  tone_k=(2.0, 40.0), burst_p: float = 0.01, burst_k=(2.0, 20.0), burst_len=(1, 8),
                  bandpass: bool = True) -> np.ndarray:
    """float32 power [S][T][C] shaped like channelised noise with interference,
    for flagger tests that do not need a voltage run: each cell is exponential
    (the power of a complex Gaussian) with mean mu_k = a smooth bandpass,
    persistent tones add k mu_k to a fraction of the channels (same channels
    for every signal, k ~ U[tone_k]), and broadband bursts multiply whole
    spectra by 1 + k (start probability burst_p per spectrum and signal, length
    U{burst_len}, k ~ U[burst_k])."""
    out = np.empty((S, T, C), dtype=np.float32)
    k = np.arange(C)
    mu = 1000.0 * (0.6 + 0.4 * np.sin(np.pi * (k + 0.5) / C)) if bandpass else np.full(C, 1000.0)
    g = rng(seed, 20)
    n_tone = int(round(tone_frac * C))
    tch = g.choice(C, size=n_tone, replace=False) if n_tone else np.zeros(0, dtype=np.int64)
    tk = g.uniform(*tone_k, n_tone)
    for s in range(S):
        gs = rng(seed, 21, s)
        mean = np.broadcast_to(mu, (T, C)).copy()
        mean[:, tch] += tk * mu[tch]
        starts = np.nonzero(gs.random(T) < burst_p)[0]
        for m0 in starts:
            ln = int(gs.integers(burst_len[0], burst_len[1] + 1))
            mean[m0:m0 + ln] *= 1.0 + gs.uniform(*burst_k)
        out[s] = (gs.exponential(1.0, (T, C)) * mean).astype(np.float32)
    return out


# ---------------------------------------------------------------------------
# Impulsive voltage interference (the broadband, power-line spark RFI that the
# time-domain blanker of section 5 targets)
# ---------------------------------------------------------------------------
def impulse_bursts(n_samples: int, seed: int = BASE_SEED, *, duty: float = 0.025, burst_len=(16, 512),
                   k=(4.0, 40.0)):
    """Bursts common to every antenna: (start sample, length, variance factor)
    arrays.  Starts are uniform over the stream (count Poisson with mean
    duty * n / mean length, so about a fraction ``duty`` of the samples lie in
    a burst), each moved past the end of the previous burst so that no two
    overlap; lengths U{burst_len}, variance factors k ~ U[k] in units of
    sigma_t^2."""
    g = rng(seed, 30, n_samples)
    mean_len = 0.5 * (burst_len[0] + burst_len[1])
    nb = int(g.poisson(duty * n_samples / mean_len))
    starts = np.sort(g.integers(0, max(1, n_samples), nb))
    lens = g.integers(burst_len[0], burst_len[1] + 1, nb)
    ks = g.uniform(k[0], k[1], nb)
    before = np.concatenate([[0], np.cumsum(lens)[:-1]])      # samples in earlier bursts
    starts = np.maximum.accumulate(starts - before) + before  # start_i >= end_{i-1}
    return starts, lens, ks


def add_impulses(x, geom: Geom, n_samples: int, *, sigma_t: float = 12.0, seed: int = BASE_SEED,
                 duty: float = 0.025, burst_len=(16, 512), k=(4.0, 40.0), n_pol: int = 2):
    """Add impulsive RFI to int8 streams x [S][>= n_samples] in place (numpy
    array or torch tensor, on any device): each burst is one Gaussian waveform
    per polarisation (std sqrt(k) sigma_t), received by every antenna with its
    integer delay D (sample n of the waveform lands on sample n + D), so it
    correlates between antennas like a terrestrial source; then
    x = clip(x + rint(w), -127, 127).  Returns the boolean mask (numpy
    [S][n_samples]) of the samples a burst touched only for numpy input, else
    None."""
    starts, lens, ks = impulse_bursts(n_samples, seed, duty=duty, burst_len=burst_len, k=k)
    total = int(lens.sum())
    if total == 0:
        return np.zeros(x.shape[0:1] + (n_samples,), bool) if isinstance(x, np.ndarray) else None
    pos = np.repeat(starts - np.cumsum(np.concatenate([[0], lens[:-1]])), lens) + np.arange(total)
    amp = np.repeat(np.sqrt(ks) * sigma_t, lens).astype(np.float32)
    S = x.shape[0]
    if isinstance(x, np.ndarray):
        mask = np.zeros((S, n_samples), bool)
        for pol in range(n_pol):
            w = np.rint(rng(seed, 31, pol).standard_normal(total, dtype=np.float32) * amp)
            for s in range(pol, S, n_pol):
                p = pos + int(geom.D[s])
                keep = p < n_samples
                v = x[s, p[keep]].astype(np.float32) + w[keep]
                x[s, p[keep]] = np.clip(v, -127, 127).astype(np.int8)
                mask[s, p[keep]] = True
        return mask
    import torch
    dev = x.device
    pos_d = torch.from_numpy(pos).to(dev)
    amp_d = torch.from_numpy(amp).to(dev)
    gen = torch.Generator(device=dev)
    for pol in range(n_pol):
        gen.manual_seed((int(seed) * 1000003 + 31 * pol + 5) & 0x7FFFFFFFFFFFFFFF)
        w = torch.randn(total, generator=gen, device=dev, dtype=torch.float32).mul_(amp_d).round_()
        for s in range(pol, S, n_pol):
            p = pos_d + int(geom.D[s])
            keep = p < n_samples
            pk = p[keep]
            v = x[s, pk].float().add_(w[keep])
            x[s, pk] = v.clamp_(-127, 127).to(torch.int8)
        del w
    return None
