"""Pins of the gated-correlator oracle (section 5: visibilities accumulated
per pulse-phase gate) and of the pulse-phase gates, against the ungated X
oracle, worked gate patterns and a pulsed common signal; and the library's
host gate function against the oracle (host code, no GPU)."""
import math

import numpy as np
import pytest

import oracle
import paper_0910_1517_amd as corr


def test_bins_sum_to_the_ungated_visibilities():
    rng = np.random.default_rng(1)
    S, T, C = 6, 40, 5
    q = rng.integers(-127, 128, size=(S, T, C, 2)).astype(np.int8)
    gate = rng.integers(0, 4, size=T).astype(np.uint8)  # value 3 is outside n_bins = 3
    A = oracle.xengine_int_gated(q, gate, 3)
    assert np.array_equal(A.sum(0), oracle.xengine_int(q[:, gate < 3]))
    assert np.array_equal(oracle.xengine_int_gated(q, np.zeros(T, np.uint8), 1)[0], oracle.xengine_int(q))
    Y = rng.normal(size=(S, T, C)) + 1j * rng.normal(size=(S, T, C))
    V = oracle.xengine_gated(Y, gate, 3)
    assert np.allclose(V.sum(0), oracle.xengine(Y[:, gate < 3]), rtol=1e-13, atol=1e-12)
    assert np.all(oracle.xengine_gated(Y, np.full(T, 7, np.uint8), 2) == 0)  # nothing gated in


def test_worked_gate_patterns():
    N, fs = 1024, 1.024e6  # one spectrum per millisecond
    # period of exactly 10 spectra, 10 bins: spectrum m sits at phase (m + 1/2) / 10
    g = oracle.pulsar_gates(0, 35, N, fs, 0.0, 10e-3, 10)
    assert g.tolist() == [m % 10 for m in range(35)]
    # t0 one spectrum later shifts the pattern; spectrum0 continues it
    assert oracle.pulsar_gates(0, 20, N, fs, 1e-3, 10e-3, 10).tolist() == [(m - 1) % 10 for m in range(20)]
    assert oracle.pulsar_gates(7, 20, N, fs, 0.0, 10e-3, 10).tolist() == [(m + 7) % 10 for m in range(20)]
    # on / off: two bins over a 4-spectrum period
    assert oracle.pulsar_gates(0, 8, N, fs, 0.0, 4e-3, 2).tolist() == [0, 0, 1, 1, 0, 0, 1, 1]
    assert set(oracle.pulsar_gates(0, 100, N, fs, 0.3, 7.7e-3, 1).tolist()) == {0}


def test_gates_are_equidistributed_for_an_incommensurate_period():
    n, nb = 20000, 8
    g = oracle.pulsar_gates(0, n, 4096, 66.666666e6, 0.0, 1.5578e-3, nb)  # 25.35 spectra per period
    counts = np.bincount(g, minlength=nb)
    assert counts.sum() == n and np.all(np.abs(counts - n / nb) < 0.02 * n / nb)


def test_pulsed_common_signal_appears_in_its_gate_only():
    """A signal common to all antennas, present only in the spectra of bin 0
    (the pulse), gives cross visibilities of mean A^2 per spectrum in bin 0
    and zero mean in bin 1."""
    rng = np.random.default_rng(3)
    S, T, C, A = 4, 4000, 3, 2.0
    gate = oracle.pulsar_gates(0, T, 1024, 1.024e6, 0.0, 4e-3, 2)
    pulse = (gate == 0)[None, :, None]
    c = rng.normal(size=(1, T, C)) + 1j * rng.normal(size=(1, T, C))
    Y = rng.normal(size=(S, T, C)) + 1j * rng.normal(size=(S, T, C)) + A * c * pulse
    V = oracle.xengine_gated(Y, gate, 2)
    n0, n1 = int((gate == 0).sum()), int((gate == 1).sum())
    p01 = oracle.pair_index(0, 1)
    on = V[0, :, p01].real / n0 / (2 * A * A)      # E|A c|^2 = 2 A^2
    off = V[1, :, p01].real / n1 / (2 * A * A)
    assert np.all(np.abs(on - 1) < 0.15) and np.all(np.abs(off) < 0.1)


@pytest.mark.parametrize("args", [(0, 1000, 4096, 66.666666e6, 0.0, 1.5578e-3, 16),
                                  (123456789, 5000, 1024, 33.333333e6, -0.25, 0.0897, 2),
                                  (5, 300, 512, 1.0e7, 12.5, 3.3e-5, 255)])
def test_library_gates_match_the_oracle(args):
    g, counts = corr.pulsar_gates(*args)
    ref = oracle.pulsar_gates(*args)
    assert np.array_equal(g, ref)
    assert np.array_equal(counts, np.bincount(ref, minlength=args[-1]))
