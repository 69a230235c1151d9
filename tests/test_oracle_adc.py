"""Pins of the oracle's ADC input unpacking (sections 2.3.2 and 3.3: four
inputs per acquisition card, 8-bit or 4-bit samples, demultiplexed and
unpacked to 8 bits) against hand-written cases, every byte value, and round
trips through a packer written here."""
import numpy as np
import pytest

import oracle

# two's complement value of each 4-bit code 0..15, written out
NIBBLE = [0, 1, 2, 3, 4, 5, 6, 7, -8, -7, -6, -5, -4, -3, -2, -1]


def pack(x, bits):
    """int8 rows [4 cards][n] -> raw card streams (the inverse, written here)."""
    rows, n = x.shape
    cards = rows // 4
    v = x.reshape(cards, 4, n).transpose(0, 2, 1)  # [card][t][input]
    if bits == 8:
        return np.ascontiguousarray(v.astype(np.int8).view(np.uint8).reshape(cards, 4 * n))
    u = (v.astype(np.int16) & 0xF).astype(np.uint8)  # 4-bit codes
    return np.ascontiguousarray((u[..., 0::2] | (u[..., 1::2] << 4)).reshape(cards, 2 * n))


def test_hand_cases():
    assert oracle.adc_unpack(np.array([[0x01, 0x02, 0xFF, 0x80]], np.uint8), 1, 8).ravel().tolist() == [1, 2, -1, -128]
    # low nibble first: 0x8F -> inputs 0, 1 = -1, -8; 0x71 -> inputs 2, 3 = 1, 7
    assert oracle.adc_unpack(np.array([[0x8F, 0x71]], np.uint8), 1, 4).ravel().tolist() == [-1, -8, 1, 7]
    # two time samples, two cards: rows are card-major, input-minor
    raw = np.array([[0x10, 0x32, 0x54, 0x76], [0xF8, 0x9A, 0xBC, 0xDE]], np.uint8)
    x = oracle.adc_unpack(raw, 2, 4)
    assert x.tolist() == [[0, 4], [1, 5], [2, 6], [3, 7], [-8, -4], [-1, -5], [-6, -2], [-7, -3]]


def test_every_byte_value():
    b = np.arange(256, dtype=np.uint8)
    raw8 = np.repeat(b, 4)[None]  # time t = byte value, all four inputs equal
    x8 = oracle.adc_unpack(raw8, 256, 8)
    assert np.array_equal(x8, np.tile(b.view(np.int8), (4, 1)))
    raw4 = np.repeat(b, 2)[None]  # both bytes of time t = t
    x4 = oracle.adc_unpack(raw4, 256, 4)
    lo = [NIBBLE[v & 0xF] for v in range(256)]
    hi = [NIBBLE[v >> 4] for v in range(256)]
    assert x4.tolist() == [lo, hi, lo, hi]


@pytest.mark.parametrize("bits", [8, 4])
def test_round_trip_and_card_padding(bits):
    rng = np.random.default_rng(bits)
    lo_v, hi_v = (-128, 127) if bits == 8 else (-8, 7)
    x = rng.integers(lo_v, hi_v + 1, size=(12, 1001)).astype(np.int8)
    raw = pack(x, bits)
    assert np.array_equal(oracle.adc_unpack(raw, x.shape[1], bits), x)
    padded = np.concatenate([raw, np.full((raw.shape[0], 48), 0xA5, np.uint8)], axis=1)  # bytes past the stream
    assert np.array_equal(oracle.adc_unpack(padded, x.shape[1], bits), x)
    assert np.array_equal(oracle.adc_unpack(raw, 17, bits), x[:, :17])
