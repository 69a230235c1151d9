"""ADC demultiplexing and 4-bit unpacking (sections 2.3.2 and 3.3) through
the C ABI against the oracle: bit-exact on random bytes (every value),
ragged lengths, card counts, and padded strides whose padding must not be
written."""
import numpy as np
import pytest

import oracle
import paper_0910_1517_amd as corr

pytestmark = pytest.mark.gpu

CASES = [  # (bits, cards, n, raw padding, row padding)
    (4, 1, 16, 0, 0),
    (4, 3, 4096 * 3 + 16 * 5 + 7, 32, 48),
    (4, 16, 4096, 0, 16),
    (8, 1, 16, 0, 0),
    (8, 3, 4096 * 3 + 16 * 5 + 7, 16, 32),
    (8, 16, 8192 + 3, 0, 0),
    (4, 2, 1, 0, 16),
    (8, 2, 15, 0, 0),
    (4, 5, 17, 16, 0),
]


@pytest.mark.parametrize("case", CASES, ids=["b%d-c%d-n%d" % c[:3] for c in CASES])
def test_unpack_matches_oracle(case):
    import torch
    bits, cards, n, rpad, xpad = case
    print("adc", case, flush=True)
    rng = np.random.default_rng(n + cards + bits)
    rbytes = n * 4 * bits // 8
    rrs = (rbytes + 15) // 16 * 16 + rpad
    raw = rng.integers(0, 256, size=(cards, rrs), dtype=np.uint8)
    rs = (n + 15) // 16 * 16 + xpad
    x = torch.full((4 * cards, rs), 0x5A, dtype=torch.int8, device="cuda")
    corr.adc_unpack(torch.from_numpy(raw).cuda(), x, bits=bits, n=n)
    torch.cuda.synchronize()
    got = x.cpu().numpy()
    ref = oracle.adc_unpack(raw[:, :rbytes], n, bits)
    assert np.array_equal(got[:, :n], ref)
    assert np.all(got[:, n:] == 0x5A), "row padding written"
