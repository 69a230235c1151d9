"""Host-side checks of the Python binding's buffer validation (the C-ABI
takes raw pointers and cannot see sizes, so the binding checks device,
dtype, layout and the bytes behind each pointer before a call)."""
import pytest
import torch

import paper_0910_1517_amd as corr


class FakeDev:
    """A CPU tensor presented as a device tensor: only the attributes the
    check reads."""

    def __init__(self, t):
        self.t = t
        self.is_cuda = True
        self.dtype = t.dtype
        self.shape = t.shape

    def __getattr__(self, k):
        return getattr(self.t, k)


def test_need_accepts_exact_and_larger_buffers():
    corr._need(FakeDev(torch.zeros(16, dtype=torch.float32)), "a", 64, torch.float32)
    corr._need(FakeDev(torch.zeros(17, dtype=torch.float32)), "a", 64)
    corr._need(None, "a", 64, optional=True)


def test_need_rejects_small_wrong_or_host_buffers():
    with pytest.raises(ValueError, match="holds 60 bytes, needs 64"):
        corr._need(FakeDev(torch.zeros(15, dtype=torch.float32)), "a", 64)
    with pytest.raises(TypeError):
        corr._need(FakeDev(torch.zeros(16, dtype=torch.float64)), "a", 64, torch.float32)
    with pytest.raises(ValueError, match="device tensor"):
        corr._need(torch.zeros(16), "a", 64)
    with pytest.raises(ValueError, match="required"):
        corr._need(None, "a", 64)
    with pytest.raises(ValueError, match="contiguous"):
        corr._need(FakeDev(torch.zeros(8, 8).t()), "a", 64)


def test_need_counts_bytes_from_the_view_not_the_storage_start():
    base = torch.zeros(64, dtype=torch.uint8)
    corr._need(FakeDev(base[16:]), "a", 48)
    with pytest.raises(ValueError, match="holds 48 bytes"):
        corr._need(FakeDev(base[16:]), "a", 49)


def test_rows_layout_and_extent():
    x = torch.zeros(4, 64, dtype=torch.int8)
    corr._need(FakeDev(x[:, :40]), "x", corr._rows_bytes(4, 64, 40), torch.int8, rows=True)
    corr._need(FakeDev(x.view(-1)), "x", corr._rows_bytes(4, 64, 64), rows=True)  # flat buffer
    with pytest.raises(ValueError, match="unit stride"):
        corr._need(FakeDev(x.t()), "x", 1, rows=True)
    # the last row's bytes are counted up to whole 16-byte chunks
    assert corr._rows_bytes(3, 64, 33) == 2 * 64 + 48
    assert corr._rows_bytes(0, 64, 33) == 0
    with pytest.raises(ValueError, match="needs"):
        corr._need(FakeDev(torch.zeros(2 * 64 + 40, dtype=torch.int8)), "x", corr._rows_bytes(3, 64, 33), rows=True)


def test_a_short_view_of_a_larger_buffer_is_rejected():
    a = torch.zeros(64, dtype=torch.float32)
    with pytest.raises(ValueError, match="holds 252 bytes, needs 256"):
        corr._need(FakeDev(a[:-1]), "acc", 256)
    # rows: the last row may be read up to its 16-byte chunk, if the storage has it
    x = torch.zeros(2, 64, dtype=torch.int8)
    corr._need(FakeDev(x[:, :33]), "x", 64 + 48, rows=True)
    with pytest.raises(ValueError, match="holds 33 bytes"):  # no storage past the row
        corr._need(FakeDev(torch.zeros(1, 33, dtype=torch.int8)), "x", 48, rows=True)
