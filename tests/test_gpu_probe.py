"""The read probe (the library's bandwidth measurement aid, pecann_read_probe):
every thread runs every pass over ragged sizes and repeated, rotated passes,
folds what it read into one word and writes nothing but its sink, and only
when that word equals the key.  On a zero buffer the fold of a thread is
fixed by the pass count alone, so the key that sets the sink is known."""
import ctypes

import pytest
import torch

from paper_2312_03940_amd import pecann

pytestmark = pytest.mark.gpu


def _zero_fold(passes):
    acc = 0
    for r in range(passes):
        acc = (acc * 2654435761 + r) & 0xFFFFFFFF
    return acc


@pytest.mark.parametrize("nbytes,passes", [(16, 1), (1 << 20, 3), ((1 << 20) + 16 * 37, 2),
                                           (64 << 20, 4), (4096 + 16, 9)])
def test_read_probe_zero_buffer_sets_sink_only_on_its_fold(nbytes, passes):
    lib = pecann.load()
    print(f"read probe: {nbytes} bytes x {passes} passes", flush=True)
    buf = torch.zeros(nbytes // 4 + 16, dtype=torch.float32, device="cuda")  # guard words past nbytes
    sink = torch.zeros(4, dtype=torch.int32, device="cuda")
    want = _zero_fold(passes)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for key, hit in ((want, 1), ((want + 1) & 0xFFFFFFFF, 0)):
        sink.zero_()
        st = lib.pecann_read_probe(ctypes.c_void_p(buf.data_ptr()), nbytes, passes, key,
                                   ctypes.c_void_p(sink.data_ptr()), stream)
        assert st == 0, pecann.load().pecann_last_error()
        torch.cuda.synchronize()
        assert sink.tolist() == [hit, 0, 0, 0]
    assert torch.count_nonzero(buf).item() == 0


def test_read_probe_rejects_bad_sizes():
    lib = pecann.load()
    buf = torch.zeros(64, dtype=torch.float32, device="cuda")
    sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for nbytes, passes in ((0, 1), (24, 1), (256, 0)):
        st = lib.pecann_read_probe(ctypes.c_void_p(buf.data_ptr()), nbytes, passes, 0,
                                   ctypes.c_void_p(sink.data_ptr()), stream)
        assert st == 1  # PECANN_EINVAL
