"""The measurement hook behind the roofline context: the streaming-read probe
reads every element of its buffer once per pass."""
import ctypes

import pytest
import torch

pytestmark = pytest.mark.gpu


def test_stream_read_reads_everything():
    assert torch.cuda.is_available()
    from paper_2203_14354_amd import _lib
    lib = _lib.load()
    n_vec, passes, blocks = 1_000_003, 3, 64
    x = torch.ones(n_vec * 4, dtype=torch.float32, device="cuda")
    out = torch.zeros(blocks * 256, dtype=torch.float32, device="cuda")
    _lib.check(lib.xp_stream_read(ctypes.c_void_p(x.data_ptr()), n_vec, passes, blocks,
                                  ctypes.c_void_p(out.data_ptr()), None))
    torch.cuda.synchronize()
    # each thread sums 4 ones per vector it reads; every vector is read once per pass
    assert float(out.double().sum()) == 4.0 * n_vec * passes
