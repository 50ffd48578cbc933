"""lb_copy_probe, the STREAM-like copy that bench.py times as the practical
memory ceiling: it copies exactly, on sizes that fill whole per-block
chunks (2 GiB: 8192 chunks of 256 KiB) and ragged ones, and refuses
misaligned, overlapping or null buffers on the host before any launch."""
import ctypes as C

import pytest

from paper_1109_6672_amd import lbddf

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n_floats", [4, 4 * 1000 + 4, 4 * 1025, 4 * 2048 * 256 * 4 * 3 + 36, 1 << 24, 1 << 29])
def test_copy_probe_copies_exactly(gpu, n_floats):
    import torch

    print(f"[case] copy probe, {n_floats * 4} bytes", flush=True)
    g = torch.Generator(device="cuda").manual_seed(n_floats)
    x = torch.rand(n_floats, device="cuda", generator=g)
    y = torch.full_like(x, -1.0)
    lbddf.copy_probe(x, y)
    torch.cuda.synchronize()
    assert torch.equal(x, y)


def test_copy_probe_refuses_bad_buffers(gpu):
    import torch

    lib = lbddf.load()
    x = torch.zeros(1024, device="cuda")
    y = torch.zeros(1024, device="cuda")
    p, q = x.data_ptr(), y.data_ptr()
    assert lib.lb_copy_probe(C.c_void_p(p + 4), C.c_void_p(q), 64, None) == lbddf.LB_EINVAL  # misaligned
    assert lib.lb_copy_probe(C.c_void_p(p), C.c_void_p(q), 60, None) == lbddf.LB_EINVAL  # not 16-byte units
    assert lib.lb_copy_probe(C.c_void_p(p), C.c_void_p(p + 1024), 2048, None) == lbddf.LB_EINVAL  # overlap
    assert lib.lb_copy_probe(None, C.c_void_p(q), 64, None) == lbddf.LB_EINVAL
    assert lib.lb_copy_probe(C.c_void_p(p), C.c_void_p(q), 0, None) == lbddf.LB_OK
    torch.cuda.synchronize()
