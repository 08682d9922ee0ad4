"""ft_upload: a gather list of pinned-host segments lands byte-exact in device
memory with one call, whatever the sizes (empty, sub-vector tails, chunk
boundaries, more segments than one launch takes); invalid lists are rejected
before anything is enqueued."""
import ctypes as ct
import sys

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_2509_10757_amd import binding as ft
    return ft.Context(ft.default_limits(max_batch_frames=4, max_map_points=1024, max_inflight=1))


def _host(ctx, nbytes):
    addr = ctx.ft_host_alloc(nbytes)
    return addr, np.ctypeslib.as_array((ct.c_uint8 * nbytes).from_address(addr))


def test_gather_copy_is_byte_exact(ctx):
    rng = np.random.default_rng(7)
    sizes = [0, 1, 15, 16, 17, 4096, 32767, 32768, 32769, 100_000] + list(rng.integers(0, 70_000, 70))
    offs, o = [], 0
    for n in sizes:
        offs.append(o)
        o += (int(n) + 15) // 16 * 16 + 16
    addr, h = _host(ctx, o)
    h[:] = rng.integers(0, 256, o, dtype=np.uint8)
    dev = torch.full((o,), 0xA5, dtype=torch.uint8, device="cuda")
    segs = [(addr + a, dev.data_ptr() + a, int(n)) for a, n in zip(offs, sizes)]
    say("segments", len(segs), "bytes", sum(sizes))
    ctx.ft_upload(segs)
    torch.cuda.synchronize()
    got = dev.cpu().numpy()
    for a, n in zip(offs, sizes):
        n = int(n)
        assert np.array_equal(got[a:a + n], h[a:a + n])
        assert np.all(got[a + n:(a + n + 15) // 16 * 16] == 0xA5)   # nothing past the segment
    ctx.ft_host_free(addr)


def test_invalid_lists_are_rejected(ctx):
    from paper_2509_10757_amd import binding as ft
    addr, h = _host(ctx, 4096)
    dev = torch.zeros(4096, dtype=torch.uint8, device="cuda")
    d = dev.data_ptr()
    bad = [[(addr + 16, d, 4096)],            # runs past the block
           [(addr + 8, d, 16)],               # misaligned source
           [(addr, d + 4, 16)],               # misaligned destination
           [(addr, d, -1)],                   # negative size
           [(addr, d, 16), (d, d + 64, 16)]]  # a source outside every host block
    for segs in bad:
        assert ctx.ft_upload(segs, check=False) == ft.FT_ERR_INVALID_ARGUMENT
    torch.cuda.synchronize()
    assert int(dev.sum()) == 0                 # nothing was enqueued
    ctx.ft_upload([])                          # empty list: no-op
    ctx.ft_host_free(addr)
    with pytest.raises(ft.FtError):
        ctx.ft_host_free(addr)                 # double free
