"""Measurement probes (fhv_probe): the copy moves the first half of the
buffer onto the second; every atomic probe leaves each line holding the
value its passes define (one uncontended atomic per line and pass) and
touches nothing else."""
from __future__ import annotations

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_15460_amd import fhv
    fhv.lib()
    return fhv


@pytest.mark.parametrize("cached", [False, True])
def test_probe_copy(F, cached):
    import torch
    g = torch.Generator().manual_seed(5)
    n = (3 << 20) + 96            # bytes, a multiple of 32 that is not a power of two
    host = torch.randint(0, 256, (n,), dtype=torch.uint8, generator=g)
    buf = host.cuda()
    F.probe(F.FHV_PROBE_COPY_CACHED if cached else F.FHV_PROBE_COPY, buf)
    torch.cuda.synchronize()
    out = buf.cpu().numpy()
    h = host.numpy()
    assert np.array_equal(out[: n // 2], h[: n // 2])
    assert np.array_equal(out[n // 2:], h[: n // 2])


@pytest.mark.parametrize("cached", [False, True])
def test_probe_read_and_write(F, cached):
    """The read probe leaves a 0xFF buffer as it was; the write probe sets
    every byte to 0xFF and nothing beyond (both access forms)."""
    import torch
    n = (5 << 20) + 48            # bytes, a multiple of 16 that is not a power of two
    buf = torch.full((n + 64,), 0x11, dtype=torch.uint8, device="cuda")
    F.probe(F.FHV_PROBE_WRITE_CACHED if cached else F.FHV_PROBE_WRITE, buf[:n])
    torch.cuda.synchronize()
    out = buf.cpu().numpy()
    assert np.all(out[:n] == 0xFF) and np.all(out[n:] == 0x11)
    F.probe(F.FHV_PROBE_READ_CACHED if cached else F.FHV_PROBE_READ, buf[:n])
    torch.cuda.synchronize()
    assert np.array_equal(buf.cpu().numpy(), out)


@pytest.mark.parametrize("line,n_lines,passes", [(128, 1000, 3), (8, 5000, 2), (4096, 17, 5),
                                                 (128, 600_000, 2)])
def test_probe_atomics(F, line, n_lines, passes):
    import torch
    nbytes = line * n_lines + line // 2        # a partial last line is not touched
    print(f"probe line={line} lines={n_lines} passes={passes}", flush=True)
    for kind in (F.FHV_PROBE_ADD_U32, F.FHV_PROBE_EXCH_U32, F.FHV_PROBE_MIN_U64):
        buf = torch.full((nbytes,), 0x5A, dtype=torch.uint8, device="cuda")
        if kind == F.FHV_PROBE_MIN_U64:
            buf.fill_(0xFF)
        before = buf.cpu().numpy().copy()
        F.probe(kind, buf, line, passes)
        torch.cuda.synchronize()
        out = buf.cpu().numpy()
        lines = out[: line * n_lines].reshape(n_lines, line)
        w = lines[:, :8].copy().view(np.uint32).reshape(n_lines, 2)
        if kind == F.FHV_PROBE_ADD_U32:
            assert np.all(w[:, 0] == np.uint32(0x5A5A5A5A + passes))
            assert np.all(lines[:, 4:] == 0x5A)
        elif kind == F.FHV_PROBE_EXCH_U32:
            assert np.all(w[:, 0] == passes)
            # each thread adds what its exchanges returned: the start value,
            # then 1 .. passes-1, over every line it handles
            per_line = np.uint64(0x5A5A5A5A) + np.uint64(passes * (passes - 1) // 2)
            got = w[:, 1].astype(np.uint64)
            # the grid has at least one thread per line for these sizes
            assert np.all(got == per_line % np.uint64(1 << 32))
            assert np.all(lines[:, 8:] == 0x5A)
        else:
            v = lines[:, :8].copy().view(np.uint64).ravel()
            want = (np.uint64(1) << np.uint64(32)) | np.arange(n_lines, dtype=np.uint64)
            assert np.array_equal(v, want)
            assert np.all(lines[:, 8:] == 0xFF)
        assert np.array_equal(out[line * n_lines:], before[line * n_lines:])


def test_probe_rejects_bad_arguments(F):
    import ctypes as C
    import torch
    buf = torch.zeros(4096, dtype=torch.uint8, device="cuda")
    L = F.lib()
    p = C.c_void_p(buf.data_ptr())
    for kind, nbytes, line, passes in ((9, 4096, 128, 1), (8, 40, 0, 0), (1, 4096, 96, 1), (1, 4096, 4, 1),
                                       (1, 4096, 8192, 1), (1, 64, 128, 1), (1, 4096, 128, 0),
                                       (1, 4096, 128, 1025), (0, 48, 0, 0), (0, 16, 0, 0)):
        assert L.fhv_probe(F.ctx(), kind, p, nbytes, line, passes, None) == -1
    assert L.fhv_probe(F.ctx(), 1, C.c_void_p(buf.data_ptr() + 4), 4000, 128, 1, None) == -1
