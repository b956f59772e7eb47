"""GPU check of the entry point that allocates nothing: sfft_dense_topk_noalloc
against sfft_dense_topk (caller-provided scratch) on the same spectra, on two
calls in a row (the second with fewer, shorter spectra, so that stale
contents of the shared static scratch would show), bit-exact; and the count
limit rejected before anything is launched.  Calls go through the C ABI."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_1201_2501_amd import sfft
    lib = sfft.load()
    lib.sfft_dense_topk_noalloc.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                            ctypes.c_double, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_void_p]
    lib.sfft_dense_topk_noalloc.restype = ctypes.c_int32
    lib.sfft_dense_topk_noalloc_max_count.restype = ctypes.c_uint32
    return torch, torch.device("cuda:0"), sfft, lib


def spectra(torch, dev, count, n, seed, ties):
    g = torch.Generator(device="cpu").manual_seed(seed)
    s = torch.complex(torch.randn(count, n, generator=g), torch.randn(count, n, generator=g)).to(torch.complex64)
    if ties:   # repeated magnitudes across chunk boundaries: ties go to the smaller index
        s[:, 1::7] = s[:, 0:1]
    return s.to(dev).contiguous()


def run_both(torch, dev, sfft, lib, spec, cap, scale, keep):
    count, n = spec.shape
    ref_idx, ref_val, ref_cnt = sfft.dense_topk(spec, cap, scale, keep)
    idx = torch.full((count, cap), -1, dtype=torch.int64, device=dev)
    val = torch.full((count, cap), float("nan"), dtype=torch.complex128, device=dev)
    cnt = torch.full((count,), -1, dtype=torch.int32, device=dev)
    st = lib.sfft_dense_topk_noalloc(spec.data_ptr(), n, count, cap, scale, keep, idx.data_ptr(), val.data_ptr(),
                                     cnt.data_ptr(), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == sfft.SFFT_OK, sfft.sfft_last_error()
    torch.cuda.synchronize()
    assert torch.equal(cnt, ref_cnt)
    assert torch.equal(idx, ref_idx)
    assert torch.equal(torch.view_as_real(val), torch.view_as_real(ref_val))
    return cnt


def test_noalloc_topk_matches_scratch_version_twice(env):
    torch, dev, sfft, lib = env
    big = spectra(torch, dev, 48, 1 << 16, 1, ties=True)
    small = spectra(torch, dev, 5, 1 << 12, 2, ties=False)
    say("noalloc top-k 48 x 2^16 then 5 x 2^12")
    c1 = run_both(torch, dev, sfft, lib, big, 300, 1.0 / 256.0, -1.0)
    assert int(c1.min()) == 300
    c2 = run_both(torch, dev, sfft, lib, small, 40, 1.0 / 64.0, 0.02)
    assert int(c2.max()) <= 40


def test_noalloc_topk_rejects_counts_above_its_scratch(env):
    torch, dev, sfft, lib = env
    m = int(lib.sfft_dense_topk_noalloc_max_count())
    assert m == 64
    spec = torch.zeros((m + 1, 1 << 10), dtype=torch.complex64, device=dev)
    idx = torch.zeros((m + 1, 8), dtype=torch.int64, device=dev)
    val = torch.zeros((m + 1, 8), dtype=torch.complex128, device=dev)
    cnt = torch.full((m + 1,), 7, dtype=torch.int32, device=dev)
    say("noalloc top-k count limit")
    st = lib.sfft_dense_topk_noalloc(spec.data_ptr(), 1 << 10, m + 1, 8, 1.0, -1.0, idx.data_ptr(), val.data_ptr(),
                                     cnt.data_ptr(), None)
    assert st == sfft.SFFT_EINVAL and "static scratch" in sfft.sfft_last_error()
    torch.cuda.synchronize()
    assert int(cnt.min()) == 7 and int(cnt.max()) == 7     # nothing was launched
