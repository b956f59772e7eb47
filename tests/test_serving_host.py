"""Host-side checks of the serving runtime's pure functions (no GPU): the
shape a request maps to, the device-size query that admission relies on, and
descriptor validation."""
import ctypes

import pytest

from paper_1201_2501_amd import sfft
from oracle.window import default_w


def test_server_desc_defaults():
    d = sfft.sfft_server_desc_init()
    assert d.budget_bytes == 16 << 30 and d.slots == 32 and d.instances == 2
    assert d.delta_exact == 1e-9 and d.delta_general == 1e-6 and d.theta == 0.25


@pytest.mark.parametrize("n,k,mode,B,dense", [
    (1 << 22, 256, sfft.SFFT_MODE_EXACT, 1024, False),
    (1 << 22, 200, sfft.SFFT_MODE_EXACT, 1024, False),     # k rounded up to 256
    (1 << 20, 64, sfft.SFFT_MODE_GENERAL, 1024, False),
    (1 << 24, 1024, sfft.SFFT_MODE_EXACT, 4096, False),
    (1 << 16, 1024, sfft.SFFT_MODE_EXACT, 4096, True),     # window longer than the signal
    (1 << 16, 8, sfft.SFFT_MODE_EXACT, 64, False),
    (1 << 16, 200, sfft.SFFT_MODE_GENERAL, 4096, True),
])
def test_server_shape_policy(n, k, mode, B, dense):
    sd = sfft.sfft_server_desc_init()
    d, is_dense, nbytes = sfft.sfft_server_shape(sd, n, k, mode)
    kb = 1 << max(3, (k - 1).bit_length())
    assert d.k == kb and d.cap == kb and d.B == B and d.mode == mode and d.max_batch == sd.slots
    delta = sd.delta_exact if mode == sfft.SFFT_MODE_EXACT else sd.delta_general
    w = default_w(n, B, 0.5, delta)
    assert is_dense == dense == (w >= n)
    if not dense:
        assert d.w == w
        # one instance = the plan's workspace + the server's staging buffers
        staging = sd.slots * (8 + 8 + kb * 8 + kb * 16 + 4 + 16)
        assert nbytes == sfft.sfft_plan_device_bytes(d) + staging
    else:
        assert nbytes >= sd.slots * n * 8


def test_plan_device_bytes_scales_with_batch_and_rejects_bad_descs():
    d = sfft.sfft_desc_init(1 << 20, 64, 512)
    d.max_batch = 1
    one = sfft.sfft_plan_device_bytes(d)
    d.max_batch = 3
    three = sfft.sfft_plan_device_bytes(d)
    d.max_batch = 5
    five = sfft.sfft_plan_device_bytes(d)
    assert one > 0 and three > one and five - three == three - one   # linear in the batch
    bad = sfft.sfft_desc_init(1 << 20, 64, 500)                      # B not a power of two
    assert sfft.sfft_plan_device_bytes(bad) == 0


@pytest.mark.parametrize("field,value", [("slots", 0), ("instances", 0), ("budget_bytes", 0), ("theta", 0.0),
                                         ("delta_exact", 1.5), ("delta_general", 0.0), ("instances", 17)])
def test_server_create_rejects_bad_descs(field, value):
    lib = sfft.load()
    d = sfft.sfft_server_desc_init()
    setattr(d, field, value)
    h = ctypes.c_void_p()
    assert lib.sfft_server_create(ctypes.byref(d), ctypes.byref(h)) == sfft.SFFT_EINVAL
    assert not h.value


@pytest.mark.parametrize("n,k,mode,status", [(3 << 20, 64, 0, sfft.SFFT_ENOTPOW2), (1 << 20, 0, 0, sfft.SFFT_EINVAL),
                                             (1 << 20, 2048, 0, sfft.SFFT_EINVAL), (1 << 20, 64, 5, sfft.SFFT_EINVAL),
                                             (1 << 8, 8, 0, sfft.SFFT_ENOTPOW2)])
def test_server_shape_rejects_bad_requests(n, k, mode, status):
    lib = sfft.load()
    sd = sfft.sfft_server_desc_init()
    d = sfft.PlanDesc()
    dense = ctypes.c_int32(0)
    assert lib.sfft_server_shape(ctypes.byref(sd), n, k, mode, ctypes.byref(d), ctypes.byref(dense), None) == status


def test_server_calls_reject_null_server():
    lib = sfft.load()
    res = sfft.RequestResult()
    st = sfft.ServerStats()
    assert lib.sfft_server_poll(None, 1, ctypes.byref(res)) == sfft.SFFT_EINVAL
    assert lib.sfft_server_wait(None, 1, 0.0, ctypes.byref(res)) == sfft.SFFT_EINVAL
    assert lib.sfft_server_stats(None, ctypes.byref(st)) == sfft.SFFT_EINVAL
    assert lib.sfft_server_destroy(None) == sfft.SFFT_OK
