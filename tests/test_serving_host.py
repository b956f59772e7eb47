"""Host-side checks of the serving runtime's pure functions (no GPU): the
shape a request maps to, the device-size query that admission relies on, and
descriptor validation."""
import ctypes
import time

import pytest

from paper_1201_2501_amd import sfft
from oracle.window import default_w


def test_server_desc_defaults():
    d = sfft.sfft_server_desc_init()
    assert d.budget_bytes == 16 << 30 and d.slots == 32 and d.instances == 2
    assert d.delta_exact == 1e-9 and d.delta_general == 1e-6 and d.theta == 0.25


def path_model_dense(n, mode, samples, streamed):
    """The server's path model: predicted solo milliseconds of each path."""
    if mode == sfft.SFFT_MODE_EXACT:
        sparse = sfft.SFFT_SERVER_EXACT_MS + 1e-6 * (sfft.SFFT_SERVER_GATHER_NS * (samples - streamed) +
                                                    sfft.SFFT_SERVER_STREAM_NS * streamed)
    else:
        sparse = sfft.SFFT_SERVER_GENERAL_MS + 1e-6 * sfft.SFFT_SERVER_GENERAL_NS * samples
    return sparse > sfft.SFFT_SERVER_DENSE_MS + 1e-6 * sfft.SFFT_SERVER_DENSE_NS * n


@pytest.mark.parametrize("n,k,mode,B,dense", [
    (1 << 22, 8, sfft.SFFT_MODE_EXACT, 64, False),         # measured solo: sparse 0.14 ms, dense 0.20
    (1 << 24, 256, sfft.SFFT_MODE_EXACT, 1024, False),     # sparse 0.38, dense 0.54
    (1 << 24, 1024, sfft.SFFT_MODE_EXACT, 4096, True),     # sparse 1.03, dense 0.56
    (1 << 22, 256, sfft.SFFT_MODE_EXACT, 1024, True),      # sparse 0.31, dense 0.22
    (1 << 22, 8, sfft.SFFT_MODE_GENERAL, 256, True),       # sparse 0.84, dense 0.22
    (1 << 20, 1024, sfft.SFFT_MODE_EXACT, 4096, True),
    (1 << 16, 1024, sfft.SFFT_MODE_EXACT, 4096, True),     # window longer than the signal
    (1 << 16, 8, sfft.SFFT_MODE_EXACT, 64, True),          # sparse 0.15, dense 0.13
    (1 << 16, 200, sfft.SFFT_MODE_GENERAL, 4096, True),
])
def test_server_shape_policy(n, k, mode, B, dense):
    sd = sfft.sfft_server_desc_init()
    d, is_dense, nbytes = sfft.sfft_server_shape(sd, n, k, mode)
    kb = 1 << max(3, (k - 1).bit_length())
    assert d.k == kb and d.cap == kb and d.B == B and d.mode == mode and d.max_batch == sd.slots
    delta = sd.delta_exact if mode == sfft.SFFT_MODE_EXACT else sd.delta_general
    w = default_w(n, B, 0.5, delta, kind=1)      # served shapes use the Kaiser-Bessel window
    assert d.window == 1
    assert is_dense == dense
    if w < n:
        # the path model decides, from the sparse plan's gathered and
        # streamed samples
        sparse = sfft.PlanDesc.from_buffer_copy(d)
        sparse.w = w
        samples = sfft.sfft_plan_samples(sparse)
        streamed = sfft.sfft_plan_stream_rounds(sparse) * n
        assert sparse.hash_mode == (1 if mode == sfft.SFFT_MODE_EXACT else 0)
        assert samples > 0 and dense == path_model_dense(n, mode, samples, streamed)
    if not dense:
        assert d.w == w
        # one instance = the plan's workspace + the server's staging buffers
        staging = sd.slots * (8 + 8 + kb * 8 + kb * 16 + 4 + 16)
        assert nbytes == sfft.sfft_plan_device_bytes(d) + staging
    else:
        assert d.w == n and nbytes >= sd.slots * n * 8


def test_server_flags_force_a_path():
    n, k = 1 << 20, 64
    sd = sfft.sfft_server_desc_init()
    sd.flags = sfft.SFFT_SERVER_SPARSE_ONLY
    assert not sfft.sfft_server_shape(sd, n, k, sfft.SFFT_MODE_GENERAL)[1]
    sd.flags = 0
    assert sfft.sfft_server_shape(sd, n, k, sfft.SFFT_MODE_GENERAL)[1]
    assert sfft.sfft_server_shape(sd, 1 << 16, 1024, sfft.SFFT_MODE_EXACT)[1]    # w >= n: dense anyway
    sd.flags = sfft.SFFT_SERVER_DENSE_ONLY
    assert sfft.sfft_server_shape(sd, 1 << 24, 8, sfft.SFFT_MODE_EXACT)[1]


def level_count(n, B_r, t=16):
    """LocateInner levels: region widths n/B_r, shrinking by t/4, while above 1."""
    W, lev = n // B_r, 0
    while W > 1:
        lev += 1
        W = W * 4 / t
    return lev


def test_plan_samples_closed_forms():
    # exact: the pair of each round of group 0 (rounds up to the first at b_min
    # bins, plus patience + 1), w_r + 1 samples each
    d = sfft.sfft_desc_init(1 << 20, 64, 256, 24576)
    d.b_min, d.patience, d.rounds = 32, 5, 24
    Bs = [max(256 >> r, 32) for r in range(24)]
    first_floor = next(r for r in range(23) if Bs[r + 1] == Bs[r])
    expect = sum(24576 // 256 * Bs[r] + 1 for r in range(first_floor + 5 + 1))
    assert sfft.sfft_plan_samples(d) == expect == 61449
    # general: every round's LocateInner pairs and EstimateValues hashings
    n, B, w = 1 << 18, 256, 15872
    g = sfft.sfft_desc_init(n, 8, B, w)
    g.mode = sfft.SFFT_MODE_GENERAL
    g.rounds = 7
    expect = 0
    for r in range(7):
        k_r = max(1, 8 >> (2 * r))
        B_r = min(B, max(B >> r, 1 << (4 * k_r - 1).bit_length()))
        expect += (2 * level_count(n, B_r) * g.R_loc + g.R_est) * (w // B * B_r)
    assert sfft.sfft_plan_samples(g) == expect == 1285880
    bad = sfft.sfft_desc_init(1 << 20, 64, 500)
    assert sfft.sfft_plan_samples(bad) == 0


def test_general_b_min_floors_the_round_schedule():
    """General mode with b_min = B keeps B and w in every round (the fixed
    schedule the practical one is measured against); the host's gathered
    samples follow the oracle's round schedule either way."""
    from oracle.general import round_schedule
    from oracle.params import SfftParams
    n, k, B, w = 1 << 20, 64, 1024, 64512
    for b_min in (0, 256, B):
        g = sfft.sfft_desc_init(n, k, B, w)
        g.mode, g.rounds, g.b_min = sfft.SFFT_MODE_GENERAL, 7, b_min
        p = SfftParams(n=n, k=k, B=B, w=w, seed=0, rounds=7, b_min=b_min)
        expect = 0
        for r in range(7):
            k_r, B_r, w_r = round_schedule(p, r)
            assert B_r == min(B, max(B >> r, 1 << (4 * k_r - 1).bit_length(), b_min)) and w_r == w // B * B_r
            expect += (2 * level_count(n, B_r) * g.R_loc + g.R_est) * w_r
        assert sfft.sfft_plan_samples(g) == expect
        if b_min == B:
            assert expect == 7 * (2 * level_count(n, B) * g.R_loc + g.R_est) * w


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
                                         ("delta_exact", 1.5), ("delta_general", 0.0), ("instances", 17),
                                         ("flags", 0x6), ("flags", 0x10)])
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


# ---- the scheduler on the fake device (no GPU: batches finish on a host timer)
FAKE_X = 0x1000          # a request's signal pointer is never read on the fake device


class FakeServer:
    def __init__(self, **fields):
        self.lib = sfft.load()
        d = sfft.sfft_server_desc_init()
        d.flags = sfft.SFFT_SERVER_FAKE_DEVICE
        for k, v in fields.items():
            setattr(d, k, v)
        self.desc = d
        self.h = ctypes.c_void_p()
        assert self.lib.sfft_server_create(ctypes.byref(d), ctypes.byref(self.h)) == sfft.SFFT_OK

    def submit(self, n, k, mode=sfft.SFFT_MODE_EXACT, seed=0):
        req = sfft.Request(x_dev=FAKE_X, n=n, seed=seed, k=k, mode=mode, idx_host=None, val_host=None)
        t = ctypes.c_uint64(0)
        st = self.lib.sfft_server_submit(self.h, ctypes.byref(req), ctypes.byref(t))
        return st, t.value

    def wait(self, ticket):
        res = sfft.RequestResult()
        st = self.lib.sfft_server_wait(self.h, ticket, 10000.0, ctypes.byref(res))
        return st, res

    def stats(self):
        st = sfft.ServerStats()
        assert self.lib.sfft_server_stats(self.h, ctypes.byref(st)) == sfft.SFFT_OK
        return st

    def close(self):
        assert self.lib.sfft_server_destroy(self.h) == sfft.SFFT_OK


def test_fake_server_rejects_a_shape_larger_than_the_budget():
    srv = FakeServer(budget_bytes=1 << 20)
    try:
        st, _ = srv.submit(1 << 22, 256)
        assert st == sfft.SFFT_EBUDGET
        st, _ = srv.submit(1000, 16)
        assert st == sfft.SFFT_ENOTPOW2
        assert srv.stats().completed == 0
    finally:
        srv.close()


def test_fake_server_budget_eviction_and_peak():
    sd = sfft.sfft_server_desc_init()
    sd.slots = 4
    shapes = [(1 << 22, 8), (1 << 23, 64), (1 << 24, 8)]     # sparse-path shapes under the path model
    assert not any(sfft.sfft_server_shape(sd, n, k, 0)[1] for n, k in shapes)
    sizes = [sfft.sfft_server_shape(sd, n, k, 0)[2] for n, k in shapes]
    budget = max(sizes) + min(sizes) // 2
    srv = FakeServer(slots=4, instances=1, budget_bytes=budget, fake_service_ms=2.0)
    try:
        tickets = []
        for rep in range(4):
            for n, k in shapes:
                st, t = srv.submit(n, k, seed=rep)
                assert st == sfft.SFFT_OK
                tickets.append(t)
        for t in tickets:
            st, res = srv.wait(t)
            assert st == sfft.SFFT_OK and res.count == 0 and res.latency_ms >= res.service_ms >= 1.5
        s = srv.stats()
        assert s.completed == len(tickets) and s.failed == 0
        assert s.peak_bytes <= budget and s.evictions >= 2 and s.bytes_in_use <= budget
    finally:
        srv.close()


def test_fake_server_batches_requests_that_wait():
    srv = FakeServer(slots=8, instances=1, fake_service_ms=30.0)
    try:
        tickets = [srv.submit(1 << 20, 64, seed=s)[1] for s in range(9)]
        outs = [srv.wait(t) for t in tickets]
        assert all(st == sfft.SFFT_OK for st, _ in outs)
        s = srv.stats()
        # the first request runs alone; the 8 that arrived meanwhile share one batch
        assert s.batches == 2 and abs(s.mean_batch - 4.5) < 1e-9
        assert outs[-1][1].queue_ms >= 20.0
        assert s.p50_ms <= s.p99_ms
    finally:
        srv.close()


def test_fake_server_cancels_requests_that_have_not_launched():
    srv = FakeServer(slots=1, instances=1, fake_service_ms=40.0)
    lib = srv.lib
    try:
        tickets = [srv.submit(1 << 20, 64, seed=s)[1] for s in range(4)]
        assert lib.sfft_server_cancel(srv.h, tickets[3]) == sfft.SFFT_OK
        assert lib.sfft_server_cancel(srv.h, tickets[2]) == sfft.SFFT_OK
        assert lib.sfft_server_cancel(srv.h, 10 ** 6) == sfft.SFFT_EINVAL
        time.sleep(0.01)                    # the first request is running (40 ms of service)
        assert lib.sfft_server_cancel(srv.h, tickets[0]) == sfft.SFFT_EAGAIN
        assert srv.wait(tickets[0])[0] == sfft.SFFT_OK
        # the second is launched when the first finishes: either withdrawn or served
        st1 = lib.sfft_server_cancel(srv.h, tickets[1])
        assert st1 in (sfft.SFFT_OK, sfft.SFFT_EAGAIN)
        assert srv.wait(tickets[1])[0] == (sfft.SFFT_ECANCELED if st1 == sfft.SFFT_OK else sfft.SFFT_OK)
        assert srv.wait(tickets[2])[0] == sfft.SFFT_ECANCELED
        assert srv.wait(tickets[3])[0] == sfft.SFFT_ECANCELED
        s = srv.stats()
        assert s.completed == (1 if st1 == sfft.SFFT_OK else 2) and s.failed == 0
    finally:
        srv.close()


def test_fake_server_keeps_dense_instances_resident():
    """Dense-path instances are not evicted: two sparse shapes that fit beside
    the dense one only one at a time are evicted around it, every request is
    served and the dense shape is built once."""
    sd = sfft.sfft_server_desc_init()
    sd.slots = 2
    dense = (1 << 16, 600, 0)
    sparse = [(1 << 22, 8, 0), (1 << 23, 64, 0)]
    assert sfft.sfft_server_shape(sd, *dense)[1] and not any(sfft.sfft_server_shape(sd, *s)[1] for s in sparse)
    dbytes = sfft.sfft_server_shape(sd, *dense)[2]
    sizes = [sfft.sfft_server_shape(sd, *s)[2] for s in sparse]
    budget = dbytes + max(sizes) + min(sizes) // 2
    srv = FakeServer(slots=2, instances=1, budget_bytes=budget, fake_service_ms=1.0)
    try:
        for rep in range(5):
            tickets = [srv.submit(*sh, seed=rep)[1] for sh in [dense] + sparse]
            for t in tickets:
                st, res = srv.wait(t)
                assert st == sfft.SFFT_OK, res.message
        s = srv.stats()
        assert s.completed == 15 and s.failed == 0 and s.peak_bytes <= budget
        assert s.evictions >= 4                  # the sparse shapes take turns
        assert s.instances == 2                  # the dense instance and one sparse
    finally:
        srv.close()


def test_fake_server_fails_a_shape_that_cannot_fit_beside_dense_instances():
    """A shape whose instance does not fit beside the resident dense-path
    instances fails with SFFT_EBUDGET and a message that says why; with
    SFFT_SERVER_EVICT_DENSE the dense instance is evicted instead."""
    sd = sfft.sfft_server_desc_init()
    sd.slots = 2
    dense = (1 << 16, 600, 0)
    sparse = (1 << 22, 64, 0)
    dbytes = sfft.sfft_server_shape(sd, *dense)[2]
    sbytes = sfft.sfft_server_shape(sd, *sparse)[2]
    budget = max(dbytes, sbytes) + min(dbytes, sbytes) // 2
    for flags, expect in ((0, sfft.SFFT_EBUDGET), (sfft.SFFT_SERVER_EVICT_DENSE, sfft.SFFT_OK)):
        srv = FakeServer(slots=2, instances=1, budget_bytes=budget, fake_service_ms=1.0,
                         flags=sfft.SFFT_SERVER_FAKE_DEVICE | flags)
        try:
            st, res = srv.wait(srv.submit(*dense)[1])
            assert st == sfft.SFFT_OK and res.message == b""
            st, res = srv.wait(srv.submit(*sparse)[1])
            assert st == expect
            if expect == sfft.SFFT_EBUDGET:
                assert b"dense-path instances" in res.message
                assert srv.stats().failed == 1
            else:
                assert srv.stats().evictions == 1
        finally:
            srv.close()


def test_fake_server_many_shapes_tight_budget_with_cancels():
    """Instances are built on threads of their own and idle ones (dense-path
    ones too, with SFFT_SERVER_EVICT_DENSE) are evicted under a budget barely
    above the largest instance: every request of a stream over 24 shapes
    (with cancels) ends served or canceled, none fails, and the budget
    holds."""
    import random
    rng = random.Random(7)
    shapes = [(1 << e, k, m) for e in (16, 18, 20, 22) for k in (8, 100, 600) for m in (0, 1)]
    sd = sfft.sfft_server_desc_init()
    sd.slots = 4
    sizes = [sfft.sfft_server_shape(sd, *s)[2] for s in shapes]
    for budget_factor, instances, service in ((1.05, 1, 0.5), (1.5, 2, 0.0), (3.0, 3, 2.0)):
        budget = int(max(sizes) * budget_factor)
        srv = FakeServer(slots=4, instances=instances, budget_bytes=budget, fake_service_ms=service,
                         flags=sfft.SFFT_SERVER_FAKE_DEVICE | sfft.SFFT_SERVER_EVICT_DENSE)
        try:
            tickets, canceled = [], 0
            for i in range(300):
                n, k, m = rng.choice(shapes)
                st, t = srv.submit(n, k, m, seed=i)
                assert st == sfft.SFFT_OK
                tickets.append(t)
                if rng.random() < 0.05 and srv.lib.sfft_server_cancel(srv.h, t) == sfft.SFFT_OK:
                    canceled += 1
            done = 0
            for t in tickets:
                res = sfft.RequestResult()
                st = srv.lib.sfft_server_wait(srv.h, t, 20000.0, ctypes.byref(res))
                assert st in (sfft.SFFT_OK, sfft.SFFT_ECANCELED)
                done += st == sfft.SFFT_OK
            s = srv.stats()
            assert done + canceled == len(tickets) and s.completed == done and s.failed == 0
            assert s.peak_bytes <= budget and s.bytes_in_use <= budget
        finally:
            srv.close()
