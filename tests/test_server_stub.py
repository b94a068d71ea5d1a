"""The served form's queue and admission on a stub executor (CPU, no GPU).

``ssa_server_create_stub`` runs the real queue, slot and pool bookkeeping of the
continuous-batching server with the kernel launches replaced by a counter: an admitted
request reports its stopping test passed after ``ticks`` ticks and then completes like a
real one (finalized one tick, reported the next).  Requests above the batched engine's
n_max go to the long path (``ssa_server_enable_long``), which sizes each by its
single-series plan.  Checked here: the pool is never overcommitted and returns to full;
a request the pool cannot hold blocks everything behind it (no overtaking); a class
without a free slot lets the other class pass; a request larger than the pool is refused
at submission; overload queues up and drains; every id completes exactly once.
"""
import ctypes

import pytest

from paper_0911_4498_amd import ssa

FAKE = 0x1000  # never dereferenced by the stub executor


@pytest.fixture(scope="module")
def lib():
    return ssa.load()


class Stub:
    def __init__(self, lib, slots, pool_bytes, ticks=3, long_slots=0, n_max=20480, n_long_max=1 << 20):
        self.lib = lib
        h = ctypes.c_void_p()
        opts = ssa.SsaOpts()
        assert lib.ssa_server_create_stub(n_max, 32, slots, ctypes.byref(opts), pool_bytes, ticks,
                                          ctypes.byref(h)) == 0
        self.h = h
        if long_slots:
            assert lib.ssa_server_enable_long(h, n_long_max, long_slots) == 0
        self.cap = slots + long_slots
        self.done = []

    def bytes(self, N, L, k):
        b = ctypes.c_size_t(0)
        assert self.lib.ssa_server_request_bytes(self.h, N, L, k, ctypes.byref(b)) == 0
        return b.value

    def submit(self, rid, N, L, k):
        return self.lib.ssa_server_submit(self.h, rid, rid, FAKE, N, L, k, FAKE, FAKE, FAKE, None, None)

    def step(self):
        buf = (ctypes.c_longlong * self.cap)()
        n = ctypes.c_int(0)
        assert self.lib.ssa_server_step(self.h, buf, self.cap, ctypes.byref(n)) == 0
        got = [buf[i] for i in range(n.value)]
        self.done += got
        return got

    def status(self):
        q, a, f = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_int(0)
        free = ctypes.c_size_t(0)
        assert self.lib.ssa_server_status(self.h, ctypes.byref(q), ctypes.byref(a), ctypes.byref(f),
                                          ctypes.byref(free)) == 0
        return q.value, a.value, f.value, free.value

    def close(self):
        self.lib.ssa_server_destroy(self.h)


def test_long_requests_wait_for_the_pool_and_block_later_ones(lib):
    probe = Stub(lib, 4, 1 << 40, long_slots=4)
    bl = probe.bytes(200000, 50000, 20)   # long: sized by its single-series plan
    bs = probe.bytes(4000, 2000, 16)      # short: a batched-engine region
    probe.close()
    assert bl > 10 * bs
    pool = int(2.5 * bl) + (1 << 16)
    srv = Stub(lib, 4, pool, ticks=3, long_slots=4)
    _, _, _, free0 = srv.status()
    for rid in range(3):
        assert srv.submit(rid, 200000, 50000, 20) == 0        # two fit, the third waits
    assert srv.submit(10, 4000, 2000, 16) == 0                # behind a request waiting for memory
    srv.step()
    q, a, f, free = srv.status()
    assert (q, a) == (2, 2), (q, a)                            # no overtaking
    assert free >= 0 and free0 - free >= 2 * bl
    ticks = 0
    while len(srv.done) < 4:
        srv.step()
        ticks += 1
        assert ticks < 100
        q, a, f, free = srv.status()
        assert free <= free0
    assert srv.done[:2] == [0, 1] and sorted(srv.done) == [0, 1, 2, 10]
    assert srv.status() == (0, 0, 0, free0)
    srv.close()


def test_full_class_lets_the_other_class_pass(lib):
    srv = Stub(lib, 2, 1 << 40, ticks=4, long_slots=1)
    assert srv.submit(0, 100000, 50000, 20) == 0   # takes the only long slot
    assert srv.submit(1, 100000, 50000, 20) == 0   # waits for a long slot
    assert srv.submit(2, 5000, 2500, 8) == 0       # a short request passes it
    srv.step()
    q, a, f, _ = srv.status()
    assert (q, a) == (1, 2)
    for _ in range(100):
        srv.step()
        if len(srv.done) == 3:
            break
    assert sorted(srv.done) == [0, 1, 2] and srv.done[-1] == 1
    srv.close()


def test_refusals(lib):
    srv = Stub(lib, 2, 1 << 20, long_slots=1)
    assert srv.submit(0, 300000, 100000, 20) == ssa.SSA_ENOMEM   # can never fit the pool
    assert srv.submit(1, 4000, 2000, 40) == ssa.SSA_EINVAL       # k above k_max
    assert srv.submit(2, (1 << 20) + 1, 1000, 8) == ssa.SSA_EINVAL  # above n_long_max
    srv.close()
    short_only = Stub(lib, 2, 1 << 30)
    assert short_only.submit(0, 100000, 50000, 20) == ssa.SSA_EINVAL  # long path not enabled
    short_only.close()


def test_overload_drains_with_bounded_occupancy(lib):
    srv = Stub(lib, 3, 1 << 36, ticks=2, long_slots=2)
    ids = list(range(40))
    for rid in ids:
        N = 3000 + 97 * rid if rid % 3 else 40000 + 1000 * rid
        assert srv.submit(rid, N, N // 2, 8) == 0
    _, _, _, free0 = srv.status()
    for _ in range(400):
        srv.step()
        q, a, f, free = srv.status()
        assert a + f <= 5
        if len(srv.done) == len(ids):
            break
    assert sorted(srv.done) == ids and len(set(srv.done)) == len(ids)
    assert srv.status() == (0, 0, 0, free0)
    srv.close()
