"""Host-side tests of the streaming server's scheduling: the server source is
built against host-only stand-ins of the HIP runtime and kernels
(tests/native/mock_runtime.cpp), whose "launches" complete a set delay after
they are recorded.  Covers FIFO admission under overload (no deadlock with a
client that consumes results in order), batching of consecutive equal
shapes, the memory budget, and refusal of impossible requests."""
import ctypes as C
import os
import subprocess
import threading
import time

import numpy as np
import pytest

import synth
from paper_2602_03529_amd import _lib as L

HERE = os.path.dirname(os.path.abspath(__file__))
NATIVE = os.path.join(HERE, "native")
LIB = os.path.join(NATIVE, "libtok_serve_mock.so")


@pytest.fixture(scope="module")
def lib():
    r = subprocess.run(["bash", os.path.join(NATIVE, "build_mock_server.sh")], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    lb = C.CDLL(LIB)
    vp, sz, i32 = C.c_void_p, C.c_size_t, C.c_int
    lb.tok_server_create.argtypes = [vp, sz, i32, i32, C.POINTER(vp)]
    lb.tok_server_submit.argtypes = [vp, C.POINTER(L.Request), C.POINTER(C.c_uint64)]
    lb.tok_server_wait.argtypes = [vp, C.c_uint64, i32, C.POINTER(L.Result)]
    lb.tok_server_release.argtypes = [vp, C.c_uint64]
    lb.tok_server_stats.argtypes = [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32), C.POINTER(sz),
                                    C.POINTER(sz)]
    lb.tok_server_destroy.argtypes = [vp]
    lb.mock_set_delay_us.argtypes = [C.c_longlong]
    lb.mock_fail_next_encodes.argtypes = [C.c_int]
    return lb


class Server:
    def __init__(self, lib, budget, slots, max_batch, delay_us):
        self.lib = lib
        lib.mock_set_delay_us(delay_us)
        self.h = C.c_void_p()
        assert lib.tok_server_create(C.c_void_p(1), budget, slots, max_batch, C.byref(self.h)) == 0
        self.keep = {}

    def submit(self, i, T, H, W):
        a = np.zeros((T, H, W, 3), np.uint8)
        a[0, 0, 0, 0] = i % 251
        req = L.Request(T, H, W, a.ctypes.data, L.DropDesc(1, 0.1, 3, i, 0, None))
        t = C.c_uint64()
        rc = self.lib.tok_server_submit(self.h, C.byref(req), C.byref(t))
        if rc == 0:
            self.keep[t.value] = a
        return rc, t.value

    def wait(self, t, timeout_ms=20000):
        r = L.Result()
        rc = self.lib.tok_server_wait(self.h, t, timeout_ms, C.byref(r))
        return rc, r

    def stats(self):
        q, r, f = C.c_int(), C.c_int(), C.c_int()
        u, p = C.c_size_t(), C.c_size_t()
        self.lib.tok_server_stats(self.h, C.byref(q), C.byref(r), C.byref(f), C.byref(u), C.byref(p))
        return dict(queued=q.value, running=r.value, finished=f.value, in_use=u.value, peak=p.value)

    def close(self):
        self.lib.tok_server_destroy(self.h)


def test_overload_with_in_order_client_never_stalls(lib):
    """Poisson arrivals of mixed resolutions faster than the stand-in kernels
    finish; the client waits for and releases results in submission order."""
    budget = 8 << 30
    sv = Server(lib, budget, slots=4, max_batch=4, delay_us=100000)
    reqs = synth.make_requests(48, 400.0, 17, seed=3)
    tickets = [None] * len(reqs)

    def submitter():
        t0 = time.perf_counter()
        for i, r in enumerate(reqs):
            d = r.arrival_s - (time.perf_counter() - t0)
            if d > 0:
                time.sleep(d)
            rc, t = sv.submit(i, r.T, r.H, r.W)
            assert rc == 0
            tickets[i] = t

    th = threading.Thread(target=submitter)
    th.start()
    for i in range(len(reqs)):
        while tickets[i] is None:
            time.sleep(0.0005)
        rc, r = sv.wait(tickets[i])
        assert rc == 0, ("stalled", i, sv.stats())
        assert r.status == 0
        assert C.cast(r.codes, C.POINTER(C.c_float))[0] == float(i % 251)
        assert C.cast(r.idx, C.POINTER(C.c_int32))[0] == i % 251
        lib.tok_server_release(sv.h, tickets[i])
    th.join()
    st = sv.stats()
    assert st["peak"] <= budget and st["in_use"] == 0 and st["finished"] == len(reqs)
    sv.close()


def test_batches_are_runs_of_consecutive_equal_shapes(lib):
    sv = Server(lib, 1 << 30, slots=1, max_batch=4, delay_us=150000)
    A, B = (5, 32, 32), (5, 48, 32)
    shapes = [A, A, A, B, A, A]
    ts, t_sub = [], []
    for i, s in enumerate(shapes):
        t_sub.append(time.perf_counter())
        ts.append(sv.submit(i, *s)[1])
        if i == 0:  # let clip 0 start alone before the others queue up behind it
            while sv.stats()["running"] == 0:
                time.sleep(0.001)
    sizes, done = [], []
    for i, t in enumerate(ts):
        rc, r = sv.wait(t)
        assert rc == 0 and r.status == 0
        sizes.append(r.batch_size)
        done.append(t_sub[i] + r.total_ms / 1e3)
    # clip 0 runs alone (admitted at once), then 1+2, then 3 (shape B), then 4+5
    assert sizes == [1, 2, 2, 1, 2, 2], sizes
    assert all(b >= a - 0.005 for a, b in zip(done, done[1:]))  # FIFO completion with one slot
    for t in ts:
        lib.tok_server_release(sv.h, t)
    sv.close()


def test_impossible_request_refused_and_others_served(lib):
    sv = Server(lib, 256 << 20, slots=2, max_batch=2, delay_us=1000)
    rc, _ = sv.submit(0, 17, 1080, 1920)
    assert rc == -5  # TOK_EBUDGET
    rc, _ = sv.submit(1, 4, 32, 32)
    assert rc == -2  # TOK_ESHAPE (T % 4 != 1)
    rc, t = sv.submit(2, 5, 32, 32)
    assert rc == 0
    rc, r = sv.wait(t)
    assert rc == 0 and r.status == 0
    lib.tok_server_release(sv.h, t)
    sv.close()


def test_budget_bounds_concurrency(lib):
    """Room for one clip: all clips still finish, one at a time, under budget."""
    one = 0
    sv = Server(lib, 1 << 30, slots=4, max_batch=1, delay_us=20000)
    ts = [sv.submit(i, 9, 128, 128)[1] for i in range(3)]
    for t in ts:
        rc, r = sv.wait(t)
        assert rc == 0 and r.status == 0
        lib.tok_server_release(sv.h, t)
        one = max(one, sv.stats()["peak"])
    assert one <= 1 << 30
    sv.close()


def test_failed_launch_leaves_no_view_of_its_block(lib):
    """A batch whose launch fails returns its result block to the arena; the
    failed request must not keep a view of it: the next batch reuses the same
    block, and neither waiting on nor releasing the failed request may shift
    the next clip's views or free its block."""
    sv = Server(lib, 1 << 30, slots=1, max_batch=1, delay_us=20000)
    lib.mock_fail_next_encodes(1)
    rc, ta = sv.submit(7, 5, 32, 32)
    assert rc == 0
    rc, ra = sv.wait(ta)
    assert rc == 0 and ra.status == -4  # TOK_EDEVICE
    rc, tb = sv.submit(9, 5, 32, 32)
    assert rc == 0
    rc, rb = sv.wait(tb)
    assert rc == 0 and rb.status == 0 and rb.batch_size == 1
    assert C.cast(rb.codes, C.POINTER(C.c_float))[0] == 9.0
    assert lib.tok_server_release(sv.h, ta) == 0
    in_use = sv.stats()["in_use"]
    assert in_use > 0  # the second clip's block is still held
    rc, rb2 = sv.wait(tb)
    assert rc == 0 and rb2.codes == rb.codes
    assert C.cast(rb2.codes, C.POINTER(C.c_float))[0] == 9.0
    assert lib.tok_server_release(sv.h, tb) == 0
    assert sv.stats()["in_use"] == 0
    sv.close()
