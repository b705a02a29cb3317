"""The continuous-batching scheduler on the CPU (simulate mode: no device
work; a request finishes after a scripted number of epochs): admission by
device-memory budget in strict arrival order, runs joining and leaving at
epoch boundaries, arena accounting, and completion bookkeeping."""
import os

import numpy as np
import pytest

from paper_2108_10209_amd import n2f, synth

pytestmark = pytest.mark.skipif(not os.path.exists(n2f.LIB_PATH), reason="libn2f.so not built")


def _drive(srv, reqs, arena, max_steps=100000):
    """Submit everything, step until all finished; check invariants each step."""
    for r in reqs:
        srv.submit(r["id"], H=r["H"], W=r["W"], C=r["C"], sim_epochs=r["epochs"])
    done, step = [], 0
    admitted_order = []
    while len(done) < len(reqs):
        active, queued = srv.step(1)
        used, largest = srv.memory()
        assert used <= arena and largest <= arena - used
        done += srv.poll()
        step += 1
        assert step < max_steps
    return done, step


def test_all_requests_finish_and_arena_is_returned():
    arena = 3 * n2f.workspace_bytes(512, 512, 1)
    srv = n2f.Server(arena, simulate=True, max_active=64)
    rng = np.random.default_rng(0)
    reqs = [dict(id=i, H=int(rng.integers(32, 600)), W=int(rng.integers(32, 600)), C=int(rng.choice([1, 3])),
                 epochs=int(rng.integers(1, 40))) for i in range(60)]
    done, steps = _drive(srv, reqs, arena)
    assert sorted(i for i, _ in done) == list(range(60))
    assert all(st == n2f.OK for _, st in done)
    used, largest = srv.memory()
    assert used == 0 and largest == arena


def test_strict_arrival_order_admission():
    """A large request at the head of the queue is not overtaken by small
    ones that would fit: admission follows arrival order."""
    big = n2f.workspace_bytes(1024, 1024, 1)
    small = n2f.workspace_bytes(64, 64, 1)
    arena = big + small // 2      # the big request fits only when the arena is otherwise empty
    srv = n2f.Server(arena, simulate=True, max_active=64)
    srv.submit(0, H=64, W=64, C=1, sim_epochs=10)          # occupies part of the arena for 10 epochs
    srv.submit(1, H=1024, W=1024, C=1, sim_epochs=1)       # does not fit until 0 leaves
    for i in range(2, 6):
        srv.submit(i, H=64, W=64, C=1, sim_epochs=1)
    order = []
    for _ in range(30):
        srv.step(1)
        order += [i for i, _ in srv.poll()]
        if len(order) == 6:
            break
    assert order.index(0) < order.index(1) < min(order.index(i) for i in range(2, 6))


def test_max_active_and_join_leave_at_epoch_boundaries():
    arena = 100 * n2f.workspace_bytes(64, 64, 1)
    srv = n2f.Server(arena, simulate=True, max_active=3)
    for i in range(7):
        srv.submit(i, H=64, W=64, C=1, sim_epochs=2 + i)
    seen = []
    t = 0
    finish_step = {}
    while len(finish_step) < 7:
        active, queued = srv.step(1)
        t += 1
        assert active <= 3
        for i, _ in srv.poll():
            finish_step[i] = t
    # first three start at step 1 and finish after their own epoch counts
    assert finish_step[0] == 2 and finish_step[1] == 3 and finish_step[2] == 4
    # request 3 joins when request 0 leaves (after step 2) and runs 5 epochs
    assert finish_step[3] == 2 + 5


def test_request_that_never_fits_is_rejected():
    arena = n2f.workspace_bytes(64, 64, 1)
    srv = n2f.Server(arena, simulate=True)
    with pytest.raises(n2f.N2FError) as e:
        srv.submit(1, H=512, W=512, C=1, sim_epochs=1)
    assert e.value.code == n2f.ENOMEM
    with pytest.raises(n2f.N2FError) as e:
        srv.submit(2, H=1, W=512, C=1, sim_epochs=1)
    assert e.value.code == n2f.EINVAL


def test_serving_trace_generator():
    reqs = synth.serving_trace(n=400, rate=2.0, seed=5)
    sides = np.array([[r.H, r.W] for r in reqs]).ravel()
    assert sides.min() >= 128 and sides.max() <= 2048
    assert abs(np.mean([r.C == 3 for r in reqs]) - 0.3) < 0.08
    arr = np.array([r.arrival for r in reqs])
    assert np.all(np.diff(arr) > 0) and abs(arr[-1] / 400 - 0.5) < 0.1


def test_cancel_queued_and_active_requests():
    """Cancelling (the serving failure path): a queued request leaves the
    queue, an active one leaves at once and frees its arena range; both are
    reported once with ECANCELED, the others finish normally, and an id that
    is no longer queued or active is refused."""
    unit = n2f.workspace_bytes(128, 128, 1)
    arena = 2 * unit
    srv = n2f.Server(arena, simulate=True, max_active=2)
    for i in range(4):
        srv.submit(i, H=128, W=128, C=1, sim_epochs=5)
    srv.step(1)                       # 0 and 1 active, 2 and 3 queued
    assert srv.memory()[0] == 2 * unit
    srv.cancel(1)                     # active
    srv.cancel(3)                     # queued
    assert dict(srv.poll()) == {1: n2f.ECANCELED, 3: n2f.ECANCELED}
    assert srv.memory()[0] == unit    # 1's range is free again
    with pytest.raises(n2f.N2FError):
        srv.cancel(3)
    with pytest.raises(n2f.N2FError):
        srv.submit(0, H=8, W=8, C=1, sim_epochs=1)   # id 0 is active
    done = {}
    for _ in range(20):
        srv.step(1)
        done.update(srv.poll())
    assert done == {0: n2f.OK, 2: n2f.OK}
    assert srv.memory() == (0, arena)


def test_cpu_tensors_refused_on_the_host():
    """Host tensors never reach the library: every binding entry point that
    takes images refuses them (and non-contiguous or non-FP32 ones) before
    any call into it."""
    import torch
    x = torch.zeros((1, 16, 16), dtype=torch.float32)
    with pytest.raises(ValueError):
        n2f.denoise(x)
    with pytest.raises(ValueError):
        n2f.Run(x)
    with pytest.raises(ValueError):
        n2f.Batch([x])
    srv = n2f.Server(1 << 30, simulate=True)
    with pytest.raises(ValueError):
        srv.submit(0, x, x.clone())
    with pytest.raises(ValueError):
        srv.submit(1, x.to(torch.float64), x.clone())
    with pytest.raises(ValueError):
        srv.submit(2, x.transpose(1, 2), x.clone())
    assert srv.step(1) == (0, 0)      # nothing was queued
