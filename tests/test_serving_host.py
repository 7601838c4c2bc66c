"""Host logic of the continuous-batching serving loop (no GPU).

The loop's batch calls (sem_batch_create/add/step/poll/release and
sem_solve_workspace_bytes) are replaced by a fake backend in which solve k
finishes after a fixed number of steps. The tests check the admission policy
(FIFO, at most max_slots in flight, waiting while the HBM budget is full, an
error for a request that can never fit), slot reuse, and the accounting of
latencies, occupancy and peak workspace.
"""
import types

import numpy as np
import pytest
import torch

from paper_2110_01716_amd import serving
from paper_2110_01716_amd import sem as real_sem


class FakeBatch:
    def __init__(self, max_slots):
        self.max_slots = max_slots
        self.slots = {}          # slot -> [steps left, request order]
        self.admitted = []       # rhs tags in admission order
        self.max_in_flight = 0

    def add(self, rhs, steps):
        free = [k for k in range(self.max_slots) if k not in self.slots]
        assert free, "admitted beyond max_slots"
        k = free[0]
        self.slots[k] = steps
        self.admitted.append(int(rhs[0]))
        self.max_in_flight = max(self.max_in_flight, len(self.slots))
        return k


def fake_sem(steps_of_mesh, ws_of_mesh):
    st = {}

    def create(max_slots, stream=None):
        st["b"] = FakeBatch(max_slots)
        return st["b"]

    def add(b, mh, ph, rhs, x, opts=None):
        return b.add(rhs, steps_of_mesh[mh])

    def step(b, iters=1):
        for k in b.slots:
            if b.slots[k] > 0:
                b.slots[k] -= 1
        return len(b.slots)

    def poll(b, slot):
        return {"status": real_sem.RUNNING if b.slots[slot] > 0 else real_sem.SEM_OK, "iters": 1}

    def release(b, slot):
        del b.slots[slot]

    return types.SimpleNamespace(
        sem_batch_create=create, sem_batch_add=add, sem_batch_step=step, sem_batch_poll=poll,
        sem_batch_release=release, sem_batch_destroy=lambda b: None,
        sem_solve_workspace_bytes=lambda mh, ph: ws_of_mesh[mh],
        solve_opts=lambda **kw: kw, RUNNING=real_sem.RUNNING, SEM_OK=real_sem.SEM_OK), st


def resident(n):
    return [(types.SimpleNamespace(h=k, E=8, Np=64), types.SimpleNamespace(h=100 + k)) for k in range(n)]


def requests(mesh_ids, arrivals=None):
    out = []
    for i, m in enumerate(mesh_ids):
        out.append(serving.Request(rid=i, mesh=m, rhs=torch.full((4,), float(i)),
                                   arrival=0.0 if arrivals is None else arrivals[i]))
    return out


@pytest.fixture
def patch(monkeypatch):
    def install(steps_of_mesh, ws_of_mesh):
        fs, st = fake_sem(steps_of_mesh, ws_of_mesh)
        monkeypatch.setattr(serving, "sem", fs)
        monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)
        return st
    return install


def test_fifo_admission_within_slot_limit(patch):
    st = patch({0: 3, 1: 5}, {0: 10, 1: 10})
    srv = serving.Server(resident(2), max_slots=2, hbm_budget=10 ** 9)
    reqs = requests([0, 1, 0, 1, 0, 0, 1])
    stats = srv.run(reqs, realtime=False)
    b = st["b"]
    assert stats.completed == len(reqs)
    assert b.admitted == list(range(len(reqs)))        # arrival order
    assert b.max_in_flight == 2 and max(stats.occupancy) == 2
    assert all(r.done >= r.admitted >= r.arrival for r in reqs)
    assert len(stats.latencies) == len(reqs) and min(stats.latencies) >= 0.0
    assert stats.rejected_for_memory == 0
    assert not b.slots                                   # every slot released


def test_waits_for_memory_and_respects_budget(patch):
    # mesh 1's workspace takes most of the budget: it runs alone
    st = patch({0: 2, 1: 4}, {0: 30, 1: 80})
    srv = serving.Server(resident(2), max_slots=8, hbm_budget=100)
    reqs = requests([0, 1, 0, 1, 0])
    stats = srv.run(reqs, realtime=False)
    assert stats.completed == len(reqs)
    assert stats.peak_ws_bytes <= 100
    assert stats.rejected_for_memory > 0
    assert st["b"].admitted == list(range(len(reqs)))    # still first come, first served


def test_request_that_can_never_fit_is_an_error(patch):
    patch({0: 1}, {0: 500})
    srv = serving.Server(resident(1), max_slots=4, hbm_budget=100)
    with pytest.raises(MemoryError):
        srv.run(requests([0]), realtime=False)


def test_realtime_arrivals_and_summary(patch):
    patch({0: 2, 1: 3}, {0: 10, 1: 10})
    srv = serving.Server(resident(2), max_slots=4, hbm_budget=10 ** 6)
    arr = serving.poisson_arrivals(12, rate=2000.0, n_meshes=2, seed=5)
    assert arr[0][0] == 0.0 and all(b[0] >= a[0] for a, b in zip(arr, arr[1:]))
    reqs = requests([m for _, m in arr], [t for t, _ in arr])
    stats = srv.run(reqs, realtime=True)
    s = stats.summary()
    assert s["completed"] == 12 and s["steps"] >= 3
    assert s["p99_ms"] >= s["p50_ms"] >= 0.0
    assert 1.0 <= s["mean_batch"] <= 4.0
    assert all(r.admitted >= r.arrival for r in reqs)
