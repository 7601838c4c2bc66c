"""Continuous-batching serving loop for Poisson solves on resident meshes.

Requests (mesh id, right-hand side) arrive over time. Every mesh keeps its
geometric factors, gather-scatter map and p-multigrid hierarchy resident on the
device (built once). The loop:

  * admits waiting requests in arrival order while a batch slot is free and
    the solve's workspace (sem_solve_workspace_bytes) fits the HBM budget;
  * advances every admitted solve by one flexible-CG iteration per step: each
    phase of the iteration is one launch over all active solves
    (sem_batch_step), so requests that arrived while others were running join
    at the next iteration boundary and their work overlaps on the device;
  * retires finished solves, frees their slots and workspace, records the
    latency from arrival to result.

Each solve's arithmetic depends only on its own data (per-problem reductions
in a fixed order), so a result is bitwise the same alone or in any mix.

The method being served is the paper's pressure solve (FP64 flexible CG with
an FP32 pMG V-cycle, Implementation section); batching independent solves is
a systems pattern on top of it, not part of the paper.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import sem


@dataclass
class Request:
    rid: int
    mesh: int
    rhs: object          # device tensor, consistent and masked
    arrival: float       # seconds from the start of the run
    x: object = None     # device tensor for the solution
    admitted: float = None
    done: float = None
    info: dict = None
    slot: int = -1


@dataclass
class ResidentMesh:
    mesh: "sem.Mesh"
    pmg: "sem.Pmg"
    ws_bytes: int
    E: int
    Np: int


@dataclass
class ServeStats:
    latencies: list = field(default_factory=list)
    occupancy: list = field(default_factory=list)
    completed: int = 0
    wall: float = 0.0
    steps: int = 0
    peak_ws_bytes: int = 0
    rejected_for_memory: int = 0

    def summary(self) -> dict:
        lat = np.array(self.latencies) if self.latencies else np.array([np.nan])
        return {
            "completed": self.completed,
            "solves_per_s": self.completed / self.wall if self.wall > 0 else 0.0,
            "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(np.mean(lat) * 1e3),
            "mean_batch": float(np.mean(self.occupancy)) if self.occupancy else 0.0,
            "steps": self.steps,
            "wall_s": self.wall,
            "peak_workspace_GB": self.peak_ws_bytes / 1e9,
            "admission_waits_for_memory": self.rejected_for_memory,
        }


class Server:
    """Holds resident meshes and runs request streams through one batch."""

    def __init__(self, meshes, max_slots: int = 32, hbm_budget: int | None = None,
                 solve_opts: dict | None = None, stream=None):
        import torch
        self.torch = torch
        self.res = []
        for m, p in meshes:
            self.res.append(ResidentMesh(m, p, sem.sem_solve_workspace_bytes(m.h, p.h), m.E, m.Np))
        self.max_slots = max_slots
        if hbm_budget is None:
            free, _ = torch.cuda.mem_get_info()
            hbm_budget = int(free * 0.8)
        self.hbm_budget = hbm_budget
        self.opts = sem.solve_opts(**(solve_opts or {"rtol": 1e-8}))
        self.batch = sem.sem_batch_create(max_slots, stream)

    def close(self):
        if self.batch is not None:
            sem.sem_batch_destroy(self.batch)
            self.batch = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, requests: list, realtime: bool = True) -> ServeStats:
        """Serve `requests` (sorted by arrival). realtime=False ignores arrival
        times (everything is waiting at t=0)."""
        torch = self.torch
        st = ServeStats()
        pending = sorted(requests, key=lambda r: r.arrival)
        waiting: list[Request] = []
        active: dict[int, Request] = {}
        used = 0
        nxt = 0
        t0 = time.perf_counter()
        now = 0.0
        while nxt < len(pending) or waiting or active:
            now = time.perf_counter() - t0
            while nxt < len(pending) and (not realtime or pending[nxt].arrival <= now):
                waiting.append(pending[nxt])
                nxt += 1
            # admission: FIFO, slot and memory permitting
            while waiting and len(active) < self.max_slots:
                r = waiting[0]
                rm = self.res[r.mesh]
                if used + rm.ws_bytes > self.hbm_budget:
                    if not active:
                        raise MemoryError(f"request {r.rid} needs {rm.ws_bytes} B, budget {self.hbm_budget} B")
                    st.rejected_for_memory += 1
                    break
                waiting.pop(0)
                if r.x is None:
                    r.x = torch.empty_like(r.rhs)
                r.slot = sem.sem_batch_add(self.batch, rm.mesh.h, rm.pmg.h, r.rhs, r.x, self.opts)
                r.admitted = time.perf_counter() - t0
                active[r.slot] = r
                used += rm.ws_bytes
                st.peak_ws_bytes = max(st.peak_ws_bytes, used)
            if not active:
                if nxt < len(pending):
                    delay = pending[nxt].arrival - (time.perf_counter() - t0)
                    if delay > 0:
                        time.sleep(min(delay, 0.001))
                continue
            st.occupancy.append(len(active))
            sem.sem_batch_step(self.batch, 1)
            st.steps += 1
            for slot in list(active):
                info = sem.sem_batch_poll(self.batch, slot)
                if info["status"] == sem.RUNNING:
                    continue
                r = active.pop(slot)
                r.done = time.perf_counter() - t0
                r.info = info
                sem.sem_batch_release(self.batch, slot)
                used -= self.res[r.mesh].ws_bytes
                st.latencies.append(r.done - r.arrival)
                st.completed += 1
        torch.cuda.synchronize()
        st.wall = time.perf_counter() - t0
        return st


def poisson_arrivals(n: int, rate: float, n_meshes: int, seed: int) -> list[tuple[float, int]]:
    """(arrival time, mesh index) for n requests: exponential inter-arrival
    times at `rate` per second, mesh drawn uniformly; seeded."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n)
    t = np.cumsum(gaps) - gaps[0]
    meshes = rng.integers(0, n_meshes, size=n)
    return list(zip(t.tolist(), meshes.tolist()))
