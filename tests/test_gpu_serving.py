"""Continuous-batching serving loop: requests on resident meshes, admitted by
HBM footprint, each result bitwise identical to the same solve run alone."""
import numpy as np
import pytest

from paper_2110_01716_amd import workloads as wl

from gpu_util import dev, print_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    from paper_2110_01716_amd import sem, serving
    sem.load()
    bms = [wl.box_mesh(n, N=7, deform=0.05, seed=1000 + n) for n in (2, 3, 4)]
    meshes = [(sem.Mesh.from_box(bm), None) for bm in bms]
    meshes = [(m, sem.Pmg(m)) for m, _ in meshes]
    rhs = {(k, j): dev(wl.random_rhs(bm, 2000 + 10 * k + j)) for k, bm in enumerate(bms) for j in range(3)}
    return sem, serving, bms, meshes, rhs


def _alone(sem, meshes, rhs, k, j):
    import torch
    m, p = meshes[k]
    x = torch.empty_like(rhs[(k, j)])
    sem.sem_pcg_solve(m.h, p.h, rhs[(k, j)], x, sem.solve_opts(rtol=1e-8))
    return x


def _requests(serving, rhs, arrivals):
    reqs = []
    for i, (t, k) in enumerate(arrivals):
        reqs.append(serving.Request(rid=i, mesh=k, rhs=rhs[(k, i % 3)], arrival=t))
    return reqs


def test_serving_results_equal_alone(env):
    import torch
    sem, serving, bms, meshes, rhs = env
    print_case("serving-identity")
    srv = serving.Server(meshes, max_slots=4)
    arrivals = serving.poisson_arrivals(12, rate=400.0, n_meshes=3, seed=7)
    reqs = _requests(serving, rhs, arrivals)
    st = srv.run(reqs, realtime=True)
    srv.close()
    assert st.completed == 12
    assert max(st.occupancy) >= 2  # solves really overlapped
    for r in reqs:
        assert r.info["status"] == 0 and r.info["relres"] <= 1e-8
        assert torch.equal(r.x, _alone(sem, meshes, rhs, r.mesh, r.rid % 3))
    s = st.summary()
    assert s["p99_ms"] >= s["p50_ms"] > 0


def test_serving_admission_by_memory(env):
    import torch
    sem, serving, bms, meshes, rhs = env
    print_case("serving-memory")
    ws = [sem.sem_solve_workspace_bytes(m.h, p.h) for m, p in meshes]
    budget = max(ws) + min(ws)  # at most two small solves, or the big one alone
    srv = serving.Server(meshes, max_slots=8, hbm_budget=budget)
    reqs = _requests(serving, rhs, [(0.0, k % 3) for k in range(9)])
    st = srv.run(reqs, realtime=False)
    srv.close()
    assert st.completed == 9
    assert st.peak_ws_bytes <= budget
    assert st.rejected_for_memory > 0
    for r in reqs:
        assert torch.equal(r.x, _alone(sem, meshes, rhs, r.mesh, r.rid % 3))
