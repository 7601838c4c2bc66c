"""Benchmark of the SEM Poisson hot path on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-solve] [--no-cpu]

Workload: 64^3 = 262,144 hex elements, N = 7 (89.9M DOFs, 134.2M local GLL
points), unit box deformed by x_i += 0.05 sin(2 pi x_j + phi) sin(2 pi x_k + phi)
with seeded phases, homogeneous Dirichlet boundary, synthetic inputs (the
paper's reactor meshes are not available).

Timed region: K steps after W warm-up steps; a step is one FP64 application of
the local SEM Laplacian Ax over all elements (inputs resident in HBM), bracketed
by torch.cuda.synchronize(); HIP events on the library's stream give the
kernel time. value = Ax GDOF/s with DOF = E N^3.

The same line reports:
  * roofline of the Ax kernel: 64 algorithmic bytes per local point (u, six
    geometric factors, Au in FP64) over the event-timed kernel duration,
    against 8 TB/s;
  * the Poisson time-to-solution at relative residual 1e-8 for FP64 Jacobi-PCG
    and for FP64 flexible CG preconditioned by the FP32 p-multigrid V-cycle
    (N = 7 -> 3 -> 1, Chebyshev-Jacobi degree 2, coarse FP64 Jacobi-PCG to
    1e-2) on the 48^3 mesh (and the 64^3 mesh with --solve-c2);
  * cpu_baseline: the FP64 NumPy oracle's Ax on a bounded sample of the same
    workload on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def build_mesh(sem, spec):
    from paper_2110_01716_amd import workloads as wl
    t = time.time()
    bm = wl.box_mesh(spec["n"], N=spec["N"], deform=spec["deform"], seed=spec["seed"])
    log(f"generated {spec['n']}^3 N={spec['N']} mesh in {time.time() - t:.1f}s")
    t = time.time()
    m = sem.Mesh.from_box(bm)
    log(f"mesh setup on device in {time.time() - t:.1f}s")
    return bm, m


def time_ax(sem, m, E, Np, steps, warmup):
    import torch
    u = torch.rand((E, Np), dtype=torch.float64, device="cuda") * 2 - 1
    Au = torch.empty_like(u)
    for _ in range(warmup):
        sem.sem_ax(m.h, u, Au)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in ev:
        a.record()
        sem.sem_ax(m.h, u, Au)
        b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = [a.elapsed_time(b) for a, b in ev]
    del u, Au
    return wall, ms


def solve_pair(sem, bm, m, label, skip_pcg=False):
    import torch
    from paper_2110_01716_amd import workloads as wl
    out = {}
    b = torch.from_numpy(wl.random_rhs(bm, 2000)).to("cuda")
    x = torch.empty_like(b)
    t = time.time()
    p = sem.Pmg(m)
    out["pmg_setup_s"] = time.time() - t
    info = sem.sem_pcg_solve(m.h, p.h, b, x, sem.solve_opts(rtol=1e-8))  # warm
    torch.cuda.synchronize()
    t = time.perf_counter()
    info = sem.sem_pcg_solve(m.h, p.h, b, x, sem.solve_opts(rtol=1e-8))
    torch.cuda.synchronize()
    out["pmg_fp32"] = {"seconds": time.perf_counter() - t, "iters": info["iters"], "relres": info["relres"],
                       "relres_true": info["relres_true"], "coarse_iters": info["coarse_iters"]}
    log(label, "pmg", out["pmg_fp32"])
    if skip_pcg:
        p.close()
        return out
    xp = x.clone()
    t = time.perf_counter()
    info = sem.sem_pcg_solve(m.h, None, b, x, sem.solve_opts(rtol=1e-8, maxit=20000))
    torch.cuda.synchronize()
    out["pcg_fp64"] = {"seconds": time.perf_counter() - t, "iters": info["iters"], "relres": info["relres"],
                       "relres_true": info["relres_true"]}
    log(label, "pcg", out["pcg_fp64"])
    out["speedup_pmg_vs_pcg"] = out["pcg_fp64"]["seconds"] / out["pmg_fp32"]["seconds"]
    out["rel_diff_pmg_vs_pcg"] = float((xp - x).abs().max() / x.abs().max())
    p.close()
    return out


def cpu_baseline(bm_spec, budget_s=12.0):
    """Oracle Ax (FP64 NumPy) on a bounded sample of the workload, 1 thread."""
    from threadpoolctl import threadpool_limits
    from oracle import operators as ops
    from paper_2110_01716_amd import workloads as wl
    n = 16
    bm = wl.box_mesh(n, N=bm_spec["N"], deform=bm_spec["deform"], seed=bm_spec["seed"])
    with threadpool_limits(limits=1):
        G, _, _ = ops.geometric_factors(bm.N, bm.x, bm.y, bm.z)
        u = np.random.default_rng(0).uniform(-1, 1, bm.x.shape)
        reps, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < budget_s:
            ops.ax_local(bm.N, G, u)
            reps += 1
        dt = (time.perf_counter() - t0) / reps
    return {"value": bm.E * bm.N ** 3 / dt / 1e9, "unit": "GDOF/s", "cores": 1, "kind": "oracle",
            "sample": f"FP64 NumPy oracle Ax on a {n}^3-element N={bm.N} deformed box "
                      f"(same construction as the workload), {reps} repetitions, one thread"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--solve-c2", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--skip-pcg", action="store_true", help="time only the pMG solve")
    ap.add_argument("--solve-only", action="store_true", help="skip the Ax steps (profiling the solve)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run a plain 1 GiB device copy first (counter calibration under a profiler)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); this build has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2110_01716_amd import sem, workloads as wl
    sem.load()
    if a.calib_copy:
        src = torch.rand(1 << 27, dtype=torch.float64, device="cuda")  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: 3 x 1 GiB read + 1 GiB write")
        del src, dst
    spec = dict(wl.config_meshes()["ax_64x64x64_N7"])
    spec["n"] = a.n
    if a.solve_only:
        spec3 = wl.config_meshes()["pmg_48x48x48_N7"]
        bm3, m3 = build_mesh(sem, spec3)
        print(json.dumps({"poisson": {"48x48x48_N7": solve_pair(sem, bm3, m3, "c3", a.skip_pcg)}}), flush=True)
        return
    bm, m = build_mesh(sem, spec)
    E, N = bm.E, bm.N
    Np = (N + 1) ** 3
    dofs = E * N ** 3
    wall, ms = time_ax(sem, m, E, Np, a.steps, a.warmup)
    ms_avg = float(np.mean(ms))
    ms_med = float(np.median(ms))
    bytes_per_launch = 64 * E * Np
    gbs = bytes_per_launch / (ms_avg * 1e-3) / 1e9
    value = dofs / (wall / a.steps) / 1e9
    res = {
        "metric": "Ax GDOF/s & HBM GB/s; Poisson time-to-1e-8: FP64 PCG vs FP32-pMG",
        "value": round(value, 3),
        "unit": "GDOF/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(wall / a.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"deformed box {a.n}^3 hex elements, N=7, FP64 Ax (local SEM Laplacian)",
                   "elements": E, "N": N, "dofs_EN3": dofs, "local_points": E * Np},
        "ax": {"ms_mean": round(ms_avg, 4), "ms_median": round(ms_med, 4), "ms_min": round(min(ms), 4),
               "gdofs_kernel": round(dofs / (ms_avg * 1e-3) / 1e9, 3), "hbm_gbs": round(gbs, 1)},
        "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None},
    }
    log("ax", res["ax"])
    if not a.no_solve:
        poisson = {}
        if a.solve_c2:
            poisson["64x64x64_N7"] = solve_pair(sem, bm, m, "c2")
        m.close()
        del bm
        spec3 = wl.config_meshes()["pmg_48x48x48_N7"]
        bm3, m3 = build_mesh(sem, spec3)
        poisson["48x48x48_N7"] = solve_pair(sem, bm3, m3, "c3", a.skip_pcg)
        m3.close()
        res["poisson"] = poisson
    if not a.no_cpu:
        res["cpu_baseline"] = cpu_baseline(spec)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
