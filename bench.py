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
    1e-2) on the 48^3 mesh (and the 64^3 mesh with --solve-c2), plus the
    same solve with GMRES(6) and with the Chebyshev-accelerated Schwarz
    smoothers (ASM, RAS);
  * the Helmholtz operator (A_L + lambda B) u (72 B per point) on the same
    mesh, and Helmholtz Jacobi-PCG solves on the 48^3 mesh;
  * projection onto prior solutions: per-solve time and iterations of the
    pMG solve over a sequence of 40 smoothly varying right-hand sides on the
    48^3 mesh for L_max = 0, 8 and 30;
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

# HBM bytes per FP64 Ax launch (64^3, N=7) from rocprofv3 FETCH_SIZE x 2.0 +
# WRITE_SIZE x 1.0 (scales from the library's copy kernel on 1 GiB), taken on the Ax kernel
# whose source hashes to `source_sha16`; reported only while it still matches.
AX_COUNTERS = {"source_sha16": "7a4238109b8e6ce7", "traffic_GB_per_launch": 8.590091,
               "summary": "profiles/ax_64x64x64_N7_fp64_hbm_counters.txt"}


def ax_source_sha16() -> str:
    import hashlib
    src = open(os.path.join(ROOT, "paper_2110_01716_amd", "csrc", "sem_kernels.hip")).read()
    t = src[src.index("// ax-kernel-begin"):src.index("// ax-kernel-end")]
    return hashlib.sha256(t.encode()).hexdigest()[:16]


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


def time_ax(sem, m, E, Np, steps, warmup, lam=None):
    """Event-timed FP64 Ax (lam=None) or Helmholtz (A_L + lam B) u launches."""
    import torch
    u = torch.rand((E, Np), dtype=torch.float64, device="cuda") * 2 - 1
    Au = torch.empty_like(u)

    def op():
        if lam is None:
            sem.sem_ax(m.h, u, Au)
        else:
            sem.sem_helmholtz(m.h, u, Au, lam)

    for _ in range(warmup):
        op()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in ev:
        a.record()
        op()
        b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = [a.elapsed_time(b) for a, b in ev]
    del u, Au
    return wall, ms


def bench_ax_orders(sem, steps=20, warmup=5):
    """Event-timed Ax at the orders of the batched workload's hierarchies
    (N = 5, 7, 9), FP64 and FP32, each on a deformed box of ~55M local points."""
    import torch
    from paper_2110_01716_amd import workloads as wl
    out = {}
    for N, n in ((5, 64), (7, 48), (9, 38)):
        bm = wl.box_mesh(n, N=N, deform=0.05, seed=1001)
        m = sem.Mesh.from_box(bm)
        E, Np = bm.E, bm.Np
        del bm
        for dt, bpp in ((torch.float64, 64), (torch.float32, 32)):
            u = torch.rand((E, Np), dtype=dt, device="cuda") * 2 - 1
            Au = torch.empty_like(u)
            for _ in range(warmup):
                sem.sem_ax(m.h, u, Au)
            torch.cuda.synchronize()
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
            for a_, b_ in ev:
                a_.record()
                sem.sem_ax(m.h, u, Au)
                b_.record()
            torch.cuda.synchronize()
            ms = float(np.mean([a_.elapsed_time(b_) for a_, b_ in ev]))
            gbs = bpp * E * Np / (ms * 1e-3) / 1e9
            out[f"N{N}_{'f64' if bpp == 64 else 'f32'}"] = {
                "elements": E, "local_points": E * Np, "bytes_per_point": bpp, "ms_mean": round(ms, 4),
                "GBs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4), "gdofs": round(E * N ** 3 / ms / 1e6, 2)}
            del u, Au
        m.close()
    return out


def time_stream(sem, n, steps, warmup):
    """Event-timed bandwidth probe (sem_stream) on n doubles per array: copy
    (16 B per element), STREAM triad (24 B) and the FP64 Ax read:write mix of
    seven streams in, one out (64 B, as Ax per local point)."""
    import torch
    n -= n % 2
    src = torch.empty((7, n), dtype=torch.float64, device="cuda").uniform_(-1, 1)
    dst = torch.empty(n, dtype=torch.float64, device="cuda")
    out = {"elements": n}
    for name, nin, bpe in (("copy", 1, 16), ("triad", 2, 24), ("ax_mix_7r1w", 7, 64)):
        for _ in range(warmup):
            sem.sem_stream(nin, src, dst, 0.5, n)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        for a, b in ev:
            a.record()
            sem.sem_stream(nin, src, dst, 0.5, n)
            b.record()
        torch.cuda.synchronize()
        ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
        out[name] = {"bytes_per_element": bpe, "ms_mean": round(ms, 4), "GBs": round(bpe * n / (ms * 1e-3) / 1e9, 1)}
    del src, dst
    return out


def load_xstar_samples(n):
    """Sampled FP64 oracle solution of the n^3 mixed-precision workload
    (tests/golden, written by make_oracle_solution_samples.py), or None."""
    path = os.path.join(ROOT, "tests", "golden", f"pmg_{n}x{n}x{n}_N7_rhs2000_xstar_samples.txt")
    if not os.path.exists(path):
        return None
    meta, idx, val = {}, [], []
    for line in open(path):
        if line.startswith("#"):
            parts = line[1:].split()
            if len(parts) == 2:
                try:
                    meta[parts[0]] = float(parts[1])
                except ValueError:
                    pass
            continue
        i, v = line.split()
        idx.append(int(i))
        val.append(float(v))
    return {"meta": meta, "idx": np.array(idx, dtype=np.int64), "val": np.array(val), "file": os.path.relpath(path, ROOT)}


def solution_errors(x, samples, xref):
    """Relative max-norm error of x against the oracle's x* at the sampled
    DOFs (scaled by max |x*| over all DOFs) and against a full reference."""
    import torch
    e = {}
    if samples is not None:
        it = torch.from_numpy(samples["idx"]).to(x.device)
        xs = x.reshape(-1)[it].cpu().numpy()
        e["err_vs_oracle_sampled"] = float(np.max(np.abs(xs - samples["val"])) / samples["meta"]["xstar_max_abs"])
    if xref is not None:
        e["err_vs_ref_max"] = float((x - xref).abs().max() / xref.abs().max())
    return e


def time_to_error(sem, m, p, b, x, samples, xref, rtols, target=1e-8, maxit=None):
    """Solve at decreasing rtol until the solution error (max of the sampled
    oracle error and the full-reference error) is <= target; every solve is
    timed from the call to its return. Returns the per-rtol records and the
    first rtol that meets the target with its time."""
    import torch
    runs = []
    hit = None
    for rtol in rtols:
        o = sem.solve_opts(rtol=rtol, maxit=maxit) if maxit else sem.solve_opts(rtol=rtol)
        torch.cuda.synchronize()
        t = time.perf_counter()
        info = sem.sem_pcg_solve(m.h, p.h if p is not None else None, b, x, o)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t
        rec = {"rtol": rtol, "seconds": round(sec, 5), "iters": info["iters"], "relres_true": info["relres_true"]}
        rec.update(solution_errors(x, samples, xref))
        runs.append(rec)
        err = max(v for k, v in rec.items() if k.startswith("err_"))
        if err <= target:
            hit = {"rtol": rtol, "seconds": rec["seconds"], "iters": rec["iters"], "error": err}
            break
    return {"runs": runs, "to_target": hit, "target_error": target}


def timed_solve(sem, m, p, b, x, opts, gmres_K=0):
    """One solve timed from the call to its return (inputs resident)."""
    import torch
    torch.cuda.synchronize()
    t = time.perf_counter()
    if gmres_K:
        info = sem.sem_gmres_solve(m.h, p.h, gmres_K, b, x, opts)
    else:
        info = sem.sem_pcg_solve(m.h, p.h if p is not None else None, b, x, opts)
    torch.cuda.synchronize()
    return {"seconds": time.perf_counter() - t, "iters": info["iters"], "relres": info["relres"],
            "relres_true": info["relres_true"], "coarse_iters": info["coarse_iters"]}


def reference_solution(sem, m, b, samples):
    """FlexCG preconditioned by pMG with FP64 smoothing, to relative residual
    1e-12: the full-vector reference for solution errors (its own error
    against the oracle's x* at the sampled DOFs is reported with it)."""
    import torch
    pr = sem.Pmg(m, smoother_dtype="f64")
    xref = torch.empty_like(b)
    rec = timed_solve(sem, m, pr, b, xref, sem.solve_opts(rtol=1e-12, maxit=200))
    pr.close()
    rec["solver"] = "FP64 FlexCG + pMG with FP64 smoothing, rtol 1e-12"
    rec.update(solution_errors(xref, samples, None))
    return xref, rec


def solve_pair(sem, bm, m, label, skip_pcg=False, samples=None, smoothers=True, rtols=(1e-8, 1e-9, 1e-10, 1e-11),
               pcg_rtols=None):
    """FP32-pMG FlexCG (and GMRES(6), Schwarz smoothers) vs FP64 Jacobi-PCG on
    one mesh: times at rtol 1e-8, then the time each solver needs for a
    solution error <= 1e-8 (rtol lowered by decades until it holds), errors
    taken against the sampled oracle x* (if given) and a full FP64 reference."""
    import torch
    from paper_2110_01716_amd import workloads as wl
    out = {}
    b = torch.from_numpy(wl.random_rhs(bm, 2000)).to("cuda")
    x = torch.empty_like(b)
    t = time.time()
    p = sem.Pmg(m)
    out["pmg_setup_s"] = time.time() - t
    o8 = sem.solve_opts(rtol=1e-8)
    sem.sem_pcg_solve(m.h, p.h, b, x, o8)  # warm
    out["pmg_fp32"] = timed_solve(sem, m, p, b, x, o8)
    xp = x.clone()
    log(label, "pmg", out["pmg_fp32"])
    if smoothers:
        sem.sem_gmres_solve(m.h, p.h, 6, b, x, o8)  # warm
        out["pmg_fp32_gmres6"] = timed_solve(sem, m, p, b, x, o8, gmres_K=6)
        log(label, "pmg-gmres6", out["pmg_fp32_gmres6"])
        ras = None
        for sm in ("asm", "ras"):
            t = time.time()
            ps = sem.Pmg(m, smoother=sm)
            setup_s = time.time() - t
            sem.sem_pcg_solve(m.h, ps.h, b, x, o8)  # warm
            rec = timed_solve(sem, m, ps, b, x, o8)
            rec.update({"setup_s": round(setup_s, 2), "rho": ps.info()["rho"][:2]})
            out[f"pmg_fp32_cheb_{sm}"] = rec
            log(label, f"pmg-{sm}", rec)
            if sm == "ras":
                ras = ps  # kept for its time to the target error below
            else:
                ps.close()
    xref, out["reference"] = reference_solution(sem, m, b, samples)
    log(label, "reference", out["reference"])
    out["pmg_fp32"].update(solution_errors(xp, samples, xref))
    if samples is not None:
        out["oracle_samples"] = {"file": samples["file"], "count": int(len(samples["idx"])),
                                 "oracle_iters": int(samples["meta"].get("iters", 0)),
                                 "oracle_relres_true": samples["meta"].get("relres_true")}
    tte = {"pmg_fp32": time_to_error(sem, m, p, b, x, samples, xref, rtols)}
    log(label, "pmg time-to-error", tte["pmg_fp32"])
    if smoothers and ras is not None:
        tte["pmg_fp32_cheb_ras"] = time_to_error(sem, m, ras, b, x, samples, xref, rtols)
        log(label, "pmg-ras time-to-error", tte["pmg_fp32_cheb_ras"])
        ras.close()
    if not skip_pcg:
        xw = torch.empty_like(b)
        sem.sem_pcg_solve(m.h, None, b, xw, sem.solve_opts(maxit=3), check=False)  # workspace
        tte["pcg_fp64"] = time_to_error(sem, m, None, b, xw, samples, xref, pcg_rtols or rtols, maxit=50000)
        log(label, "pcg time-to-error", tte["pcg_fp64"])
        r0 = tte["pcg_fp64"]["runs"][0]
        out["pcg_fp64"] = {k: r0[k] for k in ("seconds", "iters", "relres_true") if k in r0}
        out["pcg_fp64"].update({k: v for k, v in r0.items() if k.startswith("err_")})
        out["speedup_pmg_vs_pcg"] = out["pcg_fp64"]["seconds"] / out["pmg_fp32"]["seconds"]
        if tte["pmg_fp32"]["to_target"] and tte["pcg_fp64"]["to_target"]:
            tte["speedup_pmg_vs_pcg_at_equal_error"] = round(
                tte["pcg_fp64"]["to_target"]["seconds"] / tte["pmg_fp32"]["to_target"]["seconds"], 2)
        ras_hit = tte.get("pmg_fp32_cheb_ras", {}).get("to_target")
        if ras_hit and tte["pcg_fp64"]["to_target"]:
            tte["speedup_pmg_ras_vs_pcg_at_equal_error"] = round(
                tte["pcg_fp64"]["to_target"]["seconds"] / ras_hit["seconds"], 2)
        del xw
    out["time_to_1e-8_solution_error"] = tte
    p.close()
    del xref, xp
    return out


def bench_projection(sem, bm, m, steps=40, lmaxes=(0, 8, 30), gmres_K=6):
    """Successive right-hand sides (smooth in time, 8 modes + 1e-3 rough
    noise, dt = 0.05) solved to 1e-8 by flexible CG + pMG, with the starting
    guess projected onto the last L_max solutions; L_max = 0 is the plain
    solve. Reports per-solve time and iterations averaged over all steps."""
    import torch
    from paper_2110_01716_amd import workloads as wl
    at = wl.rhs_sequence_fn(bm, modes=8, noise=1e-3, dt=0.05, seed=4000, device="cuda")
    p = sem.Pmg(m)
    opts = sem.solve_opts(rtol=1e-8)
    x = torch.empty(bm.x.shape, dtype=torch.float64, device="cuda")
    sem.sem_pcg_solve(m.h, p.h, at(0), x, opts)  # warm
    out = {"steps": steps, "rhs": "8 smooth modes + 1e-3 rough noise, dt 0.05", "rtol": 1e-8}
    runs = [(L, 0) for L in lmaxes] + [(lmaxes[-1], gmres_K)]
    for L, K in runs:
        pr = sem.Projection(m, L, gmres_K=K) if L else None
        secs, its, rel0, worst = [], [], [], 0.0
        for k in range(steps):
            b = at(k)
            torch.cuda.synchronize()
            t = time.perf_counter()
            info = pr.solve(p, b, x, opts) if pr else sem.sem_pcg_solve(m.h, p.h, b, x, opts)
            torch.cuda.synchronize()
            secs.append(time.perf_counter() - t)
            its.append(info["iters"])
            rel0.append(info["relres_initial"])
            worst = max(worst, info["relres_true"])
            del b
        key = f"L{L}" + (f"_gmres{K}" if K else "")
        out[key] = {"s_per_solve": round(float(np.mean(secs)), 5), "iters_mean": round(float(np.mean(its)), 2),
                        "iters_last10": its[-10:], "relres_initial_median": float(np.median(rel0)),
                        "relres_true_max": worst}
        log("projection", key, out[key])
        if pr:
            pr.close()
    base = out["L0"]["s_per_solve"]
    for L in lmaxes[1:]:
        out[f"speedup_L{L}_vs_L0"] = round(base / out[f"L{L}"]["s_per_solve"], 3)
    kg = f"L{lmaxes[-1]}_gmres{gmres_K}"
    out[f"speedup_{kg}_vs_L0"] = round(base / out[kg]["s_per_solve"], 3)
    p.close()
    return out


def bench_helmholtz_solve(sem, bm, m, lams=(1e2, 1e4)):
    """FP64 Jacobi-PCG on (A + lam B) x = b (the velocity-substep operator) to 1e-8."""
    import torch
    from paper_2110_01716_amd import workloads as wl
    b = torch.from_numpy(wl.random_rhs(bm, 2001)).to("cuda")
    x = torch.empty_like(b)
    out = {}
    for lam in lams:
        o = sem.solve_opts(rtol=1e-8, maxit=20000, lam=lam)
        sem.sem_pcg_solve(m.h, None, b, x, o)  # warm
        torch.cuda.synchronize()
        t = time.perf_counter()
        info = sem.sem_pcg_solve(m.h, None, b, x, o)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t
        out[f"lambda_{lam:g}"] = {"seconds": round(sec, 5), "iters": info["iters"],
                                  "ms_per_iter": round(sec / max(info["iters"], 1) * 1e3, 4),
                                  "relres_true": info["relres_true"]}
        log("helmholtz-pcg", lam, out[f"lambda_{lam:g}"])
    return out


def bench_batched(sem, count=256, sequential=True):
    """Independent Dirichlet problems (m^3 elements, m ~ U{2..12}; N ~ U{5,7,9};
    deformed boxes; seeded RHS) solved by FP64 flexible CG + FP32 pMG: one
    batched call (each phase one launch over all problems) vs one call each."""
    import torch
    from paper_2110_01716_amd import workloads as wl
    t = time.time()
    specs = wl.batched_problem_specs(count)
    meshes, pmgs, bs = [], [], []
    for k, sp in enumerate(specs):
        bm = wl.box_mesh(sp["n"], N=sp["N"], deform=sp["deform"], seed=sp["seed"])
        m = sem.Mesh.from_box(bm)
        meshes.append(m)
        pmgs.append(sem.Pmg(m))
        bs.append(torch.from_numpy(wl.random_rhs(bm, 2000 + k)).to("cuda"))
    setup = time.time() - t
    npts = sum(m.E * m.Np for m in meshes)
    xb = [torch.empty_like(b) for b in bs]
    opts = sem.solve_opts(rtol=1e-8)
    sem.sem_pcg_solve_batched([m.h for m in meshes], [p.h for p in pmgs], bs, xb, opts)  # warm
    torch.cuda.synchronize()
    time.sleep(0.05)  # separates the timed solve from the others in a kernel trace
    t = time.perf_counter()
    rc, infos = sem.sem_pcg_solve_batched([m.h for m in meshes], [p.h for p in pmgs], bs, xb, opts)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t
    time.sleep(0.05)
    out = {"problems": count, "local_points": npts, "setup_s": round(setup, 2), "batched_s": round(tb, 4),
           "batched_solves_per_s": round(count / tb, 1), "status_ok": all(i["status"] == 0 for i in infos),
           "max_relres_true": max(i["relres_true"] for i in infos),
           "iters_mean": float(np.mean([i["iters"] for i in infos])), "iters_max": max(i["iters"] for i in infos),
           # one launch per phase over all unfinished problems; the last problem to finish reports the whole call
           "kernel_launches": max(i["launches"] for i in infos)}
    if sequential:
        xs = [torch.empty_like(b) for b in bs]
        launches = 0
        t = time.perf_counter()
        for m, p, b, x in zip(meshes, pmgs, bs, xs):
            launches += sem.sem_pcg_solve(m.h, p.h, b, x, opts)["launches"]
        torch.cuda.synchronize()
        ts = time.perf_counter() - t
        out["sequential_s"] = round(ts, 4)
        out["sequential_kernel_launches"] = launches
        out["speedup_batched_vs_sequential"] = round(ts / tb, 2)
        out["bitwise_equal_to_alone"] = all(torch.equal(a, b) for a, b in zip(xs, xb))
    for p in pmgs:
        p.close()
    for m in meshes:
        m.close()
    return out


def bench_serving(sem, rates=(10, 20, 50, 100, 200, 500), window_s=2.0, max_slots=32):
    """Poisson arrivals on 16 resident N=7 deformed-box meshes of m^3 elements,
    m = round(8 + 32 i / 15); each request solves to 1e-8 (FP64 flexible CG,
    FP32 pMG); admission by HBM footprint; p50/p99 arrival-to-result latency."""
    import torch
    from paper_2110_01716_amd import serving, workloads as wl
    t = time.time()
    sides = wl.serving_mesh_sides()
    resident, pool = [], {}
    for k, n in enumerate(sides):
        bm = wl.box_mesh(n, N=7, deform=0.05, seed=1000 + k)
        m = sem.Mesh.from_box(bm)
        resident.append((m, sem.Pmg(m)))
        for j in range(2):
            pool[(k, j)] = torch.from_numpy(wl.random_rhs(bm, 2000 + 2 * k + j)).to("cuda")
        del bm
    setup = time.time() - t
    srv = serving.Server(resident, max_slots=max_slots)
    warm = [serving.Request(rid=k, mesh=k, rhs=pool[(k, 0)], arrival=0.0) for k in range(len(sides))]
    srv.run(warm, realtime=False)
    out = {"meshes": sides, "setup_s": round(setup, 1), "max_slots": max_slots,
           "hbm_budget_GB": round(srv.hbm_budget / 1e9, 1), "rates": {}}
    for rate in rates:
        n = int(min(max(rate * window_s, 24), 240))
        arr = serving.poisson_arrivals(n, rate, len(sides), seed=5000 + rate)
        reqs = [serving.Request(rid=i, mesh=k, rhs=pool[(k, i % 2)], arrival=tt) for i, (tt, k) in enumerate(arr)]
        st = srv.run(reqs, realtime=True)
        s = st.summary()
        s["offered_rate"] = rate
        s["requests"] = n
        s["all_ok"] = all(r.info["status"] == 0 for r in reqs)
        out["rates"][str(rate)] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in s.items()}
        log("serving", rate, out["rates"][str(rate)])
    srv.close()
    for m, p in resident:
        p.close()
        m.close()
    return out


def _oracle_ax_worker(args):
    """One host core: the oracle's Ax on an n^3-element sample mesh, repeated
    for `budget` seconds with one BLAS thread. Returns (E, N, seconds per Ax)."""
    n, N, deform, seed, budget = args
    from threadpoolctl import threadpool_limits
    from oracle import operators as ops
    from paper_2110_01716_amd import workloads as wl
    bm = wl.box_mesh(n, N=N, deform=deform, seed=seed)
    with threadpool_limits(limits=1):
        G, _, _ = ops.geometric_factors(bm.N, bm.x, bm.y, bm.z)
        u = np.random.default_rng(0).uniform(-1, 1, bm.x.shape)
        reps, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < budget:
            ops.ax_local(bm.N, G, u)
            reps += 1
        dt = (time.perf_counter() - t0) / reps
    return bm.E, bm.N, dt


def cpu_baseline(bm_spec, budget_s=8.0):
    """The FP64 NumPy oracle on the host cores: its Ax run by one process per
    core (affinity mask) on a 16^3-element sample of the workload's mesh
    construction, summed over cores; plus the oracle's solves on the tiny
    manufactured problem (direct and Jacobi-PCG) and its pMG-FlexCG on an
    8^3-element box, with the 48^3 figure that follows per element-iteration."""
    import multiprocessing as mp
    cores = len(os.sched_getaffinity(0))
    n = 16
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(cores) as pool:
        res = pool.map(_oracle_ax_worker, [(n, bm_spec["N"], bm_spec["deform"], bm_spec["seed"], budget_s)] * cores)
    wall = time.perf_counter() - t0
    value = sum(E * N ** 3 / dt for E, N, dt in res) / 1e9
    out = {"value": value, "unit": "GDOF/s", "cores": cores, "kind": "oracle",
           "sample": f"FP64 NumPy oracle Ax on a {n}^3-element N={bm_spec['N']} deformed box (same construction as "
                     f"the workload), one process per core on {cores} cores, one BLAS thread each, "
                     f"{budget_s:.0f} s of repetitions per core, rates summed",
           "host_cpu_count": os.cpu_count(), "affinity_cores": cores, "ax_wall_s": round(wall, 1),
           "ax_ms_per_core": round(float(np.mean([dt for _, _, dt in res])) * 1e3, 2)}
    out["solves"] = oracle_solves()
    return out


def oracle_solves():
    """Oracle solves on the host (BLAS threads on all cores): the tiny
    manufactured problem by assembly + sparse direct solve and by Jacobi-PCG
    to 1e-8, and pMG-FlexCG to 1e-8 on an 8^3-element N=7 deformed box."""
    import scipy.sparse.linalg as spla
    from oracle import operators as ops, pmg as opmg, solvers as osv
    from paper_2110_01716_amd import workloads as wl
    out = {}
    bm = wl.box_mesh(4, N=7)
    G, B, _ = ops.geometric_factors(7, bm.x, bm.y, bm.z)
    b = ops.assemble_rhs(7, B, bm.gid, bm.dirichlet, wl.manufactured_source(bm))
    t0 = time.perf_counter()
    A, ids, _ = ops.assemble(7, G, bm.gid, bm.dirichlet)
    idsall, bu = ops.to_unique(bm.gid, b)
    spla.spsolve(A.tocsc(), bu[np.searchsorted(idsall, ids)])
    out["tiny_4^3_N7_direct_s"] = round(time.perf_counter() - t0, 3)
    dinv = ops.jacobi_inverse(7, G, bm.gid, bm.dirichlet)
    t0 = time.perf_counter()
    res = osv.pcg(lambda v: ops.apply_A(7, G, bm.gid, bm.dirichlet, v), lambda r: dinv * r,
                  lambda x, y: ops.dot(bm.gid, x, y), b, rtol=1e-8)
    out["tiny_4^3_N7_jacobi_pcg_s"] = round(time.perf_counter() - t0, 3)
    out["tiny_4^3_N7_jacobi_pcg_iters"] = res.iters
    bm = wl.box_mesh(8, N=7, deform=0.05, seed=1002)
    t0 = time.perf_counter()
    lv = opmg.build_levels(7, bm.x, bm.y, bm.z, bm.gid, bm.dirichlet)
    out["pmg_8^3_N7_setup_s"] = round(time.perf_counter() - t0, 2)
    b = wl.random_rhs(bm, 2000)
    t0 = time.perf_counter()
    res = opmg.pmg_flexcg(lv, b, opmg.VCycleOpts(), rtol=1e-8)
    solve = time.perf_counter() - t0
    out["pmg_8^3_N7_solve_s"] = round(solve, 2)
    out["pmg_8^3_N7_iters"] = res.iters
    out["pmg_48^3_N7_extrapolated_s"] = round(solve / max(res.iters, 1) / bm.E * 48 ** 3 * 13, 1)
    out["note"] = ("48^3 figure extrapolated per element-iteration at 13 iterations; the measured 48^3 oracle "
                   "solve (build host) is in the header of the sampled-solution file")
    return out


def oracle_timings():
    """Host timings of the FP64 oracle only (no GPU): its Ax with BLAS on all
    host cores, and the oracle solves of cpu_baseline."""
    from oracle import operators as ops
    from paper_2110_01716_amd import workloads as wl
    out = {"cores": os.cpu_count(), "affinity": len(os.sched_getaffinity(0))}
    for n in (4, 16):
        bm = wl.box_mesh(n, N=7, deform=0.05 if n > 4 else 0.0, seed=1000 + n)
        G, _, _ = ops.geometric_factors(7, bm.x, bm.y, bm.z)
        u = np.random.default_rng(0).uniform(-1, 1, bm.x.shape)
        reps, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < 3.0:
            ops.ax_local(7, G, u)
            reps += 1
        dt = (time.perf_counter() - t0) / reps
        out[f"ax_{n}^3_N7_ms"] = round(dt * 1e3, 3)
        out[f"ax_{n}^3_N7_gdofs"] = round(bm.E * 343 / dt / 1e9, 4)
    out.update(oracle_solves())
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--no-c2-solve", action="store_true", help="skip the 64^3 Jacobi-PCG / pMG solves")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--skip-pcg", action="store_true", help="time only the pMG solve")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-projection", action="store_true")
    ap.add_argument("--projection-only", action="store_true")
    ap.add_argument("--oracle-timings", action="store_true", help="host timings of the oracle only (no GPU)")
    ap.add_argument("--solve-repeat", type=int, default=0,
                    help="only the 48^3 FlexCG+pMG solve, this many times, 50 ms apart (for kernel traces)")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--batched-only", action="store_true")
    ap.add_argument("--serving-only", action="store_true")
    ap.add_argument("--solve-only", action="store_true", help="skip the Ax steps (profiling the solve)")
    ap.add_argument("--ax-orders", action="store_true", help="Ax at N = 5, 7, 9 (FP64 and FP32) only")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run a plain 1 GiB device copy first (counter calibration under a profiler)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); this build has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)

    if a.oracle_timings:
        print(json.dumps({"oracle_timings": oracle_timings()}), flush=True)
        return
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
    if a.ax_orders:
        print(json.dumps({"ax_orders": bench_ax_orders(sem, a.steps, a.warmup)}), flush=True)
        return
    if a.batched_only:
        print(json.dumps({"batched": bench_batched(sem)}), flush=True)
        return
    if a.serving_only:
        print(json.dumps({"serving": bench_serving(sem)}), flush=True)
        return
    if a.solve_repeat > 0:
        bm3, m3 = build_mesh(sem, wl.config_meshes()["pmg_48x48x48_N7"])
        p3 = sem.Pmg(m3)
        b3 = torch.from_numpy(wl.random_rhs(bm3, 2000)).to("cuda")
        x3 = torch.empty_like(b3)
        times = []
        for _ in range(a.solve_repeat):
            torch.cuda.synchronize()
            time.sleep(0.05)  # separates the solves in a trace
            t = time.perf_counter()
            info = sem.sem_pcg_solve(m3.h, p3.h, b3, x3, sem.solve_opts(rtol=1e-8))
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t)
            log("solve", info["iters"], info["coarse_iters"], round(times[-1], 5))
        print(json.dumps({"solve_repeat": {"seconds": times, "iters": info["iters"]}}), flush=True)
        return
    if a.projection_only:
        bm3, m3 = build_mesh(sem, wl.config_meshes()["pmg_48x48x48_N7"])
        print(json.dumps({"projection": bench_projection(sem, bm3, m3)}), flush=True)
        return
    if a.solve_only:
        spec3 = wl.config_meshes()["pmg_48x48x48_N7"]
        bm3, m3 = build_mesh(sem, spec3)
        print(json.dumps({"poisson": {"48x48x48_N7": solve_pair(sem, bm3, m3, "c3", a.skip_pcg,
                                                                samples=load_xstar_samples(spec3["n"]))}}),
              flush=True)
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
                     "frac": round(gbs / HBM_PEAK_GBS, 4),
                     "traffic": (AX_COUNTERS["traffic_GB_per_launch"]
                                 if ax_source_sha16() == AX_COUNTERS["source_sha16"] else None),
                     "traffic_unit": "GB per launch (algorithmic: %.3f)" % (bytes_per_launch / 1e9),
                     "kernel": "k_ax<7,double>", "bytes_per_point": 64},
    }
    log("ax", res["ax"])
    hw, hms = time_ax(sem, m, E, Np, a.steps, a.warmup, lam=10.0)
    hms_avg = float(np.mean(hms))
    hgbs = 72 * E * Np / (hms_avg * 1e-3) / 1e9
    res["helmholtz_ax"] = {"ms_mean": round(hms_avg, 4), "ms_median": round(float(np.median(hms)), 4),
                           "hbm_gbs": round(hgbs, 1), "frac": round(hgbs / HBM_PEAK_GBS, 4), "bytes_per_point": 72,
                           "kernel": "k_ax<7,double,helmholtz>"}
    log("helmholtz ax", res["helmholtz_ax"])
    st = time_stream(sem, E * Np, a.steps, a.warmup)
    log("stream", st)
    rl = res["roofline"]
    rl["realizable"] = {"probe": "sem_stream (k_stream<n_in>), FP64, %d elements per array" % st["elements"],
                        "copy_GBs": st["copy"]["GBs"], "triad_GBs": st["triad"]["GBs"],
                        "ax_mix_7r1w_GBs": st["ax_mix_7r1w"]["GBs"],
                        "triad_frac_of_peak": round(st["triad"]["GBs"] / HBM_PEAK_GBS, 4),
                        "ax_frac_of_triad": round(gbs / st["triad"]["GBs"], 4),
                        "ax_frac_of_mix": round(gbs / st["ax_mix_7r1w"]["GBs"], 4)}
    if not a.no_solve:
        poisson = {}
        if not a.no_c2_solve:
            # config 2: FP64 Jacobi-PCG to 1e-8 on the Ax mesh, beside the FP32-pMG solve
            poisson["64x64x64_N7"] = solve_pair(sem, bm, m, "c2", samples=None, smoothers=False, pcg_rtols=(1e-8,))
        m.close()
        del bm
        spec3 = wl.config_meshes()["pmg_48x48x48_N7"]
        bm3, m3 = build_mesh(sem, spec3)
        poisson["48x48x48_N7"] = solve_pair(sem, bm3, m3, "c3", a.skip_pcg, samples=load_xstar_samples(spec3["n"]))
        poisson["48x48x48_N7"]["helmholtz_jacobi_pcg"] = bench_helmholtz_solve(sem, bm3, m3)
        if not a.no_projection:
            poisson["48x48x48_N7"]["projection"] = bench_projection(sem, bm3, m3)
        m3.close()
        res["poisson"] = poisson
    if not a.no_batched:
        res["batched"] = bench_batched(sem)
        log("batched", res["batched"])
    if not a.no_serving:
        res["serving"] = bench_serving(sem)
    if not a.no_cpu:
        res["cpu_baseline"] = cpu_baseline(spec)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
