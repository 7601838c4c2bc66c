"""Write sampled values of the FP64 oracle's solution of a deformed-box Poisson
problem, for solution-error checks at sizes where the oracle cannot run inside
a test or a benchmark.

    python tests/golden/make_oracle_solution_samples.py [--n 48] [--samples 2000]

Calls only the oracle (oracle/) and the seeded input generators
(paper_2110_01716_amd/workloads.py). The problem is the mixed-precision
workload's: n^3 hex elements, N = 7, unit box deformed with seeded phases
(mesh seed 1002), homogeneous Dirichlet boundary, right-hand side seeded
uniform [-1, 1] (seed 2000). x* is the oracle's FP64 flexible CG preconditioned
by its FP64 p-multigrid V-cycle (7 -> 3 -> 1, Chebyshev-Jacobi degree 2,
coarse Jacobi-PCG to 1e-2), run to relative residual 1e-12.

Output (text): a header with the recipe, the iteration count, the final
relative residual and global statistics of x* over unique DOFs (max |x*|,
the unique-DOF 2-norm), then one line per sample: the local index
e * (N+1)^3 + p of a non-Dirichlet node, and x* there to 17 significant digits.
Samples are distinct unique DOFs chosen by a seeded generator.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import operators as ops, pmg as opmg  # noqa: E402
from paper_2110_01716_amd import workloads as wl  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=48)
    ap.add_argument("--samples", type=int, default=2000)
    ap.add_argument("--rtol", type=float, default=1e-12)
    ap.add_argument("--sample-seed", type=int, default=7001)
    a = ap.parse_args()
    N, mesh_seed, rhs_seed = 7, 1002, 2000
    t0 = time.time()
    bm = wl.box_mesh(a.n, N=N, deform=0.05, seed=mesh_seed)
    b = wl.random_rhs(bm, rhs_seed)
    lv = opmg.build_levels(N, bm.x, bm.y, bm.z, bm.gid, bm.dirichlet)
    t_setup = time.time() - t0
    print(f"setup {t_setup:.1f}s rho={[lv_.rho for lv_ in lv[:-1]]}", flush=True)
    t0 = time.time()
    res = opmg.pmg_flexcg(lv, b, opmg.VCycleOpts(), rtol=a.rtol, maxit=100)
    t_solve = time.time() - t0
    print(f"solve {t_solve:.1f}s iters={res.iters} relres={res.relres:.3e}", flush=True)
    x = res.x
    # true residual, unique-DOF norms
    r = b - lv[0].A(x)
    relres_true = np.sqrt(ops.dot(bm.gid, r, r) / ops.dot(bm.gid, b, b))
    xnorm = np.sqrt(ops.dot(bm.gid, x, x))
    xmax = float(np.max(np.abs(x)))
    # distinct unique DOFs: the first copy (in local order) of each global ID
    flat_gid = bm.gid.ravel()
    _, first = np.unique(flat_gid, return_index=True)
    free = first[bm.dirichlet.ravel()[first] == 0]
    rng = np.random.default_rng(a.sample_seed)
    pick = np.sort(rng.choice(free, size=a.samples, replace=False))
    out = os.path.join(HERE, f"pmg_{a.n}x{a.n}x{a.n}_N{N}_rhs{rhs_seed}_xstar_samples.txt")
    with open(out, "w") as f:
        f.write("# Sampled FP64 oracle solution x* of a deformed-box Poisson problem.\n")
        f.write(f"# Written by tests/golden/make_oracle_solution_samples.py --n {a.n} "
                f"--samples {a.samples} --rtol {a.rtol:g} --sample-seed {a.sample_seed}\n")
        f.write(f"# mesh: box_mesh({a.n}, N={N}, deform=0.05, seed={mesh_seed}); rhs: random_rhs(seed={rhs_seed})\n")
        f.write("# solver: oracle pmg_flexcg, levels 7->3->1, Chebyshev-Jacobi degree 2 (1+1 sweeps), "
                "coarse Jacobi-PCG to 1e-2, all FP64\n")
        f.write(f"# iters {res.iters}\n# relres_recurrence {res.relres:.6e}\n# relres_true {relres_true:.6e}\n")
        f.write(f"# xstar_max_abs {xmax:.17e}\n# xstar_norm2_unique {xnorm:.17e}\n")
        f.write(f"# n_unique {len(first)}\n# samples {a.samples}\n")
        f.write(f"# oracle_setup_s {t_setup:.1f}\n# oracle_solve_s {t_solve:.1f}\n"
                f"# host_cores {len(os.sched_getaffinity(0))}\n")
        f.write("# local_index value\n")
        for i in pick:
            f.write(f"{int(i)} {x.ravel()[i]:.17e}\n")
    print(f"wrote {out} (setup {t_setup:.0f}s, solve {t_solve:.0f}s)", flush=True)


if __name__ == "__main__":
    main()
