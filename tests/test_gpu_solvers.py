"""GPU parity of the solvers through the C ABI: Jacobi-PCG, the pMG hierarchy
(coarse geometry and IDs, transfers, rho), one V-cycle in FP64 and FP32,
pMG-preconditioned flexible CG, error paths, and batched / continuous-batching
solves (each result identical to its solve alone)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import operators as ops
from oracle import pmg as opmg
from paper_2110_01716_amd import workloads as wl

from gpu_util import dev, host, print_case, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sem():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    from paper_2110_01716_amd import sem as s
    s.load()
    return s


def direct_solution(bm, b):
    G, _, _ = ops.geometric_factors(bm.N, bm.x, bm.y, bm.z)
    A, ids, _ = ops.assemble(bm.N, G, bm.gid, bm.dirichlet)
    idsall, bu = ops.to_unique(bm.gid, b)
    xin = spla.spsolve(A.tocsc(), bu[np.searchsorted(idsall, ids)])
    return ops.scatter_unique(bm.gid, ids, xin)


def gpu_rhs_manufactured(sem, m, bm):
    import torch
    f = dev(wl.manufactured_source(bm))
    b = torch.empty_like(f)
    sem.sem_mass(m.h, f, b)
    sem.sem_gs(m.h, b, apply_mask=True)
    return b


def test_jacobi_pcg_tiny_manufactured(sem):
    """4^3 undeformed elements, N=7, manufactured RHS, FP64 Jacobi-PCG to 1e-8."""
    import torch
    print_case("pcg-tiny")
    bm = wl.box_mesh(4, N=7)
    m = sem.Mesh.from_box(bm)
    b = gpu_rhs_manufactured(sem, m, bm)
    x = torch.empty_like(b)
    info = sem.sem_pcg_solve(m.h, None, b, x, sem.solve_opts(rtol=1e-8))
    assert info["status"] == 0 and info["relres"] <= 1e-8
    assert info["relres_true"] <= 2e-8
    G, B, _ = ops.geometric_factors(7, bm.x, bm.y, bm.z)
    bo = ops.assemble_rhs(7, B, bm.gid, bm.dirichlet, wl.manufactured_source(bm))
    xs = direct_solution(bm, bo)
    xg = host(x)
    err_1e8 = rel_err(xg, xs)
    assert err_1e8 <= 1e-7
    # spectral accuracy of the discrete solution itself
    assert np.max(np.abs(xg - wl.manufactured_solution(bm))) < 1e-5
    # the solution itself to 1e-8 relative against the oracle's direct solve
    info = sem.sem_pcg_solve(m.h, None, b, x, sem.solve_opts(rtol=1e-10))
    assert info["status"] == 0 and info["relres_true"] <= 2e-10
    err = rel_err(host(x), xs)
    print(f"tiny manufactured: error {err_1e8:.2e} at rtol 1e-8, {err:.2e} at rtol 1e-10", flush=True)
    assert err <= 1e-8


def test_jacobi_pcg_matches_oracle_iterates(sem):
    import torch
    from oracle import solvers
    print_case("pcg-iterates")
    bm = wl.box_mesh(3, 2, 3, N=5, deform=0.05, seed=3)
    m = sem.Mesh.from_box(bm)
    b = wl.random_rhs(bm, 4)
    bd = dev(b)
    x = torch.empty_like(bd)
    info = sem.sem_pcg_solve(m.h, None, bd, x, sem.solve_opts(fixed_iters=25))
    assert info["iters"] == 25
    G, _, _ = ops.geometric_factors(5, bm.x, bm.y, bm.z)
    dinv = ops.jacobi_inverse(5, G, bm.gid, bm.dirichlet)
    res = solvers.pcg(lambda v: ops.apply_A(5, G, bm.gid, bm.dirichlet, v), lambda r: dinv * r,
                      lambda a, c: ops.dot(bm.gid, a, c), b, fixed_iters=25)
    assert rel_err(host(x), res.x) <= 1e-10
    assert abs(info["relres"] - res.relres) <= 1e-8 * res.relres


def test_solver_error_paths(sem):
    import torch
    print_case("errors")
    bm = wl.box_mesh(2, N=3, deform=0.05, seed=1)
    m = sem.Mesh.from_box(bm)
    zero = torch.zeros((bm.E, bm.Np), dtype=torch.float64, device="cuda")
    x = torch.full_like(zero, 5.0)
    info = sem.sem_pcg_solve(m.h, None, zero, x)
    assert info["status"] == 0 and info["iters"] == 0 and float(x.abs().max()) == 0.0
    b = dev(wl.random_rhs(bm, 1))
    b[0, 3] = float("nan")
    info = sem.sem_pcg_solve(m.h, None, b, x, check=False)
    assert info["rc"] == sem.SEM_ENAN
    b = dev(wl.random_rhs(bm, 1))
    info = sem.sem_pcg_solve(m.h, None, b, x, sem.solve_opts(maxit=3), check=False)
    assert info["rc"] == sem.SEM_ENOCONV and info["iters"] == 3


def _levels_oracle(bm, rho=None):
    return opmg.build_levels(bm.N, bm.x, bm.y, bm.z, bm.gid, bm.dirichlet, rho=rho)


HIERARCHIES = {5: [5, 2, 1], 7: [7, 3, 1], 9: [9, 4, 1]}


@pytest.mark.parametrize("N", [5, 7, 9])
def test_pmg_hierarchy_matches_oracle(sem, N):
    import torch
    from oracle import solvers
    from oracle.counter_rng import start_vector
    print_case("pmg-hierarchy", N)
    bm = wl.box_mesh(3, 2, 2, N=N, deform=0.05, seed=6)
    m = sem.Mesh.from_box(bm)
    p = sem.Pmg(m)
    info = p.info()
    assert info["orders"] == HIERARCHIES[N]
    lv = _levels_oracle(bm)
    # fine-level rho from the same splitmix64 start vector
    assert abs(info["rho"][0] - lv[0].rho) <= 1e-10 * lv[0].rho
    for l in (1, 2):
        h = p.level(l)
        o = lv[l]
        n = o.x.size
        xs = [torch.empty(o.x.shape, dtype=torch.float64, device="cuda") for _ in range(3)]
        gid = torch.empty(o.x.shape, dtype=torch.int64, device="cuda")
        dr = torch.empty(o.x.shape, dtype=torch.uint8, device="cuda")
        sem.sem_mesh_export_nodes(h, xs[0], xs[1], xs[2], gid, dr)
        for a, b in zip(xs, (o.x, o.y, o.z)):
            assert rel_err(host(a), b) <= 1e-13
        g = host(gid)
        pairs = np.unique(np.stack([g.ravel(), o.gid.ravel()], 1), axis=0)
        assert len(pairs) == len(np.unique(g)) == len(np.unique(o.gid))
        np.testing.assert_array_equal(host(dr), o.dirichlet)
        assert info["n_unique"][l] == len(np.unique(o.gid))
        # coarse geometric factors and diagonal
        G = torch.empty((bm.E, 6, o.x.shape[1]), dtype=torch.float64, device="cuda")
        D = torch.empty(o.x.shape, dtype=torch.float64, device="cuda")
        sem.sem_mesh_export(h, G, None, D)
        assert rel_err(host(G), o.G) <= 1e-12
        assert rel_err(host(D), o.dinv) <= 1e-12
        del n
        if l == 1:
            # smoothed coarse level: the oracle's power iteration on its own
            # operator, started from the splitmix64 vector of the GPU's coarse IDs
            v0 = ops.mask(o.dirichlet, start_vector(g))
            rho_o = solvers.power_rho(o.A, o.dinv, o.dot, v0, iters=20)
            assert abs(info["rho"][1] - rho_o) <= 1e-9 * rho_o


def test_pmg_coarse_ids_on_relabelled_mesh(sem):
    print_case("pmg-relabel")
    bm = wl.box_mesh(2, 3, 2, N=7, deform=0.05, seed=7)
    rb = wl.relabel(bm, 5)
    m = sem.Mesh.from_box(rb)
    p = sem.Pmg(m, rho_override=[2.0, 2.0])
    info = p.info()
    assert info["n_unique"][1] == (2 * 3 + 1) * (3 * 3 + 1) * (2 * 3 + 1)
    assert info["n_unique"][2] == 3 * 4 * 3


@pytest.mark.parametrize("N", [5, 7, 9])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_transfers_match_oracle(sem, dtype, N):
    import torch
    print_case("transfers", dtype, N)
    bm = wl.box_mesh(2, 3, 2, N=N, deform=0.05, seed=8)
    m = sem.Mesh.from_box(bm)
    p = sem.Pmg(m, smoother_dtype=dtype, rho_override=[2.0, 2.0])
    lv = _levels_oracle(bm, rho=[2.0, 2.0])
    tf = torch.float32 if dtype == "f32" else torch.float64
    tol = 2e-6 if dtype == "f32" else 1e-13
    rng = np.random.default_rng(0)
    for l in (0, 1):
        tc = torch.float64 if l == 1 else tf
        f, c = lv[l], lv[l + 1]
        rf = ops.mask(f.dirichlet, ops.gs(f.gid, rng.uniform(-1, 1, f.x.shape)) / f.mult)
        out = torch.zeros(c.x.shape, dtype=tc, device="cuda")
        sem.sem_pmg_transfer(p.h, l, 1, dev(rf, tf), out)
        assert rel_err(host(out), opmg.restrict(lv, l, rf)) <= tol
        zc = ops.mask(c.dirichlet, ops.gs(c.gid, rng.uniform(-1, 1, c.x.shape)) / c.mult)
        base = rng.uniform(-1, 1, f.x.shape)
        xf = dev(base, tf)
        sem.sem_pmg_transfer(p.h, l, 0, dev(zc, tc), xf)
        assert rel_err(host(xf), base + opmg.prolong(lv, l, zc)) <= tol


def _vcycle_case(sem, dtype, coarse_iters=6, N=7):
    import torch
    bm = wl.box_mesh(3, 2, 3, N=N, deform=0.05, seed=9)
    lv = _levels_oracle(bm)
    rho = [lv[0].rho, lv[1].rho]
    m = sem.Mesh.from_box(bm)
    p = sem.Pmg(m, smoother_dtype=dtype, rho_override=rho, coarse_fixed_iters=coarse_iters)
    r = wl.random_rhs(bm, 12)
    z = torch.zeros((bm.E, bm.Np), dtype=torch.float64, device="cuda")
    sem.sem_pmg_apply(p.h, dev(r), z)
    o = opmg.VCycleOpts(coarse_fixed_iters=coarse_iters)
    zo = opmg.vcycle(lv, r, o)
    return host(z), zo


@pytest.mark.parametrize("N", [5, 7, 9])
def test_vcycle_fp64_matches_oracle(sem, N):
    print_case("vcycle-f64", N)
    z, zo = _vcycle_case(sem, "f64", N=N)
    assert rel_err(z, zo) <= 1e-12


@pytest.mark.parametrize("N", [5, 7, 9])
def test_vcycle_fp32_matches_oracle(sem, N):
    print_case("vcycle-f32", N)
    z, zo = _vcycle_case(sem, "f32", N=N)
    assert rel_err(z, zo) <= 1e-5


@pytest.mark.parametrize("dtype,N", [("f32", 7), ("f64", 7), ("f32", 5), ("f32", 9)])
def test_pmg_flexcg_solution(sem, dtype, N):
    import torch
    print_case("flexcg", dtype, N)
    bm = wl.box_mesh(3, 3, 2, N=N, deform=0.05, seed=10)
    m = sem.Mesh.from_box(bm)
    p = sem.Pmg(m, smoother_dtype=dtype)
    b = wl.random_rhs(bm, 2)
    bd = dev(b)
    x = torch.empty_like(bd)
    info = sem.sem_pcg_solve(m.h, p.h, bd, x, sem.solve_opts(rtol=1e-10))
    assert info["status"] == 0 and info["iters"] < 40
    xs = direct_solution(bm, b)
    assert rel_err(host(x), xs) <= 1e-8
    assert info["relres_true"] <= 1e-9
    assert info["coarse_iters"] > 0


@pytest.mark.parametrize("smoother", ["jacobi", "ras"])
def test_pmg_anisotropic_strongly_deformed(sem, smoother):
    """Elements stretched 8:1 (a 1 x 1 x 8 box cut into 4 x 4 x 4 elements)
    and deformed so that the Jacobian determinant varies 6.7-fold over the
    mesh: a harder operator for the FP32 smoothing and the point-Jacobi /
    Schwarz smoothers (pMG with Chebyshev-Jacobi needs about 90 iterations
    here instead of 13). The FP32-pMG solve still reaches the oracle's direct
    solution to 1e-8, and so does Jacobi-PCG, in more iterations."""
    import torch
    print_case("anisotropic", smoother)
    bm = wl.box_mesh(4, 4, 4, N=7, deform=0.12, seed=21, hi=(1.0, 1.0, 8.0))
    m = sem.Mesh.from_box(bm)
    p = sem.Pmg(m, smoother=smoother)
    b = wl.random_rhs(bm, 22)
    bd = dev(b)
    xs = direct_solution(bm, b)
    x = torch.empty_like(bd)
    info = sem.sem_pcg_solve(m.h, p.h, bd, x, sem.solve_opts(rtol=1e-10, maxit=300))
    assert info["status"] == 0, info
    assert info["relres_true"] <= 1e-9
    assert rel_err(host(x), xs) <= 1e-8
    xj = torch.empty_like(bd)
    ij = sem.sem_pcg_solve(m.h, None, bd, xj, sem.solve_opts(rtol=1e-11, maxit=20000))
    print(f"anisotropic {smoother}: pMG {info['iters']} iterations, Jacobi-PCG {ij['iters']}", flush=True)
    assert ij["status"] == 0 and ij["iters"] > info["iters"]
    assert rel_err(host(xj), xs) <= 1e-8
    p.close()


@pytest.mark.parametrize("shape", [(3, 2, 1), (1, 1, 1)])
@pytest.mark.parametrize("smoother", ["jacobi", "ras"])
def test_pmg_single_layer_mesh(sem, smoother, shape):
    """Degenerate hierarchy: one element across z (or a single element), so
    every node of the N=1 coarse level lies on the Dirichlet boundary and the
    coarse system is empty. The coarse correction is zero and the smoothers
    carry the solve; a single element also has no shared nodes at all."""
    import torch
    print_case("single-layer", smoother, shape)
    bm = wl.box_mesh(*shape, N=7, deform=0.05, seed=12)
    m = sem.Mesh.from_box(bm)
    p = sem.Pmg(m, smoother=smoother)
    b = wl.random_rhs(bm, 3)
    bd = dev(b)
    x = torch.empty_like(bd)
    info = sem.sem_pcg_solve(m.h, p.h, bd, x, sem.solve_opts(rtol=1e-10, maxit=200))
    assert info["status"] == 0, info
    assert rel_err(host(x), direct_solution(bm, b)) <= 1e-8


def test_batched_equals_alone_bitwise(sem):
    import torch
    print_case("batched")
    specs = [(2, 5, 1), (3, 7, 2), (2, 9, 3), (3, 5, 4)]
    meshes, pmgs, bs, xs_alone, xs_batch = [], [], [], [], []
    for n, N, seed in specs:
        bm = wl.box_mesh(n, N=N, deform=0.05, seed=1000 + seed)
        m = sem.Mesh.from_box(bm)
        meshes.append(m)
        pmgs.append(sem.Pmg(m))
        bs.append(dev(wl.random_rhs(bm, 2000 + seed)))
        xs_alone.append(torch.empty_like(bs[-1]))
        xs_batch.append(torch.empty_like(bs[-1]))
    alone = []
    for m, p, b, x in zip(meshes, pmgs, bs, xs_alone):
        alone.append(sem.sem_pcg_solve(m.h, p.h, b, x, sem.solve_opts(rtol=1e-8)))
    rc, infos = sem.sem_pcg_solve_batched([m.h for m in meshes], [p.h for p in pmgs], bs, xs_batch,
                                          sem.solve_opts(rtol=1e-8))
    assert rc == 0
    for a, bi, xa, xb in zip(alone, infos, xs_alone, xs_batch):
        assert a["iters"] == bi["iters"]
        assert torch.equal(xa, xb)
    # launch counts: every solve queues kernels; the batched call shares one
    # launch per phase among the problems in flight, so it queues fewer than
    # the solves one by one, and no problem finishes after the whole call
    assert all(a["launches"] > 0 for a in alone) and all(i["launches"] > 0 for i in infos)
    total = max(i["launches"] for i in infos)
    assert max(a["launches"] for a in alone) <= total < sum(a["launches"] for a in alone)


def test_batched_mixed_coarse_tolerances_equal_alone(sem):
    """Hierarchies with different coarse tolerances in one batched call: each
    problem is solved with its own (bitwise equal to its solve alone)."""
    import torch
    print_case("batched-coarse-rtol")
    bm = wl.box_mesh(3, N=5, deform=0.05, seed=1007)
    m = sem.Mesh.from_box(bm)
    pa, pb = sem.Pmg(m, coarse_rtol=1e-2), sem.Pmg(m, coarse_rtol=1e-6)
    b = dev(wl.random_rhs(bm, 2007))
    o = sem.solve_opts(rtol=1e-8)
    xa, xb = torch.empty_like(b), torch.empty_like(b)
    ia = sem.sem_pcg_solve(m.h, pa.h, b, xa, o)
    ib = sem.sem_pcg_solve(m.h, pb.h, b, xb, o)
    assert ia["coarse_iters"] != ib["coarse_iters"]  # the tolerances do differ in effect
    ya, yb = torch.empty_like(b), torch.empty_like(b)
    rc, infos = sem.sem_pcg_solve_batched([m.h, m.h], [pa.h, pb.h], [b, b], [ya, yb], o)
    assert rc == 0
    assert [i["coarse_iters"] for i in infos] == [ia["coarse_iters"], ib["coarse_iters"]]
    assert torch.equal(ya, xa) and torch.equal(yb, xb)
    pa.close()
    pb.close()


def test_batched_solutions_match_oracle(sem):
    """The batched configuration's problem mix (N = 5, 7 and 9, hierarchies
    5->2->1, 7->3->1, 9->4->1, deformed boxes of different sizes) solved in
    one batched call by FP64 flexible CG + FP32 pMG at rtol 1e-10: every
    solution within 1e-8 of the oracle's direct solve."""
    import torch
    print_case("batched-oracle")
    specs = [(2, 5, 11), (3, 7, 12), (2, 9, 13), (3, 5, 14), (1, 9, 15), (2, 7, 16)]
    bms = [wl.box_mesh(n, N=N, deform=0.05, seed=1000 + sd) for n, N, sd in specs]
    meshes = [sem.Mesh.from_box(bm) for bm in bms]
    pmgs = [sem.Pmg(m) for m in meshes]
    bh = [wl.random_rhs(bm, 2000 + k) for k, bm in enumerate(bms)]
    bs = [dev(b) for b in bh]
    xs = [torch.empty_like(b) for b in bs]
    rc, infos = sem.sem_pcg_solve_batched([m.h for m in meshes], [p.h for p in pmgs], bs, xs,
                                          sem.solve_opts(rtol=1e-10))
    assert rc == 0
    for bm, b, x, info in zip(bms, bh, xs, infos):
        assert info["status"] == 0 and info["relres_true"] <= 1.05e-10
        assert rel_err(host(x), direct_solution(bm, b)) <= 1e-8, (bm.N, bm.E)


def test_continuous_batching_equals_alone(sem):
    import torch
    print_case("continuous")
    bms = [wl.box_mesh(n, N=7, deform=0.05, seed=1000 + n) for n in (2, 3, 4)]
    meshes = [sem.Mesh.from_box(bm) for bm in bms]
    pmgs = [sem.Pmg(m) for m in meshes]
    bs = [dev(wl.random_rhs(bm, 7 + k)) for k, bm in enumerate(bms)]
    alone = [torch.empty_like(b) for b in bs]
    for m, p, b, x in zip(meshes, pmgs, bs, alone):
        sem.sem_pcg_solve(m.h, p.h, b, x)
    mixed = [torch.empty_like(b) for b in bs]
    B = sem.sem_batch_create(2)
    s0 = sem.sem_batch_add(B, meshes[0].h, pmgs[0].h, bs[0], mixed[0])
    s1 = sem.sem_batch_add(B, meshes[1].h, pmgs[1].h, bs[1], mixed[1])
    sem.sem_batch_step(B, 3)
    with pytest.raises(sem.SemError):
        sem.sem_batch_add(B, meshes[2].h, pmgs[2].h, bs[2], mixed[2])
    done = {}
    pending = [2]
    slots = {s0: 0, s1: 1}
    for _ in range(200):
        n = sem.sem_batch_step(B, 1)
        for s, k in list(slots.items()):
            info = sem.sem_batch_poll(B, s)
            if info["status"] != sem.RUNNING:
                done[k] = info
                sem.sem_batch_release(B, s)
                del slots[s]
                if pending:
                    kk = pending.pop()
                    slots[sem.sem_batch_add(B, meshes[kk].h, pmgs[kk].h, bs[kk], mixed[kk])] = kk
        if not slots:
            break
    sem.sem_batch_destroy(B)
    assert sorted(done) == [0, 1, 2]
    for k in range(3):
        assert done[k]["status"] == 0
        assert torch.equal(alone[k], mixed[k])


@pytest.mark.parametrize("degree,pre,post", [(1, 1, 1), (3, 1, 1), (2, 2, 1), (2, 1, 0), (2, 0, 1), (3, 2, 2)])
def test_vcycle_schedules_match_oracle(sem, degree, pre, post):
    """Every Chebyshev degree / sweep-count combination of the V-cycle (the
    fused first and last smoothing steps and the folded precision
    conversions) against the oracle, FP64 smoothing, fixed coarse iterations."""
    import torch
    print_case("vcycle-schedule", degree, pre, post)
    bm = wl.box_mesh(4, 3, 3, N=5, deform=0.05, seed=19)  # 12 coarse DOFs: no exact CG breakdown in 5 steps
    lv = _levels_oracle(bm)
    rho = [lv[0].rho, lv[1].rho]
    m = sem.Mesh.from_box(bm)
    p = sem.Pmg(m, smoother_dtype="f64", rho_override=rho, coarse_fixed_iters=5, cheb_degree=degree, pre=pre,
                post=post)
    r = wl.random_rhs(bm, 21)
    z = torch.zeros((bm.E, bm.Np), dtype=torch.float64, device="cuda")
    sem.sem_pmg_apply(p.h, dev(r), z)
    zo = opmg.vcycle(lv, r, opmg.VCycleOpts(degree=degree, pre=pre, post=post, coarse_fixed_iters=5))
    assert rel_err(host(z), zo) <= 1e-11
    # FP32 smoothing: same schedule within single-precision rounding
    p32 = sem.Pmg(m, smoother_dtype="f32", rho_override=rho, coarse_fixed_iters=5, cheb_degree=degree, pre=pre,
                  post=post)
    z32 = torch.zeros_like(z)
    sem.sem_pmg_apply(p32.h, dev(r), z32)
    assert rel_err(host(z32), zo) <= 2e-5
