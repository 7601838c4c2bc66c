"""Checks of the seeded input generators (shapes, IDs, flags, determinism)."""
import numpy as np

from paper_2110_01716_amd import workloads as wl


def test_box_mesh_counts_and_ids():
    m = wl.box_mesh(4, N=7)
    assert m.x.shape == (64, 512) and m.gid.dtype == np.int64
    assert len(np.unique(m.gid)) == 29 ** 3
    # interior unique nodes
    ids, first = np.unique(m.gid.ravel(), return_index=True)
    assert np.sum(m.dirichlet.ravel()[first] == 0) == 27 ** 3
    # copies of a node share coordinates bitwise
    for c in (m.x, m.y, m.z):
        _, inv = np.unique(m.gid.ravel(), return_inverse=True)
        mn = np.full(len(ids), np.inf)
        mx = np.full(len(ids), -np.inf)
        np.minimum.at(mn, inv, c.ravel())
        np.maximum.at(mx, inv, c.ravel())
        assert np.all(mn == mx)


def test_deformed_mesh_consistent_and_seeded():
    a = wl.box_mesh(3, N=5, deform=0.05, seed=4)
    b = wl.box_mesh(3, N=5, deform=0.05, seed=4)
    c = wl.box_mesh(3, N=5, deform=0.05, seed=5)
    assert np.array_equal(a.x, b.x) and not np.array_equal(a.x, c.x)
    ids, inv = np.unique(a.gid.ravel(), return_inverse=True)
    mn = np.full(len(ids), np.inf)
    mx = np.full(len(ids), -np.inf)
    np.minimum.at(mn, inv, a.y.ravel())
    np.maximum.at(mx, inv, a.y.ravel())
    assert np.all(mn == mx)


def test_random_rhs_consistent_masked():
    m = wl.box_mesh(3, N=3, deform=0.05, seed=1)
    b = wl.random_rhs(m, 7)
    assert np.all(b[m.dirichlet != 0] == 0)
    assert np.all(np.abs(b) <= 1)
    _, inv = np.unique(m.gid.ravel(), return_inverse=True)
    s = np.zeros(inv.max() + 1)
    np.maximum.at(s, inv, b.ravel())
    assert np.allclose(s[inv], np.maximum(b.ravel(), s[inv]))
    assert np.array_equal(b, wl.random_rhs(m, 7))


def test_relabel_preserves_structure():
    m = wl.box_mesh(2, N=3)
    r = wl.relabel(m, 3)
    assert np.array_equal(r.x, m.x[r.meta["perm"]])
    assert len(np.unique(r.gid)) == len(np.unique(m.gid))


def test_named_workloads():
    cfg = wl.config_meshes()
    assert cfg["ax_64x64x64_N7"]["n"] == 64
    specs = wl.batched_problem_specs()
    assert len(specs) == 256 and {s["N"] for s in specs} == {5, 7, 9}
    assert wl.serving_mesh_sides() == [8, 10, 12, 14, 17, 19, 21, 23, 25, 27, 29, 31, 34, 36, 38, 40]


def test_rhs_sequence_consistent_masked_and_device_path():
    import torch
    m = wl.box_mesh(3, 2, 2, N=4, deform=0.05, seed=3)
    seq = wl.rhs_sequence(m, 3, modes=4, noise=1e-2, seed=5)
    order = np.argsort(m.gid.ravel(), kind="stable")
    for b in seq:
        v = b.ravel()[order]
        g = m.gid.ravel()[order]
        same = g[1:] == g[:-1]
        assert np.all(v[1:][same] == v[:-1][same])  # every copy of a node equal
        assert np.all(b[m.dirichlet != 0] == 0)
        assert np.max(np.abs(b)) > 0.1
    at = wl.rhs_sequence_fn(m, modes=4, noise=1e-2, seed=5, device="cpu")
    for k, b in enumerate(seq):
        assert np.max(np.abs(at(k).numpy() - b)) <= 1e-13
    # consecutive steps are close, distant ones are not
    d1 = np.max(np.abs(seq[1] - seq[0]))
    assert d1 < 0.5 * np.max(np.abs(seq[0]))


def test_rotate_elements_keeps_the_mesh():
    from oracle import operators as ops
    m = wl.box_mesh(3, 2, 2, N=3, deform=0.05, seed=2)
    r = wl.rotate_elements(m, 5)
    assert len(set(r.meta["rot"].tolist())) > 4
    _, _, detJ = ops.geometric_factors(3, r.x, r.y, r.z)
    assert detJ.min() > 0
    for e in range(m.E):
        assert sorted(m.gid[e]) == sorted(r.gid[e])
        order = np.argsort(r.gid[e])
        assert np.array_equal(r.x[e][order], m.x[e][np.argsort(m.gid[e])])


def test_oracle_solution_samples_file():
    """The stored oracle samples of the 48^3 mixed-precision workload are
    well formed: 2000 distinct local indices inside the mesh, the oracle's
    true residual at 1e-12, and max |x*| at least every sampled |x*|."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        "pmg_48x48x48_N7_rhs2000_xstar_samples.txt")
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
    idx = np.array(idx)
    assert len(idx) == int(meta["samples"]) == 2000
    assert np.all(np.diff(idx) > 0) and idx[0] >= 0 and idx[-1] < 48 ** 3 * 512
    assert meta["relres_true"] <= 1e-12
    assert int(meta["n_unique"]) == (48 * 7 + 1) ** 3
    assert np.max(np.abs(val)) <= meta["xstar_max_abs"]
