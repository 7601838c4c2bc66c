"""Helpers shared by the GPU tests (host <-> device copies, oracle setups)."""
import numpy as np

from oracle import operators as ops


def dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda").contiguous()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().to("cpu").numpy()


def empty_like_np(a, dtype=None):
    import torch
    dt = dtype or torch.float64
    return torch.empty(a.shape, dtype=dt, device="cuda")


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def oracle_setup(bm):
    G, B, detJ = ops.geometric_factors(bm.N, bm.x, bm.y, bm.z)
    return G, B, detJ


def print_case(*parts):
    print("CASE", *parts, flush=True)
