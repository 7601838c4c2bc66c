"""ctypes binding of libsem (the C ABI declared in include/sem.h).

Argument marshalling only: every step of the solve runs in the HIP library.
Device buffers are torch tensors on a ROCm device (torch is used for device
memory and streams); host arrays are numpy arrays. The library must be built
(python -m paper_2110_01716_amd.build_lib); loading fails loudly otherwise.

Functions keep the C names (sem_mesh_create, sem_ax, sem_gs, sem_pmg_setup,
sem_pcg_solve, ...). Small wrapper classes (Mesh, Pmg, Batch) own the handles.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsem.so")

SEM_OK, SEM_EINVAL, SEM_EGEOM, SEM_ENOMEM, SEM_EHIP, SEM_ENOCONV, SEM_ENAN, SEM_EBUSY = 0, -1, -2, -3, -4, -5, -6, -7
SEM_F64, SEM_F32 = 0, 1
RUNNING = 1


class SemError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str):
        super().__init__(f"{where}: {detail} (status {code})")
        self.code = code


class sem_mesh_desc(C.Structure):
    _fields_ = [("N", C.c_int32), ("E", C.c_int64), ("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p),
                ("gid", C.c_void_p), ("dirichlet", C.c_void_p), ("stream", C.c_void_p)]


class sem_mesh_info(C.Structure):
    _fields_ = [("N", C.c_int32), ("E", C.c_int64), ("n_local", C.c_int64), ("n_unique", C.c_int64),
                ("n_interior", C.c_int64), ("n_shared_nodes", C.c_int64), ("n_shared_entries", C.c_int64),
                ("resident_bytes", C.c_int64), ("min_detJ", C.c_double), ("volume", C.c_double)]


class sem_pmg_opts(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("orders", C.c_int32 * 8), ("smoother_dtype", C.c_int),
                ("cheb_degree", C.c_int32), ("pre", C.c_int32), ("post", C.c_int32), ("eig_lo", C.c_double),
                ("eig_hi", C.c_double), ("power_iters", C.c_int32), ("rho_override", C.c_void_p),
                ("coarse_rtol", C.c_double), ("coarse_maxit", C.c_int32), ("coarse_fixed_iters", C.c_int32),
                ("coarse_check_every", C.c_int32), ("smoother", C.c_int32)]


SEM_SMOOTH_CHEB_JACOBI, SEM_SMOOTH_CHEB_ASM, SEM_SMOOTH_CHEB_RAS = 0, 1, 2
_SMOOTHERS = {"jacobi": 0, "asm": 1, "ras": 2, 0: 0, 1: 1, 2: 2}


class sem_pmg_info(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("orders", C.c_int32 * 8), ("rho", C.c_double * 8),
                ("n_unique", C.c_int64 * 8), ("resident_bytes", C.c_int64)]


class sem_solve_opts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("maxit", C.c_int32), ("check_every", C.c_int32),
                ("fixed_iters", C.c_int32), ("lam", C.c_double)]


class sem_solve_info(C.Structure):
    _fields_ = [("iters", C.c_int32), ("status", C.c_int32), ("relres", C.c_double),
                ("relres_true", C.c_double), ("coarse_iters", C.c_int64), ("seconds", C.c_double),
                ("relres_initial", C.c_double), ("launches", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_P = C.c_void_p
_SIGS = {
    "sem_reference": (C.c_int, [C.c_int, _P, _P, _P]),
    "sem_interpolation": (C.c_int, [C.c_int, C.c_int, _P]),
    "sem_mesh_create": (C.c_int, [C.POINTER(sem_mesh_desc), C.POINTER(_P)]),
    "sem_mesh_destroy": (C.c_int, [_P]),
    "sem_mesh_query": (C.c_int, [_P, C.POINTER(sem_mesh_info)]),
    "sem_mesh_export": (C.c_int, [_P, _P, _P, _P, _P]),
    "sem_mesh_export_nodes": (C.c_int, [_P, _P, _P, _P, _P, _P, _P]),
    "sem_ax": (C.c_int, [_P, C.c_int, _P, _P, C.c_int64, C.c_int64, _P]),
    "sem_helmholtz": (C.c_int, [_P, C.c_int, _P, _P, C.c_double, _P]),
    "sem_gs": (C.c_int, [_P, C.c_int, _P, C.c_int, _P]),
    "sem_mass": (C.c_int, [_P, C.c_int, _P, _P, _P]),
    "sem_dot": (C.c_int, [_P, C.c_int, _P, _P, C.POINTER(C.c_double), _P]),
    "sem_dot_noalloc": (C.c_int, [_P, C.c_int, _P, _P, C.POINTER(C.c_double), _P]),
    "sem_pmg_opts_default": (None, [C.POINTER(sem_pmg_opts)]),
    "sem_pmg_setup": (C.c_int, [_P, C.POINTER(sem_pmg_opts), C.POINTER(_P)]),
    "sem_pmg_destroy": (C.c_int, [_P]),
    "sem_pmg_query": (C.c_int, [_P, C.POINTER(sem_pmg_info)]),
    "sem_pmg_level": (C.c_int, [_P, C.c_int, C.POINTER(_P)]),
    "sem_pmg_transfer": (C.c_int, [_P, C.c_int, C.c_int, _P, _P, _P]),
    "sem_pmg_apply": (C.c_int, [_P, _P, _P, _P]),
    "sem_solve_opts_default": (None, [C.POINTER(sem_solve_opts)]),
    "sem_pcg_solve": (C.c_int, [_P, _P, _P, _P, C.POINTER(sem_solve_opts), C.POINTER(sem_solve_info), _P]),
    "sem_pcg_solve_batched": (C.c_int, [C.c_int, _P, _P, _P, _P, C.POINTER(sem_solve_opts),
                                        C.POINTER(sem_solve_info), _P]),
    "sem_solve_workspace_bytes": (C.c_size_t, [_P, _P]),
    "sem_batch_create": (C.c_int, [C.c_int, _P, C.POINTER(_P)]),
    "sem_batch_destroy": (C.c_int, [_P]),
    "sem_batch_add": (C.c_int, [_P, _P, _P, _P, _P, C.POINTER(sem_solve_opts), C.POINTER(C.c_int)]),
    "sem_batch_step": (C.c_int, [_P, C.c_int, C.POINTER(C.c_int)]),
    "sem_batch_poll": (C.c_int, [_P, C.c_int, C.POINTER(sem_solve_info)]),
    "sem_batch_release": (C.c_int, [_P, C.c_int]),
    "sem_pmg_smoother_apply": (C.c_int, [_P, C.c_int, _P, _P, _P]),
    "sem_gmres_solve": (C.c_int, [_P, _P, C.c_int, _P, _P, C.POINTER(sem_solve_opts), C.POINTER(sem_solve_info), _P]),
    "sem_proj_create": (C.c_int, [_P, C.c_int, C.POINTER(_P)]),
    "sem_proj_destroy": (C.c_int, [_P]),
    "sem_proj_size": (C.c_int, [_P, C.POINTER(C.c_int)]),
    "sem_proj_reset": (C.c_int, [_P]),
    "sem_proj_set_gmres": (C.c_int, [_P, C.c_int]),
    "sem_proj_export": (C.c_int, [_P, C.c_int, _P, _P, _P]),
    "sem_pcg_solve_projected": (C.c_int, [_P, _P, _P, _P, C.POINTER(sem_solve_opts), C.POINTER(sem_solve_info), _P]),
    "sem_stream": (C.c_int, [C.c_int, _P, _P, C.c_double, C.c_int64, _P]),
    "sem_status_string": (C.c_char_p, [C.c_int]),
    "sem_last_error": (C.c_char_p, []),
}

_lib = None


def load(path: str = LIB_PATH) -> C.CDLL:
    """Load libsem.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} not found: build it with `python -m paper_2110_01716_amd.build_lib`")
    lib = C.CDLL(path)
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    return list(_SIGS)


def _check(rc: int, where: str):
    if rc != SEM_OK:
        lib = load()
        raise SemError(rc, where, lib.sem_last_error().decode(errors="replace"))


def _ptr(t) -> int:
    """Device/host address of a torch tensor or numpy array (None -> 0)."""
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        if not t.flags["C_CONTIGUOUS"]:
            raise ValueError("numpy array must be C-contiguous")
        return t.ctypes.data
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def _stream(stream=None):
    if stream is not None:
        return stream
    import torch
    return torch.cuda.current_stream().cuda_stream


def _dtype_code(t) -> int:
    import torch
    if t.dtype == torch.float64:
        return SEM_F64
    if t.dtype == torch.float32:
        return SEM_F32
    raise TypeError(f"unsupported dtype {t.dtype}")


# ---------------------------------------------------------------------------
# C names
# ---------------------------------------------------------------------------

def sem_reference(N: int):
    lib = load()
    x, w, D = np.zeros(N + 1), np.zeros(N + 1), np.zeros((N + 1, N + 1))
    _check(lib.sem_reference(N, _ptr(x), _ptr(w), _ptr(D)), "sem_reference")
    return x, w, D


def sem_interpolation(Nc: int, Nf: int):
    lib = load()
    J = np.zeros((Nf + 1, Nc + 1))
    _check(lib.sem_interpolation(Nc, Nf, _ptr(J)), "sem_interpolation")
    return J


def sem_mesh_create(N, x, y, z, gid, dirichlet=None, stream=None):
    lib = load()
    E = x.shape[0]
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (x, y, z)]
    g = np.ascontiguousarray(gid, dtype=np.int64)
    d = None if dirichlet is None else np.ascontiguousarray(dirichlet, dtype=np.uint8)
    desc = sem_mesh_desc(N, E, _ptr(arrs[0]), _ptr(arrs[1]), _ptr(arrs[2]), _ptr(g), _ptr(d), _stream(stream))
    h = C.c_void_p()
    _check(lib.sem_mesh_create(C.byref(desc), C.byref(h)), "sem_mesh_create")
    return h


def sem_mesh_destroy(h):
    _check(load().sem_mesh_destroy(h), "sem_mesh_destroy")


def sem_mesh_query(h) -> dict:
    info = sem_mesh_info()
    _check(load().sem_mesh_query(h, C.byref(info)), "sem_mesh_query")
    return {k: getattr(info, k) for k, _ in info._fields_}


def sem_mesh_export(h, G=None, B=None, dinv=None, stream=None):
    _check(load().sem_mesh_export(h, _ptr(G), _ptr(B), _ptr(dinv), _stream(stream)), "sem_mesh_export")


def sem_mesh_export_nodes(h, x=None, y=None, z=None, gid=None, dirichlet=None, stream=None):
    _check(load().sem_mesh_export_nodes(h, _ptr(x), _ptr(y), _ptr(z), _ptr(gid), _ptr(dirichlet),
                                        _stream(stream)), "sem_mesh_export_nodes")


def sem_ax(h, u, Au, e0=0, ne=None, E=None, stream=None):
    if ne is None:
        ne = (E if E is not None else u.shape[0]) - e0
    _check(load().sem_ax(h, _dtype_code(u), _ptr(u), _ptr(Au), e0, ne, _stream(stream)), "sem_ax")


def sem_helmholtz(h, u, Au, lam, stream=None):
    _check(load().sem_helmholtz(h, _dtype_code(u), _ptr(u), _ptr(Au), float(lam), _stream(stream)),
           "sem_helmholtz")


def sem_gs(h, v, apply_mask=True, stream=None):
    _check(load().sem_gs(h, _dtype_code(v), _ptr(v), 1 if apply_mask else 0, _stream(stream)), "sem_gs")


def sem_mass(h, u, Bu, stream=None):
    _check(load().sem_mass(h, _dtype_code(u), _ptr(u), _ptr(Bu), _stream(stream)), "sem_mass")


def sem_dot(h, a, b, stream=None) -> float:
    r = C.c_double()
    _check(load().sem_dot(h, _dtype_code(a), _ptr(a), _ptr(b), C.byref(r), _stream(stream)), "sem_dot")
    return r.value


def sem_stream(n_in, src, dst, s=1.0, n=None, stream=None):
    """dst = src[0] + s * (src[1] + ... + src[n_in-1]); src is a [n_in, n] FP64 tensor."""
    n = dst.numel() if n is None else n
    _check(load().sem_stream(n_in, _ptr(src), _ptr(dst), s, n, _stream(stream)), "sem_stream")


def sem_dot_noalloc(h, a, b, stream=None) -> float:
    r = C.c_double()
    _check(load().sem_dot_noalloc(h, _dtype_code(a), _ptr(a), _ptr(b), C.byref(r), _stream(stream)),
           "sem_dot_noalloc")
    return r.value


def pmg_opts(**kw) -> sem_pmg_opts:
    o = sem_pmg_opts()
    load().sem_pmg_opts_default(C.byref(o))
    keep = []
    for k, v in kw.items():
        if k == "orders":
            o.n_levels = len(v)
            for i, n in enumerate(v):
                o.orders[i] = n
        elif k == "rho_override":
            if v is None:
                o.rho_override = None
            else:
                arr = np.ascontiguousarray(v, dtype=np.float64)
                keep.append(arr)
                o.rho_override = arr.ctypes.data
        elif k == "smoother_dtype":
            o.smoother_dtype = {"f32": SEM_F32, "f64": SEM_F64, SEM_F32: SEM_F32, SEM_F64: SEM_F64}[v]
        elif k == "smoother":
            o.smoother = _SMOOTHERS[v] if isinstance(v, str) else int(v)
        else:
            setattr(o, k, v)
    o._keep = keep
    return o


def sem_pmg_setup(mesh, opts: sem_pmg_opts | None = None):
    h = C.c_void_p()
    _check(load().sem_pmg_setup(mesh, C.byref(opts) if opts is not None else None, C.byref(h)), "sem_pmg_setup")
    return h


def sem_pmg_destroy(h):
    _check(load().sem_pmg_destroy(h), "sem_pmg_destroy")


def sem_pmg_query(h) -> dict:
    info = sem_pmg_info()
    _check(load().sem_pmg_query(h, C.byref(info)), "sem_pmg_query")
    L = info.n_levels
    return {"n_levels": L, "orders": list(info.orders)[:L], "rho": list(info.rho)[:L],
            "n_unique": list(info.n_unique)[:L], "resident_bytes": info.resident_bytes}


def sem_pmg_level(h, level: int):
    out = C.c_void_p()
    _check(load().sem_pmg_level(h, level, C.byref(out)), "sem_pmg_level")
    return out


def sem_pmg_transfer(h, level, direction, src, dst, stream=None):
    _check(load().sem_pmg_transfer(h, level, direction, _ptr(src), _ptr(dst), _stream(stream)), "sem_pmg_transfer")


def sem_pmg_apply(h, r, z, stream=None):
    _check(load().sem_pmg_apply(h, _ptr(r), _ptr(z), _stream(stream)), "sem_pmg_apply")


def solve_opts(**kw) -> sem_solve_opts:
    """sem_solve_opts with defaults; `lam` (or `lambda_`) is the Helmholtz shift."""
    o = sem_solve_opts()
    load().sem_solve_opts_default(C.byref(o))
    for k, v in kw.items():
        setattr(o, "lam" if k in ("lam", "lambda_", "helmholtz_lambda") else k, v)
    return o


def sem_pcg_solve(mesh, pmg, b, x, opts: sem_solve_opts | None = None, stream=None, check=True) -> dict:
    info = sem_solve_info()
    rc = load().sem_pcg_solve(mesh, pmg, _ptr(b), _ptr(x), C.byref(opts) if opts is not None else None,
                              C.byref(info), _stream(stream))
    if check and rc not in (SEM_OK,):
        _check(rc, "sem_pcg_solve")
    d = info.as_dict()
    d["rc"] = rc
    return d


def sem_pcg_solve_batched(meshes, pmgs, bs, xs, opts: sem_solve_opts | None = None, stream=None, check=True):
    n = len(meshes)
    M = (C.c_void_p * n)(*[m.value for m in meshes])
    P = None if pmgs is None else (C.c_void_p * n)(*[(p.value if p is not None else None) for p in pmgs])
    Bp = (C.c_void_p * n)(*[_ptr(b) for b in bs])
    Xp = (C.c_void_p * n)(*[_ptr(x) for x in xs])
    infos = (sem_solve_info * n)()
    rc = load().sem_pcg_solve_batched(n, M, P, Bp, Xp, C.byref(opts) if opts is not None else None, infos,
                                      _stream(stream))
    if check and rc != SEM_OK:
        _check(rc, "sem_pcg_solve_batched")
    return rc, [i.as_dict() for i in infos]


def sem_solve_workspace_bytes(mesh, pmg=None) -> int:
    return int(load().sem_solve_workspace_bytes(mesh, pmg))


def sem_batch_create(max_slots: int, stream=None):
    h = C.c_void_p()
    _check(load().sem_batch_create(max_slots, _stream(stream), C.byref(h)), "sem_batch_create")
    return h


def sem_batch_destroy(h):
    _check(load().sem_batch_destroy(h), "sem_batch_destroy")


def sem_batch_add(h, mesh, pmg, b, x, opts: sem_solve_opts | None = None) -> int:
    slot = C.c_int(-1)
    _check(load().sem_batch_add(h, mesh, pmg, _ptr(b), _ptr(x), C.byref(opts) if opts is not None else None,
                                C.byref(slot)), "sem_batch_add")
    return slot.value


def sem_batch_step(h, iters: int = 1) -> int:
    n = C.c_int(0)
    _check(load().sem_batch_step(h, iters, C.byref(n)), "sem_batch_step")
    return n.value


def sem_batch_poll(h, slot: int) -> dict:
    info = sem_solve_info()
    _check(load().sem_batch_poll(h, slot, C.byref(info)), "sem_batch_poll")
    return info.as_dict()


def sem_batch_release(h, slot: int):
    _check(load().sem_batch_release(h, slot), "sem_batch_release")


def sem_pmg_smoother_apply(h, level, r, z, stream=None):
    _check(load().sem_pmg_smoother_apply(h, int(level), _ptr(r), _ptr(z), _stream(stream)), "sem_pmg_smoother_apply")


def sem_gmres_solve(mesh, pmg, K, b, x, opts: sem_solve_opts | None = None, stream=None, check=True) -> dict:
    info = sem_solve_info()
    rc = load().sem_gmres_solve(mesh, pmg, int(K), _ptr(b), _ptr(x), C.byref(opts) if opts is not None else None,
                                C.byref(info), _stream(stream))
    if check and rc != SEM_OK:
        _check(rc, "sem_gmres_solve")
    d = info.as_dict()
    d["rc"] = rc
    return d


def sem_proj_create(mesh, L_max: int):
    h = C.c_void_p()
    _check(load().sem_proj_create(mesh, L_max, C.byref(h)), "sem_proj_create")
    return h


def sem_proj_destroy(h):
    _check(load().sem_proj_destroy(h), "sem_proj_destroy")


def sem_proj_size(h) -> int:
    n = C.c_int(0)
    _check(load().sem_proj_size(h, C.byref(n)), "sem_proj_size")
    return n.value


def sem_proj_reset(h):
    _check(load().sem_proj_reset(h), "sem_proj_reset")


def sem_proj_set_gmres(h, K: int):
    _check(load().sem_proj_set_gmres(h, int(K)), "sem_proj_set_gmres")


def sem_proj_export(h, i, p=None, Ap=None, stream=None):
    _check(load().sem_proj_export(h, i, _ptr(p), _ptr(Ap), _stream(stream)), "sem_proj_export")


def sem_pcg_solve_projected(proj, pmg, b, x, opts: sem_solve_opts | None = None, stream=None, check=True) -> dict:
    info = sem_solve_info()
    rc = load().sem_pcg_solve_projected(proj, pmg, _ptr(b), _ptr(x), C.byref(opts) if opts is not None else None,
                                        C.byref(info), _stream(stream))
    if check and rc != SEM_OK:
        _check(rc, "sem_pcg_solve_projected")
    d = info.as_dict()
    d["rc"] = rc
    return d


def sem_status_string(code: int) -> str:
    return load().sem_status_string(code).decode()


# ---------------------------------------------------------------------------
# owning wrappers
# ---------------------------------------------------------------------------

class Mesh:
    """A resident mesh built from host arrays (e.g. workloads.BoxMesh)."""

    def __init__(self, N, x, y, z, gid, dirichlet=None, stream=None):
        self.N = N
        self.E = x.shape[0]
        self.Np = (N + 1) ** 3
        self.h = sem_mesh_create(N, x, y, z, gid, dirichlet, stream)

    @classmethod
    def from_box(cls, bm, stream=None):
        return cls(bm.N, bm.x, bm.y, bm.z, bm.gid, bm.dirichlet, stream)

    def info(self):
        return sem_mesh_query(self.h)

    def close(self):
        if self.h is not None:
            sem_mesh_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Pmg:
    def __init__(self, mesh: Mesh, **opts):
        self.mesh = mesh
        self.opts = pmg_opts(**opts) if opts else None
        self.h = sem_pmg_setup(mesh.h, self.opts)

    def info(self):
        return sem_pmg_query(self.h)

    def level(self, l):
        return sem_pmg_level(self.h, l)

    def close(self):
        if self.h is not None:
            sem_pmg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Projection:
    """Space of earlier solutions on one mesh (sem_proj_*)."""

    def __init__(self, mesh: Mesh, L_max: int = 30, gmres_K: int = 0):
        self.mesh = mesh
        self.L_max = L_max
        self.h = sem_proj_create(mesh.h, L_max)
        if gmres_K:
            sem_proj_set_gmres(self.h, gmres_K)

    @property
    def size(self) -> int:
        return sem_proj_size(self.h)

    def reset(self):
        sem_proj_reset(self.h)

    def solve(self, pmg, b, x, opts: sem_solve_opts | None = None, stream=None, check=True) -> dict:
        return sem_pcg_solve_projected(self.h, pmg.h if isinstance(pmg, Pmg) else pmg, b, x, opts,
                                       stream=stream, check=check)

    def export(self, i, p=None, Ap=None, stream=None):
        sem_proj_export(self.h, i, p, Ap, stream)

    def close(self):
        if self.h is not None:
            sem_proj_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
