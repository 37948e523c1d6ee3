"""ctypes binding of libparo (argument marshalling only).

Each function mirrors the C entry point of the same name in
``include/paro.h``: torch tensors on the current HIP device are passed as
raw device pointers, the current torch stream as the hipStream_t.  No
arithmetic of the method happens here.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("PARO_LIB") or os.path.join(HERE, "libparo.so")

PARO_OK, PARO_EINVAL, PARO_ENOMEM, PARO_ENOTSPD = 0, -1, -2, -3
PARO_ESINGULAR, PARO_ENOCONV, PARO_EDEVICE = -4, -5, -6
PARO_FP64, PARO_FP32_INNER = 0, 1
NT_MAX = 64

c_i32, c_i64, c_dbl, c_vp = (ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                             ctypes.c_void_p)


class Box(ctypes.Structure):
    _fields_ = [("nx", c_i32), ("ny", c_i32), ("nz", c_i32),
                ("lo", c_dbl * 3), ("hi", c_dbl * 3)]

    @classmethod
    def cube(cls, nc, lo, hi):
        ncs = (nc, nc, nc) if isinstance(nc, int) else tuple(nc)
        los = (lo,) * 3 if isinstance(lo, (int, float)) else tuple(lo)
        his = (hi,) * 3 if isinstance(hi, (int, float)) else tuple(hi)
        return cls(ncs[0], ncs[1], ncs[2], (c_dbl * 3)(*los),
                   (c_dbl * 3)(*his))


class Opts(ctypes.Structure):
    _fields_ = [("N", c_i32), ("m", c_i32), ("max_steps", c_i32),
                ("pcg_maxit", c_i32), ("precision", c_i32),
                ("sigma_mode", c_i32), ("sigma", c_dbl),
                ("lambda_tol", c_dbl), ("resid_tol", c_dbl),
                ("pcg_rtol", c_dbl), ("inner_rtol", c_dbl),
                ("pcg_reduce", c_dbl)]


class Report(ctypes.Structure):
    _fields_ = [("status", c_i32), ("steps", c_i32), ("pcg_iters", c_i64),
                ("refinements", c_i64), ("n_dof", c_i64), ("nnz", c_i64),
                ("max_dlambda", c_dbl), ("max_resid", c_dbl),
                ("sigma", c_dbl), ("seconds", c_dbl), ("reorth", c_i64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


ST_NAMES = ["cg_spmm", "cg_rupd", "cg_pupd", "start", "refine", "rr_spmm",
            "gram", "small_eig", "rotate", "cg_final"]


class Timing(ctypes.Structure):
    _fields_ = [("launches", c_i64 * len(ST_NAMES)),
                ("ms", c_dbl * len(ST_NAMES)), ("cg_iters", c_i64),
                ("cg_col_iters", c_i64)]

    def as_dict(self):
        return {"stages": {n: {"launches": self.launches[i],
                               "ms": self.ms[i]}
                           for i, n in enumerate(ST_NAMES)},
                "cg_iters": self.cg_iters,
                "cg_col_iters": self.cg_col_iters}


class ServerStats(ctypes.Structure):
    _fields_ = [("queued", c_i32), ("active", c_i32), ("done", c_i64),
                ("arena_used", ctypes.c_size_t),
                ("arena_bytes", ctypes.c_size_t), ("ticks", c_i64)]


class KsOpts(ctypes.Structure):
    _fields_ = [("max_iter", c_i32), ("poisson_maxit", c_i32),
                ("mixing", c_dbl), ("occupancy", c_dbl), ("scf_tol", c_dbl),
                ("poisson_rtol", c_dbl), ("kerker_q0", c_dbl)]


class KsReport(ctypes.Structure):
    _fields_ = [("status", c_i32), ("iterations", c_i32),
                ("paro_pcg_iters", c_i64), ("poisson_iters", c_i64),
                ("residual", c_dbl), ("max_dlambda", c_dbl),
                ("max_resid", c_dbl), ("sigma", c_dbl), ("seconds", c_dbl)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ParoError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"paro error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """The loaded libparo.so (raises if it was never built)."""
    global _lib
    if _lib is not None:
        return _lib
    # torch must be loaded first: its HIP runtime then satisfies libparo's
    # libamdhip64 dependency, so the process holds one runtime and device
    # pointers / streams from torch are valid in libparo.  Loading libparo
    # first would map a second HIP/HSA runtime that sees no device.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with "
            "`python -m paper_1405_0260_amd.build` (no CPU fallback exists)")
    L = ctypes.CDLL(LIB_PATH)
    P = c_vp
    PP = ctypes.POINTER(c_vp)
    sig = {
        "paro_default_opts": (None, [ctypes.POINTER(Opts)]),
        "paro_query": (c_i32, [ctypes.POINTER(Box), ctypes.POINTER(Opts),
                               ctypes.POINTER(c_i64), ctypes.POINTER(c_i64),
                               ctypes.POINTER(ctypes.c_size_t)]),
        "paro_assemble": (c_i32, [ctypes.POINTER(Box), P,
                                  ctypes.POINTER(Opts), P, ctypes.c_size_t, P,
                                  ctypes.POINTER(P)]),
        "paro_init": (c_i32, [P, P, P, P, P]),
        "paro_step": (c_i32, [P, P, P, P, ctypes.POINTER(Report)]),
        "paro_solve": (c_i32, [P, P, P, P, P, ctypes.POINTER(Report)]),
        "paro_destroy": (None, [P]),
        "paro_last_error": (ctypes.c_char_p, []),
        "paro_strerror": (ctypes.c_char_p, [c_i32]),
        "paro_export_csr": (c_i32, [P, P, P, P, P, ctypes.POINTER(c_dbl), P]),
        "paro_spmm": (c_i32, [P, c_i32, P, P, c_i32, P]),
        "paro_gram": (c_i32, [P, P, P, P, c_i32, P]),
        "paro_gram_noalloc": (c_i32, [P, P, P, c_i64, c_i32, P]),
        "paro_elements": (c_i64, [ctypes.POINTER(Box)]),
        "paro_estimate": (c_i32, [ctypes.POINTER(Box), P, P, P, c_i32, c_i32,
                                  P, P]),
        "paro_mark_workspace_bytes": (ctypes.c_size_t, []),
        "paro_mark": (c_i32, [P, c_i64, c_dbl, c_i32, P,
                              ctypes.POINTER(c_i64), P, ctypes.c_size_t, P]),
        "paro_prolong": (c_i32, [ctypes.POINTER(Box), P, P, c_i32, P]),
        "paro_mesh_create": (c_i32, [ctypes.POINTER(Box), ctypes.POINTER(P)]),
        "paro_mesh_from_arrays": (c_i32, [ctypes.POINTER(Box), c_i64, P,
                                          c_i64, P, P, P,
                                          ctypes.POINTER(P)]),
        "paro_mesh_info": (c_i32, [P, ctypes.POINTER(c_i64),
                                   ctypes.POINTER(c_i64),
                                   ctypes.POINTER(c_i64)]),
        "paro_mesh_arrays": (c_i32, [P, P, P, P, P, P]),
        "paro_mesh_refine": (c_i32, [P, P, ctypes.POINTER(P)]),
        "paro_mesh_destroy": (None, [P]),
        "paro_mesh_query": (c_i32, [P, ctypes.POINTER(Opts),
                                    ctypes.POINTER(c_i64),
                                    ctypes.POINTER(c_i64),
                                    ctypes.POINTER(ctypes.c_size_t)]),
        "paro_mesh_assemble": (c_i32, [P, P, ctypes.POINTER(Opts), P,
                                       ctypes.c_size_t, P,
                                       ctypes.POINTER(P)]),
        "paro_mesh_estimate": (c_i32, [P, P, P, c_i32, c_i32, P, P]),
        "paro_mesh_prolong_workspace_bytes": (ctypes.c_size_t, [P, P]),
        "paro_mesh_prolong": (c_i32, [P, P, P, P, c_i32, P, ctypes.c_size_t,
                                      P]),
        "paro_small_geneig": (c_i32, [P, P, c_i32, P, P, P, P]),
        "paro_pcg": (c_i32, [P, P, P, c_i32, P, P]),
        "paro_set_timing": (c_i32, [P, c_i32]),
        "paro_set_graphs": (None, [c_i32]),
        "paro_set_persistent": (None, [c_i32]),
        "paro_set_matrix_free": (None, [c_i32]),
        "paro_set_clusters": (c_i32, [P, P, c_i32, P]),
        "paro_nonlocal_query": (c_i32, [P, c_i32, ctypes.POINTER(ctypes.c_size_t)]),
        "paro_set_nonlocal": (c_i32, [P, P, c_i32, P, ctypes.c_size_t, P]),
        "paro_set_autotune": (None, [c_i32]),
        "paro_tuned": (c_i32, [P, ctypes.POINTER(c_i32),
                               ctypes.POINTER(c_i32)]),
        "paro_set_tuning": (c_i32, [P, c_i32, c_i32]),
        "paro_get_timing": (c_i32, [P, ctypes.POINTER(Timing)]),
        "paro_batch_workspace_bytes": (ctypes.c_size_t, [c_i32]),
        "paro_batch_init": (c_i32, [PP, c_i32, PP, PP, PP, P,
                                    ctypes.c_size_t, P]),
        "paro_batch_step": (c_i32, [PP, c_i32, PP, PP, P, ctypes.c_size_t,
                                    P, ctypes.POINTER(Report)]),
        "paro_batch_solve": (c_i32, [PP, c_i32, PP, PP, PP, P,
                                     ctypes.c_size_t, P,
                                     ctypes.POINTER(Report)]),
        "paro_server_create": (c_i32, [P, ctypes.c_size_t, c_i32, P,
                                       ctypes.POINTER(P)]),
        "paro_server_submit": (c_i32, [P, ctypes.POINTER(Box), P,
                                       ctypes.POINTER(Opts), P, P, P,
                                       ctypes.POINTER(c_i64)]),
        "paro_server_tick": (c_i32, [P, ctypes.POINTER(c_i64), c_i32,
                                     ctypes.POINTER(c_i32),
                                     ctypes.POINTER(ServerStats)]),
        "paro_server_report": (c_i32, [P, c_i64, ctypes.POINTER(Report)]),
        "paro_server_destroy": (None, [P]),
        "paro_ks_default_opts": (None, [ctypes.POINTER(KsOpts)]),
        "paro_ks_query": (c_i32, [ctypes.POINTER(Box),
                                  ctypes.POINTER(ctypes.c_size_t)]),
        "paro_update_potential": (c_i32, [P, P, P]),
        "paro_sigma": (c_dbl, [P]),
        "paro_ks_solve": (c_i32, [P, P, ctypes.POINTER(KsOpts), P,
                                  ctypes.c_size_t, P, P, P, P, P, P,
                                  ctypes.POINTER(KsReport)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(rc, allow=()):
    if rc != PARO_OK and rc not in allow:
        raise ParoError(rc, lib().paro_last_error().decode())
    return rc


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr()


def _stream(stream):
    if stream is not None:
        return stream
    import torch
    return torch.cuda.current_stream().cuda_stream


def _f64(t, shape: Sequence[int], name: str):
    import torch
    if t.dtype != torch.float64:
        raise ValueError(f"{name}: expected float64, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: expected shape {tuple(shape)}, "
                         f"got {tuple(t.shape)}")


def paro_default_opts() -> Opts:
    o = Opts()
    lib().paro_default_opts(ctypes.byref(o))
    return o


def default_opts(**kw) -> Opts:
    o = paro_default_opts()
    for k, v in kw.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


def paro_query(box: Box, opts: Opts):
    n, z, b = c_i64(), c_i64(), ctypes.c_size_t()
    _check(lib().paro_query(ctypes.byref(box), ctypes.byref(opts),
                            ctypes.byref(n), ctypes.byref(z), ctypes.byref(b)))
    return n.value, z.value, b.value


class Problem:
    """An assembled problem: host handle plus the caller-owned workspace."""

    def __init__(self, handle, box, opts, workspace, n, nnz):
        self.handle = handle
        self.box = box
        self.opts = opts
        self.workspace = workspace
        self.n = n
        self.nnz = nnz
        self.Nt = opts.N + opts.m

    def __del__(self):
        try:
            if self.handle:
                lib().paro_destroy(self.handle)
                self.handle = None
        except Exception:
            pass


def paro_assemble(box: Box, V, opts: Opts, stream=None,
                  workspace=None) -> Problem:
    """Assemble on the device; V: float64 device tensor of all vertices."""
    import torch
    n, z, nbytes = paro_query(box, opts)
    _f64(V, ((box.nx + 1) * (box.ny + 1) * (box.nz + 1),), "V")
    if workspace is None:
        workspace = torch.empty(nbytes + 256, dtype=torch.uint8,
                                device=V.device)
    base = workspace.data_ptr()
    off = (-base) % 256
    h = c_vp()
    _check(lib().paro_assemble(ctypes.byref(box), _ptr(V), ctypes.byref(opts),
                               base + off, workspace.numel() - off,
                               _stream(stream), ctypes.byref(h)))
    return Problem(h, box, opts, workspace, n, z)


def paro_init(p: Problem, U0, lam, U, stream=None):
    _f64(U0, (p.n, p.Nt), "U0")
    _f64(U, (p.n, p.Nt), "U")
    _f64(lam, (p.Nt,), "lambda")
    _check(lib().paro_init(p.handle, _ptr(U0), _ptr(lam), _ptr(U),
                           _stream(stream)))


def paro_step(p: Problem, lam, U, stream=None, report=True):
    _f64(U, (p.n, p.Nt), "U")
    _f64(lam, (p.Nt,), "lambda")
    r = Report()
    _check(lib().paro_step(p.handle, _ptr(lam), _ptr(U), _stream(stream),
                           ctypes.byref(r) if report else None),
           allow=(PARO_ENOCONV,))
    return r if report else None


def paro_solve(p: Problem, U0, lam, U, stream=None) -> Report:
    _f64(U0, (p.n, p.Nt), "U0")
    _f64(U, (p.n, p.Nt), "U")
    _f64(lam, (p.Nt,), "lambda")
    r = Report()
    _check(lib().paro_solve(p.handle, _ptr(U0), _ptr(lam), _ptr(U),
                            _stream(stream), ctypes.byref(r)),
           allow=(PARO_ENOCONV,))
    return r


def paro_destroy(p: Problem):
    if p.handle:
        lib().paro_destroy(p.handle)
        p.handle = None


def paro_export_csr(p: Problem, stream=None):
    import torch
    dev = p.workspace.device
    rowptr = torch.empty(p.n + 1, dtype=torch.int32, device=dev)
    col = torch.empty(p.nnz, dtype=torch.int32, device=dev)
    valA = torch.empty(p.nnz, dtype=torch.float64, device=dev)
    valM = torch.empty(p.nnz, dtype=torch.float64, device=dev)
    sigma = c_dbl()
    _check(lib().paro_export_csr(p.handle, _ptr(rowptr), _ptr(col),
                                 _ptr(valA), _ptr(valM), ctypes.byref(sigma),
                                 _stream(stream)))
    return rowptr, col, valA, valM, sigma.value


def paro_spmm(p: Problem, which: int, X, Y, stream=None):
    ncols = X.shape[1]
    _f64(X, (p.n, ncols), "X")
    _f64(Y, (p.n, ncols), "Y")
    _check(lib().paro_spmm(p.handle, which, _ptr(X), _ptr(Y), ncols,
                           _stream(stream)))


def paro_gram(p: Problem, W, Y, G, stream=None):
    ncols = W.shape[1]
    _f64(W, (p.n, ncols), "W")
    _f64(Y, (p.n, ncols), "Y")
    _f64(G, (ncols, ncols), "G")
    _check(lib().paro_gram(p.handle, _ptr(W), _ptr(Y), _ptr(G), ncols,
                           _stream(stream)))


def paro_gram_noalloc(W, Y, G, stream=None):
    """G = W^T Y without a problem or workspace (the library's static
    device scratch; allocates nothing)."""
    n, ncols = W.shape
    _f64(W, (n, ncols), "W")
    _f64(Y, (n, ncols), "Y")
    _f64(G, (ncols, ncols), "G")
    _check(lib().paro_gram_noalloc(_ptr(W), _ptr(Y), _ptr(G), n, ncols,
                                   _stream(stream)))


PARO_MARK_DORFLER = 0
PARO_MARK_MAXIMUM = 1


def paro_elements(box: Box) -> int:
    return lib().paro_elements(ctypes.byref(box))


def paro_estimate(box: Box, V, lam, U, nreq, eta, stream=None):
    """Residual estimator per element of the first nreq columns of U (see
    include/paro.h) into eta (paro_elements(box) doubles)."""
    n, ncols = U.shape
    _f64(V, ((box.nx + 1) * (box.ny + 1) * (box.nz + 1),), "V")
    _f64(lam, (ncols,), "lambda")
    _f64(eta, (paro_elements(box),), "eta")
    _check(lib().paro_estimate(ctypes.byref(box), _ptr(V), _ptr(lam),
                               _ptr(U), ncols, nreq, _ptr(eta),
                               _stream(stream)))


def paro_mark(eta, theta, strategy=PARO_MARK_DORFLER, stream=None):
    """Marked elements (uint8 device tensor) and their count."""
    import torch
    nbytes = lib().paro_mark_workspace_bytes()
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=eta.device)
    off = (-ws.data_ptr()) % 256
    marked = torch.empty(eta.shape[0], dtype=torch.uint8, device=eta.device)
    cnt = c_i64()
    _check(lib().paro_mark(_ptr(eta), eta.shape[0], theta, strategy,
                           _ptr(marked), ctypes.byref(cnt),
                           ctypes.c_void_p(ws.data_ptr() + off), nbytes,
                           _stream(stream)))
    return marked, cnt.value


def paro_prolong(box: Box, Uc, Uf, stream=None):
    """Orbitals of the box's mesh -> the mesh with twice the cells."""
    ncols = Uc.shape[1]
    _check(lib().paro_prolong(ctypes.byref(box), _ptr(Uc), _ptr(Uf), ncols,
                              _stream(stream)))


# ------------------------------------------------- general bisection meshes

class Mesh:
    """A bisection mesh of a box (host object of the library).  Arrays
    come back as numpy copies."""

    def __init__(self, handle, box):
        self.handle = handle
        self.box = box

    @classmethod
    def kuhn(cls, box: Box) -> "Mesh":
        h = c_vp()
        _check(lib().paro_mesh_create(ctypes.byref(box), ctypes.byref(h)))
        return cls(h, box)

    @classmethod
    def from_arrays(cls, box: Box, X, tets, tags, parents=None) -> "Mesh":
        import numpy as np
        X = np.ascontiguousarray(X, dtype=np.float64)
        tets = np.ascontiguousarray(tets, dtype=np.int32)
        tags = np.ascontiguousarray(tags, dtype=np.int32)
        if parents is not None:
            parents = np.ascontiguousarray(parents, dtype=np.int32)
        h = c_vp()
        _check(lib().paro_mesh_from_arrays(
            ctypes.byref(box), X.shape[0], X.ctypes.data, tets.shape[0],
            tets.ctypes.data, tags.ctypes.data,
            None if parents is None else parents.ctypes.data,
            ctypes.byref(h)))
        return cls(h, box)

    def info(self):
        """(vertices, elements, dofs)."""
        nv, ne, n = c_i64(), c_i64(), c_i64()
        _check(lib().paro_mesh_info(self.handle, ctypes.byref(nv),
                                    ctypes.byref(ne), ctypes.byref(n)))
        return nv.value, ne.value, n.value

    def arrays(self):
        """dict of X, tets, tags, parents, dof (numpy)."""
        import numpy as np
        nv, ne, _ = self.info()
        out = {"X": np.empty((nv, 3)), "tets": np.empty((ne, 4), np.int32),
               "tags": np.empty(ne, np.int32),
               "parents": np.empty((nv, 2), np.int32),
               "dof": np.empty(nv, np.int32)}
        _check(lib().paro_mesh_arrays(
            self.handle, out["X"].ctypes.data, out["tets"].ctypes.data,
            out["tags"].ctypes.data, out["parents"].ctypes.data,
            out["dof"].ctypes.data))
        return out

    def refine(self, marked) -> "Mesh":
        """Bisect the marked elements (host bool/uint8 array or a device
        uint8 tensor) with the conforming closure."""
        import numpy as np
        if hasattr(marked, "cpu"):
            marked = marked.cpu().numpy()
        m = np.ascontiguousarray(marked, dtype=np.uint8)
        _, ne, _ = self.info()
        if m.shape != (ne,):
            raise ValueError(f"marked must have {ne} entries")
        h = c_vp()
        _check(lib().paro_mesh_refine(self.handle, m.ctypes.data,
                                      ctypes.byref(h)))
        return Mesh(h, self.box)

    def close(self):
        if self.handle:
            lib().paro_mesh_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def paro_mesh_query(mesh: Mesh, opts: Opts):
    n, z, b = c_i64(), c_i64(), ctypes.c_size_t()
    _check(lib().paro_mesh_query(mesh.handle, ctypes.byref(opts),
                                 ctypes.byref(n), ctypes.byref(z),
                                 ctypes.byref(b)))
    return n.value, z.value, b.value


def paro_mesh_assemble(mesh: Mesh, V, opts: Opts, stream=None,
                       workspace=None) -> Problem:
    """Assemble on a mesh; V: float64 device tensor of all vertices."""
    import torch
    n, z, nbytes = paro_mesh_query(mesh, opts)
    nv, _, _ = mesh.info()
    _f64(V, (nv,), "V")
    if workspace is None:
        workspace = torch.empty(nbytes + 256, dtype=torch.uint8,
                                device=V.device)
    base = workspace.data_ptr()
    off = (-base) % 256
    h = c_vp()
    _check(lib().paro_mesh_assemble(mesh.handle, _ptr(V), ctypes.byref(opts),
                                    base + off, workspace.numel() - off,
                                    _stream(stream), ctypes.byref(h)))
    p = Problem(h, mesh.box, opts, workspace, n, z)
    p.mesh = mesh  # keeps the host mesh alive with the problem
    return p


def paro_mesh_estimate(p: Problem, lam, U, nreq, eta, stream=None):
    """Indicator per element of the mesh p was assembled on."""
    n, ncols = U.shape
    _f64(U, (p.n, ncols), "U")
    _f64(lam, (ncols,), "lambda")
    _, ne, _ = p.mesh.info()
    _f64(eta, (ne,), "eta")
    _check(lib().paro_mesh_estimate(p.handle, _ptr(lam), _ptr(U), ncols,
                                    nreq, _ptr(eta), _stream(stream)))


def paro_mesh_prolong(coarse: Mesh, fine: Mesh, Uc, Uf, stream=None):
    """Orbitals of `coarse` -> the refined mesh `fine` (P1 transfer)."""
    import torch
    ncols = Uc.shape[1]
    nbytes = lib().paro_mesh_prolong_workspace_bytes(coarse.handle,
                                                     fine.handle)
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=Uc.device)
    off = (-ws.data_ptr()) % 256
    _check(lib().paro_mesh_prolong(coarse.handle, fine.handle, _ptr(Uc),
                                   _ptr(Uf), ncols,
                                   ctypes.c_void_p(ws.data_ptr() + off),
                                   nbytes, _stream(stream)))


def paro_small_geneig(A, B, theta, C, info, stream=None):
    n = A.shape[0]
    _f64(A, (n, n), "A")
    _f64(B, (n, n), "B")
    _f64(theta, (n,), "theta")
    _f64(C, (n, n), "C")
    _check(lib().paro_small_geneig(_ptr(A), _ptr(B), n, _ptr(theta), _ptr(C),
                                   _ptr(info), _stream(stream)))


def paro_pcg(p: Problem, B, X, stream=None):
    """Solve (H - s M) X = B from the start X (in place); returns the CG
    iteration count of every column."""
    ncols = B.shape[1]
    _f64(B, (p.n, ncols), "B")
    _f64(X, (p.n, ncols), "X")
    iters = (c_i32 * ncols)()
    _check(lib().paro_pcg(p.handle, _ptr(B), _ptr(X), ncols, iters,
                          _stream(stream)))
    return list(iters)


def paro_set_graphs(on: bool = True):
    """Run CG chunks as captured HIP graphs (on) or kernel by kernel (off,
    the default); process-wide."""
    lib().paro_set_graphs(1 if on else 0)


def paro_set_clusters(p: Problem, sizes=(), stream=None):
    """Cluster-wise projection over consecutive column clusters of the given
    sizes (summing to N + m); an empty sequence restores the full one."""
    arr = (c_i32 * max(1, len(sizes)))(*sizes)
    _check(lib().paro_set_clusters(p.handle, ctypes.cast(arr, ctypes.c_void_p),
                                   len(sizes), _stream(stream)))


def paro_set_nonlocal(p: Problem, zeta=None, stream=None):
    """Add the nonlocal term with projector values zeta (n x k device
    tensor, FP64); None removes it.  The workspace is allocated here and
    kept on the problem object."""
    import torch
    if zeta is None:
        _check(lib().paro_set_nonlocal(p.handle, None, 0, None, 0,
                                       _stream(stream)))
        p._nl_ws = None
        return
    k = zeta.shape[1]
    _f64(zeta, (p.n, k), "zeta")
    nbytes = ctypes.c_size_t(0)
    _check(lib().paro_nonlocal_query(p.handle, k, ctypes.byref(nbytes)))
    ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=zeta.device)
    off = (-ws.data_ptr()) % 256
    _check(lib().paro_set_nonlocal(p.handle, _ptr(zeta), k,
                                   ws.data_ptr() + off, nbytes.value,
                                   _stream(stream)))
    p._nl_ws = ws


def paro_set_persistent(on: bool = True):
    """Run every CG iteration of a call in one cooperative launch."""
    lib().paro_set_persistent(1 if on else 0)


def paro_set_matrix_free(on: bool = True):
    """FP64 z-marching CG SpMM forms the stencil coefficients from the
    potential (on, the default) or reads the stored ones (off); the same
    bits either way.  Process-wide."""
    lib().paro_set_matrix_free(1 if on else 0)


def paro_set_autotune(on: bool = True):
    """Autotune the CG SpMM per problem shape at assembly (default on)."""
    lib().paro_set_autotune(1 if on else 0)


def paro_tuned(p: Problem):
    """(SpMM variant, real block count) chosen for the problem: variant -1
    untuned, 0 for the row-sweep SpMM, 0/1/2 (1, 2 or 4 chunks per unit)
    for the z-marching one."""
    v, b = c_i32(), c_i32()
    _check(lib().paro_tuned(p.handle, ctypes.byref(v), ctypes.byref(b)))
    return v.value, b.value


def paro_set_tuning(p: Problem, variant: int, blocks: int):
    """Pin the SpMM variant and real block count of a problem (variant -1 or
    0; up to 2 for a z-marching problem)."""
    _check(lib().paro_set_tuning(p.handle, variant, blocks))


def paro_set_timing(p: Problem, on: bool = True):
    _check(lib().paro_set_timing(p.handle, 1 if on else 0))


def paro_get_timing(p: Problem) -> Timing:
    t = Timing()
    _check(lib().paro_get_timing(p.handle, ctypes.byref(t)))
    return t


# ----------------------------------------------------------------- batches

def _ptrs(items):
    return (c_vp * len(items))(*items)


class Batch:
    """Launch-table memory for batched calls over up to `capacity`
    problems (device bytes from paro_batch_workspace_bytes)."""

    def __init__(self, capacity: int, device=None):
        import torch
        self.capacity = capacity
        nbytes = lib().paro_batch_workspace_bytes(capacity)
        if nbytes == 0:
            raise ValueError("capacity must be >= 1")
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8,
                              device=device or "cuda")
        base = self.ws.data_ptr()
        self.off = (-base) % 256
        self.ptr = base + self.off
        self.bytes = self.ws.numel() - self.off

    def _args(self, probs):
        if len(probs) > self.capacity:
            raise ValueError(f"{len(probs)} problems > capacity "
                             f"{self.capacity}")
        return _ptrs([p.handle.value if isinstance(p.handle, c_vp)
                      else p.handle for p in probs])


def _batch_checks(probs, U0s, lams, Us):
    for k, p in enumerate(probs):
        if U0s is not None:
            _f64(U0s[k], (p.n, p.Nt), f"U0[{k}]")
        _f64(Us[k], (p.n, p.Nt), f"U[{k}]")
        _f64(lams[k], (p.Nt,), f"lambda[{k}]")


def paro_batch_init(batch: Batch, probs, U0s, lams, Us, stream=None):
    _batch_checks(probs, U0s, lams, Us)
    _check(lib().paro_batch_init(
        batch._args(probs), len(probs), _ptrs([_ptr(t) for t in U0s]),
        _ptrs([_ptr(t) for t in lams]), _ptrs([_ptr(t) for t in Us]),
        batch.ptr, batch.bytes, _stream(stream)))


def paro_batch_step(batch: Batch, probs, lams, Us, stream=None, report=True):
    """One ParO step of every problem; returns per-problem reports."""
    _batch_checks(probs, None, lams, Us)
    reps = (Report * len(probs))() if report else None
    _check(lib().paro_batch_step(
        batch._args(probs), len(probs), _ptrs([_ptr(t) for t in lams]),
        _ptrs([_ptr(t) for t in Us]), batch.ptr, batch.bytes,
        _stream(stream), reps))
    return list(reps) if report else None


def paro_batch_solve(batch: Batch, probs, U0s, lams, Us, stream=None):
    """Whole solves of every problem; returns per-problem reports (a
    problem that did not converge has status PARO_ENOCONV)."""
    _batch_checks(probs, U0s, lams, Us)
    reps = (Report * len(probs))()
    _check(lib().paro_batch_solve(
        batch._args(probs), len(probs), _ptrs([_ptr(t) for t in U0s]),
        _ptrs([_ptr(t) for t in lams]), _ptrs([_ptr(t) for t in Us]),
        batch.ptr, batch.bytes, _stream(stream), reps),
        allow=(PARO_ENOCONV,))
    return list(reps)


# ----------------------------------------------------------------- serving

class Server:
    """Continuous-batching request loop (paro_server_*).  The device arena
    is a torch uint8 tensor of `arena_bytes`; inputs and results are host
    numpy arrays (results are filled when a request retires)."""

    def __init__(self, arena_bytes: int, max_active: int = 64, device=None,
                 stream=None):
        import torch
        self.arena = torch.empty(arena_bytes + 256, dtype=torch.uint8,
                                 device=device or "cuda")
        base = self.arena.data_ptr()
        off = (-base) % 256
        self.handle = c_vp()
        self.max_active = max_active
        self._keep = {}
        _check(lib().paro_server_create(base + off, arena_bytes, max_active,
                                        _stream(stream),
                                        ctypes.byref(self.handle)))

    def submit(self, box: Box, V, opts: Opts, U0):
        """Queue a request; V and U0 are float64 numpy arrays (copied)."""
        import numpy as np
        V = np.ascontiguousarray(V, dtype=np.float64)
        U0 = np.ascontiguousarray(U0, dtype=np.float64)
        Nt = opts.N + opts.m
        lam = np.zeros(Nt)
        U = np.zeros((U0.shape[0], Nt))
        rid = c_i64()
        _check(lib().paro_server_submit(
            self.handle, ctypes.byref(box), V.ctypes.data, ctypes.byref(opts),
            U0.ctypes.data, lam.ctypes.data, U.ctypes.data,
            ctypes.byref(rid)))
        self._keep[rid.value] = (lam, U)
        return rid.value

    def tick(self, max_done: int = 1024):
        """One scheduling round; returns (retired ids, stats)."""
        ids = (c_i64 * max_done)()
        nd = c_i32()
        st = ServerStats()
        _check(lib().paro_server_tick(self.handle, ids, max_done,
                                      ctypes.byref(nd), ctypes.byref(st)))
        return [ids[k] for k in range(nd.value)], st

    def result(self, rid: int):
        """(lambda, U, report) of a retired request."""
        r = Report()
        _check(lib().paro_server_report(self.handle, rid, ctypes.byref(r)))
        lam, U = self._keep.pop(rid)
        return lam, U, r

    def close(self):
        if self.handle:
            lib().paro_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------- Kohn-Sham

def ks_default_opts(**kw) -> KsOpts:
    o = KsOpts()
    lib().paro_ks_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


def paro_update_potential(p: Problem, V, stream=None):
    _f64(V, ((p.box.nx + 1) * (p.box.ny + 1) * (p.box.nz + 1),), "V")
    _check(lib().paro_update_potential(p.handle, _ptr(V), _stream(stream)))


def paro_sigma(p: Problem) -> float:
    return lib().paro_sigma(p.handle)


def paro_ks_solve(p: Problem, Vext, U0, lam, U, opts: KsOpts = None,
                  rho=None, stream=None, workspace=None, history=None):
    """Kohn-Sham outer iteration (see paro_ks_solve in include/paro.h);
    returns the report (status PARO_ENOCONV if max_iter was reached).
    history: optional float64 numpy array of max_iter values that receives
    the density residual of every outer iteration."""
    import numpy as np
    import torch
    opts = opts or ks_default_opts()
    _f64(Vext, ((p.box.nx + 1) * (p.box.ny + 1) * (p.box.nz + 1),), "Vext")
    _f64(U0, (p.n, p.Nt), "U0")
    _f64(U, (p.n, p.Nt), "U")
    _f64(lam, (p.Nt,), "lambda")
    if rho is not None:
        _f64(rho, (p.n,), "rho")
    nbytes = ctypes.c_size_t()
    _check(lib().paro_ks_query(ctypes.byref(p.box), ctypes.byref(nbytes)))
    if workspace is None:
        workspace = torch.empty(nbytes.value + 256, dtype=torch.uint8,
                                device=U.device)
    base = workspace.data_ptr()
    off = (-base) % 256
    rep = KsReport()
    hptr = None
    if history is not None:
        if not (isinstance(history, np.ndarray) and history.dtype ==
                np.float64 and history.size >= opts.max_iter and
                history.flags.c_contiguous):
            raise ValueError("history: contiguous float64, max_iter values")
        hptr = history.ctypes.data
    _check(lib().paro_ks_solve(p.handle, _ptr(Vext), ctypes.byref(opts),
                               base + off, workspace.numel() - off, _ptr(U0),
                               _ptr(lam), _ptr(U), _ptr(rho), hptr,
                               _stream(stream), ctypes.byref(rep)),
           allow=(PARO_ENOCONV,))
    return rep
