"""Helpers for the GPU tests: device tensors for a workload and the
oracle's matrices for the same inputs (no method arithmetic here)."""
import sys

import numpy as np

from oracle import fem, paro as oparo
from paper_1405_0260_amd import binding as pb
from paper_1405_0260_amd import inputs


def device():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a HIP device")
    return torch.device("cuda:0")


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(device())


def box_of(ncs, lo, hi):
    ncs = (ncs,) * 3 if np.isscalar(ncs) else tuple(ncs)
    lo = (lo,) * 3 if np.isscalar(lo) else tuple(lo)
    hi = (hi,) * 3 if np.isscalar(hi) else tuple(hi)
    import ctypes
    return pb.Box(ncs[0], ncs[1], ncs[2], (ctypes.c_double * 3)(*lo),
                  (ctypes.c_double * 3)(*hi))


def assemble(ncs, lo, hi, V, N, m=0, **opts):
    note(f"assemble {ncs} [{lo},{hi}] N={N} m={m} {opts}")
    o = pb.default_opts(N=N, m=m, **opts)
    return pb.paro_assemble(box_of(ncs, lo, hi), to_dev(V), o)


def workload_problem(w: inputs.Workload, **opts):
    return assemble(w.nc, w.lo, w.hi, w.V, w.N, w.m, **opts)


def oracle_matrices(ncs, lo, hi, V):
    mesh = fem.kuhn_mesh(ncs, lo, hi)
    H, M = fem.hamiltonian(mesh, V)
    return H, M, oparo.shift_from_potential(V)


def solve(prob, U0, sync=True):
    import torch
    lam = torch.zeros(prob.Nt, dtype=torch.float64, device=device())
    U = torch.zeros(prob.n, prob.Nt, dtype=torch.float64, device=device())
    rep = pb.paro_solve(prob, to_dev(U0), lam, U)
    if sync:
        torch.cuda.synchronize()
    return lam.cpu().numpy(), U.cpu().numpy(), rep
