"""Seeded synthetic inputs for the ParO eigenproblems.

This module only draws random numbers and evaluates the given potential
functions at mesh vertices.  It holds none of the method's arithmetic (no
finite-element assembly, no solver), so the CPU oracle and the HIP path can
both be fed from it without sharing any computation.

Every workload is a box [lo, hi]^3 cut into nc^3 cubes (nc cells per axis);
potential values are given at all (nc+1)^3 vertices, x fastest.  The
interior degrees of freedom number (nc-1)^3.  Initial orbitals are standard
normal draws of shape (n_dof, N + m), rows = interior dofs (x fastest),
columns = orbitals.

Random-number recipe (numpy PCG64 via ``default_rng``):
  * harmonic oscillator V = |x|^2 / 2 (no random numbers);
  * soft-Coulomb V = -sum_k Z_k / sqrt(|x - R_k|^2 + 0.1): from one
    generator, first ``Z = integers(1, zmax + 1, size=K)`` then
    ``R = uniform(-r, r, size=(K, 3))``;
  * orbitals: ``default_rng(seed).standard_normal((n_dof, N + m))``.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

SOFT_EPS = 0.1  # softening constant of the soft-Coulomb potential


@dataclasses.dataclass
class Workload:
    """One eigenproblem: box, grid, nodal potential, orbital counts, start."""

    name: str
    nc: int                 # cells per axis (same in x, y, z)
    lo: float
    hi: float
    N: int                  # requested orbitals
    m: int                  # buffer orbitals (Algorithm 3.2); N_t = N + m
    V: np.ndarray           # nodal potential, shape ((nc+1)^3,), x fastest
    orbital_seed: int
    kind: str = "ho"        # "ho" or "soft_coulomb"
    Z: Optional[np.ndarray] = None
    R: Optional[np.ndarray] = None
    max_steps: int = 200

    @property
    def n_dof(self) -> int:
        return (self.nc - 1) ** 3

    @property
    def Nt(self) -> int:
        return self.N + self.m

    def U0(self) -> np.ndarray:
        return initial_orbitals(self.n_dof, self.Nt, self.orbital_seed)


def vertex_coords(nc, lo, hi) -> np.ndarray:
    """Coordinates of all vertices, x fastest, shape (nv, 3).  nc is an int
    or (nx, ny, nz); lo, hi are scalars or 3-vectors."""
    ncs = (nc, nc, nc) if np.isscalar(nc) else tuple(int(c) for c in nc)
    lo = np.broadcast_to(np.asarray(lo, dtype=np.float64), (3,))
    hi = np.broadcast_to(np.asarray(hi, dtype=np.float64), (3,))
    axes = [lo[a] + (hi[a] - lo[a]) / ncs[a] * np.arange(ncs[a] + 1)
            for a in range(3)]
    z, y, x = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)


def harmonic_potential(nc: int, lo: float, hi: float) -> np.ndarray:
    X = vertex_coords(nc, lo, hi)
    return 0.5 * np.sum(X * X, axis=1)


def soft_coulomb_centres(seed: int, count: int, zmax: int, r: float):
    rng = np.random.default_rng(seed)
    Z = rng.integers(1, zmax + 1, size=count).astype(np.float64)
    R = rng.uniform(-r, r, size=(count, 3))
    return Z, R


def soft_coulomb_at(X: np.ndarray, Z, R) -> np.ndarray:
    """The soft-Coulomb potential of centres (Z, R) at the points X (the
    vertices of any mesh)."""
    V = np.zeros(X.shape[0])
    for zk, rk in zip(Z, R):
        d2 = np.sum((X - rk) ** 2, axis=1)
        V -= zk / np.sqrt(d2 + SOFT_EPS)
    return V


def soft_coulomb_potential(nc, lo, hi, Z, R) -> np.ndarray:
    return soft_coulomb_at(vertex_coords(nc, lo, hi), Z, R)


def initial_orbitals(n_dof: int, Nt: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).standard_normal((n_dof, Nt))


# --------------------------------------------------------------------------
# The named workloads.
# --------------------------------------------------------------------------

def harmonic(nc=24, N=4, m=0, seed=1, lo=-6.0, hi=6.0, max_steps=30,
             name=None) -> Workload:
    """3D harmonic oscillator V = |x|^2/2; continuum spectrum n + 3/2."""
    return Workload(name or f"harmonic_{nc}c_N{N}", nc, lo, hi, N, m,
                    harmonic_potential(nc, lo, hi), seed, "ho",
                    max_steps=max_steps)


def molecule(nc=64, N=16, m=8, pot_seed=2, seed=12, centres=8, zmax=6,
             spread=3.0, lo=-10.0, hi=10.0, max_steps=400,
             name=None) -> Workload:
    """Synthetic molecule: soft-Coulomb centres with random charges."""
    Z, R = soft_coulomb_centres(pot_seed, centres, zmax, spread)
    return Workload(name or f"softcoulomb_{nc}c_N{N}", nc, lo, hi, N, m,
                    soft_coulomb_potential(nc, lo, hi, Z, R), seed,
                    "soft_coulomb", Z, R, max_steps=max_steps)


def harmonic_24():
    """24^3 cells on [-6,6]^3, N = 4, 30 ParO steps, orbital seed 1."""
    return harmonic()


def molecule_64():
    """8 soft-Coulomb centres (Z in 1..6, R in [-3,3]^3, seed 2) on
    [-10,10]^3 with 64^3 cells, N = 16 (+ m buffer), orbital seed 12."""
    return molecule()


def kohn_sham_96(nc=96):
    """20 soft-Coulomb centres (Z in 1..8, R in [-5,5]^3, seed 3) on
    [-14,14]^3 with 96^3 cells, N = 32 occupied orbitals, seed 13."""
    return molecule(nc=nc, N=32, m=8, pot_seed=3, seed=13, centres=20,
                    zmax=8, spread=5.0, lo=-14.0, hi=14.0,
                    name=f"kohnsham_{nc}c_N32")


def batch_64(count: int = 64, seed: int = 4, nc_lo=16, nc_hi=48,
             n_lo=2, n_hi=24) -> List[Workload]:
    """Uneven batch: nc ~ U{nc_lo..nc_hi}, N ~ U{n_lo..n_hi}, half harmonic
    (box +-6), half soft-Coulomb (8 centres, Z 1..6, R in [-3,3]^3, box
    +-10).  Member j draws its potential and orbitals from seed 4000 + j.
    Buffers: harmonic members close the shell above N; soft-Coulomb
    members carry N // 2 + 4 buffer orbitals."""
    rng = np.random.default_rng(seed)
    ncs = rng.integers(nc_lo, nc_hi + 1, size=count)
    Ns = rng.integers(n_lo, n_hi + 1, size=count)
    kinds = rng.integers(0, 2, size=count)
    out = []
    for j in range(count):
        nc, N = int(ncs[j]), int(Ns[j])
        s = 4000 + j
        if kinds[j] == 0:
            m = harmonic_buffer(N)
            out.append(harmonic(nc=nc, N=N, m=m, seed=s, max_steps=300,
                                name=f"b{j}_ho_{nc}c_N{N}"))
        else:
            out.append(molecule(nc=nc, N=N, m=N // 2 + 4, pot_seed=s,
                                seed=s + 100000, max_steps=1000,
                                name=f"b{j}_sc_{nc}c_N{N}"))
    return out


def harmonic_buffer(N: int) -> int:
    """Buffer orbitals that close the harmonic shell above N (shell sizes
    1, 3, 6, 10, ... give closures at 1, 4, 10, 20, 35) plus one."""
    closure = 1
    k = 1
    while closure < N:
        k += 1
        closure += k * (k + 1) // 2
    nxt = closure + (k + 1) * (k + 2) // 2
    return nxt - N if nxt - N <= 16 else closure - N + 1


def gaussian_projectors(nc: int, lo: float, hi: float, centres: np.ndarray,
                        width: float = 1.0, height: float = 1.0) -> np.ndarray:
    """Synthetic nonlocal projectors: one Gaussian per centre,
    zeta_j(x) = height exp(-|x - R_j|^2 / (2 width^2)), sampled at the
    interior vertices (n_dof x len(centres), x fastest)."""
    X = vertex_coords(nc, lo, hi)
    m = nc + 1
    inner = np.zeros((m, m, m), dtype=bool)
    inner[1:-1, 1:-1, 1:-1] = True
    Xi = X[inner.reshape(-1)]
    d2 = ((Xi[:, None, :] - np.asarray(centres)[None, :, :]) ** 2).sum(-1)
    return height * np.exp(-d2 / (2.0 * width * width))


def serve_requests(count: int, seed: int = 5, big_fraction: float = 0.25,
                   big_nc: int = 64) -> List[Workload]:
    """Request mix of the served stream: a fraction `big_fraction` of
    soft-Coulomb problems like the 64^3, N = 16 workload (own potential per
    request), the rest drawn like the members of the uneven batch.
    Request j draws from seed 5000 + j."""
    rng = np.random.default_rng(seed)
    big = rng.random(count) < big_fraction
    ncs = rng.integers(16, 49, size=count)
    Ns = rng.integers(2, 25, size=count)
    kinds = rng.integers(0, 2, size=count)
    out = []
    for j in range(count):
        s = 5000 + j
        if big[j]:
            out.append(molecule(nc=big_nc, N=16, m=8, pot_seed=s,
                                seed=s + 100000, max_steps=1000,
                                name=f"r{j}_sc_{big_nc}c_N16"))
        elif kinds[j] == 0:
            N = int(Ns[j])
            out.append(harmonic(nc=int(ncs[j]), N=N, m=harmonic_buffer(N),
                                seed=s, max_steps=300,
                                name=f"r{j}_ho_{ncs[j]}c_N{N}"))
        else:
            N = int(Ns[j])
            out.append(molecule(nc=int(ncs[j]), N=N, m=N // 2 + 4,
                                pot_seed=s, seed=s + 100000, max_steps=1000,
                                name=f"r{j}_sc_{ncs[j]}c_N{N}"))
    return out


def arrivals(count: int, rate_hz: float, seed: int = 5) -> np.ndarray:
    """Poisson arrival times (seconds) of ``count`` requests."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_hz, size=count))
