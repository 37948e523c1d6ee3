"""Writes the stored expected values under tests/golden/.

Calls only the oracle (and the seeded input generators).  Each output file
records the command and the oracle routine that produced it.

    python tests/golden/make_golden.py [name ...]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import fem, paro, reference  # noqa: E402
from paper_1405_0260_amd import inputs  # noqa: E402


def save(name, arr, header):
    path = os.path.join(HERE, name)
    np.savetxt(path, np.atleast_1d(arr), fmt="%.17g",
               header=header + "\nwritten by: python tests/golden/make_golden.py")
    print("wrote", path)


def harmonic_48c():
    nc = 48
    mesh = fem.kuhn_mesh(nc, -6.0, 6.0)
    H, M = fem.hamiltonian(mesh, inputs.harmonic_potential(nc, -6.0, 6.0))
    lam, _ = reference.sparse_lowest(H, M, 10, -0.5)
    save("harmonic_48c_lowest10.txt", lam,
         "Lowest 10 P1 eigenvalues, V=|x|^2/2, box [-6,6]^3, 48^3 Kuhn cells\n"
         "oracle.reference.sparse_lowest (shift-invert Lanczos)")


def harmonic_24c():
    """Config of the 30-step plain FP64 run: the converged pairs and the
    ParO iterate after 30 steps from the seeded start."""
    w = inputs.harmonic_24()
    mesh = fem.kuhn_mesh(w.nc, w.lo, w.hi)
    H, M = fem.hamiltonian(mesh, w.V)
    lam, _ = reference.sparse_lowest(H, M, 10, -0.5)
    save("harmonic_24c_lowest10.txt", lam,
         "Lowest 10 P1 eigenvalues, V=|x|^2/2, box [-6,6]^3, 24^3 Kuhn cells\n"
         "oracle.reference.sparse_lowest (shift-invert Lanczos)")
    r = paro.paro_solve(H, M, w.U0(), w.N, V_nodal=w.V, max_steps=30,
                        rtol=1e-12)
    save("harmonic_24c_paro30_lambda.txt", r.lam_all,
         "ParO iterate after 30 steps, N=4, m=0, orbital seed 1, sigma=0,\n"
         "PCG rtol 1e-12: oracle.paro.paro_solve")
    hist = np.array(r.lam_history)
    save("harmonic_24c_paro30_history.txt", hist,
         "Ritz values per ParO step (row 0 = Rayleigh-Ritz of the seeded "
         "start)\noracle.paro.paro_solve, same run as paro30_lambda")


def molecule_64c():
    w = inputs.molecule_64()
    mesh = fem.kuhn_mesh(w.nc, w.lo, w.hi)
    H, M = fem.hamiltonian(mesh, w.V)
    s = paro.shift_from_potential(w.V)
    t = time.time()
    lam, _ = reference.sparse_lowest(H, M, w.Nt + 1, s)
    save("softcoulomb_64c_lowest.txt", lam,
         f"Lowest {w.Nt + 1} P1 eigenvalues of the 8-centre soft-Coulomb "
         "workload, 64^3 cells on [-10,10]^3\n"
         f"oracle.reference.sparse_lowest about sigma={s!r} "
         f"({time.time() - t:.0f} s)")


def linear_96c(nc=96, workers=None):
    """The linear eigenproblem of the 96^3 Kohn-Sham workload's external
    potential (20 centres, N = 32, m = 8): the oracle's ParO run from the
    seeded start to convergence (shift-invert Lanczos does not fit: its
    sparse LU at 857,375 dofs needs tens of GB).  The source problems of
    each step run in worker processes; the iterates are the serial ones."""
    w = inputs.kohn_sham_96(nc=nc)
    mesh = fem.kuhn_mesh(w.nc, w.lo, w.hi)
    H, M = fem.hamiltonian(mesh, w.V)
    workers = workers or min(8, os.cpu_count() or 1)
    t = time.time()

    def progress(k, lam, U):
        if k % 25 == 0:
            print(f"  step {k}: lambda_N {lam[w.N - 1]!r} "
                  f"({time.time() - t:.0f} s)", flush=True)

    r = paro.paro_solve(H, M, w.U0(), w.N, V_nodal=w.V, max_steps=3000,
                        lambda_tol=1e-13, resid_tol=1e-9, rtol=1e-11,
                        workers=workers, callback=progress)
    assert r.converged, "oracle ParO did not converge"
    rho = paro.residuals(H, M, r.lam_all, r.U_all)
    save(f"linear_{nc}c_lowest.txt", r.lam_all,
         f"All {w.Nt} Ritz values (the lowest {w.N} are the answer) of the "
         f"{nc}^3 linear problem of the 20-centre workload, box [-14,14]^3\n"
         f"oracle.paro.paro_solve to lambda_tol 1e-13, resid_tol 1e-9, "
         f"PCG rtol 1e-11, {r.steps} steps, sigma={r.sigma!r}, max residual "
         f"of the requested pairs {rho[:w.N].max():.3e} "
         f"({time.time() - t:.0f} s, {workers} worker processes)")


def _member_lowest(name, ws, members, title):
    """Lowest N eigenvalues of the chosen members of a problem list
    (shift-invert Lanczos about the oracle's shift), one line per member:
    'j name lam_1 ... lam_N' (the name identifies the member's recipe, so a
    reader can tell a different list apart)."""
    lines = []
    for j in members:
        w = ws[j]
        mesh = fem.kuhn_mesh(w.nc, w.lo, w.hi)
        H, M = fem.hamiltonian(mesh, w.V)
        s = paro.shift_from_potential(w.V) - 0.5
        # Lanczos can miss a copy of a degenerate eigenvalue near the end
        # of the wanted range: ask for the whole buffered range plus more,
        # twice with different counts, and keep the N lowest only if the
        # two agree.
        lam, _ = reference.sparse_lowest(H, M, w.Nt + 2, s)
        lam2, _ = reference.sparse_lowest(H, M, w.Nt + 6, s)
        assert np.allclose(lam[:w.N], lam2[:w.N], rtol=1e-12, atol=0), \
            (w.name, lam[:w.N], lam2[:w.N])
        lines.append(f"{j} {w.name} " +
                     " ".join(f"{x:.17g}" for x in lam[:w.N]))
        print(f"  {w.name}: {lam[:min(3, w.N)]}", flush=True)
    path = os.path.join(HERE, name)
    with open(path, "w") as f:
        f.write(f"# {title}\n# oracle.reference.sparse_lowest (shift-invert "
                "Lanczos about the oracle's shift - 0.5), lowest N per member"
                "\n# line: member index, member name, then its N requested "
                "eigenvalues\n"
                "# written by: python tests/golden/make_golden.py\n")
        f.write("\n".join(lines) + "\n")
    print("wrote", path)


def batch_sample():
    _member_lowest("batch64_sample_lowest.txt", inputs.batch_64(),
                   [3, 7, 15, 22, 26, 44, 47],
                   "Sampled members of the 64-problem uneven batch "
                   "(paper_1405_0260_amd.inputs.batch_64)")


def serve_sample():
    _member_lowest("serve_sample_lowest.txt", inputs.serve_requests(64),
                   [1, 2, 10, 14, 18],
                   "Sampled requests of the served stream "
                   "(paper_1405_0260_amd.inputs.serve_requests(64))")


JOBS = {"harmonic_48c": harmonic_48c, "harmonic_24c": harmonic_24c,
        "molecule_64c": molecule_64c, "linear_96c": linear_96c,
        "batch_sample": batch_sample, "serve_sample": serve_sample}

if __name__ == "__main__":
    for name in (sys.argv[1:] or list(JOBS)):
        JOBS[name]()
