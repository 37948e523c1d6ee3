"""General bisection meshes on the GPU against the oracle.

Every mesh here is the oracle's (adapt.from_kuhn / adapt.refine) handed to
the library as arrays, so no oracle input comes from the library: the CSR
operator against the oracle's assembly, ParO solves and steps against
dense eigenpairs and the oracle's iterates, the estimator against the
oracle's, the transfer against the oracle's prolongation, a whole adaptive
run driven by the oracle's marks against the oracle's adaptive ParO, and
a mesh problem in a batch bitwise equal to the same problem alone.  The
library's own refinement is checked on the host (test_mesh_host.py) and in
one GPU-only adaptive loop by properties."""
import ctypes

import numpy as np
import pytest

from oracle import adapt, fem, paro as oparo, reference
from paper_1405_0260_amd import binding as pb
from paper_1405_0260_amd import inputs
import gpu_util as gu
from paro_checks import m_orthonormality_error, rel_lambda_err, subspace_sine

pytestmark = pytest.mark.gpu

LO, HI = -5.0, 5.0
Z, R = np.array([3.0, 1.5]), np.array([[0.4, -0.3, 0.2], [-1.2, 0.8, -0.5]])


def _box(nc, lo=LO, hi=HI):
    ncs = (nc,) * 3 if np.isscalar(nc) else tuple(nc)
    lo = (lo,) * 3 if np.isscalar(lo) else tuple(lo)
    hi = (hi,) * 3 if np.isscalar(hi) else tuple(hi)
    return pb.Box(ncs[0], ncs[1], ncs[2], (ctypes.c_double * 3)(*lo),
                  (ctypes.c_double * 3)(*hi))


def _vfun(X):
    return inputs.soft_coulomb_at(X, Z, R)


def _oracle_mesh(nc=6, rounds=3, seed=0, frac=0.12):
    """A locally refined oracle mesh: random marks near the centres."""
    rng = np.random.default_rng(seed)
    m = adapt.from_kuhn(nc, LO, HI)
    for _ in range(rounds):
        c = m.X[m.tets].mean(axis=1)
        d = np.min(np.linalg.norm(c[:, None, :] - R[None], axis=2), axis=1)
        k = max(1, int(frac * m.tets.shape[0]))
        near = np.argsort(d, kind="stable")[:2 * k]
        m = adapt.refine(m, np.sort(rng.choice(near, size=k, replace=False)))
    return m


def _lib_mesh(o, nc=6):
    return pb.Mesh.from_arrays(_box(nc), o.X, o.tets, o.tags, o.parents)


def _problem(o, N, m=0, nc=6, **kw):
    mesh = _lib_mesh(o, nc)
    gu.note(f"mesh problem: {o.X.shape[0]} vertices, {o.tets.shape[0]} "
            f"elements, N={N} m={m}")
    return pb.paro_mesh_assemble(mesh, gu.to_dev(_vfun(o.X)),
                                 pb.default_opts(N=N, m=m, **kw))


def _oracle_ops(o):
    V = _vfun(o.X)
    H, M = fem.hamiltonian(o.fem_mesh(), V)
    return H, M, oparo.shift_from_potential(V)


def _export(p):
    import torch
    dev = gu.device()
    rp = torch.zeros(p.n + 1, dtype=torch.int32, device=dev)
    col = torch.zeros(p.nnz, dtype=torch.int32, device=dev)
    A = torch.zeros(p.nnz, dtype=torch.float64, device=dev)
    Mv = torch.zeros(p.nnz, dtype=torch.float64, device=dev)
    sig = ctypes.c_double()
    pb._check(pb.lib().paro_export_csr(p.handle, rp.data_ptr(),
                                       col.data_ptr(), A.data_ptr(),
                                       Mv.data_ptr(), ctypes.byref(sig),
                                       None))
    import scipy.sparse as sp
    rp, col = rp.cpu().numpy(), col.cpu().numpy()
    shape = (p.n, p.n)
    return (sp.csr_matrix((A.cpu().numpy(), col, rp), shape=shape),
            sp.csr_matrix((Mv.cpu().numpy(), col, rp), shape=shape),
            sig.value)


@pytest.mark.parametrize("rounds", [0, 3])
def test_csr_operator_matches_the_oracle_assembly(rounds):
    o = _oracle_mesh(rounds=rounds)
    p = _problem(o, N=2)
    A, M, s = _export(p)
    H, Mo, so = _oracle_ops(o)
    assert s == so
    As = (H - so * Mo).tocsr()
    assert abs(A - As).max() <= 1e-13 * abs(As).max()
    assert abs(M - Mo).max() <= 1e-13 * abs(Mo).max()
    # Sorted column indices per row, the diagonal among them.
    for r in range(0, p.n, max(1, p.n // 50)):
        cols = A.indices[A.indptr[r]:A.indptr[r + 1]]
        assert np.all(np.diff(cols) > 0) and r in cols


@pytest.mark.parametrize("rounds", [2, 4])
def test_solve_on_a_refined_mesh_matches_dense(rounds):
    o = _oracle_mesh(rounds=rounds, seed=rounds)
    N, m = 3, 2
    p = _problem(o, N=N, m=m, max_steps=600, lambda_tol=1e-13,
                 resid_tol=1e-9)
    U0 = inputs.initial_orbitals(p.n, N + m, 7)
    lam, U, rep = gu.solve(p, U0)
    assert rep.status == 0, rep.as_dict()
    H, M, _ = _oracle_ops(o)
    ref, Uref = reference.dense_lowest(H, M, N + m + 1)
    assert rel_lambda_err(lam[:N], ref[:N]) < 1e-9
    assert m_orthonormality_error(M, U) < 1e-11
    assert subspace_sine(M, U[:, :1], Uref[:, :1]) < 1e-6


def test_steps_match_the_oracle_iterates():
    """Thirty public steps against the oracle's ParO history."""
    import torch
    o = _oracle_mesh(rounds=3, seed=9)
    N, m = 2, 2
    p = _problem(o, N=N, m=m, pcg_rtol=1e-12)
    U0 = inputs.initial_orbitals(p.n, N + m, 11)
    lam = torch.zeros(N + m, dtype=torch.float64, device=gu.device())
    U = torch.zeros(p.n, N + m, dtype=torch.float64, device=gu.device())
    pb.paro_init(p, gu.to_dev(U0), lam, U)
    hist = [lam.cpu().numpy().copy()]
    for _ in range(30):
        pb.paro_step(p, lam, U)
        hist.append(lam.cpu().numpy().copy())
    H, M, _ = _oracle_ops(o)
    r = oparo.paro_solve(H, M, U0, N, V_nodal=_vfun(o.X), max_steps=30,
                         rtol=1e-12, lambda_tol=0.0, resid_tol=0.0)
    for k in range(31):
        assert rel_lambda_err(hist[k], r.lam_history[k]) < 1e-9, k


def test_estimator_matches_the_oracle():
    o = _oracle_mesh(rounds=3, seed=3)
    H, M, _ = _oracle_ops(o)
    lam, U = reference.dense_lowest(H, M, 4)
    ref = adapt.estimator(o, _vfun(o.X), lam[:3], U[:, :3])
    import torch
    p = _problem(o, N=3, m=1)
    eta = torch.zeros(o.tets.shape[0], dtype=torch.float64,
                      device=gu.device())
    pb.paro_mesh_estimate(p, gu.to_dev(lam), gu.to_dev(U), 3, eta)
    got = eta.cpu().numpy()
    assert np.allclose(got, ref, rtol=1e-10, atol=1e-13 * ref.max())


def test_transfer_matches_the_oracle_prolongation():
    import torch
    coarse = _oracle_mesh(rounds=1, seed=4)
    fine = adapt.refine(adapt.refine(coarse, np.arange(0, coarse.tets.shape[0],
                                                       5)), [3, 11, 40])
    U = np.random.default_rng(8).standard_normal(
        (int((coarse.dof >= 0).sum()), 5))
    ref = adapt.prolong(coarse, fine, U)
    lc, lf = _lib_mesh(coarse), _lib_mesh(fine)
    Uf = torch.zeros(ref.shape, dtype=torch.float64, device=gu.device())
    pb.paro_mesh_prolong(lc, lf, gu.to_dev(U), Uf)
    assert np.array_equal(Uf.cpu().numpy(), ref)


def test_uniform_mesh_problem_agrees_with_the_box_problem():
    """The Kuhn mesh as a general mesh: the same operator (CSR vs the
    stencil's CSR copy) and the same converged pairs."""
    nc = 7
    box = _box(nc)
    X = inputs.vertex_coords(nc, LO, HI)
    V = _vfun(X)
    opts = dict(N=3, m=2, max_steps=500, lambda_tol=1e-13, resid_tol=1e-9)
    pm = pb.paro_mesh_assemble(pb.Mesh.kuhn(box), gu.to_dev(V),
                               pb.default_opts(**opts))
    pbx = pb.paro_assemble(box, gu.to_dev(V), pb.default_opts(**opts))
    A1, M1, s1 = _export(pm)
    A2, M2, s2 = _export(pbx)
    assert s1 == s2
    assert abs(A1 - A2).max() <= 1e-13 * abs(A2).max()
    assert abs(M1 - M2).max() <= 1e-13 * abs(M2).max()
    U0 = inputs.initial_orbitals(pm.n, 5, 3)
    l1, _, r1 = gu.solve(pm, U0)
    l2, _, r2 = gu.solve(pbx, U0)
    assert r1.status == r2.status == 0
    assert rel_lambda_err(l1[:3], l2[:3]) < 1e-11


def test_component_calls_on_a_mesh_problem():
    """paro_spmm (H X, M X) and paro_pcg ((H - s M) X = B) on a mesh."""
    import torch
    o = _oracle_mesh(rounds=2, seed=6)
    p = _problem(o, N=4)
    H, M, s = _oracle_ops(o)
    X = np.random.default_rng(2).standard_normal((p.n, 4))
    Y = torch.zeros(p.n, 4, dtype=torch.float64, device=gu.device())
    for which, op in ((2, H), (1, M)):  # H X, M X
        pb.paro_spmm(p, which, gu.to_dev(X), Y)
        want = op @ X
        assert np.abs(Y.cpu().numpy() - want).max() <= 1e-12 * np.abs(want).max()
    B = M @ X
    Xs = torch.zeros(p.n, 4, dtype=torch.float64, device=gu.device())
    pb.paro_pcg(p, gu.to_dev(B), Xs)
    A = (H - s * M).tocsr()
    r = B - A @ Xs.cpu().numpy()
    assert np.linalg.norm(r) <= 2e-10 * np.linalg.norm(B)


def test_mesh_problem_in_a_batch_is_bitwise_its_solve_alone():
    import torch
    o = _oracle_mesh(rounds=3, seed=12)
    w = inputs.harmonic(nc=10, N=3, m=3, seed=5)
    pm = _problem(o, N=2, m=2, max_steps=400, lambda_tol=1e-12,
                  resid_tol=1e-9)
    pbx = gu.workload_problem(w, max_steps=400, lambda_tol=1e-12,
                              resid_tol=1e-9)
    probs = [pm, pbx]
    U0s = [inputs.initial_orbitals(pm.n, 4, 1), w.U0()]
    batch = pb.Batch(2)
    lams = [torch.zeros(p.Nt, dtype=torch.float64, device=gu.device())
            for p in probs]
    Us = [torch.zeros(p.n, p.Nt, dtype=torch.float64, device=gu.device())
          for p in probs]
    reps = pb.paro_batch_solve(batch, probs, [gu.to_dev(u) for u in U0s],
                               lams, Us)
    torch.cuda.synchronize()
    for k, p in enumerate(probs):
        assert reps[k].status == 0
        la, Ua, ra = gu.solve(p, U0s[k])
        assert ra.steps == reps[k].steps
        assert np.array_equal(la, lams[k].cpu().numpy())
        assert np.array_equal(Ua, Us[k].cpu().numpy())


def test_adaptive_run_with_the_oracles_marks_matches_the_oracle():
    """Algorithm 3.1 with Step 2 on the oracle's meshes: each refining step
    carries the GPU orbitals over with the library's transfer, assembles
    on the new mesh and steps there.  The meshes and marks are the
    oracle's (adapt.adaptive_paro with the same theta and steps)."""
    import torch
    m0 = adapt.from_kuhn(5, LO, HI)
    N, Nt = 2, 4
    U0 = inputs.initial_orbitals(int((m0.dof >= 0).sum()), Nt, 21)
    steps, refine_steps = 14, range(4, 8)
    ref = adapt.adaptive_paro(m0, _vfun, U0, N, steps=steps, theta=0.4,
                              refine_steps=refine_steps)
    # Replay the oracle's mesh sequence: refine with the oracle at the same
    # steps from its own estimator (the run is deterministic).
    meshes = [m0]
    mesh = m0
    V = _vfun(mesh.X)
    H, M = fem.hamiltonian(mesh.fem_mesh(), V)
    lam_o, U_o = oparo.rayleigh_ritz(H, M, U0)
    for step in range(steps):
        if step in refine_steps:
            eta = adapt.estimator(mesh, V, lam_o[:N], U_o[:, :N])
            new = adapt.refine(mesh, adapt.dorfler_mark(eta, 0.4))
            U_o = adapt.prolong(mesh, new, U_o)
            mesh = new
            V = _vfun(mesh.X)
            H, M = fem.hamiltonian(mesh.fem_mesh(), V)
        s = oparo.shift_from_potential(V)
        A = (H - s * M).tocsr()
        lam_o, U_o, _ = oparo.paro_step(H, M, A, 1.0 / A.diagonal(), lam_o,
                                        U_o, s, 1e-12, 10 * U_o.shape[0])
        meshes.append(mesh)
    assert np.allclose(lam_o, ref.lam, rtol=1e-12, atol=0)
    # The GPU run over the same meshes.
    dev = gu.device()
    lib_meshes = {id(mm): _lib_mesh(mm, 5) for mm in meshes}

    def assemble(mm):
        return pb.paro_mesh_assemble(
            lib_meshes[id(mm)], gu.to_dev(_vfun(mm.X)),
            pb.default_opts(N=N, m=Nt - N, pcg_rtol=1e-12))

    cur = meshes[0]
    p = assemble(cur)
    lam = torch.zeros(Nt, dtype=torch.float64, device=dev)
    U = torch.zeros(p.n, Nt, dtype=torch.float64, device=dev)
    pb.paro_init(p, gu.to_dev(U0), lam, U)
    hist = [lam.cpu().numpy().copy()]
    for step in range(steps):
        nxt = meshes[step + 1]
        if nxt is not cur:
            p2 = assemble(nxt)
            U2 = torch.zeros(p2.n, Nt, dtype=torch.float64, device=dev)
            pb.paro_mesh_prolong(lib_meshes[id(cur)], lib_meshes[id(nxt)], U,
                                 U2)
            p, U, cur = p2, U2, nxt
        pb.paro_step(p, lam, U)
        hist.append(lam.cpu().numpy().copy())
    for k in range(steps + 1):
        assert rel_lambda_err(hist[k], ref.lam_history[k]) < 1e-9, k


def test_gpu_adaptive_loop_refines_at_the_centres_and_converges():
    """The whole Step 2 on the library alone: estimate and mark on the GPU,
    refine on the host, transfer, assemble and solve on the GPU.  Every
    solve converges, the new vertices gather at the potential's centres,
    and the lowest eigenvalue on the last mesh lies well below the one on
    the coarse first mesh, which cannot resolve the wells."""
    import torch
    dev = gu.device()
    mesh = pb.Mesh.kuhn(_box(6))
    N, Nt = 1, 3
    lam0 = []
    U_prev = None
    prev_mesh = None
    for it in range(4):
        X = mesh.arrays()["X"]
        p = pb.paro_mesh_assemble(mesh, gu.to_dev(_vfun(X)),
                                  pb.default_opts(N=N, m=Nt - N,
                                                  max_steps=800,
                                                  lambda_tol=1e-12,
                                                  resid_tol=1e-9))
        if U_prev is None:
            U0 = gu.to_dev(inputs.initial_orbitals(p.n, Nt, 2))
        else:
            U0 = torch.zeros(p.n, Nt, dtype=torch.float64, device=dev)
            pb.paro_mesh_prolong(prev_mesh, mesh, U_prev, U0)
        lam = torch.zeros(Nt, dtype=torch.float64, device=dev)
        U = torch.zeros(p.n, Nt, dtype=torch.float64, device=dev)
        rep = pb.paro_solve(p, U0, lam, U)
        assert rep.status == 0, (it, rep.as_dict())
        lam0.append(float(lam[0]))
        gu.note(f"adaptive round {it}: {p.n} dofs, lambda_0 {lam0[-1]:.8f}, "
                f"{rep.steps} steps")
        _, ne, _ = mesh.info()
        eta = torch.zeros(ne, dtype=torch.float64, device=dev)
        pb.paro_mesh_estimate(p, lam, U, N, eta)
        marked, cnt = pb.paro_mark(eta, 0.5, pb.PARO_MARK_DORFLER)
        assert 0 < cnt < ne
        prev_mesh, U_prev = mesh, U
        mesh = mesh.refine(marked)
    a = mesh.arrays()
    new = a["X"][a["parents"][:, 0] >= 0]
    d = np.min(np.linalg.norm(new[:, None, :] - R[None], axis=2), axis=1)
    d_all = np.min(np.linalg.norm(a["X"][:, None, :] - R[None], axis=2),
                   axis=1)
    assert np.median(d) < 0.5 * np.median(d_all)
    assert lam0[-1] < lam0[0] - 1e-3 * abs(lam0[0]), lam0
