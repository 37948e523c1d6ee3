"""Source solves on meshes large enough that the CG SpMM leaves its plain
one-tile-per-segment form:

* 81^3 = 531,441 rows (more than 2048 tiles of 248 rows) takes the
  z-marching SpMM: 26 xy tiles per 80 x 80 plane, 16 ranges of 5 planes,
  one p.q partial per (range, tile);
* a flat 289 x 289 x 8 box (83,521-row planes, too many xy tiles for the
  z-march) keeps the row sweep with slab segments: 8 slabs of tiles, each
  of the 1024 p.q partials covering every 128th tile of a slab.

Checked against the oracle's matrix: the FP64 residual of the result, and
for FP64 the iteration count of the oracle's own Jacobi-PCG on each column
(any error in an iterate changes it)."""
import numpy as np
import pytest

from oracle import paro as oparo
from paper_1405_0260_amd import binding as pb
from paper_1405_0260_amd import inputs
import gpu_util as gu

pytestmark = pytest.mark.gpu

NC = 82  # 81^3 interior dofs
NCOLS = 4


FLAT = (290, 290, 9)   # 289 x 289 x 8 interior vertices


def _case(shape):
    if shape == "cube":
        w = inputs.harmonic(nc=NC, N=NCOLS)
        ncs, lo, hi, V = w.nc, w.lo, w.hi, w.V
    else:
        ncs, lo, hi = FLAT, (-6.0, -6.0, -1.5), (6.0, 6.0, 1.5)
        X = inputs.vertex_coords(ncs, lo, hi)
        V = 0.5 * np.sum(X * X, axis=1)
    H, M, s = gu.oracle_matrices(ncs, lo, hi, V)
    A = (H - s * M).tocsr()
    n = A.shape[0]
    assert n > 2048 * 248
    rng = np.random.default_rng(11)
    B = rng.standard_normal((n, NCOLS))
    X0 = rng.standard_normal((n, NCOLS)) * 0.01
    return (ncs, lo, hi, V), A, B, X0


@pytest.fixture(scope="module", params=["cube", "flat"])
def large_case(request):
    return request.param, _case(request.param)


@pytest.mark.parametrize("precision", [pb.PARO_FP64, pb.PARO_FP32_INNER])
def test_pcg_with_segmented_spmm_partials(large_case, precision):
    shape, ((ncs, lo, hi, V), A, B, X0) = large_case
    gu.note(f"large pcg: {shape} {ncs}, n = {A.shape[0]}, ncols = {NCOLS}, "
            f"precision = {precision}")
    prob = gu.assemble(ncs, lo, hi, V, N=NCOLS, precision=precision,
                       pcg_rtol=1e-12)
    Xd = gu.to_dev(X0)
    its = pb.paro_pcg(prob, gu.to_dev(B), Xd)
    X = Xd.cpu().numpy()
    res = np.linalg.norm(B - A @ X, axis=0) / np.linalg.norm(B, axis=0)
    assert np.max(res) <= 1.01e-12, res
    if precision == pb.PARO_FP64:
        dinv = 1.0 / A.diagonal()
        for c in range(NCOLS):
            _, k = oparo.jacobi_pcg(A, B[:, c], X0[:, c], dinv, 1e-12, 20000)
            assert abs(its[c] - k) <= 1, (c, its[c], k)


@pytest.mark.parametrize("precision", [pb.PARO_FP64, pb.PARO_FP32_INNER])
def test_batch_with_segmented_member_matches_alone(precision):
    """A batch of the 81^3 problem (z-marching SpMM) and a 12^3 one (row
    sweep, one tile per segment): the batch launches both SpMM kernels,
    each serving its own problems.  Two ParO steps, bitwise equal to the
    members stepped alone."""
    import torch
    ws = [inputs.harmonic(nc=NC, N=2, m=2, seed=31, max_steps=50),
          inputs.harmonic(nc=12, N=2, m=2, seed=32, max_steps=50)]
    gu.note(f"large batch: n = {[w.n_dof for w in ws]}, "
            f"precision = {precision}")
    probs = [gu.workload_problem(w, precision=precision, pcg_rtol=1e-10)
             for w in ws]
    U0s = [gu.to_dev(w.U0()) for w in ws]

    def outs():
        return ([torch.zeros(p.Nt, dtype=torch.float64, device=gu.device())
                 for p in probs],
                [torch.zeros(p.n, p.Nt, dtype=torch.float64,
                             device=gu.device()) for p in probs])

    batch = pb.Batch(len(probs))
    lams, Us = outs()
    pb.paro_batch_init(batch, probs, U0s, lams, Us)
    lams1, Us1 = outs()
    for p, U0, l1, U1 in zip(probs, U0s, lams1, Us1):
        pb.paro_init(p, U0, l1, U1)
    for step in range(2):
        reps = pb.paro_batch_step(batch, probs, lams, Us)
        for k, p in enumerate(probs):
            r1 = pb.paro_step(p, lams1[k], Us1[k])
            assert reps[k].status == r1.status == pb.PARO_OK, (step, k)
            assert reps[k].pcg_iters == r1.pcg_iters, (step, k)
        torch.cuda.synchronize()
        for k in range(len(probs)):
            assert torch.equal(lams[k], lams1[k]), (step, k)
            assert torch.equal(Us[k], Us1[k]), (step, k)


@pytest.mark.parametrize("precision", [pb.PARO_FP64, pb.PARO_FP32_INNER])
def test_z_march_variants_give_the_same_steps(precision):
    """The z-marching SpMM's tuning choices (1, 2 or 4 chunks per unit,
    full or halved block count) only decide which unit or block serves a
    column: three ParO steps agree bit for bit under every choice."""
    import torch
    w = inputs.harmonic(nc=NC, N=6, m=4, seed=33)
    gu.note(f"z-march variants, precision {precision}")
    pb.paro_set_autotune(False)
    try:
        p = gu.workload_problem(w, precision=precision, pcg_rtol=1e-10)
        _, ns = pb.paro_tuned(p)
        ref = None
        for var in (-1, 0, 1, 2):
            for nb in (ns, max(8, ns // 2 // 8 * 8)):
                pb.paro_set_tuning(p, var, nb)
                lam = torch.zeros(p.Nt, dtype=torch.float64,
                                  device=gu.device())
                U = torch.zeros(p.n, p.Nt, dtype=torch.float64,
                                device=gu.device())
                pb.paro_init(p, gu.to_dev(w.U0()), lam, U)
                its = [pb.paro_step(p, lam, U).pcg_iters for _ in range(3)]
                got = (lam.cpu().numpy(), U.cpu().numpy(), its)
                if ref is None:
                    ref = got
                    continue
                assert got[2] == ref[2], (var, nb)
                assert np.array_equal(got[0], ref[0]), (var, nb)
                assert np.array_equal(got[1], ref[1]), (var, nb)
        with pytest.raises(pb.ParoError):
            pb.paro_set_tuning(p, 3, ns)
    finally:
        pb.paro_set_autotune(True)


@pytest.mark.parametrize("ncols", [7, 10])
@pytest.mark.parametrize("precision", [pb.PARO_FP64, pb.PARO_FP32_INNER])
def test_matrix_free_spmm_is_bitwise_the_stored_one(ncols, precision):
    """The matrix-free z-marching SpMM (each row's coefficients formed from
    the potential at its stencil vertices) against the stored-coefficient
    one on an 81^3 box with a rough random potential: the same CG iterates
    bit for bit and the same iteration counts.  7 columns run one column
    per chunk (groups of 4 and 3 chunks), 10 columns two per chunk (groups
    of 3 and 2); columns leave the groups as they converge.  In FP32-inner
    mode both the FP32 inner SpMM (coefficients rounded from FP64) and the
    FP64 refinement SpMM change form."""
    ncs, lo, hi = NC, -8.0, 8.0
    X = inputs.vertex_coords(ncs, lo, hi)
    V = 0.5 * np.sum(X * X, axis=1) + np.random.default_rng(3).uniform(
        -2.0, 2.0, X.shape[0])
    n = (NC - 1) ** 3
    rng = np.random.default_rng(12)
    B = rng.standard_normal((n, ncols))
    X0 = rng.standard_normal((n, ncols)) * 0.01
    out = []
    try:
        for mf in (True, False):
            pb.paro_set_matrix_free(mf)
            gu.note(f"matrix-free {mf}: {ncs}^3 box, ncols {ncols}, "
                    f"precision {precision}")
            prob = gu.assemble(ncs, lo, hi, V, N=ncols, precision=precision,
                               pcg_rtol=1e-11)
            Xd = gu.to_dev(X0)
            its = pb.paro_pcg(prob, gu.to_dev(B), Xd)
            out.append((its, Xd.cpu().numpy()))
    finally:
        pb.paro_set_matrix_free(True)
    (its_mf, X_mf), (its_st, X_st) = out
    assert its_mf == its_st
    assert np.array_equal(X_mf, X_st)
    assert max(its_mf) > 20


@pytest.mark.parametrize("N,m", [(4, 2), (5, 2)])
def test_matrix_free_steps_are_bitwise_the_stored_ones(N, m):
    """ParO steps on an 81^3 box with a rough potential, CG SpMM in the
    matrix-free form (coefficients from the potential) against the
    stored-coefficient form: the same Ritz values and orbitals bit for bit
    after Step 1 and three steps, through starts, source solves whose
    columns converge at different iterations, and rotations.  6 columns
    make 3 chunks of 2, 7 columns 7 single-column chunks (groups of 4 and
    3)."""
    import torch
    ncs, lo, hi = NC, -8.0, 8.0
    X = inputs.vertex_coords(ncs, lo, hi)
    V = 0.5 * np.sum(X * X, axis=1) + np.random.default_rng(4).uniform(
        -1.0, 1.0, X.shape[0])
    n = (NC - 1) ** 3
    U0 = gu.to_dev(np.random.default_rng(5).standard_normal((n, N + m)))
    out = []
    try:
        for mf in (True, False):
            pb.paro_set_matrix_free(mf)
            gu.note(f"matrix-free {mf}: steps on {ncs}^3, N {N}, m {m}")
            prob = gu.assemble(ncs, lo, hi, V, N=N, m=m, pcg_rtol=1e-9)
            lam = torch.zeros(N + m, dtype=torch.float64, device=gu.device())
            U = torch.zeros(n, N + m, dtype=torch.float64, device=gu.device())
            pb.paro_init(prob, U0, lam, U)
            lams = [lam.cpu().numpy().copy()]
            for _ in range(3):
                pb.paro_step(prob, lam, U)
                lams.append(lam.cpu().numpy().copy())
            out.append((np.array(lams), U.cpu().numpy()))
    finally:
        pb.paro_set_matrix_free(True)
    (l_mf, U_mf), (l_st, U_st) = out
    assert np.array_equal(l_mf, l_st)
    assert np.array_equal(U_mf, U_st)
    assert np.all(np.isfinite(l_mf)) and l_mf[-1, 0] < l_mf[0, 0]


def test_matrix_free_spmm_on_an_anisotropic_box():
    """A 97 x 81 x 71-cell box of unequal spacings (96 x 80 x 70 interior
    vertices, 2168 tiles: the z-marching SpMM) with a rough potential: the
    matrix-free source solves against the oracle's own matrix (FP64
    residual; CG iteration counts within one of the oracle's Jacobi-PCG)
    and bitwise against the stored-coefficient form."""
    ncs, lo, hi = (97, 81, 71), (-7.0, -5.0, -4.5), (6.0, 5.5, 4.0)
    X = inputs.vertex_coords(ncs, lo, hi)
    V = 0.5 * np.sum(X * X, axis=1) + np.random.default_rng(8).uniform(
        -1.0, 1.0, X.shape[0])
    H, M, s = gu.oracle_matrices(ncs, lo, hi, V)
    A = (H - s * M).tocsr()
    n = A.shape[0]
    assert n == 96 * 80 * 70 and n > 2048 * 248
    ncols = 3
    rng = np.random.default_rng(21)
    B = rng.standard_normal((n, ncols))
    X0 = rng.standard_normal((n, ncols)) * 0.01
    out = []
    try:
        for mf in (True, False):
            pb.paro_set_matrix_free(mf)
            gu.note(f"matrix-free {mf}: anisotropic box {ncs}")
            prob = gu.assemble(ncs, lo, hi, V, N=ncols, pcg_rtol=1e-12)
            Xd = gu.to_dev(X0)
            its = pb.paro_pcg(prob, gu.to_dev(B), Xd)
            out.append((its, Xd.cpu().numpy()))
            del prob
    finally:
        pb.paro_set_matrix_free(True)
    (its, Xm), (its_st, Xs) = out
    assert its == its_st and np.array_equal(Xm, Xs)
    res = np.linalg.norm(B - A @ Xm, axis=0) / np.linalg.norm(B, axis=0)
    assert np.max(res) <= 1.01e-12, res
    dinv = 1.0 / A.diagonal()
    for c in range(ncols):
        _, k = oparo.jacobi_pcg(A, B[:, c], X0[:, c], dinv, 1e-12, 20000)
        assert abs(its[c] - k) <= 1, (c, its[c], k)


def test_mixed_solve_with_chunk_major_refinement_matches_fp64():
    """A whole mixed-precision solve on the 81^3 harmonic box, where the
    FP64 refinement iterate is chunk-major (the emitting rotation writes
    x0 and b that way, the residual is a z-march, X is unpacked after the
    solves): the same Ritz values as the plain FP64 solve."""
    w = inputs.harmonic(nc=NC, N=4, m=inputs.harmonic_buffer(4),
                        max_steps=400)
    U0 = w.U0()
    out = {}
    for prec in (pb.PARO_FP64, pb.PARO_FP32_INNER):
        gu.note(f"81^3 harmonic solve, precision {prec}")
        prob = gu.workload_problem(w, precision=prec)
        lam, U, rep = gu.solve(prob, U0)
        assert rep.status == 0, rep.as_dict()
        assert np.all(np.isfinite(U))
        out[prec] = lam[:w.N]
    rel = np.abs(out[pb.PARO_FP32_INNER] - out[pb.PARO_FP64]) / np.abs(
        out[pb.PARO_FP64])
    assert np.max(rel) <= 1e-10, rel
    # The continuum values 3/2 and 5/2 within the mesh's O(h^2) error.
    assert abs(out[pb.PARO_FP64][0] - 1.5) < 0.05
    assert np.all(np.abs(out[pb.PARO_FP64][1:] - 2.5) < 0.1)
