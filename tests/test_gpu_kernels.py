"""Kernel-level parity of the HIP path against the oracle (GPU).

Each stage of a ParO step is called through the C ABI on seeded inputs and
compared element by element with the oracle or with the plain library
definition (a matmul, a dense eigensolve)."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from oracle import paro as oparo
from paper_1405_0260_amd import binding as pb
from paper_1405_0260_amd import inputs
import gpu_util as gu

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


ASSEMBLY_CASES = [
    ("harmonic_24", 24, -6.0, 6.0, "ho"),
    ("softcoulomb_10", 10, -6.0, 6.0, "sc"),
    ("noncubic_4x5x6", (4, 5, 6), (-1.0, 0.0, 2.0), (1.0, 3.0, 2.5), "rand"),
    ("minimal_2", 2, -1.0, 1.0, "ho"),
    ("slab_9x3x7", (9, 3, 7), -2.0, 2.0, "sc"),
]


def case_potential(ncs, lo, hi, kind):
    X = inputs.vertex_coords(ncs, lo, hi)
    if kind == "ho":
        return 0.5 * np.sum(X * X, axis=1)
    if kind == "sc":
        Z, R = inputs.soft_coulomb_centres(2, 8, 6, 3.0)
        return inputs.soft_coulomb_potential(ncs, lo, hi, Z, R)
    return np.random.default_rng(5).uniform(-3, 2, X.shape[0])


@pytest.mark.parametrize("name,ncs,lo,hi,kind", ASSEMBLY_CASES,
                         ids=[c[0] for c in ASSEMBLY_CASES])
def test_assembly_matches_oracle(name, ncs, lo, hi, kind):
    V = case_potential(ncs, lo, hi, kind)
    H, M, s = gu.oracle_matrices(ncs, lo, hi, V)
    A = (H - s * M).tocsr()
    A.sort_indices()
    prob = gu.assemble(ncs, lo, hi, V, N=1)
    rowptr, col, valA, valM, sigma = pb.paro_export_csr(prob)
    _torch().cuda.synchronize()
    assert sigma == s
    # Pattern: bit-exact.
    assert np.array_equal(rowptr.cpu().numpy(), A.indptr.astype(np.int32))
    assert np.array_equal(col.cpu().numpy(), A.indices.astype(np.int32))
    Mo = M.tocsr()
    Mo.sort_indices()
    assert np.array_equal(Mo.indices, A.indices)
    # Values: same sums in another order.
    va, vm = valA.cpu().numpy(), valM.cpu().numpy()
    assert np.max(np.abs(va - A.data)) <= 1e-13 * np.max(np.abs(A.data))
    assert np.max(np.abs(vm - Mo.data)) <= 1e-14 * np.max(np.abs(Mo.data))


@pytest.fixture(scope="module")
def sc_problem():
    w = inputs.molecule(nc=13, N=4, m=0, lo=-6.0, hi=6.0)
    H, M, s = gu.oracle_matrices(w.nc, w.lo, w.hi, w.V)
    prob = gu.workload_problem(w)
    return w, H, M, s, prob


@pytest.mark.parametrize("ncols", [1, 2, 3, 4, 16, 24, 33, 64])
@pytest.mark.parametrize("which", [0, 1, 2])
def test_spmm_matches_oracle(sc_problem, ncols, which):
    w, H, M, s, prob = sc_problem
    torch = _torch()
    X = np.random.default_rng(ncols).standard_normal((prob.n, ncols))
    Y = torch.empty(prob.n, ncols, dtype=torch.float64, device=gu.device())
    pb.paro_spmm(prob, which, gu.to_dev(X), Y)
    ref = {0: (H - s * M) @ X, 1: M @ X, 2: H @ X}[which]
    got = Y.cpu().numpy()
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.fixture(scope="module")
def wide_problem():
    """N + m = 64 columns (the largest block the kernels take)."""
    w = inputs.molecule(nc=13, N=60, m=4, lo=-6.0, hi=6.0)
    return w, None, None, None, gu.workload_problem(w)


@pytest.mark.parametrize("ncols", [1, 5, 16, 17, 32, 48, 64])
def test_gram_matches_matmul(wide_problem, ncols):
    """W^T Y on FP64 matrix cores, non-symmetric operands (checks the MFMA
    operand and result lane layouts tile by tile)."""
    w, H, M, s, prob = wide_problem
    torch = _torch()
    rng = np.random.default_rng(100 + ncols)
    W = rng.standard_normal((prob.n, ncols))
    Yh = rng.standard_normal((prob.n, ncols)) + 0.5
    G = torch.empty(ncols, ncols, dtype=torch.float64, device=gu.device())
    pb.paro_gram(prob, gu.to_dev(W), gu.to_dev(Yh), G)
    ref = W.T @ Yh
    got = G.cpu().numpy()
    err = np.max(np.abs(got - ref))
    assert err <= 1e-13 * np.sqrt(prob.n) * np.max(np.abs(ref)), err


def _geneig(A, B):
    torch = _torch()
    n = A.shape[0]
    th = torch.empty(n, dtype=torch.float64, device=gu.device())
    C = torch.empty(n, n, dtype=torch.float64, device=gu.device())
    info = torch.zeros(1, dtype=torch.int32, device=gu.device())
    pb.paro_small_geneig(gu.to_dev(A), gu.to_dev(B), th, C, info)
    return th.cpu().numpy(), C.cpu().numpy(), int(info.cpu().numpy()[0])


def _spd(rng, n, cond=10.0):
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return (Q * np.geomspace(1.0, cond, n)) @ Q.T


@pytest.mark.parametrize("n", [1, 2, 3, 7, 16, 24, 31, 32, 48, 64])
def test_small_geneig_matches_eigh(n):
    rng = np.random.default_rng(n)
    B = _spd(rng, n)
    A = rng.standard_normal((n, n))
    A = A + A.T
    th, C, info = _geneig(A, B)
    assert info == 0
    ref = sla.eigh(A, B, eigvals_only=True)
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(th - ref)) <= 1e-12 * scale
    assert np.max(np.abs(C.T @ B @ C - np.eye(n))) <= 1e-12
    assert np.max(np.abs(A @ C - B @ C * th)) <= 1e-11 * scale
    # Sign rule: the largest-magnitude entry of each column is positive.
    idx = np.argmax(np.abs(C), axis=0)
    assert np.all(C[idx, np.arange(n)] > 0)


def test_small_geneig_degenerate_and_ordered():
    rng = np.random.default_rng(3)
    n = 12
    B = _spd(rng, n, 5.0)
    L = np.linalg.cholesky(B)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    d = np.array([-2.0, -2.0, -2.0, 0.5, 0.5, 1.0, 1.0, 1.0, 1.0, 3.0, 7.0,
                  7.0])
    A = L @ (Q * d) @ Q.T @ L.T
    th, C, info = _geneig(A, B)
    assert info == 0
    assert np.max(np.abs(th - d)) <= 1e-12 * 7
    assert np.all(np.diff(th) >= -1e-13)
    assert np.max(np.abs(C.T @ B @ C - np.eye(n))) <= 1e-12


@pytest.mark.parametrize("diag,expect", [
    ([2.0, 1.0, 3.0, 0.0, 1.0, 1.0], 4),
    ([1.0, -1.0, 1.0], 2),
])
def test_small_geneig_reports_non_positive_pivot(diag, expect):
    n = len(diag)
    _, _, info = _geneig(np.eye(n), np.diag(diag))
    assert info == expect


@pytest.mark.parametrize("precision", [pb.PARO_FP64, pb.PARO_FP32_INNER])
@pytest.mark.parametrize("ncols", [1, 4, 7])
def test_pcg_matches_direct_solve_and_oracle(precision, ncols):
    w = inputs.molecule(nc=13, N=7, m=0, lo=-6.0, hi=6.0)
    H, M, s = gu.oracle_matrices(w.nc, w.lo, w.hi, w.V)
    A = (H - s * M).tocsr()
    prob = gu.workload_problem(w, precision=precision, pcg_rtol=1e-12)
    rng = np.random.default_rng(7)
    B = rng.standard_normal((prob.n, ncols))
    X0 = rng.standard_normal((prob.n, ncols)) * 0.1
    Xd = gu.to_dev(X0)
    its = pb.paro_pcg(prob, gu.to_dev(B), Xd)
    X = Xd.cpu().numpy()
    ref = spla.spsolve(A.tocsc(), B)
    ref = ref.reshape(prob.n, ncols)
    rel = np.linalg.norm(X - ref, axis=0) / np.linalg.norm(ref, axis=0)
    assert np.max(rel) < 1e-9
    res = np.linalg.norm(B - A @ X, axis=0) / np.linalg.norm(B, axis=0)
    assert np.max(res) <= 1.01e-12
    if precision == pb.PARO_FP64:
        dinv = 1.0 / A.diagonal()
        for c in range(ncols):
            _, k = oparo.jacobi_pcg(A, B[:, c], X0[:, c], dinv, 1e-12, 10000)
            assert abs(its[c] - k) <= 1, (c, its[c], k)
