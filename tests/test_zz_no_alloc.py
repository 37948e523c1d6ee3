"""The allocation-free Gram (paro_gram_noalloc) against paro_gram (GPU):
same kernels, same segments, so the same bits; two calls in a row, the
second smaller than the first (the static scratch keeps the first call's
contents), and a third after a paro_gram call on another shape."""
import numpy as np
import pytest

from paper_1405_0260_amd import binding as pb
from paper_1405_0260_amd import inputs
import gpu_util as gu

pytestmark = pytest.mark.gpu


def _blocks(n, ncols, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, ncols)), rng.standard_normal((n, ncols))


def _reference(nc, ncols, W, Y):
    """paro_gram on a problem with n dofs and N + m = ncols."""
    import torch
    w = inputs.harmonic(nc=nc, N=ncols)
    p = gu.workload_problem(w)
    G = torch.zeros(ncols, ncols, dtype=torch.float64, device=gu.device())
    pb.paro_gram(p, gu.to_dev(W), gu.to_dev(Y), G)
    torch.cuda.synchronize()
    return G.cpu().numpy()


def _noalloc(W, Y):
    import torch
    ncols = W.shape[1]
    G = torch.full((ncols, ncols), np.nan, dtype=torch.float64,
                   device=gu.device())
    pb.paro_gram_noalloc(gu.to_dev(W), gu.to_dev(Y), G)
    torch.cuda.synchronize()
    return G.cpu().numpy()


def test_noalloc_gram_matches_paro_gram_twice_then_smaller():
    cases = [(40, 64, 1), (17, 24, 2), (9, 5, 3)]   # (cells, ncols, seed)
    for nc, ncols, seed in cases:
        n = (nc - 1) ** 3
        gu.note(f"noalloc gram: n = {n}, ncols = {ncols}")
        W, Y = _blocks(n, ncols, seed)
        got = _noalloc(W, Y)
        ref = _reference(nc, ncols, W, Y)
        exact = W.T @ Y
        assert np.array_equal(got, ref), (nc, ncols)
        assert np.allclose(got, exact, rtol=1e-12,
                           atol=1e-12 * np.abs(exact).max())


def test_noalloc_gram_rejects_sizes_beyond_its_scratch():
    import torch
    W = torch.zeros(10, 65, dtype=torch.float64, device=gu.device())
    G = torch.zeros(65, 65, dtype=torch.float64, device=gu.device())
    with pytest.raises(pb.ParoError):
        pb.paro_gram_noalloc(W, W, G)
