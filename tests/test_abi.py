"""Host-side checks of the C ABI (CPU only: no kernel is launched).

The library must load, export every entry point declared in
include/paro.h, and answer the host-only queries and argument checks."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import fem
from paper_1405_0260_amd import binding as pb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "paro.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(pb.LIB_PATH):
        from paper_1405_0260_amd import build
        build.build()
    return pb.lib()


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(paro_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ("paro_query", "paro_assemble", "paro_step", "paro_solve",
              "paro_init", "paro_destroy"):
        assert s in syms


def test_library_exports_every_declared_symbol(lib):
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


@pytest.mark.parametrize("ncs", [(2, 2, 2), (3, 3, 3), (24, 24, 24),
                                 (4, 5, 6), (7, 3, 9)])
def test_query_matches_oracle_mesh(lib, ncs):
    mesh = fem.kuhn_mesh(ncs, 0.0, 1.0)
    K, _, _ = fem.assemble(mesh, np.zeros(mesh.X.shape[0]))
    box = pb.Box(ncs[0], ncs[1], ncs[2], (ctypes.c_double * 3)(0, 0, 0),
                 (ctypes.c_double * 3)(1, 1, 1))
    n, z, ws = pb.paro_query(box, pb.default_opts(N=1))
    assert n == mesh.n_dof and z == K.nnz
    assert ws > 8 * 2 * z


def test_default_options(lib):
    o = pb.paro_default_opts()
    assert (o.N, o.m, o.precision, o.sigma_mode) == (1, 0, pb.PARO_FP64, 0)
    assert o.pcg_rtol == 1e-10 and o.lambda_tol == 1e-12
    assert o.pcg_reduce == 0.0
    assert o.max_steps == 200 and o.pcg_maxit == 10000


def test_workspace_grows_with_columns_and_precision(lib):
    box = pb.Box.cube(16, -1, 1)
    _, _, a = pb.paro_query(box, pb.default_opts(N=4))
    _, _, b = pb.paro_query(box, pb.default_opts(N=8))
    _, _, c = pb.paro_query(box, pb.default_opts(N=8, precision=1))
    assert a < b < c


@pytest.mark.parametrize("box,opts,code", [
    (pb.Box.cube(1, 0, 1), dict(N=1), pb.PARO_EINVAL),
    (pb.Box.cube(8, 0, 1), dict(N=40, m=30), pb.PARO_EINVAL),
    (pb.Box.cube(2, 0, 1), dict(N=2), pb.PARO_EINVAL),
    (pb.Box.cube(8, 0, 1), dict(N=1, precision=7), pb.PARO_EINVAL),
    (pb.Box.cube(8, 0, 1), dict(N=0), pb.PARO_EINVAL),
    (pb.Box.cube(8, 1, 0), dict(N=1), pb.PARO_EINVAL),
    (pb.Box.cube(8, 0, 1), dict(N=1, pcg_rtol=0.0), pb.PARO_EINVAL),
    (pb.Box.cube(8, 0, 1), dict(N=1, pcg_reduce=1.0), pb.PARO_EINVAL),
    (pb.Box.cube(8, 0, 1), dict(N=1, pcg_reduce=-0.1), pb.PARO_EINVAL),
])
def test_query_rejects_bad_arguments(lib, box, opts, code):
    with pytest.raises(pb.ParoError) as e:
        pb.paro_query(box, pb.default_opts(**opts))
    assert e.value.code == code
    assert lib.paro_last_error().decode() not in ("", "no error")


def test_strerror(lib):
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert lib.paro_strerror(code).decode()


def test_server_host_side_checks(lib):
    """Creation and submission are host-only: a fake (never dereferenced)
    arena address is enough to check sizes and errors."""
    fake = ctypes.c_void_p(1 << 40)
    srv = ctypes.c_void_p()
    assert lib.paro_server_create(fake, 1 << 20, 0, None,
                                  ctypes.byref(srv)) == pb.PARO_EINVAL
    assert lib.paro_server_create(ctypes.c_void_p((1 << 40) + 8), 1 << 20, 4,
                                  None, ctypes.byref(srv)) == pb.PARO_EINVAL
    assert lib.paro_server_create(fake, 1 << 25, 4, None,
                                  ctypes.byref(srv)) == pb.PARO_OK
    box = pb.Box.cube(48, -6.0, 6.0)
    o = pb.default_opts(N=4, m=2)
    V = np.zeros(49 ** 3)
    U0 = np.zeros((47 ** 3, 6))
    lam = np.zeros(6)
    U = np.zeros_like(U0)
    rid = ctypes.c_int64()
    # 32 MiB cannot hold a 48^3 problem at all.
    assert lib.paro_server_submit(srv, ctypes.byref(box), V.ctypes.data,
                                  ctypes.byref(o), U0.ctypes.data,
                                  lam.ctypes.data, U.ctypes.data,
                                  ctypes.byref(rid)) == pb.PARO_ENOMEM
    small = pb.Box.cube(4, -1.0, 1.0)
    V2 = np.zeros(5 ** 3)
    U2 = np.zeros((27, 6))
    assert lib.paro_server_submit(srv, ctypes.byref(small), V2.ctypes.data,
                                  ctypes.byref(o), U2.ctypes.data,
                                  lam.ctypes.data, U2.ctypes.data,
                                  ctypes.byref(rid)) == pb.PARO_OK
    assert rid.value == 1
    rep = pb.Report()
    assert lib.paro_server_report(srv, rid.value,
                                  ctypes.byref(rep)) == pb.PARO_EINVAL
    lib.paro_server_destroy(srv)


def test_kohn_sham_defaults_and_workspace_query(lib):
    o = pb.ks_default_opts()
    assert o.poisson_maxit == 0 and o.mixing == 0.3 and o.occupancy == 2.0
    small = ctypes.c_size_t(0)
    big = ctypes.c_size_t(0)
    assert lib.paro_ks_query(ctypes.byref(pb.Box.cube(10, -6.0, 6.0)),
                             ctypes.byref(small)) == pb.PARO_OK
    assert lib.paro_ks_query(ctypes.byref(pb.Box.cube(20, -6.0, 6.0)),
                             ctypes.byref(big)) == pb.PARO_OK
    # densities, potentials and the sine tables grow with the grid
    assert big.value > small.value > 8 * 9 ** 3 * 4
