"""MI355X (gfx950) parallel orbital-updating eigensolver.

The compute lives in ``libparo.so`` (HIP kernels behind the C ABI declared
in ``include/paro.h``); ``paper_1405_0260_amd.binding`` marshals torch
device tensors into it.  The binding raises if the library is missing:
there is no CPU fallback.
"""
from .binding import (  # noqa: F401
    Box, Opts, ParoError, Problem, Report, default_opts, lib, paro_assemble,
    paro_default_opts, paro_destroy, paro_export_csr, paro_gram, paro_init,
    paro_pcg, paro_query, paro_set_timing, paro_get_timing, Timing,
    paro_small_geneig, paro_solve, paro_spmm, paro_step, Batch,
    paro_batch_init, paro_batch_step, paro_batch_solve, Server, ServerStats,
    KsOpts, KsReport, ks_default_opts, paro_update_potential, paro_sigma,
    paro_ks_solve,
    PARO_OK, PARO_EINVAL, PARO_ENOMEM, PARO_ENOTSPD, PARO_ESINGULAR,
    PARO_ENOCONV, PARO_EDEVICE, PARO_FP64, PARO_FP32_INNER,
)
