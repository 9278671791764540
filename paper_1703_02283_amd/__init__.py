"""MI355X-native inverse matrix p-th roots (Bini-type iteration, Section II of
Lass, Kuehne, Plessl, arXiv 1703.02283).

The work is done by libipr.so (HIP kernels for gfx950 behind a C ABI,
declared in include/ipr.h). This package is a thin ctypes binding whose
functions carry the C names; torch supplies device memory and streams only.
There is no CPU fallback: if the library is not built, every call raises.
"""
from .binding import (  # noqa: F401
    IPR_OK, IPR_EARG, IPR_EMAXITER, IPR_EFLOOR, IPR_EDIVERGED, IPR_EHIP, IPR_EGUARD,
    IPR_INIT_IDENTITY, IPR_INIT_PAPER_EQ3, IPR_INIT_POLY, IPR_INIT_LEARNED, IPR_INIT_USER,
    IPR_EVAL_COUPLED, IPR_EVAL_LITERAL, IPR_EVAL_NEWTON_SCHULZ,
    IPR_FP64, IPR_BF16, IPR_FP16, IPR_FP8_E4M3, IPR_FP64_INT8_EMUL, IPR_MLP_NPARAM,
    IPR_STORE_NONE, IPR_STORE_FLOAT, IPR_STORE_FIXED,
    IprSchedule, IprResult, IprError, library_path, load,
    ipr_schedule_default, ipr_workspace_size, ipr_solve, ipr_solve_batched, ipr_gemm, ipr_lowdin,
    ipr_solve_noalloc, IPR_NOALLOC_SCRATCH_BYTES, ipr_eigvalsh,
    ipr_gemm_lowp, ipr_gemm_lowp_workspace, ipr_gemm_emul, ipr_gemm_emul_workspace, ipr_norms,
    ipr_features, ipr_mlp_forward, ipr_mlp_train_step, ipr_mlp_workspace, ipr_last_error, ipr_tune_batched,
    ipr_get_batched_tiles, ipr_set_batched_tiles, IPR_BATCH_BUCKETS, ipr_spectral_counts,
)
