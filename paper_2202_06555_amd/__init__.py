"""MI355X-native evaluation of anchored cut-HDMR expansions with sparse-grid
components (Eftekhari & Scheidegger, arXiv 2202.06555): HIP kernels for
gfx950 behind the C ABI of include/hdmr.h, with a thin ctypes binding."""
from .hdmr import (  # noqa: F401
    EXPORTS, MIXED, PLAIN_FP64, HdmrError, Model, asg_build_components, hdmr_eval, hdmr_eval_batched, hdmr_eval_grad,
    hdmr_eval_noalloc, hdmr_model_naive, hdmr_build_report, hdmr_quadrature,
    hdmr_eval_stats,
    hdmr_export_component, hdmr_free, hdmr_get_info, hdmr_init, hdmr_last_error, hdmr_model_from_surpluses, hdmr_model_load, hdmr_model_save,
    hdmr_timing_enable,
    hdmr_timing_read, lib,
)
from . import surrogate  # noqa: F401,E402
