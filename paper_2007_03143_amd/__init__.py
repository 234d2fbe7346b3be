"""MI355X-native XC integration (arXiv 2007.03143): E_xc, V_xc and N_e of a
Kohn-Sham density over an SSF-partitioned Mura-Knowles x Lebedev grid,
computed by the HIP kernels of libxc_mi355x.so behind the C ABI in
include/xc.h. This package is the thin ctypes binding; it has no CPU
fallback and raises ImportError when the library is not built."""
from .binding import (XcContext, XcError, xc_abi_version, xc_context_build_grid,
                      xc_context_create, xc_context_destroy,
                      xc_context_export_batches, xc_context_export_grid,
                      xc_context_integrate, xc_context_integrate_noalloc,
                      xc_context_integrate_uks,
                      xc_context_stats, xc_integrate, STATIC_SCRATCH_BYTES,
                      xc_context_set_timing, xc_context_set_phi_cache,
                      xc_context_footprint,
                      xc_context_timing, PHASES,
                      xc_engine_create, xc_engine_add_request, xc_engine_submit,
                      xc_engine_step, xc_engine_poll, xc_engine_release,
                      xc_engine_stats, xc_engine_destroy,
                      xc_strerror, XC_OK, XC_ERR_INVALID_ARG, XC_ERR_UNSUPPORTED,
                      XC_ERR_NOMEM, XC_ERR_DEVICE, XC_ERR_STATE, XC_ERR_BUSY, XC_LDA_SVWN5,
                      XC_GGA_PBE, XC_FP64, LIB_PATH)

__all__ = ["XcContext", "XcError", "xc_abi_version", "xc_context_build_grid",
           "xc_context_create", "xc_context_destroy", "xc_context_export_batches",
           "xc_context_export_grid", "xc_context_integrate",
           "xc_context_integrate_noalloc", "xc_context_integrate_uks", "STATIC_SCRATCH_BYTES", "xc_context_stats",
           "xc_integrate", "xc_strerror", "LIB_PATH", "xc_context_set_timing",
           "xc_context_set_phi_cache", "xc_context_footprint",
           "xc_context_timing", "PHASES", "xc_engine_create", "xc_engine_add_request",
           "xc_engine_submit", "xc_engine_step", "xc_engine_poll", "xc_engine_release",
           "xc_engine_stats", "xc_engine_destroy"]
