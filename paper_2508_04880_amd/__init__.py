"""MI355X-native noisy statevector engine: TUSQ's error characterisation on
the host and its depth-first tree traversal as gfx950 HIP kernels, behind the
C ABI of ``include/tusq.h``.

``_lib`` is the ctypes binding.  It is loaded on first use of any name below
and raises ImportError when ``libtusq.so`` has not been built: there is no
fallback path.  (The package itself imports without the library so that
``python -m paper_2508_04880_amd.build`` can build it.)"""

_EXPORTS = (
    "C64", "C128", "CACHING", "CHECKPOINT", "DFTT", "HYBRID", "NAIVE", "WANT_DIST", "WANT_NORMS", "WANT_SAMPLES",
    "Circuit", "Context", "Result", "Tree", "TusqError", "lib", "tusq_cancel",
    "tusq_ctx_create", "tusq_ecm_build", "tusq_job_times", "tusq_opts", "tusq_opts_default",
    "tusq_plan_counters", "tusq_plan_dump", "tusq_plan_dump_programs", "tusq_poll", "tusq_run", "tusq_run_batch",
    "tusq_run_tree", "tusq_run_tree_noalloc", "tusq_batch_autotune", "tusq_batch_shape", "tusq_submit", "tusq_autotune", "tusq_wait", "LIB_PATH", "ABI_VERSION", "tusq_thermal_pauli_probs",
)


def __getattr__(name):
    if name in _EXPORTS:
        from . import _lib
        return getattr(_lib, name)
    raise AttributeError(name)


__all__ = list(_EXPORTS)
