"""MI355X-native partial-circulant LASSO recovery (ISTA / ADMM with A = P C).

The compute path is the HIP library libcscirc.so (C ABI in include/cscirc.h);
this package only marshals torch tensors into it.
"""
from ._lib import (CsError, LIB_PATH, EXPORTS, load, circ_apply, circ_apply_T,  # noqa: F401
                   circ_apply_direct, circ_apply_T_direct,
                   circ_norm_bound, box_blur_generator, ista_solve, ista_solve_noalloc, admm_solve, cpadmm_solve, ista_solve_batched, admm_solve_batched, batched_schedule, batch_offsets,
                   unrolled_ckpt_bytes, unrolled_ista_fwd, unrolled_ista_bwd,
                   apply2, apply2_T, norm_bound2, ista_solve2, admm_solve2, timing_enable, timing_read, version,
                   set_solver_path, check_device, PATH_AUTO, PATH_TWO_PASS, PATH_PERSISTENT,
                   workspace_bytes, set_workspace)


def __getattr__(name):
    if name == "UnrolledISTA":
        from . import _lib
        cls = _lib._unrolled_function()
        globals()["UnrolledISTA"] = cls
        return cls
    raise AttributeError(name)
