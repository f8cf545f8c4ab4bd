"""ctypes binding of libcscirc.so: argument marshalling only.

Every function takes torch tensors that already live on the GPU, checks dtype,
device, contiguity and length, and passes raw device pointers plus the current
HIP stream to the C ABI declared in include/cscirc.h.  All arithmetic runs in
the library's HIP kernels; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcscirc.so")

CS_OK, CS_EINVAL, CS_ENOMEM, CS_EHIP, CS_ENOTSUP = 0, -1, -2, -3, -4
_NAMES = {CS_EINVAL: "CS_EINVAL", CS_ENOMEM: "CS_ENOMEM", CS_EHIP: "CS_EHIP", CS_ENOTSUP: "CS_ENOTSUP"}

EXPORTS = ["cs_circ_apply", "cs_circ_apply_T", "cs_circ_apply_direct", "cs_circ_apply_T_direct", "cs_circ_norm_bound", "cs_box_blur_generator", "cs_ista_solve",
           "cs_admm_solve", "cs_cpadmm_solve", "cs_ista_solve_noalloc", "cs_ista_solve_batched", "cs_admm_solve_batched", "cs_batched_schedule",
           "cs_unrolled_ckpt_bytes", "cs_unrolled_ista_fwd",
           "cs_unrolled_ista_bwd", "cs2_apply", "cs2_apply_T", "cs2_norm_bound", "cs2_ista_solve",
           "cs2_admm_solve", "cs_workspace_bytes", "cs_set_workspace", "cs_set_solver_path", "cs_check_device",
           "cs_timing_enable",
           "cs_timing_read", "cs_last_error", "cs_version"]


class CsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (_NAMES.get(status, str(status)), msg))
        self.status = status


_lib = None


def load():
    """Load the built library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libcscirc.so is not built (%s); run __graft_entry__.build() "
                          "or python paper_1707_02244_amd/build.py" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    P, I64, I32, F = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_float
    sig = {
        "cs_circ_apply": [P, I64, I32, P, P, P],
        "cs_circ_apply_T": [P, I64, I32, P, P, P],
        "cs_circ_apply_direct": [P, I64, I32, P, P, P],
        "cs_circ_apply_T_direct": [P, I64, I32, P, P, P],
        "cs_circ_norm_bound": [P, I64, P, P],
        "cs_box_blur_generator": [P, I64, I32, P, P],
        "cs_ista_solve": [P, I64, I32, P, F, F, I32, P, P, P],
        "cs_admm_solve": [P, I64, I32, P, F, F, I32, I32, P, P, P, P, P],
        "cs_ista_solve_noalloc": [P, I64, I32, P, F, F, I32, P, P],
        "cs_cpadmm_solve": [P, I64, P, I64, P, F, F, F, F, I32, P, P, P, P, P, P],
        "cs_ista_solve_batched": [I32, P, P, P, P, P, P, P, P, I32, P, P],
        "cs_admm_solve_batched": [I32, P, P, P, P, P, P, P, P, I32, I32, P, P, P, P],
        "cs_batched_schedule": [ctypes.c_char_p, ctypes.c_size_t],
        "cs_unrolled_ckpt_bytes": [I64, I32, I32, I32, I32],
        "cs_unrolled_ista_fwd": [P, I64, I32, I32, P, P, P, I32, I32, P, P, P],
        "cs_unrolled_ista_bwd": [P, I64, I32, I32, P, P, P, I32, I32, P, P, P, P, P, P],
        "cs2_apply": [P, P, I32, I32, P, P, P],
        "cs2_apply_T": [P, P, I32, I32, P, P, P],
        "cs2_norm_bound": [P, P, I32, I32, P, P],
        "cs2_ista_solve": [P, P, I32, I32, P, F, F, I32, P, P, P],
        "cs2_admm_solve": [P, P, I32, I32, P, F, F, I32, I32, P, P, P, P, P],
        "cs_workspace_bytes": [I64, I32, I32],
        "cs_set_workspace": [P, ctypes.c_size_t],
        "cs_set_solver_path": [I32],
        "cs_check_device": [P],
        "cs_timing_enable": [I32],
        "cs_timing_read": [ctypes.c_char_p, ctypes.POINTER(I64), ctypes.POINTER(ctypes.c_double)],
        "cs_last_error": [],
        "cs_version": [],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.cs_last_error.restype = ctypes.c_char_p
    lib.cs_unrolled_ckpt_bytes.restype = ctypes.c_size_t
    lib.cs_workspace_bytes.restype = ctypes.c_size_t
    _lib = lib
    return lib


def _check(st):
    if st != CS_OK:
        raise CsError(st, load().cs_last_error().decode())


def _ptr(t, name, numel=None):
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch.Tensor" % name)
    if t.dtype != torch.float32:
        raise TypeError("%s must be float32, got %s" % (name, t.dtype))
    if not t.is_cuda:
        raise ValueError("%s must be on the GPU" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if numel is not None and t.numel() != numel:
        raise ValueError("%s has %d elements, expected %d" % (name, t.numel(), numel))
    return ctypes.c_void_p(t.data_ptr())


def _stream(t):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def circ_apply(c, d, x, y=None):
    """y = P C x (m = n/d outputs)."""
    import torch
    n = c.numel()
    if y is None:
        y = torch.empty(n // d, device=c.device, dtype=torch.float32)
    _check(load().cs_circ_apply(_ptr(c, "c"), n, d, _ptr(x, "x", n), _ptr(y, "y", n // d), _stream(c)))
    return y


def circ_apply_T(c, d, r, x=None):
    """x = C^T P^T r (n outputs)."""
    import torch
    n = c.numel()
    if x is None:
        x = torch.empty(n, device=c.device, dtype=torch.float32)
    _check(load().cs_circ_apply_T(_ptr(c, "c"), n, d, _ptr(r, "r", n // d), _ptr(x, "x", n), _stream(c)))
    return x


def circ_apply_direct(c, d, x, y=None):
    """y = P C x evaluated directly (no FFT): one inner product over c per
    output, O(n m) work; a baseline beside circ_apply."""
    import torch
    n = c.numel()
    if y is None:
        y = torch.empty(n // d, device=c.device, dtype=torch.float32)
    _check(load().cs_circ_apply_direct(_ptr(c, "c"), n, d, _ptr(x, "x", n), _ptr(y, "y", n // d), _stream(c)))
    return y


def circ_apply_T_direct(c, d, r, x=None):
    """x = C^T P^T r evaluated directly (no FFT), O(n m) work."""
    import torch
    n = c.numel()
    if x is None:
        x = torch.empty(n, device=c.device, dtype=torch.float32)
    _check(load().cs_circ_apply_T_direct(_ptr(c, "c"), n, d, _ptr(r, "r", n // d), _ptr(x, "x", n), _stream(c)))
    return x


def circ_norm_bound(c, out=None):
    """max_k |c_hat_k|^2 as a 1-element device tensor."""
    import torch
    if out is None:
        out = torch.empty(1, device=c.device, dtype=torch.float32)
    _check(load().cs_circ_norm_bound(_ptr(c, "c"), c.numel(), _ptr(out, "out", 1), _stream(c)))
    return out


def box_blur_generator(c, L, out=None):
    """Generator of C B for the order-L box blur B (Section 7): out[k] is
    the mean of c over the L samples starting at k, circularly."""
    import torch
    n = c.numel()
    if out is None:
        out = torch.empty(n, device=c.device, dtype=torch.float32)
    _check(load().cs_box_blur_generator(_ptr(c, "c"), n, int(L), _ptr(out, "out", n), _stream(c)))
    return out


def ista_solve(c, d, y, lam, tau, iters, x=None, obj=None):
    """ISTA (Alg. 1) from x(0) = 0; returns x(iters)."""
    import torch
    n = c.numel()
    if x is None:
        x = torch.empty(n, device=c.device, dtype=torch.float32)
    _check(load().cs_ista_solve(_ptr(c, "c"), n, d, _ptr(y, "y", n // d), float(lam), float(tau),
                                int(iters), _ptr(x, "x", n), _ptr(obj, "obj", iters), _stream(c)))
    return x


def ista_solve_noalloc(c, d, y, lam, tau, iters, x):
    """ISTA through the allocation-free entry point (n <= 2^20); x is the
    caller's output tensor (nothing is allocated here either)."""
    n = c.numel()
    _check(load().cs_ista_solve_noalloc(_ptr(c, "c"), n, d, _ptr(y, "y", n // d), float(lam), float(tau),
                                        int(iters), _ptr(x, "x", n), _stream(c)))
    return x


def cpadmm_solve(c, omega, y, alpha, rho, sigma, tau, iters):
    """Circulant ADMM with the arbitrary row set `omega` (host integer array,
    distinct indices; y in omega's order); returns (x, v, z, mu, nu)."""
    import numpy as np
    import torch
    n = c.numel()
    om = np.ascontiguousarray(omega, dtype=np.int64)
    out = [torch.empty(n, device=c.device, dtype=torch.float32) for _ in range(5)]
    _check(load().cs_cpadmm_solve(_ptr(c, "c"), n, ctypes.c_void_p(om.ctypes.data), len(om),
                                  _ptr(y, "y", len(om)), float(alpha), float(rho), float(sigma), float(tau),
                                  int(iters), *[_ptr(t, nm, n) for t, nm in zip(out, ("x", "v", "z", "mu", "nu"))],
                                  _stream(c)))
    return tuple(out)


def admm_solve(c, d, y, lam, rho, iters, x=None, z=None, u=None, warm=False, obj=None):
    """ADMM (Alg. 2); returns (x, z, u) after `iters` steps."""
    import torch
    n = c.numel()
    mk = lambda: torch.empty(n, device=c.device, dtype=torch.float32)
    x = mk() if x is None else x
    z = mk() if z is None else z
    u = mk() if u is None else u
    _check(load().cs_admm_solve(_ptr(c, "c"), n, d, _ptr(y, "y", n // d), float(lam), float(rho),
                                int(iters), int(bool(warm)), _ptr(x, "x", n), _ptr(z, "z", n),
                                _ptr(u, "u", n), _ptr(obj, "obj", iters), _stream(c)))
    return x, z, u


def _shape2(s):
    if s.dim() != 2:
        raise ValueError("s must be a 2-D (rows x cols) tensor")
    return int(s.shape[0]), int(s.shape[1])


def apply2(s, h, x, y=None):
    """y = P C H x on a rows x cols image (h may be None); y is rows/2 x cols/2."""
    import torch
    R, C = _shape2(s)
    if y is None:
        y = torch.empty(R // 2, C // 2, device=s.device, dtype=torch.float32)
    _check(load().cs2_apply(_ptr(s, "s"), _ptr(h, "h", R * C), R, C, _ptr(x, "x", R * C),
                            _ptr(y, "y", (R // 2) * (C // 2)), _stream(s)))
    return y


def apply2_T(s, h, r, x=None):
    """x = H^T C^T P^T r (rows x cols)."""
    import torch
    R, C = _shape2(s)
    if x is None:
        x = torch.empty(R, C, device=s.device, dtype=torch.float32)
    _check(load().cs2_apply_T(_ptr(s, "s"), _ptr(h, "h", R * C), R, C, _ptr(r, "r", (R // 2) * (C // 2)),
                              _ptr(x, "x", R * C), _stream(s)))
    return x


def norm_bound2(s, h, out=None):
    """max |DFT2(s) DFT2(h)|^2 as a 1-element device tensor."""
    import torch
    R, C = _shape2(s)
    if out is None:
        out = torch.empty(1, device=s.device, dtype=torch.float32)
    _check(load().cs2_norm_bound(_ptr(s, "s"), _ptr(h, "h", R * C), R, C, _ptr(out, "out", 1), _stream(s)))
    return out


def ista_solve2(s, h, y, lam, tau, iters, x=None, obj=None):
    """ISTA (Alg. 1) on the 2-D operator from x(0) = 0; returns x(iters)."""
    import torch
    R, C = _shape2(s)
    if x is None:
        x = torch.empty(R, C, device=s.device, dtype=torch.float32)
    _check(load().cs2_ista_solve(_ptr(s, "s"), _ptr(h, "h", R * C), R, C, _ptr(y, "y", (R // 2) * (C // 2)),
                                 float(lam), float(tau), int(iters), _ptr(x, "x", R * C),
                                 _ptr(obj, "obj", iters), _stream(s)))
    return x


def admm_solve2(s, h, y, lam, rho, iters, x=None, z=None, u=None, warm=False, obj=None):
    """ADMM (Alg. 2) on the 2-D operator; returns (x, z, u)."""
    import torch
    R, C = _shape2(s)
    mk = lambda: torch.empty(R, C, device=s.device, dtype=torch.float32)
    x = mk() if x is None else x
    z = mk() if z is None else z
    u = mk() if u is None else u
    _check(load().cs2_admm_solve(_ptr(s, "s"), _ptr(h, "h", R * C), R, C, _ptr(y, "y", (R // 2) * (C // 2)),
                                 float(lam), float(rho), int(iters), int(bool(warm)), _ptr(x, "x", R * C),
                                 _ptr(z, "z", R * C), _ptr(u, "u", R * C), _ptr(obj, "obj", iters), _stream(s)))
    return x, z, u


def _batch_dims(ns, d):
    import numpy as np
    ns = np.ascontiguousarray(ns, dtype=np.int64)
    ds = np.ascontiguousarray(np.broadcast_to(np.asarray(d, dtype=np.int32), ns.shape), dtype=np.int32)
    return ns, ds


def batch_offsets(ns, d):
    """Offsets of each signal in the concatenated n- and m-length arrays
    (d: one decimation for all signals, or one per signal)."""
    import numpy as np
    ns, ds = _batch_dims(ns, d)
    off_n = np.concatenate([[0], np.cumsum(ns)[:-1]]).astype(np.int64)
    off_m = np.concatenate([[0], np.cumsum(ns // ds)[:-1]]).astype(np.int64)
    return off_n, off_m


def ista_solve_batched(ns, d, c_cat, y_cat, lam, tau, iters, x_cat=None):
    """Batched ISTA over signals of lengths `ns` and decimations `d` (one
    value or one per signal), inputs concatenated in order; lam and tau are
    device arrays with one value per signal."""
    import torch
    ns, ds = _batch_dims(ns, d)
    off_n, off_m = batch_offsets(ns, ds)
    total_n, total_m = int(ns.sum()), int((ns // ds).sum())
    if x_cat is None:
        x_cat = torch.empty(total_n, device=c_cat.device, dtype=torch.float32)
    B = len(ns)
    P = ctypes.c_void_p
    _check(load().cs_ista_solve_batched(
        B, P(ns.ctypes.data), P(ds.ctypes.data), P(off_n.ctypes.data), P(off_m.ctypes.data),
        _ptr(c_cat, "c_cat", total_n), _ptr(y_cat, "y_cat", total_m), _ptr(lam, "lam", B), _ptr(tau, "tau", B),
        int(iters), _ptr(x_cat, "x_cat", total_n), _stream(c_cat)))
    return x_cat


def admm_solve_batched(ns, d, c_cat, y_cat, lam, rho, iters, x_cat=None, z_cat=None, u_cat=None, warm=False):
    """Batched ADMM (per-signal lam and rho, device arrays) over signals laid
    out as for ista_solve_batched; returns (x, z, u) concatenated."""
    import torch
    ns, ds = _batch_dims(ns, d)
    off_n, off_m = batch_offsets(ns, ds)
    total_n, total_m = int(ns.sum()), int((ns // ds).sum())
    dev = c_cat.device
    x_cat = torch.empty(total_n, device=dev, dtype=torch.float32) if x_cat is None else x_cat
    z_cat = torch.zeros(total_n, device=dev, dtype=torch.float32) if z_cat is None else z_cat
    u_cat = torch.zeros(total_n, device=dev, dtype=torch.float32) if u_cat is None else u_cat
    B = len(ns)
    P = ctypes.c_void_p
    _check(load().cs_admm_solve_batched(
        B, P(ns.ctypes.data), P(ds.ctypes.data), P(off_n.ctypes.data), P(off_m.ctypes.data),
        _ptr(c_cat, "c_cat", total_n), _ptr(y_cat, "y_cat", total_m), _ptr(lam, "lam", B), _ptr(rho, "rho", B),
        int(iters), 1 if warm else 0, _ptr(x_cat, "x_cat", total_n), _ptr(z_cat, "z_cat", total_n),
        _ptr(u_cat, "u_cat", total_n), _stream(c_cat)))
    return x_cat, z_cat, u_cat


def batched_schedule():
    """The last batched call's schedule and tuner trials (a dict)."""
    import json
    buf = ctypes.create_string_buffer(1 << 16)
    _check(load().cs_batched_schedule(buf, len(buf)))
    return json.loads(buf.value.decode())


def unrolled_ckpt_bytes(n, d, batch, K, every):
    return int(load().cs_unrolled_ckpt_bytes(n, d, batch, K, every))


def unrolled_ista_fwd(c, d, y, lam, tau, K, every, xK=None, ckpt=None):
    """Forward of K unrolled ISTA steps for a batch y (Bt x m) sharing c.
    Returns (x_K, checkpoints)."""
    import torch
    n = c.numel()
    Bt = y.shape[0]
    if xK is None:
        xK = torch.empty(Bt, n, device=c.device, dtype=torch.float32)
    nb = unrolled_ckpt_bytes(n, d, Bt, K, every)
    if ckpt is None:
        ckpt = torch.empty(max(nb // 4, 1), device=c.device, dtype=torch.float32)
    _check(load().cs_unrolled_ista_fwd(_ptr(c, "c"), n, d, Bt, _ptr(y, "y", Bt * (n // d)), _ptr(lam, "lam", K),
                                       _ptr(tau, "tau", K), int(K), int(every), _ptr(xK, "xK", Bt * n),
                                       _ptr(ckpt, "ckpt"), _stream(c)))
    return xK, ckpt


def unrolled_ista_bwd(c, d, y, lam, tau, K, every, ckpt, g_xK):
    """Reverse pass: (dL/dlam, dL/dtau, dL/dy) from dL/dx_K."""
    import torch
    n = c.numel()
    Bt = y.shape[0]
    g_lam = torch.empty(K, device=c.device, dtype=torch.float32)
    g_tau = torch.empty(K, device=c.device, dtype=torch.float32)
    g_y = torch.empty_like(y)
    _check(load().cs_unrolled_ista_bwd(_ptr(c, "c"), n, d, Bt, _ptr(y, "y", Bt * (n // d)), _ptr(lam, "lam", K),
                                       _ptr(tau, "tau", K), int(K), int(every), _ptr(ckpt, "ckpt"),
                                       _ptr(g_xK, "g_xK", Bt * n), _ptr(g_lam, "g_lam", K), _ptr(g_tau, "g_tau", K),
                                       _ptr(g_y, "g_y"), _stream(c)))
    return g_lam, g_tau, g_y


def _unrolled_function():
    import torch

    class UnrolledISTA(torch.autograd.Function):
        """x_K of K unrolled ISTA steps; differentiable in y, lam and tau.
        Usage: UnrolledISTA.apply(y, lam, tau, c, d, K, every)."""

        @staticmethod
        def forward(ctx, y, lam, tau, c, d, K, every):
            y, lam, tau = y.contiguous(), lam.contiguous(), tau.contiguous()
            xK, ckpt = unrolled_ista_fwd(c, d, y, lam, tau, K, every)
            ctx.save_for_backward(y, lam, tau, c, ckpt)
            ctx.cfg = (d, K, every)
            return xK

        @staticmethod
        def backward(ctx, g):
            y, lam, tau, c, ckpt = ctx.saved_tensors
            d, K, every = ctx.cfg
            g_lam, g_tau, g_y = unrolled_ista_bwd(c, d, y, lam, tau, K, every, ckpt, g.contiguous())
            return g_y, g_lam, g_tau, None, None, None, None

    return UnrolledISTA


def workspace_bytes(n, d, mode=0):
    """Bytes of the device block a single-signal call of (n, d) needs
    (mode 0 operators, 1 ISTA, 2 ADMM; one layout); 0 if (n, d) is invalid."""
    return int(load().cs_workspace_bytes(int(n), int(d), int(mode)))


def set_workspace(ws):
    """Use the caller's device block for the single-signal calls on the
    current device (ws: a float32 or uint8 CUDA tensor, kept alive by the
    caller while set), or library memory again (ws None)."""
    if ws is None:
        _check(load().cs_set_workspace(None, 0))
        return
    if not ws.is_cuda or not ws.is_contiguous():
        raise ValueError("workspace must be a contiguous GPU tensor")
    _check(load().cs_set_workspace(ctypes.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size()))


PATH_AUTO, PATH_TWO_PASS, PATH_PERSISTENT = 0, 1, 2


def set_solver_path(path):
    """0: per size (default), 1: two launches per iteration, 2: persistent."""
    _check(load().cs_set_solver_path(int(path)))


def check_device(device=None):
    """Synchronise the current stream and raise if a persistent solve's grid
    barrier hit its bound."""
    import torch
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else device
    _check(load().cs_check_device(ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)))


def timing_enable(on=True):
    """Bracket each solver kernel launch with hipEvents (diagnostics)."""
    _check(load().cs_timing_enable(1 if on else 0))


def timing_read(kernel):
    """(launches, total_ms) of the recorded launches of one kernel; clears them."""
    n = ctypes.c_int64(0)
    ms = ctypes.c_double(0.0)
    _check(load().cs_timing_read(kernel.encode(), ctypes.byref(n), ctypes.byref(ms)))
    return int(n.value), float(ms.value)


def __getattr__(name):
    if name == "UnrolledISTA":
        return _unrolled_function()
    raise AttributeError(name)


def version():
    return int(load().cs_version())
