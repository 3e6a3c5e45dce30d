"""Python binding of libjkcals (the MI355X JK-CALS hot path).

Argument marshalling only: every computation runs in the HIP kernels of
``libjkcals.so``.  The functions below carry the names of the C ABI
(``include/jk_cals.h``) and take torch tensors for device memory; the torch
stream current at call time is the stream the work is enqueued on.  There
is no CPU fallback: if the shared library is missing or fails to load,
importing the binding's functions raises.

Layouts (same as the C ABI):
* tensor: device, column-major with i_1 fastest (a flat tensor, or any
  tensor whose memory is in that order; use :func:`to_device_tensor`);
* factors, MTTKRP results, gradients: device float64, (I_n, C) row-major;
* model k owns columns [off_k, off_k + ranks[k]).
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# JKCALS_LIBRARY names another build of the library (the host-sanitizer build
# of the validation and planning code, libjkcals_asan.so); default in-tree
LIB_PATH = os.environ.get("JKCALS_LIBRARY") or os.path.join(_HERE, "libjkcals.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "jk_cals.h")

JKC_OK, JKC_EINVAL, JKC_ENOMEM, JKC_EDEVICE, JKC_ESTATE, JKC_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
JKC_FP64, JKC_SPLIT_BF16X3, JKC_SPLIT_BF16X6 = 0, 1, 2
JKC_TENSOR_F64, JKC_TENSOR_F32 = 0, 1
JKC_ST_CONVERGED, JKC_ST_FALLBACK, JKC_ST_NONFINITE = 1, 2, 4
MAX_RANK = 32

_STATUS_NAMES = {0: "JKC_OK", -1: "JKC_EINVAL", -2: "JKC_ENOMEM", -3: "JKC_EDEVICE",
                 -4: "JKC_ESTATE", -5: "JKC_EUNSUPPORTED"}


class JkcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (_STATUS_NAMES.get(status, str(status)), msg))
        self.status = status


class Problem(ctypes.Structure):
    _fields_ = [
        ("order", ctypes.c_int32),
        ("dims", ctypes.POINTER(ctypes.c_int64)),
        ("sampled_mode", ctypes.c_int32),
        ("num_models", ctypes.c_int32),
        ("ranks", ctypes.POINTER(ctypes.c_int32)),
        ("left_out", ctypes.POINTER(ctypes.c_int32)),
        ("tensor_dtype", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("copy_tensor", ctypes.c_int32),
        ("stream", ctypes.c_void_p),
        ("delete_d", ctypes.c_int32),
        ("tree_max_gib", ctypes.c_int32),
    ]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libjkcals.so (in-tree).  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libjkcals.so is not built (%s); run "
                           "`python -m paper_2112_03985_amd.build`" % LIB_PATH)
    try:
        import torch  # noqa: F401  (load torch's HIP runtime first: one runtime per process)
    except Exception:
        pass
    L = ctypes.CDLL(LIB_PATH, mode=ctypes.RTLD_GLOBAL)
    P, VP, I32, F64, SZ = ctypes.POINTER, ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.c_size_t
    sig = {
        "jk_cals_workspace_size": (I32, [P(Problem), P(SZ)]),
        "jk_cals_init": (I32, [P(Problem), VP, P(VP), VP, SZ, P(VP)]),
        "jk_cals_mttkrp": (I32, [VP, I32, VP]),
        "jk_cals_sweep": (I32, [VP, I32, VP]),
        "jk_cals_fit": (I32, [VP, I32, F64, VP, VP, VP]),
        "jk_cals_get_factors": (I32, [VP, I32, VP, VP]),
        "jk_cals_set_factors": (I32, [VP, I32, VP, VP]),
        "jk_cals_get_status": (I32, [VP, VP, VP, VP, VP]),
        "jk_cals_loss_grad": (I32, [VP, VP]),
        "jk_cals_get_grad": (I32, [VP, I32, VP, VP]),
        "jk_cals_scale_columns": (I32, [VP, I32, VP, VP, VP]),
        "jk_cals_refine": (I32, [VP, I32, VP]),
        "jk_cals_tune": (I32, [VP, I32]),
        "jk_cals_describe": (ctypes.c_char_p, [VP, I32]),
        "jk_cals_num_tilings": (I32, [VP]),
        "jk_cals_set_update_kernel": (I32, [VP, I32]),
        "jk_cals_set_sweep_graph": (I32, [VP, I32]),
        "jk_cals_set_mttkrp_tree": (I32, [VP, I32]),
        "jk_cals_set_allmode": (I32, [VP, I32]),
        "jk_cals_profile": (I32, [VP, I32]),
        "jk_cals_profile_read": (I32, [VP, VP, VP]),
        "jk_cals_set_tiling": (I32, [VP, I32, I32, I32]),
        "jk_cals_jackknife_std": (I32, [VP, I32, I32, I32, P(VP), VP, VP]),
        "jk_cals_set_compaction": (I32, [VP, I32]),
        "jk_cals_remove_slice": (I32, [P(Problem), VP, I32, VP]),
        "jk_cals_mttkrp_static": (I32, [P(Problem), VP, P(VP), I32, VP]),
        "jk_cals_destroy": (None, [VP]),
        "jk_cals_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def header_functions(path: str = HEADER) -> list:
    """Names of the functions the C header declares."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(jk_cals_[a-z_]+)\s*\(", text)))


def _check(st: int):
    if st != JKC_OK:
        raise JkcError(st, lib().jk_cals_last_error().decode())


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def _stream(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _check_buffer(t, shape, name, dtype="float64", device=None, allow_none=False):
    """Validate a caller buffer before its pointer reaches the library: a
    contiguous device tensor of the given dtype and shape (and device).
    Raises TypeError (dtype, not a tensor) or ValueError (placement, shape,
    layout); nothing is launched."""
    import torch
    if t is None:
        if allow_none:
            return
        raise ValueError("%s is required" % name)
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    want = {"float64": torch.float64, "int32": torch.int32}[dtype]
    if t.dtype != want:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if tuple(t.shape) != tuple(int(x) for x in shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if device is not None and t.device != device:
        raise ValueError("%s is on %s, the context on %s" % (name, t.device, device))


def to_device_tensor(T: np.ndarray, device="cuda"):
    """Flat device copy of T in column-major (i_1 fastest) order, the
    library's tensor layout."""
    import torch
    flat = np.ascontiguousarray(np.asarray(T).ravel(order="F"))
    return torch.from_numpy(flat).to(device)


def make_problem(dims, sampled_mode, ranks, left_out, tensor_dtype=JKC_TENSOR_F64,
                 precision=JKC_FP64, copy_tensor=1, stream=0, tree_max_gib=0):
    """Build the C problem descriptor; the returned tuple keeps the host
    arrays alive.  left_out is [K] (leave-one-out) or [K, d] (delete-d:
    row k lists the d samples model k leaves out, or d times -1)."""
    d = (ctypes.c_int64 * len(dims))(*[int(x) for x in dims])
    r = (ctypes.c_int32 * len(ranks))(*[int(x) for x in ranks])
    lo_np = np.asarray(left_out, dtype=np.int64)
    del_d = int(lo_np.shape[1]) if lo_np.ndim == 2 else 1
    flat = lo_np.reshape(-1)
    lo = (ctypes.c_int32 * len(flat))(*[int(x) for x in flat])
    prob = Problem(len(dims), d, int(sampled_mode), len(ranks), r, lo, int(tensor_dtype),
                   int(precision), int(copy_tensor), ctypes.c_void_p(stream), del_d,
                   int(tree_max_gib))
    return prob, (d, r, lo)


# ---------------------------------------------------------------------------
# Functions with the C ABI's names.
# ---------------------------------------------------------------------------

def jk_cals_workspace_size(dims, sampled_mode, ranks, left_out, tensor_dtype=JKC_TENSOR_F64,
                           precision=JKC_FP64, copy_tensor=1, tree_max_gib=0) -> int:
    prob, keep = make_problem(dims, sampled_mode, ranks, left_out, tensor_dtype, precision,
                              copy_tensor, 0, tree_max_gib)
    out = ctypes.c_size_t(0)
    _check(lib().jk_cals_workspace_size(ctypes.byref(prob), ctypes.byref(out)))
    return int(out.value)


class JkCals:
    """A JK-CALS context: the library context plus the torch-owned workspace
    (and, for copy_tensor=0, the tensor) it needs to stay alive."""

    def __init__(self, tensor, dims: Sequence[int], sampled_mode: int, ranks, left_out,
                 init: Sequence, precision: int = JKC_FP64, copy_tensor: bool = True,
                 stream=None, tree_max_gib: int = 0):
        import torch
        self.dims = [int(x) for x in dims]
        self.N = len(self.dims)
        self.sampled_mode = int(sampled_mode)
        self.ranks = np.asarray(ranks, dtype=np.int32)
        self.left_out = np.asarray(left_out, dtype=np.int32)
        self.K = len(self.ranks)
        self.C = int(self.ranks.sum())
        self.precision = int(precision)
        if tensor.dtype == torch.float64:
            tdt = JKC_TENSOR_F64
        elif tensor.dtype == torch.float32:
            tdt = JKC_TENSOR_F32
        else:
            raise TypeError("tensor must be float64 or float32")
        if not tensor.is_cuda:
            raise ValueError("tensor must be a device tensor")
        if tensor.numel() != int(np.prod(self.dims)):
            raise ValueError("tensor has %d elements, dims say %d" % (tensor.numel(), int(np.prod(self.dims))))
        for n, u in enumerate(init):
            if u.dtype != torch.float64 or not u.is_cuda or tuple(u.shape) != (self.dims[n], self.C) \
                    or not u.is_contiguous():
                raise ValueError("init[%d] must be a contiguous device float64 (%d, %d) tensor"
                                 % (n, self.dims[n], self.C))
        self.stream_handle = _stream(stream)
        self._prob, self._keep = make_problem(self.dims, sampled_mode, self.ranks, self.left_out,
                                              tdt, precision, 1 if copy_tensor else 0,
                                              self.stream_handle, tree_max_gib)
        size = ctypes.c_size_t(0)
        _check(lib().jk_cals_workspace_size(ctypes.byref(self._prob), ctypes.byref(size)))
        self.workspace_bytes = int(size.value)
        self.workspace = torch.empty(max(self.workspace_bytes, 256) + 256, dtype=torch.uint8,
                                     device=tensor.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        self._tensor = tensor                     # kept alive (needed when copy_tensor=0)
        self._init = list(init)                   # kept alive until init has run
        ptrs = (ctypes.c_void_p * self.N)(*[u.data_ptr() for u in init])
        ctx = ctypes.c_void_p(0)
        _check(lib().jk_cals_init(ctypes.byref(self._prob), ctypes.c_void_p(tensor.data_ptr()),
                                  ptrs, ctypes.c_void_p(aligned),
                                  ctypes.c_size_t(self.workspace_bytes), ctypes.byref(ctx)))
        self.ctx = ctx
        self.device = tensor.device

    # -- lifetime ---------------------------------------------------------
    def close(self):
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            lib().jk_cals_destroy(self.ctx)
            self.ctx = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- entry points -----------------------------------------------------
    def _out(self, rows, cols):
        import torch
        return torch.empty((rows, cols), dtype=torch.float64, device=self.device)

    def _mode(self, mode):
        if not 0 <= int(mode) < self.N:
            raise ValueError("mode must be in 0..%d" % (self.N - 1))
        return int(mode)

    def mttkrp(self, mode: int, out=None):
        mode = self._mode(mode)
        if out is None:
            out = self._out(self.dims[mode], self.C)
        _check_buffer(out, (self.dims[mode], self.C), "out", device=self.device)
        _check(lib().jk_cals_mttkrp(self.ctx, mode, ctypes.c_void_p(_ptr(out))))
        return out

    def sweep(self, nsweeps: int = 1, fit=None):
        _check_buffer(fit, (self.K,), "fit", device=self.device, allow_none=True)
        _check(lib().jk_cals_sweep(self.ctx, int(nsweeps), ctypes.c_void_p(_ptr(fit))))
        return fit

    def fit(self, max_iters: int, tol: float):
        iters = np.zeros(self.K, np.int32)
        fit = np.zeros(self.K, np.float64)
        status = np.zeros(self.K, np.int32)
        _check(lib().jk_cals_fit(self.ctx, int(max_iters), float(tol),
                                 iters.ctypes.data_as(ctypes.c_void_p),
                                 fit.ctypes.data_as(ctypes.c_void_p),
                                 status.ctypes.data_as(ctypes.c_void_p)))
        return iters, fit, status

    def get_factors(self, mode: int, with_lambda: bool = True):
        import torch
        out = self._out(self.dims[mode], self.C)
        lam = torch.empty(self.C, dtype=torch.float64, device=self.device) if with_lambda else None
        _check(lib().jk_cals_get_factors(self.ctx, int(mode), ctypes.c_void_p(_ptr(out)),
                                         ctypes.c_void_p(_ptr(lam))))
        return (out, lam) if with_lambda else out

    def set_factors(self, mode: int, U, lam=None):
        mode = self._mode(mode)
        _check_buffer(lam, (self.C,), "lambda", device=self.device, allow_none=True)
        _check_buffer(U, (self.dims[mode], self.C), "U", device=self.device)
        _check(lib().jk_cals_set_factors(self.ctx, mode, ctypes.c_void_p(_ptr(U)),
                                         ctypes.c_void_p(_ptr(lam))))

    def get_status(self):
        import torch
        err = torch.empty(self.K, dtype=torch.float64, device=self.device)
        fit = torch.empty(self.K, dtype=torch.float64, device=self.device)
        st = torch.empty(self.K, dtype=torch.int32, device=self.device)
        it = torch.empty(self.K, dtype=torch.int32, device=self.device)
        _check(lib().jk_cals_get_status(self.ctx, ctypes.c_void_p(_ptr(err)), ctypes.c_void_p(_ptr(fit)),
                                        ctypes.c_void_p(_ptr(st)), ctypes.c_void_p(_ptr(it))))
        return err, fit, st, it

    def loss_grad(self, loss=None):
        _check_buffer(loss, (self.K,), "loss", device=self.device, allow_none=True)
        _check(lib().jk_cals_loss_grad(self.ctx, ctypes.c_void_p(_ptr(loss))))
        return loss

    def get_grad(self, mode: int, weights=None, out=None):
        mode = self._mode(mode)
        if out is None:
            out = self._out(self.dims[mode], self.C)
        _check_buffer(out, (self.dims[mode], self.C), "out", device=self.device)
        _check_buffer(weights, (self.K,), "weights", device=self.device, allow_none=True)
        _check(lib().jk_cals_get_grad(self.ctx, mode, ctypes.c_void_p(_ptr(weights)),
                                      ctypes.c_void_p(_ptr(out))))
        return out

    def scale_columns(self, src, weights=None, out=None):
        """out(i, c) = weights[model of c] * src(i, c) for a (rows, C) block."""
        if src is None or getattr(src, "dim", lambda: 0)() != 2:
            raise ValueError("src must be a (rows, C) device tensor")
        rows = int(src.shape[0])
        _check_buffer(src, (rows, self.C), "src", device=self.device)
        if out is None:
            out = self._out(rows, self.C)
        _check_buffer(out, (rows, self.C), "out", device=self.device)
        _check_buffer(weights, (self.K,), "weights", device=self.device, allow_none=True)
        _check(lib().jk_cals_scale_columns(self.ctx, rows, ctypes.c_void_p(_ptr(src)),
                                           ctypes.c_void_p(_ptr(weights)),
                                           ctypes.c_void_p(_ptr(out))))
        return out

    def refine(self, steps: int, loss=None):
        _check_buffer(loss, (self.K,), "loss", device=self.device, allow_none=True)
        _check(lib().jk_cals_refine(self.ctx, int(steps), ctypes.c_void_p(_ptr(loss))))
        return loss

    def tune(self, reps: int = 3):
        _check(lib().jk_cals_tune(self.ctx, int(reps)))

    def jackknife_std(self, ref: int, first: int, count: int, with_matching: bool = False):
        """Alg. 2's jackknife standard deviations of the models first ..
        first+count-1 against model ``ref``: {mode: I_n x R tensor} for
        every mode except the sampled one; with_matching also returns the
        matched components (count x R int32) and signs (N x count x R)."""
        import torch
        R = int(self.ranks[ref])
        out = {n: torch.empty((self.dims[n], R), dtype=torch.float64, device="cuda")
               for n in range(self.N) if n != self.sampled_mode}
        ptrs = (ctypes.c_void_p * self.N)(*[_ptr(out.get(n)) for n in range(self.N)])
        perm = sign = None
        if with_matching:
            perm = torch.empty((count, R), dtype=torch.int32, device="cuda")
            sign = torch.empty((self.N, count, R), dtype=torch.float64, device="cuda")
        _check(lib().jk_cals_jackknife_std(self.ctx, int(ref), int(first), int(count), ptrs,
                                           ctypes.c_void_p(_ptr(perm)), ctypes.c_void_p(_ptr(sign))))
        return (out, perm, sign) if with_matching else out

    def describe(self, mode: int) -> str:
        return lib().jk_cals_describe(self.ctx, int(mode)).decode()

    def profile(self, enable: bool = True):
        _check(lib().jk_cals_profile(self.ctx, 1 if enable else 0))

    def profile_read(self):
        """(launches, milliseconds) per slot since the last read: slot n < N
        the fused MTTKRP of mode n with its split-K reduction, slot N the
        shared contraction W."""
        n = np.zeros(self.N + 1, np.int64)
        ms = np.zeros(self.N + 1, np.float64)
        _check(lib().jk_cals_profile_read(self.ctx, n.ctypes.data_as(ctypes.c_void_p),
                                          ms.ctypes.data_as(ctypes.c_void_p)))
        return n, ms

    def set_update_kernel(self, which: int):
        _check(lib().jk_cals_set_update_kernel(self.ctx, int(which)))

    def set_compaction(self, enable: bool):
        _check(lib().jk_cals_set_compaction(self.ctx, 1 if enable else 0))

    def set_sweep_graph(self, enable: bool):
        _check(lib().jk_cals_set_sweep_graph(self.ctx, 1 if enable else 0))

    def set_mttkrp_tree(self, enable: bool):
        _check(lib().jk_cals_set_mttkrp_tree(self.ctx, 1 if enable else 0))

    def set_allmode(self, enable: bool):
        _check(lib().jk_cals_set_allmode(self.ctx, 1 if enable else 0))

    def num_tilings(self) -> int:
        return int(lib().jk_cals_num_tilings(self.ctx))

    def set_tiling(self, mode: int, variant: int, splits: int):
        _check(lib().jk_cals_set_tiling(self.ctx, int(mode), int(variant), int(splits)))


def jk_cals_init(tensor, dims, sampled_mode, ranks, left_out, init, precision=JKC_FP64,
                 copy_tensor=True, stream=None) -> JkCals:
    return JkCals(tensor, dims, sampled_mode, ranks, left_out, init, precision, copy_tensor, stream)


def jk_cals_mttkrp(ctx: JkCals, mode: int, out=None):
    return ctx.mttkrp(mode, out)


def jk_cals_sweep(ctx: JkCals, nsweeps: int = 1, fit=None):
    return ctx.sweep(nsweeps, fit)


def jk_cals_fit(ctx: JkCals, max_iters: int, tol: float):
    return ctx.fit(max_iters, tol)


def jk_cals_get_factors(ctx: JkCals, mode: int):
    return ctx.get_factors(mode)


def jk_cals_set_factors(ctx: JkCals, mode: int, U, lam=None):
    return ctx.set_factors(mode, U, lam)


def jk_cals_get_status(ctx: JkCals):
    return ctx.get_status()


def jk_cals_loss_grad(ctx: JkCals, loss=None):
    return ctx.loss_grad(loss)


def jk_cals_get_grad(ctx: JkCals, mode: int, weights=None, out=None):
    return ctx.get_grad(mode, weights, out)


def jk_cals_scale_columns(ctx: JkCals, src, weights=None, out=None):
    return ctx.scale_columns(src, weights, out)


def jk_cals_refine(ctx: JkCals, steps: int, loss=None):
    return ctx.refine(steps, loss)


def jk_cals_tune(ctx: JkCals, reps: int = 3):
    return ctx.tune(reps)


def jk_cals_jackknife_std(ctx: JkCals, ref: int, first: int, count: int, with_matching=False):
    return ctx.jackknife_std(ref, first, count, with_matching)


def jk_cals_describe(ctx: JkCals, mode: int) -> str:
    return ctx.describe(mode)


def jk_cals_profile(ctx: JkCals, enable: bool = True):
    return ctx.profile(enable)


def jk_cals_profile_read(ctx: JkCals):
    return ctx.profile_read()


def jk_cals_set_update_kernel(ctx: JkCals, which: int):
    return ctx.set_update_kernel(which)


def jk_cals_set_sweep_graph(ctx: JkCals, enable: bool):
    return ctx.set_sweep_graph(enable)


def jk_cals_set_mttkrp_tree(ctx: JkCals, enable: bool):
    return ctx.set_mttkrp_tree(enable)


def jk_cals_set_allmode(ctx: JkCals, enable: bool):
    return ctx.set_allmode(enable)


def jk_cals_num_tilings(ctx: JkCals) -> int:
    return ctx.num_tilings()


def jk_cals_set_tiling(ctx: JkCals, mode: int, variant: int, splits: int):
    return ctx.set_tiling(mode, variant, splits)


def jk_cals_remove_slice(tensor, dims, sampled_mode, p, out=None, stream=None):
    """Explicitly reduced tensor of Alg. 2 (slice p of the sampled mode
    deleted), as a flat device tensor in the library layout."""
    import torch
    if tensor.dtype not in (torch.float64, torch.float32):
        raise TypeError("tensor must be float64 or float32")
    tdt = JKC_TENSOR_F64 if tensor.dtype == torch.float64 else JKC_TENSOR_F32
    if not tensor.is_cuda or not tensor.is_contiguous():
        raise ValueError("tensor must be a contiguous device tensor")
    if tensor.numel() != int(np.prod(dims)):
        raise ValueError("tensor has %d elements, dims say %d" % (tensor.numel(), int(np.prod(dims))))
    n_out = int(np.prod(dims)) // int(dims[sampled_mode]) * (int(dims[sampled_mode]) - 1)
    if out is None:
        out = torch.empty(n_out, dtype=tensor.dtype, device=tensor.device)
    if (not isinstance(out, torch.Tensor) or out.dtype != tensor.dtype or not out.is_cuda
            or out.numel() != n_out or not out.is_contiguous()):
        raise ValueError("out must be a contiguous device tensor of %d elements of the tensor's dtype"
                         % n_out)
    prob, keep = make_problem(dims, sampled_mode, [1], [-1], tdt, JKC_FP64, 1, _stream(stream))
    _check(lib().jk_cals_remove_slice(ctypes.byref(prob), ctypes.c_void_p(tensor.data_ptr()),
                                      int(p), ctypes.c_void_p(out.data_ptr())))
    return out


def jk_cals_mttkrp_static(tensor, dims, sampled_mode, ranks, left_out, factors, mode,
                          out=None, stream=None):
    """Fused MTTKRP of one mode from caller buffers, computed in the
    library's fixed device scratch (no context, no workspace, nothing
    allocated by the library; float64).  factors: N device float64
    (I_m, C) tensors (factors[mode] may be None).  out: (I_mode, C) device
    float64, allocated here when not given (pass it to allocate nothing)."""
    import torch
    dims = [int(x) for x in dims]
    N = len(dims)
    ranks = np.asarray(ranks, dtype=np.int32)
    C = int(ranks.sum())
    if not isinstance(tensor, torch.Tensor) or tensor.dtype not in (torch.float64, torch.float32):
        raise TypeError("tensor must be a float64 or float32 torch tensor")
    if not tensor.is_cuda or not tensor.is_contiguous():
        raise ValueError("tensor must be a contiguous device tensor")
    if tensor.numel() != int(np.prod(dims)):
        raise ValueError("tensor has %d elements, dims say %d" % (tensor.numel(), int(np.prod(dims))))
    if not 0 <= int(mode) < N:
        raise ValueError("mode must be in 0..%d" % (N - 1))
    mode = int(mode)
    if len(factors) != N:
        raise ValueError("factors must hold %d entries" % N)
    for m in range(N):
        if m != mode:
            _check_buffer(factors[m], (dims[m], C), "factors[%d]" % m, device=tensor.device)
    if out is None:
        out = torch.empty((dims[mode], C), dtype=torch.float64, device=tensor.device)
    _check_buffer(out, (dims[mode], C), "out", device=tensor.device)
    tdt = JKC_TENSOR_F64 if tensor.dtype == torch.float64 else JKC_TENSOR_F32
    prob, keep = make_problem(dims, sampled_mode, ranks, left_out, tdt, JKC_FP64, 1, _stream(stream))
    ptrs = (ctypes.c_void_p * N)(*[0 if (m == mode or factors[m] is None) else factors[m].data_ptr()
                                    for m in range(N)])
    _check(lib().jk_cals_mttkrp_static(ctypes.byref(prob), ctypes.c_void_p(tensor.data_ptr()),
                                       ptrs, mode, ctypes.c_void_p(out.data_ptr())))
    return out


def jk_cals_destroy(ctx: JkCals):
    ctx.close()


def jk_cals_last_error() -> str:
    return lib().jk_cals_last_error().decode()


def _make_loss_function():
    import torch

    class JKCPLoss(torch.autograd.Function):
        """Per-submodel CP least-squares loss f_k = 1/2 ||T_{-p_k} - [[U^(k)]]||^2
        over all models of a context, differentiable in the factors.

        forward(ctx, U_0, ..., U_{N-1}) -> loss[K]: installs the factors
        (device (I_n, C) float64; row p_k of the sampled mode is taken as 0)
        and runs the all-mode fused MTTKRP, the loss and the gradients in the
        library; the unweighted gradients are copied out of the context
        right away and saved with the graph node, so later calls on the same
        context (another forward, loss_grad, refine) cannot change what this
        node's backward returns.  backward(grad_loss[K]) returns
        grad_loss[k] * dF_k/dU_n on model k's columns (the library scales
        the saved gradients)."""

        @staticmethod
        def forward(fctx, jkctx, *factors):
            if len(factors) != jkctx.N:
                raise ValueError("expected %d factors" % jkctx.N)
            ones = torch.ones(jkctx.C, dtype=torch.float64, device=jkctx.device)
            for n, U in enumerate(factors):
                jkctx.set_factors(n, U.detach().contiguous(), ones)
            loss = torch.empty(jkctx.K, dtype=torch.float64, device=jkctx.device)
            jkctx.loss_grad(loss)
            fctx.jk = jkctx
            fctx.grads = [jkctx.get_grad(n) for n in range(jkctx.N)]
            return loss

        @staticmethod
        def backward(fctx, grad_loss):
            jkctx = fctx.jk
            w = grad_loss.detach().to(torch.float64).contiguous()
            grads = [jkctx.scale_columns(g, weights=w) for g in fctx.grads]
            return (None, *grads)

    return JKCPLoss


def __getattr__(name):
    if name == "JKCPLoss":
        f = _make_loss_function()
        globals()["JKCPLoss"] = f
        return f
    raise AttributeError(name)
