"""Shared helpers of the GPU parity tests (not collected by pytest)."""
import sys

import numpy as np

import oracle


def say(*a):
    """Name the case before each GPU step, flushed, so a crash still shows it."""
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def device_inputs(wl):
    import torch
    import paper_2112_03985_amd as jk
    T = jk.to_device_tensor(wl.T)
    init = [torch.from_numpy(np.ascontiguousarray(u)).cuda() for u in wl.init]
    return T, init


def make_ctx(wl, precision=0, copy_tensor=True):
    import paper_2112_03985_amd as jk
    T, init = device_inputs(wl)
    return jk.JkCals(T, wl.dims, wl.sampled_mode, wl.ranks, wl.left_out, init,
                     precision=precision, copy_tensor=copy_tensor)


def cols(wl, k):
    off = oracle.model_offsets(wl.ranks)
    return slice(int(off[k]), int(off[k] + wl.ranks[k]))


def oracle_model_mttkrp(wl, k, n, factors=None):
    """Per-submodel MTTKRP by definition: reduced tensor, reduced factors,
    output padded with a zero row at p for the sampled mode."""
    src = wl.init if factors is None else factors
    c = cols(wl, k)
    U = [np.array(src[m][:, c], dtype=np.float64) for m in range(len(wl.dims))]
    p = wl.left_out[k]
    rows = oracle.left_out_rows(p)
    nh = wl.sampled_mode
    U[nh] = oracle.reduce_init(U[nh], p)
    Tk = oracle.reduce_tensor(np.asarray(wl.T, dtype=np.float64), nh, p)
    M = oracle.mttkrp(Tk, U, n)
    if n == nh and rows:
        full = np.zeros((wl.dims[nh], M.shape[1]))
        full[np.setdiff1d(np.arange(wl.dims[nh]), rows)] = M
        M = full
    return M


def errors(a, b):
    """(normwise, elementwise) relative error of a against b: the Frobenius
    ratio ||a - b|| / ||b||, and the largest entry error relative to the
    largest entry, max|a - b| / max|b| (a single wrong entry in a large
    block shows in the second even when the first hides it)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    fro = float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))
    mb = float(np.max(np.abs(b))) if b.size else 0.0
    mx = float(np.max(np.abs(a - b)) / (mb if mb > 0 else 1.0)) if b.size else 0.0
    return fro, mx


def rel_fro(a, b):
    """Normwise relative error alone (error models stated normwise)."""
    return errors(a, b)[0]


def rel(a, b):
    """The larger of the normwise and the elementwise relative error."""
    return max(errors(a, b))


def to_np(t):
    return t.detach().cpu().numpy()
