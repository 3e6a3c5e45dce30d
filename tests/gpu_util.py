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


_FAMILY = {"mfma16x16x4": 0, "mfma4x4x4-diagonal": 1, "mfma4x4x4-strips": 2,
           "mfma16x16x32bf16": 0}


def variant_geometry(desc):
    """(wm, wn, tm, tn, bk, instr) of a tiling description
    ("f64 v34 wm1 wn4 tm7 tn2 bk16 s128 mfma16x16x4-interleaved-buffer",
    "bf16x3 v5 wm2 wn2 tm2 tn2 bk32 s8 mfma16x16x32bf16"), in the form of the
    tuned-tilings table; None for the narrow tiling."""
    f = desc.split()
    if f and f[0] == "tree":
        f = f[1:]
    suffix = f[8]
    if suffix.startswith("valu-narrow"):
        return None
    instr = 0
    if suffix.endswith("-buffer"):
        instr += 16
        suffix = suffix[: -len("-buffer")]
    if suffix.endswith("-interleaved"):
        instr += 8
        suffix = suffix[: -len("-interleaved")]
    instr += _FAMILY[suffix]
    num = [int(x.lstrip("wmntbk")) for x in f[2:7]]
    return tuple(num) + (instr,)


def shipped_tilings(wl, precision=0):
    """Tilings of the shipped tuned table (the ones bench.py times) for this
    workload and precision (0 float64, 1 bf16x3, 2 bf16x6): {slot: ((wm, wn,
    tm, tn, bk, instr), splits)}, slot N the shared contraction."""
    import os
    C = int(sum(wl.ranks))
    ldc = (C + 15) // 16 * 16
    path = os.path.join(os.path.dirname(__file__), "..", "paper_2112_03985_amd", "tuned_gfx950.txt")
    N = len(wl.dims)
    key = "gfx950 p%d f32_%d N%d d%s ldc%d " % (precision, int(wl.T.dtype == np.float32), N,
                                               "x".join(str(d) for d in wl.dims), ldc)
    out = {}
    for line in open(path):
        if not line.strip():
            continue
        k, geo, sp = line.strip().split("|")
        if not k.startswith(key):
            continue
        slot = k[len(key):]
        n = N if slot == "tree" else int(slot[len("mode"):])
        out[n] = (tuple(int(x) for x in geo.split()), int(sp))
    return out


def apply_tilings(ctx, tilings):
    """Force the given {slot: (geometry, splits)} on ctx (slot N: the shared
    contraction), finding each geometry's variant index from the
    descriptions; returns the descriptions."""
    assert tilings, "no tuned tilings for this workload"
    import paper_2112_03985_amd as jk
    N = ctx.N
    index = {}
    for v in range(ctx.num_tilings()):
        try:
            ctx.set_tiling(0, v, 1)
        except jk.JkcError:
            continue
        g = variant_geometry(ctx.describe(0))
        if g is not None:
            index[g] = v
    for n, (geo, splits) in sorted(tilings.items()):
        ctx.set_tiling(n, index[geo], splits)
    return [ctx.describe(n) for n in range(N + 1)]
