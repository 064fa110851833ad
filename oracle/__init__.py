"""FP64 CPU oracle for the colour-vibration pair search (ctypes wrapper).

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import this package.  It shares no
code with the HIP library: the arithmetic lives in ``cvib_oracle.c`` (plain C,
FP64, libm ``pow``/``cbrt``) and ``mlp_oracle.c``; this file only marshals
arguments.

Method (Section 2 of the paper): split the target colour into L*, a*, b*;
add / subtract the displacement arrays D_a = r sin(theta), D_b = r cos(theta)
to a* and b* with L* fixed; convert both colours of each pair back to RGB;
keep pairs whose per-channel RGB change encodes a pattern under the V_th /
R_novib thresholds of Section 3 / Table 1.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libcvib_oracle.so")
_SOURCES = ["cvib_oracle.c", "mlp_oracle.c", "frame_oracle.c"]


def compile_library(srcs, out: str) -> str:
    """gcc, FP64, no fast-math, OpenMP: the oracle's one build recipe."""
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math",
           "-o", tmp] + list(srcs) + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def sources() -> list[str]:
    return [os.path.join(_HERE, s) for s in _SOURCES]


def build(force: bool = True) -> str:
    """Compile the oracle."""
    if not force and os.path.exists(_SO):
        return _SO
    return compile_library(sources(), _SO)


class Grid(C.Structure):
    _fields_ = [("dr", C.c_double), ("nr", C.c_int32), ("_pad0", C.c_int32),
                ("dtheta_deg", C.c_double), ("ntheta", C.c_int32), ("_pad1", C.c_int32)]


class Rule(C.Structure):
    _fields_ = [("v_th", C.c_int32), ("_pad0", C.c_int32), ("r_novib", C.c_double),
                ("mask", C.c_uint32), ("flags", C.c_uint32)]


CAND_DTYPE = np.dtype([
    ("vp", "<f8", 3), ("vm", "<f8", 3), ("linp", "<f8", 3), ("linm", "<f8", 3),
    ("Vp", "u1", 3), ("Vm", "u1", 3), ("gamut", "u1"), ("pattern", "u1"),
    ("valid", "u1"), ("boundary", "u1"), ("dset", "u1"), ("_pad", "u1", 3)], align=True)
assert CAND_DTYPE.itemsize == 112

REC_DTYPE = np.dtype([("colour", "<u4"), ("i", "<u2"), ("j", "<u2"), ("plus", "u1", 3),
                      ("minus", "u1", 3), ("pattern", "u1"), ("flags", "u1")])
assert REC_DTYPE.itemsize == 16

SUMMARY_DTYPE = np.dtype([
    ("count", "<u4"), ("n_gamut", "<u4"), ("n_boundary", "<u4"), ("n_ambiguous", "<u4"),
    ("best_i", "<u2"),
    ("best_j", "<u2"), ("best_plus", "u1", 3), ("best_minus", "u1", 3), ("best_p", "u1"),
    ("_pad", "u1"), ("per_pattern", "<u4", 7)])
assert SUMMARY_DTYPE.itemsize == 56

# Ranges of a colour's outputs when each decision-ambiguous candidate may end
# either way (orc_reduce_bounds); keys are i << 16 | (0xFFFF - j), 0 = none.
BOUNDS_DTYPE = np.dtype([
    ("count_lo", "<u4"), ("count_hi", "<u4"), ("pat_lo", "<u4", 7), ("pat_hi", "<u4", 7),
    ("key_lo", "<u4"), ("key_hi", "<u4"), ("pkey_lo", "<u4", 7), ("pkey_hi", "<u4", 7),
    ("n_gamut", "<u4"), ("n_boundary", "<u4"), ("n_ambiguous", "<u4"), ("best_band", "u1"),
    ("pbest_band", "u1", 7), ("_pad", "<u4")])
assert BOUNDS_DTYPE.itemsize == 152

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        _lib = load_library(_SO)
    return _lib


def load_library(path: str) -> C.CDLL:
    """Load a build of the oracle's sources and declare its entry points."""
    L = C.CDLL(path)
    P = C.c_void_p
    L.orc_matrices.argtypes = [P, P, P]
    L.orc_decode.argtypes = [C.c_double]
    L.orc_decode.restype = C.c_double
    L.orc_encode.argtypes = [C.c_double]
    L.orc_encode.restype = C.c_double
    L.orc_rgb8_to_lab.argtypes = [P, C.c_int64, P]
    L.orc_lab_to_linear.argtypes = [P, C.c_int64, P]
    L.orc_lab_to_v.argtypes = [P, C.c_int64, P, P]
    L.orc_eval.argtypes = [P, C.POINTER(Grid), C.POINTER(Rule), C.c_int32, C.c_int32,
                           C.c_int32, P]
    L.orc_eval_all.argtypes = [P, C.c_int64, C.POINTER(Grid), C.POINTER(Rule), P, C.c_int32]
    L.orc_eval_list.argtypes = [P, P, C.c_int64, C.POINTER(Grid), C.POINTER(Rule), P,
                                C.c_int32]
    L.orc_search.argtypes = [P, C.c_int64, C.POINTER(Grid), C.POINTER(Rule), P, C.c_int64,
                             P, P, C.c_int32]
    L.orc_search.restype = C.c_int64
    L.orc_reduce.argtypes = [P, C.c_int64, C.POINTER(Grid), C.POINTER(Rule), P, P, P,
                             C.c_int32]
    L.orc_max_gamut_radius.argtypes = [P, C.c_int64, C.POINTER(Grid), P, C.c_int32]
    L.orc_reduce_bounds.argtypes = [P, C.c_int64, C.POINTER(Grid), C.POINTER(Rule), P, P, P, P, P,
                                    C.c_int32]
    L.orc_num_threads.restype = C.c_int32
    _mlp_bind(L)
    L.orc_philox4x64.argtypes = [P, P, P]
    L.orc_gen_frame.argtypes = [C.c_uint64, C.c_int32, C.c_int32, C.c_int32, C.c_int32, P]
    L.orc_gen_frame.restype = C.c_int32
    return L


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def grid(dr: float, nr: int, dtheta_deg: float, ntheta: int) -> Grid:
    return Grid(dr=float(dr), nr=int(nr), dtheta_deg=float(dtheta_deg), ntheta=int(ntheta))


def rule(v_th: int = 50, r_novib: float = 0.5, mask: int = 0x7F, flags: int = 0) -> Rule:
    """flags bit0: clip reading (clamp code values instead of rejecting the pair)."""
    return Rule(v_th=int(v_th), r_novib=float(r_novib), mask=int(mask), flags=int(flags))


def _as_grid(g):
    return g if isinstance(g, Grid) else grid(*g)


def _as_rule(r):
    if r is None or isinstance(r, Rule):
        return r
    return rule(*r)


def _rgb(colors) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(colors, dtype=np.uint8).reshape(-1, 3))
    return a


def matrices():
    M = np.zeros(9)
    Minv = np.zeros(9)
    W = np.zeros(3)
    lib().orc_matrices(_ptr(M), _ptr(Minv), _ptr(W))
    return M.reshape(3, 3), Minv.reshape(3, 3), W


def decode(c: float) -> float:
    return lib().orc_decode(float(c))


def encode(l: float) -> float:
    return lib().orc_encode(float(l))


def rgb8_to_lab(colors) -> np.ndarray:
    rgb = _rgb(colors)
    out = np.zeros((rgb.shape[0], 3))
    lib().orc_rgb8_to_lab(_ptr(rgb), rgb.shape[0], _ptr(out))
    return out


def lab_to_linear(lab) -> np.ndarray:
    lab = np.ascontiguousarray(np.asarray(lab, dtype=np.float64).reshape(-1, 3))
    out = np.zeros_like(lab)
    lib().orc_lab_to_linear(_ptr(lab), lab.shape[0], _ptr(out))
    return out


def lab_to_v(lab):
    """Lab -> (v [n,3] unrounded 0..255 units, gamut [n] 0/1)."""
    lab = np.ascontiguousarray(np.asarray(lab, dtype=np.float64).reshape(-1, 3))
    v = np.zeros_like(lab)
    g = np.zeros(lab.shape[0], dtype=np.uint8)
    lib().orc_lab_to_v(_ptr(lab), lab.shape[0], _ptr(v), _ptr(g))
    return v, g


def eval_one(color, g, r=None, i=0, j=0, r_zero=False, L=None) -> np.ndarray:
    rgb = _rgb(color)
    out = np.zeros(1, dtype=CAND_DTYPE)
    ru = _as_rule(r)
    (L or lib()).orc_eval(_ptr(rgb), C.byref(_as_grid(g)), C.byref(ru) if ru else None, int(i),
                   int(j), int(bool(r_zero)), _ptr(out))
    return out[0]


def eval_all(colors, g, r=None, nthreads: int = 0) -> np.ndarray:
    """Every candidate, shape [n, nr, ntheta] of CAND_DTYPE."""
    rgb = _rgb(colors)
    gg = _as_grid(g)
    out = np.zeros((rgb.shape[0], gg.nr, gg.ntheta), dtype=CAND_DTYPE)
    ru = _as_rule(r)
    lib().orc_eval_all(_ptr(rgb), rgb.shape[0], C.byref(gg), C.byref(ru) if ru else None,
                       _ptr(out), int(nthreads))
    return out


def eval_list(colors, idx, g, r=None, nthreads: int = 0, L=None) -> np.ndarray:
    """Candidates named by rows (colour index, i, j) of idx (L: another build
    of the oracle, from load_library)."""
    rgb = _rgb(colors)
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int64).reshape(-1, 3))
    out = np.zeros(idx.shape[0], dtype=CAND_DTYPE)
    ru = _as_rule(r)
    (L or lib()).orc_eval_list(_ptr(rgb), _ptr(idx), idx.shape[0], C.byref(_as_grid(g)),
                        C.byref(ru) if ru else None, _ptr(out), int(nthreads))
    return out


def search(colors, g, r, nthreads: int = 0):
    """(records [total] REC_DTYPE, offsets [n+1], n_boundary).  flags bit0 of a
    record marks a boundary candidate."""
    rgb = _rgb(colors)
    gg, ru = _as_grid(g), _as_rule(r)
    n = rgb.shape[0]
    offs = np.zeros(n + 1, dtype=np.int64)
    nb = np.zeros(1, dtype=np.int64)
    total = lib().orc_search(_ptr(rgb), n, C.byref(gg), C.byref(ru), None, 0, _ptr(offs),
                             _ptr(nb), int(nthreads))
    out = np.zeros(max(total, 1), dtype=REC_DTYPE)
    total2 = lib().orc_search(_ptr(rgb), n, C.byref(gg), C.byref(ru), _ptr(out), total,
                              _ptr(offs), _ptr(nb), int(nthreads))
    assert total2 == total
    return out[:total], offs, int(nb[0])


def reduce(colors, g, r, table: bool = False, nthreads: int = 0):
    """Per-colour summaries (SUMMARY_DTYPE [n]); with table=True also
    (count u32 [n], bins u8 [n, 36])."""
    rgb = _rgb(colors)
    gg, ru = _as_grid(g), _as_rule(r)
    n = rgb.shape[0]
    summ = np.zeros(n, dtype=SUMMARY_DTYPE)
    tc = np.zeros(n, dtype=np.uint32) if table else None
    tb = np.zeros((n, 36), dtype=np.uint8) if table else None
    lib().orc_reduce(_ptr(rgb), n, C.byref(gg), C.byref(ru), _ptr(summ),
                     _ptr(tc) if table else None, _ptr(tb) if table else None, int(nthreads))
    return (summ, tc, tb) if table else summ


def reduce_bounds(colors, g, r, bins: bool = False, rays: bool = False, nthreads: int = 0):
    """Per colour, the range every reduce output can take when each
    decision-ambiguous candidate may end either way: BOUNDS_DTYPE [n], and
    with bins (bins_lo, bins_hi) u8 [n, 36], with rays (rays_lo, rays_hi)
    u16 [n, ntheta] (largest i + 1 over must / may survivors, 0 = none).
    Returns a dict with the keys that were asked for."""
    rgb = _rgb(colors)
    gg, ru = _as_grid(g), _as_rule(r)
    n = rgb.shape[0]
    out = {"bounds": np.zeros(n, dtype=BOUNDS_DTYPE)}
    bl = bh = rl = rh = None
    if bins:
        bl, bh = np.zeros((n, 36), np.uint8), np.zeros((n, 36), np.uint8)
        out.update(bins_lo=bl, bins_hi=bh)
    if rays:
        rl, rh = np.zeros((n, gg.ntheta), np.uint16), np.zeros((n, gg.ntheta), np.uint16)
        out.update(rays_lo=rl, rays_hi=rh)
    lib().orc_reduce_bounds(_ptr(rgb), n, C.byref(gg), C.byref(ru), _ptr(out["bounds"]),
                            _ptr(bl) if bins else None, _ptr(bh) if bins else None,
                            _ptr(rl) if rays else None, _ptr(rh) if rays else None, int(nthreads))
    return out


def max_gamut_radius(colors, g, nthreads: int = 0) -> np.ndarray:
    rgb = _rgb(colors)
    out = np.zeros(rgb.shape[0], dtype=np.int32)
    lib().orc_max_gamut_radius(_ptr(rgb), rgb.shape[0], C.byref(_as_grid(g)), _ptr(out),
                               int(nthreads))
    return out


def num_threads() -> int:
    return int(lib().orc_num_threads())


# --------------------------------------------------------------------------
# MLP oracle (FP64 forward / backward / loss of the surrogate network).

def _mlp_bind(L):
    P = C.c_void_p
    L.orc_mlp_forward.argtypes = [P, C.c_int32, P, P, C.c_int64, P, P, C.c_double]
    L.orc_mlp_loss.argtypes = [P, P, P, C.c_int64, C.c_int32, C.c_double, P]
    L.orc_mlp_loss.restype = C.c_double
    L.orc_mlp_backward.argtypes = [P, C.c_int32, P, P, C.c_int64, P, P, P, P, C.c_double]
    L.orc_linear_input_grad.argtypes = [C.c_int32, C.c_int32, P, C.c_int64, P, P]


def _flat(dims, Ws, bs):
    W = np.ascontiguousarray(np.concatenate([np.asarray(w, np.float64).ravel() for w in Ws]))
    b = np.ascontiguousarray(np.concatenate([np.asarray(v, np.float64).ravel() for v in bs]))
    return np.asarray(dims, dtype=np.int32), W, b


def mlp_forward(dims, Ws, bs, x, omega0: float = 0.0) -> np.ndarray:
    """dims = [d0..dL]; Ws[l] is [d_{l+1}, d_l]; bs[l] is [d_{l+1}]; x is [B, d0].
    Returns the network output [B, dL] (ReLU hidden layers, or sin(omega0 z)
    on the first when omega0 > 0; linear output)."""
    d, W, b = _flat(dims, Ws, bs)
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    out = np.zeros((x.shape[0], int(d[-1])))
    lib().orc_mlp_forward(_ptr(d), len(d) - 1, _ptr(W), _ptr(b), x.shape[0], _ptr(x), _ptr(out),
                          float(omega0))
    return out


def mlp_loss(out, target_r, target_f, huber_delta: float):
    """Loss and its gradient w.r.t. the network output (see mlp_oracle.c)."""
    out = np.ascontiguousarray(np.asarray(out, dtype=np.float64))
    tr = np.ascontiguousarray(np.asarray(target_r, dtype=np.float64))
    tf = np.ascontiguousarray(np.asarray(target_f, dtype=np.float64))
    B, D = out.shape
    g = np.zeros_like(out)
    val = lib().orc_mlp_loss(_ptr(out), _ptr(tr), _ptr(tf), B, D, float(huber_delta), _ptr(g))
    return val, g


def mlp_backward(dims, Ws, bs, x, gout, omega0: float = 0.0):
    """Gradients of sum(gout * out) w.r.t. every layer's weights and biases."""
    d, W, b = _flat(dims, Ws, bs)
    nl = len(d) - 1
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    gout = np.ascontiguousarray(np.asarray(gout, dtype=np.float64))
    gW = np.zeros_like(W)
    gb = np.zeros_like(b)
    lib().orc_mlp_backward(_ptr(d), nl, _ptr(W), _ptr(b), x.shape[0], _ptr(x), _ptr(gout),
                           _ptr(gW), _ptr(gb), float(omega0))
    gWs, gbs, ow, ob = [], [], 0, 0
    for l in range(nl):
        o, i = int(d[l + 1]), int(d[l])
        gWs.append(gW[ow:ow + o * i].reshape(o, i))
        gbs.append(gb[ob:ob + o])
        ow += o * i
        ob += o
    return gWs, gbs


def distinct_colours(frames_u8: np.ndarray) -> np.ndarray:
    """Sorted distinct colour ids (R<<16 | G<<8 | B) of a frame stack: the plain
    definition of the de-duplication step."""
    f = np.asarray(frames_u8).reshape(-1, 3).astype(np.uint32)
    ids = (f[:, 0] << 16) | (f[:, 1] << 8) | f[:, 2]
    return np.unique(ids)


def linear_input_grad(W, gout) -> np.ndarray:
    """Gradient of sum(gout * (x W^T + b)) with respect to x: gout W, [B, d_in]
    for W [d_out, d_in] and gout [B, d_out]."""
    W = np.ascontiguousarray(np.asarray(W, dtype=np.float64))
    gout = np.ascontiguousarray(np.asarray(gout, dtype=np.float64))
    dout, din = W.shape
    gin = np.zeros((gout.shape[0], din))
    lib().orc_linear_input_grad(int(din), int(dout), _ptr(W), gout.shape[0], _ptr(gout), _ptr(gin))
    return gin


def adam_step(p, g, m, v, t: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8):
    """One Adam step (Kingma & Ba 2015, Algorithm 1) in FP64: returns the new
    (p, m, v).  m and v are the first and second moment estimates, t >= 1."""
    p, g, m, v = (np.asarray(a, dtype=np.float64) for a in (p, g, m, v))
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v


# --------------------------------------------------------------------------
# Twin of the library's synthetic frame generator (frame_oracle.c).

def philox4x64(counter, key) -> np.ndarray:
    """Philox4x64-10 (Salmon et al., SC'11) of one 4-word counter under a
    2-word key: uint64 [4]."""
    ctr = np.ascontiguousarray(np.asarray(counter, dtype=np.uint64).reshape(4))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint64).reshape(2))
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64(_ptr(ctr), _ptr(k), _ptr(out))
    return out


def gen_frame(seed: int, height: int, width: int, sites: int = 64, noise: int = 4) -> np.ndarray:
    """One synthetic frame, uint8 [height, width, 3] (the recipe in
    frame_oracle.c)."""
    out = np.zeros((height, width, 3), dtype=np.uint8)
    rc = lib().orc_gen_frame(C.c_uint64(int(seed)), int(height), int(width), int(sites), int(noise), _ptr(out))
    if rc != 0:
        raise ValueError("bad frame size, site count or noise")
    return out
