"""cvib: colour-vibration pair search on AMD Instinct MI355X (gfx950).

Python binding of ``libcvib.so`` (C-ABI declared in ``include/cvib.h``).  This
module only marshals arguments: every step of the search runs in the HIP
kernels of the library.  PyTorch supplies device memory and the current HIP
stream.  If the compiled library is missing the import of any entry point
raises; there is no CPU fallback.

Method: Hattori & Hiraki, "Accelerated and Optimized Search of Imperceptible
Color Vibration for Embedding Information into LCD images" (SIGGRAPH Asia 2022
Posters), Section 2 (pair construction in L*a*b* with L* fixed, displacement
arrays D_a = r sin(theta), D_b = r cos(theta)) and Section 3 / Table 1
(V_th / R_novib predicate).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcvib.so")

CV_OK, CV_EINVAL, CV_ECAPACITY, CV_EHIP, CV_ENOMEM, CV_ESTATE = 0, -1, -2, -3, -4, -5
CV_RGB8_TO_LAB, CV_LAB_TO_RGBF = 0, 1
CV_EMIT_ALL = 0x1
CV_PER_RAY = 0x8
CV_NO_NGAMUT = 0x10
CV_GRAPH = 0x2
CV_RULE_CLIP = 0x1
CV_TIME_EVAL, CV_TIME_WRITE, CV_TIME_CALL = 0, 1, 2

_ERRNAMES = {CV_EINVAL: "CV_EINVAL", CV_ECAPACITY: "CV_ECAPACITY", CV_EHIP: "CV_EHIP",
             CV_ENOMEM: "CV_ENOMEM", CV_ESTATE: "CV_ESTATE"}


class CvError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class cv_grid(C.Structure):
    _fields_ = [("dr", C.c_double), ("nr", C.c_int32), ("_pad0", C.c_int32),
                ("dtheta_deg", C.c_double), ("ntheta", C.c_int32), ("_pad1", C.c_int32)]


class cv_rule(C.Structure):
    _fields_ = [("v_th", C.c_int32), ("_pad0", C.c_int32), ("r_novib", C.c_double),
                ("pattern_mask", C.c_uint32), ("flags", C.c_uint32)]


PAIR_DTYPE = np.dtype([("colour", "<u4"), ("i", "<u2"), ("j", "<u2"), ("plus", "u1", 3),
                       ("minus", "u1", 3), ("pattern", "u1"), ("flags", "u1")])
SUMMARY_DTYPE = np.dtype([("count", "<u4"), ("n_gamut", "<u4"), ("best_i", "<u2"),
                          ("best_j", "<u2"), ("best_plus", "u1", 3), ("best_minus", "u1", 3),
                          ("best_p", "u1"), ("_pad", "u1"), ("per_pattern", "<u4", 7)])
TABLE_DTYPE = np.dtype([("count", "<u4"), ("bin_ridx", "u1", 36)])
PATTERN_PAIR_DTYPE = np.dtype([("i", "<u2"), ("j", "<u2"), ("plus", "u1", 3), ("minus", "u1", 3),
                               ("pattern", "u1"), ("flags", "u1")])
assert PAIR_DTYPE.itemsize == 16 and SUMMARY_DTYPE.itemsize == 48 and TABLE_DTYPE.itemsize == 40
assert PATTERN_PAIR_DTYPE.itemsize == 12

# Exported symbols (every one is declared in include/cvib.h).
EXPORTS = ("cv_context_create", "cv_context_destroy", "cv_last_error", "cv_lab_convert",
           "cv_pair_search", "cv_pair_reduce", "cv_frames_resolve", "cv_context_set_timing",
           "cv_context_kernel_time", "cv_mlp_create", "cv_mlp_destroy", "cv_mlp_num_params",
           "cv_mlp_set_params", "cv_mlp_get_params", "cv_mlp_forward", "cv_mlp_loss",
           "cv_mlp_backward", "cv_adam_step", "cv_mlp_train_steps", "cv_mlp_table_batch", "cv_mlp_save",
           "cv_mlp_load",
           "cv_surrogate_infer", "cv_frames_surrogate", "cv_context_set_autotune",
           "cv_context_set_resolve_variant", "cv_context_resolve_variant", "cv_pair_reduce_rules",
           "cv_pair_reduce_csr", "cv_context_set_gamut_cells", "cv_context_skipped",
           "cv_mlp_set_first_sine", "cv_mlp_first_sine", "cv_permute_ids", "cv_context_no_high",
           "cv_pair_reduce_noalloc", "cv_ray_search", "cv_mlp_hidden",
           "cv_mlp_save_checkpoint", "cv_mlp_load_checkpoint", "cv_mlp_checkpoint_info",
           "cv_context_set_tile_target", "cv_context_tile_target", "cv_context_set_tune_file",
           "cv_frames_generate", "cv_best_pair_search")
CV_NO_FALLBACK = 0x4
CV_PRED_GIVEN = 0x20
CV_PAIR_FOUND, CV_PAIR_SURROGATE, CV_PAIR_FALLBACK = 0x1, 0x2, 0x4
CV_RESOLVED_SURROGATE, CV_RESOLVED_EXACT, CV_RESOLVED_NONE = 0, 1, 2
CV_TIME_MLP, CV_TIME_VERIFY = 3, 4
CV_MLP_KEEP = 0x1
CV_MLP_RGB8 = 0x2
SURROGATE_DIMS = (3, 256, 256, 256, 37)
SURROGATE_OMEGA0 = 20.0   # first hidden layer sin(20 z)

_lib = None


def lib() -> C.CDLL:
    """Load libcvib.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        P, I64 = C.c_void_p, C.c_int64
        L.cv_context_create.argtypes = [C.c_int, C.POINTER(C.c_void_p)]
        L.cv_context_destroy.argtypes = [P]
        L.cv_last_error.restype = C.c_char_p
        L.cv_lab_convert.argtypes = [P, P, P, I64, C.c_int, P]
        L.cv_pair_search.argtypes = [P, P, I64, C.POINTER(cv_grid), C.POINTER(cv_rule), P, I64,
                                     P, P, C.POINTER(I64), C.c_uint32, P]
        L.cv_pair_reduce.argtypes = [P, P, I64, C.POINTER(cv_grid), C.POINTER(cv_rule), P, P, P]
        L.cv_mlp_save_checkpoint.argtypes = [P, C.c_char_p, I64, C.c_uint64]
        L.cv_mlp_load_checkpoint.argtypes = [P, C.c_char_p, C.POINTER(I64), C.POINTER(C.c_uint64)]
        L.cv_mlp_checkpoint_info.argtypes = [C.c_char_p, C.POINTER(C.c_int32), P, C.POINTER(I64),
                                             C.POINTER(C.c_uint64)]
        L.cv_mlp_hidden.argtypes = [P, C.c_int32, P, I64, P]
        L.cv_ray_search.argtypes = [P, P, I64, C.POINTER(cv_grid), C.POINTER(cv_rule), P, P, P, P, P]
        L.cv_frames_generate.argtypes = [P, P, I64, C.c_int32, C.c_int32, C.c_int32, C.c_int32, P, P]
        L.cv_best_pair_search.argtypes = [P, P, I64, C.POINTER(cv_grid), C.POINTER(cv_rule), P, P, P, P]
        L.cv_pair_reduce_noalloc.argtypes = [P, P, I64, C.POINTER(cv_grid), C.POINTER(cv_rule), P, P, P]
        L.cv_frames_resolve.argtypes = [P, P, I64, P, C.POINTER(cv_grid), C.POINTER(cv_rule), P,
                                        I64, P, P, P, P, P, P, P, P, C.c_uint32, P]
        L.cv_context_set_timing.argtypes = [P, C.c_int]
        L.cv_context_kernel_time.argtypes = [P, C.c_int, C.POINTER(C.c_double), C.POINTER(I64),
                                             C.c_int]
        L.cv_mlp_create.argtypes = [P, P, C.c_int32, C.POINTER(C.c_void_p)]
        L.cv_mlp_destroy.argtypes = [P]
        L.cv_mlp_num_params.argtypes = [P, C.POINTER(I64)]
        L.cv_mlp_set_first_sine.argtypes = [P, C.c_float]
        L.cv_mlp_first_sine.argtypes = [P, C.POINTER(C.c_float)]
        L.cv_permute_ids.argtypes = [P, P, I64, C.c_uint64, P, P]
        L.cv_mlp_set_params.argtypes = [P, P, P]
        L.cv_mlp_get_params.argtypes = [P, P, P, P]
        L.cv_mlp_forward.argtypes = [P, P, I64, P, C.c_uint32, P]
        L.cv_mlp_loss.argtypes = [P, P, P, P, I64, C.c_float, P, P, P]
        L.cv_mlp_backward.argtypes = [P, P, P, I64, P]
        L.cv_adam_step.argtypes = [P, C.c_float, C.c_float, C.c_float, C.c_float, I64, P]
        L.cv_mlp_table_batch.argtypes = [P, P, P, I64, C.c_double, P, P, P, P]
        L.cv_mlp_train_steps.argtypes = [P, P, I64, P, C.c_double, I64, C.c_float, C.c_float,
                                         C.c_float, I64, I64, P, P]
        L.cv_mlp_save.argtypes = [P, C.c_char_p]
        L.cv_mlp_load.argtypes = [P, C.c_char_p]
        L.cv_surrogate_infer.argtypes = [P, P, P, I64, C.POINTER(cv_grid), C.POINTER(cv_rule),
                                         C.c_float, C.c_int32, P, P, P, P, P, C.c_uint32, P]
        L.cv_frames_surrogate.argtypes = [P, P, P, I64, C.POINTER(cv_grid), C.POINTER(cv_rule),
                                          C.c_float, C.c_int32, P, I64, P, P, P, P, P, P, P, P,
                                          C.c_uint32, P]
        L.cv_context_set_autotune.argtypes = [P, C.c_int]
        L.cv_context_set_resolve_variant.argtypes = [P, C.c_int]
        L.cv_context_set_tile_target.argtypes = [P, C.c_int32]
        L.cv_context_tile_target.argtypes = [P, I64, C.POINTER(cv_grid), C.c_int, C.POINTER(C.c_int32),
                                             C.POINTER(C.c_int)]
        L.cv_context_set_tune_file.argtypes = [P, C.c_char_p]
        L.cv_context_resolve_variant.argtypes = [P, C.POINTER(cv_grid), C.c_int, C.POINTER(C.c_int),
                                                 C.POINTER(C.c_int)]
        L.cv_pair_reduce_rules.argtypes = [P, P, I64, C.POINTER(cv_grid), P, C.c_int32, P, P]
        L.cv_pair_reduce_csr.argtypes = [P, P, P, I64, P, P]
        L.cv_context_set_gamut_cells.argtypes = [P, C.c_int]
        L.cv_context_skipped.argtypes = [P, C.POINTER(I64), C.c_int]
        L.cv_context_no_high.argtypes = [P, C.POINTER(I64), C.c_int]
        for name in EXPORTS:
            if name != "cv_last_error":
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(rc: int) -> int:
    if rc != CV_OK:
        raise CvError(rc, lib().cv_last_error().decode())
    return rc


@dataclass(frozen=True)
class Grid:
    """r_i = (i+1) dr, i < nr; theta_j = j dtheta_deg degrees, j < ntheta."""
    dr: float
    nr: int
    dtheta_deg: float
    ntheta: int

    def c(self) -> cv_grid:
        return cv_grid(dr=self.dr, nr=self.nr, dtheta_deg=self.dtheta_deg, ntheta=self.ntheta)

    @property
    def per_colour(self) -> int:
        return self.nr * self.ntheta


@dataclass(frozen=True)
class Rule:
    """Section 3: high if change > v_th, low if change < v_th * r_novib."""
    v_th: int = 50
    r_novib: float = 0.5
    pattern_mask: int = 0x7F
    flags: int = 0

    def c(self) -> cv_rule:
        return cv_rule(v_th=self.v_th, r_novib=self.r_novib, pattern_mask=self.pattern_mask,
                       flags=self.flags)


class Context:
    """Owns a cv_context (device workspace) on one GPU."""

    def __init__(self, device: int = 0):
        h = C.c_void_p()
        _check(lib().cv_context_create(int(device), C.byref(h)))
        self.handle = h
        self.device = device

    def set_timing(self, on: bool = True):
        """Bracket the dominant search kernel with HIP events on the call's stream."""
        _check(lib().cv_context_set_timing(self.handle, int(bool(on))))

    def kernel_time(self, phase: int = 0, reset: bool = False):
        """(accumulated milliseconds, number of timed calls) of a phase:
        CV_TIME_EVAL (0), CV_TIME_WRITE (1) or CV_TIME_CALL (2)."""
        ms, n = C.c_double(0.0), C.c_int64(0)
        _check(lib().cv_context_kernel_time(self.handle, int(phase), C.byref(ms), C.byref(n),
                                            int(reset)))
        return ms.value, n.value

    def set_gamut_cells(self, on: bool = True):
        """Skip wave steps of the reduce kernels that lie in cells proven out of gamut."""
        _check(lib().cv_context_set_gamut_cells(self.handle, int(bool(on))))

    def skipped(self, reset: bool = False) -> int:
        """Candidates skipped by the gamut cells in calls made while timing was on."""
        v = C.c_int64(0)
        _check(lib().cv_context_skipped(self.handle, C.byref(v), int(bool(reset))))
        return v.value

    def no_high(self, reset: bool = False) -> int:
        """In-gamut pairs of steps proven to hold no high channel (counted,
        not encoded) in calls made while timing was on."""
        v = C.c_int64(0)
        _check(lib().cv_context_no_high(self.handle, C.byref(v), int(bool(reset))))
        return v.value

    def set_autotune(self, on: bool = True):
        """Time the per-colour resolve variants and the chunked reduce's tilings on
        the first call of each shape."""
        _check(lib().cv_context_set_autotune(self.handle, int(bool(on))))

    def set_tile_target(self, tiles: int = 0):
        """Force the chunked reduce's tiles per call (64 .. 2^20), or return to tuning (0)."""
        _check(lib().cv_context_set_tile_target(self.handle, int(tiles)))

    def tile_target(self, n: int, grid: "Grid", search: bool = True):
        """(tiles a call of this shape would use, whether they were tuned); search:
        the count pass of pair_search, else pair_reduce."""
        v, t = C.c_int32(0), C.c_int(0)
        g = grid.c()
        _check(lib().cv_context_tile_target(self.handle, int(n), C.byref(g), int(bool(search)), C.byref(v),
                                            C.byref(t)))
        return v.value, bool(t.value)

    def set_tune_file(self, path: str | None):
        """Keep the tuned choices in a file (loaded now if written for this GPU model)."""
        _check(lib().cv_context_set_tune_file(self.handle, path.encode() if path else None))

    def set_resolve_variant(self, variant: int = -1):
        """Force a per-colour resolve variant (0, 1, 2) or return to tuning (-1)."""
        _check(lib().cv_context_set_resolve_variant(self.handle, int(variant)))

    def resolve_variant(self, grid: "Grid", rays: bool = False):
        """(variant a call of this grid shape would use, whether it was tuned)."""
        v, t = C.c_int(0), C.c_int(0)
        g = grid.c()
        _check(lib().cv_context_resolve_variant(self.handle, C.byref(g), int(bool(rays)), C.byref(v),
                                                C.byref(t)))
        return v.value, bool(t.value)

    def close(self):
        if self.handle:
            lib().cv_context_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_contexts: dict[int, Context] = {}


def context(device: int | None = None) -> Context:
    dev = torch.cuda.current_device() if device is None else int(device)
    if dev not in _contexts:
        _contexts[dev] = Context(dev)
    return _contexts[dev]


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dptr(t: torch.Tensor | None):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _require(t: torch.Tensor | None, name: str, dtype: torch.dtype, numel: int,
             device: torch.device, row_bytes: int | None = None) -> None:
    """A caller's buffer the library will write: on the call's GPU, dense,
    of the expected dtype and at least `numel` elements (with row_bytes: a
    2-D uint8 tensor of rows of that many bytes)."""
    if t is None:
        return
    if not t.is_cuda or t.device != device:
        raise ValueError(f"{name} must be on {device}")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if row_bytes is not None and (t.dim() != 2 or t.shape[1] != row_bytes):
        raise ValueError(f"{name} must have shape [*, {row_bytes}]")
    if t.numel() < numel:
        raise ValueError(f"{name} holds {t.numel()} elements, the call writes {numel}")


def _colours(colors: torch.Tensor) -> torch.Tensor:
    if colors.dtype != torch.uint8 or colors.dim() != 2 or colors.shape[1] != 3:
        raise ValueError("colours must be a uint8 tensor of shape [n, 3]")
    if not colors.is_cuda:
        raise ValueError("colours must be on the GPU")
    return colors.contiguous()


def rgb8_to_lab(rgb: torch.Tensor, ctx: Context | None = None) -> torch.Tensor:
    """uint8 [n,3] sRGB -> float32 [n,3] CIE L*a*b* (D65)."""
    rgb = _colours(rgb)
    ctx = ctx or context(rgb.device.index)
    out = torch.empty((rgb.shape[0], 3), dtype=torch.float32, device=rgb.device)
    _check(lib().cv_lab_convert(ctx.handle, _dptr(rgb), _dptr(out), rgb.shape[0], CV_RGB8_TO_LAB,
                                _stream()))
    return out


def frames_generate(seeds, height: int = 2160, width: int = 3840, sites: int = 64, noise: int = 4,
                    device: int = 0, ctx: Context | None = None, out: torch.Tensor | None = None) -> torch.Tensor:
    """Synthetic sRGB8 frames on the device, uint8 [len(seeds), height, width, 3]
    (cv_frames_generate: integer recipe on Philox4x64-10 words keyed by each
    seed).  `out`, if given, must be a contiguous uint8 CUDA tensor of that
    shape."""
    sd = np.ascontiguousarray(np.asarray(list(seeds), dtype=np.uint64))
    n = int(sd.shape[0])
    shape = (n, int(height), int(width), 3)
    if out is None:
        out = torch.empty(shape, dtype=torch.uint8, device=f"cuda:{device}")
    elif (out.dtype != torch.uint8 or not out.is_cuda or not out.is_contiguous() or tuple(out.shape) != shape):
        raise ValueError(f"out must be a contiguous uint8 CUDA tensor of shape {shape}")
    ctx = ctx or context(out.device.index)
    _check(lib().cv_frames_generate(ctx.handle, sd.ctypes.data, n, int(height), int(width), int(sites),
                                    int(noise), _dptr(out), _stream()))
    return out


def lab_to_rgbf(lab: torch.Tensor, ctx: Context | None = None) -> torch.Tensor:
    """float32 [n,3] L*a*b* -> float32 [n,4]: unrounded 0..255 code values + gamut flag."""
    if lab.dtype != torch.float32 or lab.dim() != 2 or lab.shape[1] != 3 or not lab.is_cuda:
        raise ValueError("lab must be a float32 CUDA tensor of shape [n, 3]")
    lab = lab.contiguous()
    ctx = ctx or context(lab.device.index)
    out = torch.empty((lab.shape[0], 4), dtype=torch.float32, device=lab.device)
    _check(lib().cv_lab_convert(ctx.handle, _dptr(lab), _dptr(out), lab.shape[0], CV_LAB_TO_RGBF,
                                _stream()))
    return out


@dataclass
class SearchResult:
    pairs: torch.Tensor        # uint8 [total, 16] (PAIR_DTYPE records) on the GPU (sync=False: the whole buffer)
    offsets: torch.Tensor      # int64 [n + 1]
    summaries: torch.Tensor | None  # uint8 [n, 48] (SUMMARY_DTYPE)
    total: int | None          # None for sync=False: offsets[n] on the device


def pair_search(colors: torch.Tensor, grid: Grid, rule: Rule, capacity: int | None = None,
                summaries: bool = True, emit_all: bool = False, per_ray: bool = False,
                out: torch.Tensor | None = None, ctx: Context | None = None, graph: bool = False,
                offsets: torch.Tensor | None = None, summ_out: torch.Tensor | None = None,
                sync: bool = True, ngamut: bool = True) -> SearchResult:
    """Full search with stream compaction; survivors in (colour, i, j) order
    (per_ray: the largest-radius survivor of each ray, in (colour, j) order).

    With capacity None the output grows to fit (one extra search if the first
    guess is too small).  graph: capture the call once as a hipGraph and
    replay it while the arguments (pointers included: pass out, offsets and
    summ_out to reuse them) stay the same.  sync=False: nothing is read back
    (the call only enqueues work); the result's total is None, offsets[n]
    holds it on the device, and records past the capacity of `out` (which
    must then be given) are dropped.  ngamut=False: the summaries' n_gamut is
    left 0 and steps that can hold no survivor are not evaluated."""
    colors = _colours(colors)
    ctx = ctx or context(colors.device.index)
    n = colors.shape[0]
    dev = colors.device
    if offsets is None:
        offsets = torch.empty(n + 1, dtype=torch.int64, device=dev)
    _require(offsets, "offsets", torch.int64, n + 1, dev)
    summ = None
    if summaries:
        summ = summ_out if summ_out is not None else torch.empty((n, 48), dtype=torch.uint8, device=dev)
        _require(summ, "summ_out", torch.uint8, n * 48, dev)
    _require(out, "out", torch.uint8, 0, dev, row_bytes=16)
    flags = (CV_EMIT_ALL if emit_all else 0) | (CV_PER_RAY if per_ray else 0) | (CV_GRAPH if graph else 0)
    flags |= 0 if ngamut else CV_NO_NGAMUT
    if not sync:
        if out is None:
            raise ValueError("sync=False needs an output tensor")
        cap = out.shape[0] if capacity is None else min(capacity, out.shape[0])
        g, r = grid.c(), rule.c()
        _check(lib().cv_pair_search(ctx.handle, _dptr(colors), n, C.byref(g), C.byref(r), _dptr(out), cap,
                                    _dptr(offsets), _dptr(summ), None, flags, _stream()))
        return SearchResult(out, offsets, summ, None)
    if out is None:
        if capacity is None:
            full = n * grid.per_colour
            if per_ray:
                capacity = n * grid.ntheta
            else:
                capacity = full if emit_all else min(full, max(1 << 20, full // 4))
        out = torch.empty((max(capacity, 1), 16), dtype=torch.uint8, device=dev)
    cap = out.shape[0] if capacity is None else min(capacity, out.shape[0])
    total = C.c_int64(0)
    g, r = grid.c(), rule.c()
    rc = lib().cv_pair_search(ctx.handle, _dptr(colors), n, C.byref(g), C.byref(r), _dptr(out),
                              cap, _dptr(offsets), _dptr(summ), C.byref(total), flags, _stream())
    if rc == CV_ECAPACITY and capacity is None:
        out = torch.empty((total.value, 16), dtype=torch.uint8, device=dev)
        rc = lib().cv_pair_search(ctx.handle, _dptr(colors), n, C.byref(g), C.byref(r),
                                  _dptr(out), out.shape[0], _dptr(offsets), _dptr(summ),
                                  C.byref(total), flags, _stream())
    _check(rc)
    return SearchResult(out[:total.value], offsets, summ, total.value)


def pair_reduce(colors: torch.Tensor, grid: Grid, rule: Rule, summaries: bool = True,
                table: bool = False, ctx: Context | None = None):
    """Search without survivor lists: (summaries uint8 [n,48] | None, table uint8 [n,40] | None)."""
    colors = _colours(colors)
    ctx = ctx or context(colors.device.index)
    n = colors.shape[0]
    dev = colors.device
    summ = torch.empty((n, 48), dtype=torch.uint8, device=dev) if summaries else None
    tab = torch.empty((n, 40), dtype=torch.uint8, device=dev) if table else None
    g, r = grid.c(), rule.c()
    _check(lib().cv_pair_reduce(ctx.handle, _dptr(colors), n, C.byref(g), C.byref(r), _dptr(summ),
                                _dptr(tab), _stream()))
    return summ, tab


def pair_reduce_noalloc(colors: torch.Tensor, grid: Grid, rule: Rule, summ: torch.Tensor | None,
                        table: torch.Tensor | None = None, ctx: Context | None = None):
    """cv_pair_reduce_noalloc: pair_reduce into the caller's outputs (summ
    uint8 [n, 48], table uint8 [n, 40], either may be None but not both) with
    no allocation on the library's side; calls on one GPU must not overlap."""
    colors = _colours(colors)
    ctx = ctx or context(colors.device.index)
    n = colors.shape[0]
    _require(summ, "summ", torch.uint8, 48 * n, colors.device)
    _require(table, "table", torch.uint8, 40 * n, colors.device)
    g, r = grid.c(), rule.c()
    _check(lib().cv_pair_reduce_noalloc(ctx.handle, _dptr(colors), n, C.byref(g), C.byref(r),
                                        _dptr(summ), _dptr(table), _stream()))
    return summ, table


@dataclass
class RayResult:
    rays: torch.Tensor          # int16 bits of uint16 [n, ntheta]: largest valid i + 1, 0 = none
    records: torch.Tensor | None  # uint8 [n, ntheta, 16] (PAIR_DTYPE) or None
    counts: torch.Tensor        # int64 bits of uint64 [3]: evaluated, blocks tested, blocks closed
    best: torch.Tensor | None = None  # int32 bits of uint32 [n]: best key i << 16 | 0xFFFF - j, 0 = none


def ray_search(colors: torch.Tensor, grid: Grid, rule: Rule, records: bool = False, best: bool = False,
               out: RayResult | None = None, ctx: Context | None = None) -> RayResult:
    """Adaptive per-ray maxima (cv_ray_search): each ray's largest surviving
    radius index (+1), found from the outermost radius inward with blocks of
    64 radii closed by an interval bound where it can."""
    colors = _colours(colors)
    ctx = ctx or context(colors.device.index)
    n = colors.shape[0]
    dev = colors.device
    if out is None:
        out = RayResult(torch.empty((n, grid.ntheta), dtype=torch.int16, device=dev),
                        torch.empty((n, grid.ntheta, 16), dtype=torch.uint8, device=dev) if records else None,
                        torch.zeros(3, dtype=torch.int64, device=dev),
                        torch.empty(max(n, 1), dtype=torch.int32, device=dev) if best else None)
    _require(out.rays, "out.rays", torch.int16, n * grid.ntheta, dev)
    _require(out.records, "out.records", torch.uint8, n * grid.ntheta * 16, dev)
    _require(out.counts, "out.counts", torch.int64, 3, dev)
    _require(out.best, "out.best", torch.int32, n, dev)
    g, r = grid.c(), rule.c()
    _check(lib().cv_ray_search(ctx.handle, _dptr(colors), n, C.byref(g), C.byref(r), _dptr(out.rays),
                               _dptr(out.records), _dptr(out.best), _dptr(out.counts), _stream()))
    return out


@dataclass
class BestPairResult:
    best: torch.Tensor     # int32 view of uint32 [n]: i << 16 | (65535 - j), 0 = none
    pairs: torch.Tensor    # uint8 [n, 16]: cv_pair records
    counts: torch.Tensor   # int64 [3]: evaluated, blocks tested, blocks closed


def best_pair_search(colors: torch.Tensor, grid: Grid, rule: Rule, out: BestPairResult | None = None,
                     ctx: Context | None = None) -> BestPairResult:
    """Exact one-pair resolve with a global early exit (cv_best_pair_search):
    each colour's maximum-amplitude survivor, from the outermost radii inward,
    stopping at the first level of 64 radii that holds one."""
    colors = _colours(colors)
    ctx = ctx or context(colors.device.index)
    n = colors.shape[0]
    dev = colors.device
    if out is None:
        out = BestPairResult(torch.empty(max(n, 1), dtype=torch.int32, device=dev),
                             torch.empty((max(n, 1), 16), dtype=torch.uint8, device=dev),
                             torch.zeros(3, dtype=torch.int64, device=dev))
    _require(out.best, "out.best", torch.int32, n, dev)
    _require(out.pairs, "out.pairs", torch.uint8, n * 16, dev)
    _require(out.counts, "out.counts", torch.int64, 3, dev)
    g, r = grid.c(), rule.c()
    _check(lib().cv_best_pair_search(ctx.handle, _dptr(colors), n, C.byref(g), C.byref(r), _dptr(out.best),
                                     _dptr(out.pairs), _dptr(out.counts), _stream()))
    return out


def pair_reduce_csr(records: torch.Tensor, offsets: torch.Tensor, ctx: Context | None = None) -> torch.Tensor:
    """Per-colour summaries (uint8 [n, 48]) of a survivor list (uint8 [total, 16])
    with its CSR offsets (int64 [n + 1]); n_gamut is 0."""
    if not records.is_cuda or not offsets.is_cuda or offsets.dtype != torch.int64:
        raise ValueError("records and offsets must be CUDA tensors, offsets int64")
    ctx = ctx or context(offsets.device.index)
    n = offsets.numel() - 1
    summ = torch.empty((n, 48), dtype=torch.uint8, device=offsets.device)
    recs = records.contiguous() if records.numel() else torch.empty((1, 16), dtype=torch.uint8, device=offsets.device)
    _check(lib().cv_pair_reduce_csr(ctx.handle, _dptr(recs), _dptr(offsets.contiguous()), n, _dptr(summ),
                                    _stream()))
    return summ


def pair_reduce_rules(colors: torch.Tensor, grid: Grid, rules, ctx: Context | None = None) -> torch.Tensor:
    """Survivor counts of every pattern under every rule in one pass:
    int32 view of uint32 [n, len(rules), 7] (rules: Rule objects sharing one
    gamut reading)."""
    colors = _colours(colors)
    ctx = ctx or context(colors.device.index)
    n = colors.shape[0]
    arr = (cv_rule * len(rules))(*[r.c() for r in rules])
    counts = torch.empty((n, len(rules), 7), dtype=torch.int32, device=colors.device)
    g = grid.c()
    _check(lib().cv_pair_reduce_rules(ctx.handle, _dptr(colors), n, C.byref(g), C.cast(arr, C.c_void_p),
                                      len(rules), _dptr(counts), _stream()))
    return counts


def as_records(t: torch.Tensor, dtype: np.dtype) -> np.ndarray:
    """Copy a uint8 [k, itemsize] device tensor into a numpy structured array."""
    a = t.detach().cpu().contiguous().numpy()
    return a.reshape(-1).view(dtype) if a.size else np.zeros(0, dtype=dtype)


@dataclass
class FramesResult:
    colours: torch.Tensor       # uint8 [colour_cap, 3]; the first ncolours are valid
    ncolours: torch.Tensor      # int64 [1] on the GPU
    pixel_index: torch.Tensor   # uint32 (as int32) [npix]
    summaries: torch.Tensor | None   # uint8 [colour_cap, 48]
    pbest: torch.Tensor         # uint8 [colour_cap, 7, 12] (PATTERN_PAIR_DTYPE)
    rays: torch.Tensor | None   # int16 bits of uint16 [colour_cap, ntheta]
    frame_a: torch.Tensor | None
    frame_b: torch.Tensor | None
    resolved: torch.Tensor | None   # int64 [1] on the GPU


def frames_resolve(pixels: torch.Tensor, grid: Grid, rule: Rule, info: torch.Tensor | None = None,
                   summaries: bool = True, rays: bool = False, frames: bool = True,
                   graph: bool = False, out: FramesResult | None = None,
                   ctx: Context | None = None, ngamut: bool = True) -> FramesResult:
    """De-duplicate the colours of `pixels` (uint8 [..., 3] on the GPU), search
    every distinct colour, and render the two alternating frames.  Pass the
    previous result as `out` to reuse its buffers (needed for graph replays).
    ngamut=False: the summaries' n_gamut is left 0 (CV_NO_NGAMUT)."""
    if pixels.dtype != torch.uint8 or pixels.shape[-1] != 3 or not pixels.is_cuda:
        raise ValueError("pixels must be a uint8 CUDA tensor of shape [..., 3]")
    px = pixels.contiguous().reshape(-1, 3)
    npix = px.shape[0]
    ctx = ctx or context(px.device.index)
    dev = px.device
    if info is not None:
        if info.dtype != torch.uint8 or info.numel() != npix or not info.is_cuda:
            raise ValueError("info must be a uint8 CUDA tensor with one entry per pixel")
        info = info.contiguous().reshape(-1)
    cap = min(npix, 1 << 24)
    if out is not None:
        c = out.colours.shape[0] if out.colours.dim() == 2 else -1
        if c < 1:
            raise ValueError("out.colours must have shape [colour_cap, 3]")
        _require(out.colours, "out.colours", torch.uint8, 3 * c, dev)
        _require(out.ncolours, "out.ncolours", torch.int64, 1, dev)
        _require(out.pixel_index, "out.pixel_index", torch.int32, npix, dev)
        _require(out.summaries, "out.summaries", torch.uint8, 48 * c, dev)
        _require(out.pbest, "out.pbest", torch.uint8, 84 * c, dev)
        _require(out.rays, "out.rays", torch.int16, grid.ntheta * c, dev)
        _require(out.frame_a, "out.frame_a", torch.uint8, 3 * npix, dev)
        _require(out.frame_b, "out.frame_b", torch.uint8, 3 * npix, dev)
        _require(out.resolved, "out.resolved", torch.int64, 1, dev)
    if out is None:
        out = FramesResult(
            colours=torch.empty((cap, 3), dtype=torch.uint8, device=dev),
            ncolours=torch.zeros(1, dtype=torch.int64, device=dev),
            pixel_index=torch.empty(npix, dtype=torch.int32, device=dev),
            summaries=torch.empty((cap, 48), dtype=torch.uint8, device=dev) if summaries else None,
            pbest=torch.empty((cap, 7, 12), dtype=torch.uint8, device=dev),
            rays=torch.empty((cap, grid.ntheta), dtype=torch.int16, device=dev) if rays else None,
            frame_a=torch.empty((npix, 3), dtype=torch.uint8, device=dev) if frames else None,
            frame_b=torch.empty((npix, 3), dtype=torch.uint8, device=dev) if frames else None,
            resolved=torch.zeros(1, dtype=torch.int64, device=dev) if frames else None)
    g, r = grid.c(), rule.c()
    _check(lib().cv_frames_resolve(ctx.handle, _dptr(px), npix, _dptr(info), C.byref(g),
                                   C.byref(r), _dptr(out.colours), out.colours.shape[0],
                                   _dptr(out.ncolours), _dptr(out.pixel_index),
                                   _dptr(out.summaries), _dptr(out.pbest), _dptr(out.rays),
                                   _dptr(out.frame_a), _dptr(out.frame_b), _dptr(out.resolved),
                                   (CV_GRAPH if graph else 0) | (0 if ngamut else CV_NO_NGAMUT), _stream()))
    return out


# --------------------------------------------------------------------------
# Surrogate network


def init_params(dims, seed: int, first_sine: bool = False) -> np.ndarray:
    """He-normal weights (std sqrt(2 / fan_in)) and zero biases, flat FP32 in
    the library's layout (per layer W_l [d_{l+1}][d_l], then b_l), drawn from a
    Philox stream keyed by `seed`.  With first_sine the first layer (a
    sinusoidal one) starts uniform instead: W_0 in [-1/d_0, 1/d_0] and b_0 in
    [-1/sqrt(d_0), 1/sqrt(d_0)], which spreads the phases omega0 z over
    several periods across the input cube (the SIREN first-layer scheme of
    Sitzmann et al. 2020)."""
    rng = np.random.Generator(np.random.Philox(key=seed))
    parts = []
    for l in range(len(dims) - 1):
        if l == 0 and first_sine:
            parts.append(rng.uniform(-1.0 / dims[0], 1.0 / dims[0], (dims[1], dims[0])).ravel())
            parts.append(rng.uniform(-dims[0] ** -0.5, dims[0] ** -0.5, dims[1]))
            continue
        parts.append(rng.normal(0.0, np.sqrt(2.0 / dims[l]), (dims[l + 1], dims[l])).ravel())
        parts.append(np.zeros(dims[l + 1]))
    return np.concatenate(parts).astype(np.float32)


def split_params(flat, dims):
    """Flat parameters -> ([W_l], [b_l]) views."""
    flat = np.asarray(flat)
    Ws, bs, o = [], [], 0
    for l in range(len(dims) - 1):
        n = dims[l + 1] * dims[l]
        Ws.append(flat[o:o + n].reshape(dims[l + 1], dims[l]))
        o += n
        bs.append(flat[o:o + dims[l + 1]])
        o += dims[l + 1]
    return Ws, bs


class MLP:
    """A cv_mlp: FP32 master weights, gradients and Adam moments on one GPU."""

    def __init__(self, dims=SURROGATE_DIMS, ctx: Context | None = None):
        self.ctx = ctx or context()
        self.dims = tuple(int(d) for d in dims)
        d = (C.c_int32 * len(self.dims))(*self.dims)
        h = C.c_void_p()
        _check(lib().cv_mlp_create(self.ctx.handle, d, len(self.dims) - 1, C.byref(h)))
        self.handle = h
        n = C.c_int64(0)
        _check(lib().cv_mlp_num_params(h, C.byref(n)))
        self.nparams = n.value
        self.device = torch.device("cuda", self.ctx.device)

    def set_first_sine(self, omega0: float):
        """First hidden layer sin(omega0 z) (omega0 > 0) or ReLU (omega0 = 0)."""
        _check(lib().cv_mlp_set_first_sine(self.handle, float(omega0)))

    @property
    def omega0(self) -> float:
        v = C.c_float(0.0)
        _check(lib().cv_mlp_first_sine(self.handle, C.byref(v)))
        return v.value

    def set_params(self, flat):
        t = torch.as_tensor(np.asarray(flat, dtype=np.float32) if not torch.is_tensor(flat) else flat)
        t = t.to(self.device, torch.float32).contiguous()
        if t.numel() != self.nparams:
            raise ValueError(f"expected {self.nparams} parameters, got {t.numel()}")
        _check(lib().cv_mlp_set_params(self.handle, _dptr(t), _stream()))
        torch.cuda.current_stream().synchronize()

    def params(self) -> torch.Tensor:
        t = torch.empty(self.nparams, dtype=torch.float32, device=self.device)
        _check(lib().cv_mlp_get_params(self.handle, _dptr(t), None, _stream()))
        return t

    def grads(self) -> torch.Tensor:
        t = torch.empty(self.nparams, dtype=torch.float32, device=self.device)
        _check(lib().cv_mlp_get_params(self.handle, None, _dptr(t), _stream()))
        return t

    def forward(self, x: torch.Tensor, keep: bool = False, out: torch.Tensor | None = None):
        """x: float32 [B, 3] or uint8 RGB [B, 3] on the GPU -> float32 [B, dims[-1]]."""
        if not x.is_cuda or x.dim() != 2 or x.shape[1] != 3 or x.dtype not in (torch.float32, torch.uint8):
            raise ValueError("x must be a float32 or uint8 CUDA tensor of shape [B, 3]")
        x = x.contiguous()
        B = x.shape[0]
        if out is None:
            out = torch.empty((B, self.dims[-1]), dtype=torch.float32, device=self.device)
        flags = (CV_MLP_KEEP if keep else 0) | (CV_MLP_RGB8 if x.dtype == torch.uint8 else 0)
        _check(lib().cv_mlp_forward(self.handle, _dptr(x), B, _dptr(out), flags, _stream()))
        return out

    def loss(self, out, t_r, t_f, delta: float, want_grad: bool = True):
        B = out.shape[0]
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        gout = torch.empty_like(out) if want_grad else None
        _check(lib().cv_mlp_loss(self.handle, _dptr(out.contiguous()), _dptr(t_r.contiguous()),
                                 _dptr(t_f.contiguous()), B, float(delta), _dptr(loss), _dptr(gout),
                                 _stream()))
        return loss, gout

    def hidden(self, layer: int, B: int) -> torch.Tensor:
        """FP32 copy of hidden layer `layer`'s BF16 activations [B, d_layer]
        from the last kept forward pass."""
        out = torch.empty((B, self.dims[layer]), dtype=torch.float32, device=self.device)
        _check(lib().cv_mlp_hidden(self.handle, int(layer), _dptr(out), int(B), _stream()))
        return out

    def backward(self, x, gout):
        _check(lib().cv_mlp_backward(self.handle, _dptr(x.contiguous()), _dptr(gout.contiguous()),
                                     x.shape[0], _stream()))

    def adam_step(self, lr: float, t: int, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        _check(lib().cv_adam_step(self.handle, lr, beta1, beta2, eps, int(t), _stream()))

    def table_batch(self, ids: torch.Tensor, table: torch.Tensor, dr: float):
        """Training rows for colour ids (int32 [B]) from a whole-cube table
        (uint8 [2^24, 40]): (x [B, 3], t_r [B, 36], t_f [B])."""
        if table.shape[0] != 1 << 24 or ids.dtype != torch.int32:
            raise ValueError("table must hold all 2^24 rows and ids must be int32")
        B = ids.shape[0]
        x = torch.empty((B, 3), dtype=torch.float32, device=self.device)
        tr = torch.empty((B, 36), dtype=torch.float32, device=self.device)
        tf = torch.empty(B, dtype=torch.float32, device=self.device)
        _check(lib().cv_mlp_table_batch(self.handle, _dptr(ids.contiguous()), _dptr(table), B,
                                        float(dr), _dptr(x), _dptr(tr), _dptr(tf), _stream()))
        return x, tr, tf

    def train_steps(self, ids: torch.Tensor, table: torch.Tensor, dr: float, batch: int,
                    delta: float, lr_max: float, lr_min: float, step0: int, total_steps: int,
                    log: bool = True):
        """Steps over ids (int32, shuffled) in batches; returns the per-step
        losses (float32 tensor on the GPU) when log is set."""
        if table.shape[0] != 1 << 24 or ids.dtype != torch.int32 or not ids.is_cuda:
            raise ValueError("table must hold all 2^24 rows and ids must be int32 on the GPU")
        n = ids.shape[0]
        steps = -(-n // batch)
        losses = torch.empty(steps, dtype=torch.float32, device=self.device) if log else None
        _check(lib().cv_mlp_train_steps(self.handle, _dptr(ids.contiguous()), n, _dptr(table), float(dr),
                                        int(batch), float(delta), float(lr_max), float(lr_min),
                                        int(step0), int(total_steps), _dptr(losses), _stream()))
        return losses

    def save(self, path: str):
        _check(lib().cv_mlp_save(self.handle, os.fsencode(path)))

    def load(self, path: str):
        _check(lib().cv_mlp_load(self.handle, os.fsencode(path)))

    def save_checkpoint(self, path: str, step: int, key: int = 0):
        """Parameters, Adam moments, the step count and a training-order key."""
        _check(lib().cv_mlp_save_checkpoint(self.handle, os.fsencode(path), int(step), int(key) & (2 ** 64 - 1)))

    def load_checkpoint(self, path: str):
        """Restore a checkpoint of this network's shape: returns (step, key)."""
        st, k = C.c_int64(0), C.c_uint64(0)
        _check(lib().cv_mlp_load_checkpoint(self.handle, os.fsencode(path), C.byref(st), C.byref(k)))
        return st.value, k.value

    def close(self):
        if getattr(self, "handle", None):
            lib().cv_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def checkpoint_info(path: str):
    """Read and check a training checkpoint without a GPU: (dims, step, key);
    raises CvError (CV_EINVAL) for a corrupt, truncated or foreign file."""
    nl = C.c_int32(0)
    dims = (C.c_int32 * 9)()
    st, k = C.c_int64(0), C.c_uint64(0)
    _check(lib().cv_mlp_checkpoint_info(os.fsencode(path), C.byref(nl), dims, C.byref(st), C.byref(k)))
    return tuple(dims[: nl.value + 1]), st.value, k.value


def permute_ids(ids: torch.Tensor, key: int, out: torch.Tensor | None = None,
                ctx: Context | None = None) -> torch.Tensor:
    """ids (int32 on the GPU) in a keyed pseudorandom order (cv_permute_ids)."""
    ctx = ctx or context()
    if not ids.is_cuda or ids.dtype != torch.int32 or ids.dim() != 1:
        raise ValueError("ids must be a 1-D int32 CUDA tensor")
    ids = ids.contiguous()
    if out is None:
        out = torch.empty_like(ids)
    _check(lib().cv_permute_ids(ctx.handle, _dptr(ids), ids.shape[0], int(key) & (2 ** 64 - 1), _dptr(out),
                                _stream()))
    return out


def surrogate_network(seed: int = 0, ctx: Context | None = None) -> MLP:
    """The untrained surrogate network: 3 -> 256 -> 256 -> 256 -> 37 with a
    sinusoidal first layer (omega0 = 20), initialised from `seed`."""
    m = MLP(SURROGATE_DIMS, ctx)
    m.set_first_sine(SURROGATE_OMEGA0)
    m.set_params(init_params(SURROGATE_DIMS, seed, first_sine=True))
    return m


# --------------------------------------------------------------------------
# Surrogate resolve


@dataclass
class SurrogateResult:
    pairs: torch.Tensor        # uint8 [n, 12] (PATTERN_PAIR_DTYPE)
    status: torch.Tensor       # uint8 [n]: CV_RESOLVED_*
    nfallback: torch.Tensor    # int64 [1] on the GPU
    pred: torch.Tensor | None  # float32 [n, 37]
    fallback: torch.Tensor | None = None  # int32 bits of uint32 [n]: the first nfallback entries


def surrogate_infer(colors: torch.Tensor, mlp: MLP | None, grid: Grid, rule: Rule, tau: float = 0.0,
                    kbins: int = 3, fallback: bool = True, want_pred: bool = False,
                    want_list: bool = False, pred_in: torch.Tensor | None = None,
                    out: SurrogateResult | None = None, ctx: Context | None = None) -> SurrogateResult:
    """One verified pair per colour (uint8 [n, 3] on the GPU).  pred_in:
    proposals in the network's output layout (float32 [n, 37]) used instead of
    running the network (CV_PRED_GIVEN; mlp may then be None).  out: a
    previous result of the same n whose buffers are reused."""
    colors = _colours(colors)
    if mlp is None and pred_in is None:
        raise ValueError("a network or pred_in is needed")
    ctx = ctx or (mlp.ctx if mlp is not None else context(colors.device.index))
    n = colors.shape[0]
    dev = colors.device
    if pred_in is not None:
        _require(pred_in, "pred_in", torch.float32, 37 * n, dev)
    if out is None:
        out = SurrogateResult(torch.empty((n, 12), dtype=torch.uint8, device=dev),
                              torch.empty(n, dtype=torch.uint8, device=dev),
                              torch.zeros(1, dtype=torch.int64, device=dev),
                              torch.empty((n, 37), dtype=torch.float32, device=dev) if want_pred else None,
                              torch.empty(max(n, 1), dtype=torch.int32, device=dev) if want_list else None)
    _require(out.pairs, "out.pairs", torch.uint8, 12 * n, dev)
    _require(out.status, "out.status", torch.uint8, n, dev)
    _require(out.nfallback, "out.nfallback", torch.int64, 1, dev)
    _require(out.pred, "out.pred", torch.float32, 37 * n, dev)
    _require(out.fallback, "out.fallback", torch.int32, n, dev)
    pred = pred_in if pred_in is not None else out.pred
    flags = (0 if fallback else CV_NO_FALLBACK) | (CV_PRED_GIVEN if pred_in is not None else 0)
    g, r = grid.c(), rule.c()
    _check(lib().cv_surrogate_infer(ctx.handle, mlp.handle if mlp is not None else None, _dptr(colors), n,
                                    C.byref(g), C.byref(r), float(tau), int(kbins), _dptr(pred),
                                    _dptr(out.pairs), _dptr(out.status), _dptr(out.fallback),
                                    _dptr(out.nfallback), flags, _stream()))
    return out


@dataclass
class FramesSurrogateResult:
    colours: torch.Tensor
    ncolours: torch.Tensor
    pixel_index: torch.Tensor
    pairs: torch.Tensor
    status: torch.Tensor
    frame_a: torch.Tensor | None
    frame_b: torch.Tensor | None
    resolved: torch.Tensor | None
    nfallback: torch.Tensor


def frames_surrogate(pixels: torch.Tensor, mlp: MLP, grid: Grid, rule: Rule, tau: float = 0.0,
                     kbins: int = 3, fallback: bool = True, frames: bool = True,
                     out: FramesSurrogateResult | None = None,
                     ctx: Context | None = None) -> FramesSurrogateResult:
    """De-duplicate the colours of `pixels` (uint8 [..., 3]), resolve each
    through the surrogate (verified) with the exact search as fallback, and
    render the two frames."""
    if pixels.dtype != torch.uint8 or pixels.shape[-1] != 3 or not pixels.is_cuda:
        raise ValueError("pixels must be a uint8 CUDA tensor of shape [..., 3]")
    px = pixels.contiguous().reshape(-1, 3)
    npix = px.shape[0]
    ctx = ctx or mlp.ctx
    dev = px.device
    cap = min(npix, 1 << 24)
    if out is not None:
        c = out.colours.shape[0] if out.colours.dim() == 2 else -1
        if c < 1:
            raise ValueError("out.colours must have shape [colour_cap, 3]")
        _require(out.colours, "out.colours", torch.uint8, 3 * c, dev)
        _require(out.ncolours, "out.ncolours", torch.int64, 1, dev)
        _require(out.pixel_index, "out.pixel_index", torch.int32, npix, dev)
        _require(out.pairs, "out.pairs", torch.uint8, 12 * c, dev)
        _require(out.status, "out.status", torch.uint8, c, dev)
        _require(out.frame_a, "out.frame_a", torch.uint8, 3 * npix, dev)
        _require(out.frame_b, "out.frame_b", torch.uint8, 3 * npix, dev)
        _require(out.resolved, "out.resolved", torch.int64, 1, dev)
        _require(out.nfallback, "out.nfallback", torch.int64, 1, dev)
    if out is None:
        out = FramesSurrogateResult(
            colours=torch.empty((cap, 3), dtype=torch.uint8, device=dev),
            ncolours=torch.zeros(1, dtype=torch.int64, device=dev),
            pixel_index=torch.empty(npix, dtype=torch.int32, device=dev),
            pairs=torch.empty((cap, 12), dtype=torch.uint8, device=dev),
            status=torch.empty(cap, dtype=torch.uint8, device=dev),
            frame_a=torch.empty((npix, 3), dtype=torch.uint8, device=dev) if frames else None,
            frame_b=torch.empty((npix, 3), dtype=torch.uint8, device=dev) if frames else None,
            resolved=torch.zeros(1, dtype=torch.int64, device=dev) if frames else None,
            nfallback=torch.zeros(1, dtype=torch.int64, device=dev))
    g, r = grid.c(), rule.c()
    _check(lib().cv_frames_surrogate(ctx.handle, mlp.handle, _dptr(px), npix, C.byref(g), C.byref(r),
                                     float(tau), int(kbins), _dptr(out.colours), out.colours.shape[0],
                                     _dptr(out.ncolours), _dptr(out.pixel_index), _dptr(out.pairs),
                                     _dptr(out.status), _dptr(out.frame_a), _dptr(out.frame_b),
                                     _dptr(out.resolved), _dptr(out.nfallback),
                                     0 if fallback else CV_NO_FALLBACK, _stream()))
    return out
