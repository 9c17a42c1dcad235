"""Thin Python binding of libsoft.so (C-ABI in include/soft.h).

Argument marshalling only: every step of the transforms runs in the HIP
library.  Tensors are torch complex CUDA (HIP) tensors (complex128 for
SOFT_FP64, complex64 for SOFT_FP32 and SOFT_FP32_SPLIT); the binding passes
their device pointers and the current torch stream.  Loading fails loudly if
the library has not been built (``python -m paper_1808_00896_amd.build``);
there is no fallback.

The module-level functions mirror the C entry points one to one
(``soft_plan``, ``soft_forward``, ...); ``Plan`` (one bandwidth) and
``UnevenPlan`` (mixed bandwidths) wrap a plan handle with shape checks and
output allocation.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsoft.so")

SOFT_FP64 = 0
SOFT_FP32 = 1
SOFT_FP32_SPLIT = 2
PRECISIONS = {"fp64": SOFT_FP64, "fp32": SOFT_FP32, "fp32_split": SOFT_FP32_SPLIT}
SOFT_PLAN_TUNE = 1
SOFT_INPLACE_OK = 2
SOFT_PLAN_GRAPH = 4
SOFT_BETA_HALVES = 8
SOFT_DD_RECURRENCE = 16
SOFT_OK = 0
SOFT_ERR_INVALID = -1
SOFT_ERR_UNSUPPORTED = -2
SOFT_ERR_OOM = -3
SOFT_ERR_HIP = -4

_lib = None


class SoftError(RuntimeError):
    def __init__(self, status, what):
        super().__init__(f"{what}: {status_string(status)} ({status})")
        self.status = status


def lib():
    """Load libsoft.so (raises if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1808_00896_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, sz = ctypes.c_void_p, ctypes.c_size_t
        L.soft_plan.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint, ctypes.POINTER(vp)]
        L.soft_plan_uneven.argtypes = [ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.c_int, ctypes.c_uint,
                                       ctypes.POINTER(vp)]
        L.soft_plan_sizes.argtypes = [vp, ctypes.POINTER(sz), ctypes.POINTER(sz), ctypes.POINTER(sz)]
        L.soft_plan_check.argtypes = [ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.c_int, ctypes.c_uint]
        L.soft_plan_check.restype = ctypes.c_int
        L.soft_plan_offsets.argtypes = [vp, ctypes.POINTER(sz), ctypes.POINTER(sz)]
        L.soft_plan_describe.argtypes = [vp, ctypes.c_char_p, sz]
        L.soft_plan_set_dwt_shape.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        for name in ("soft_forward", "soft_inverse", "soft_adjoint", "soft_adjoint_inverse"):
            getattr(L, name).argtypes = [vp, vp, vp, vp]
        L.soft_plan_destroy.argtypes = [vp]
        L.soft_plan_set_timing.argtypes = [vp, ctypes.c_int]
        L.soft_plan_set_timing_stages.argtypes = [vp, ctypes.c_uint]
        L.soft_plan_stage_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                            ctypes.POINTER(ctypes.c_longlong), ctypes.c_int]
        L.soft_match_plan.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint, ctypes.POINTER(vp)]
        L.soft_match_sizes.argtypes = [vp, ctypes.POINTER(sz), ctypes.POINTER(sz), ctypes.POINTER(sz)]
        L.soft_match_plan_soft.argtypes = [vp, ctypes.POINTER(vp)]
        L.soft_match_coeffs.argtypes = [vp, vp, vp, vp, vp]
        L.soft_match_coeffs_vjp.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.soft_match_argmax.argtypes = [vp, vp, vp, vp]
        L.soft_match_argmax_noalloc.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp, vp]
        L.soft_match.argtypes = [vp, vp, vp, vp, vp, vp]
        L.soft_sh_forward.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp, vp]
        L.soft_sh_forward.restype = ctypes.c_int
        L.soft_match_refine.argtypes = [vp, vp, vp, vp, vp]
        L.soft_match_refine.restype = ctypes.c_int
        L.soft_match_polish.argtypes = [vp, vp, vp, ctypes.c_int, vp, vp, vp]
        L.soft_match_polish.restype = ctypes.c_int
        L.soft_match_destroy.argtypes = [vp]
        for name in ("soft_match_plan", "soft_match_sizes", "soft_match_plan_soft", "soft_match_coeffs",
                     "soft_match_coeffs_vjp", "soft_match_argmax", "soft_match_argmax_noalloc", "soft_match",
                     "soft_match_destroy"):
            getattr(L, name).restype = ctypes.c_int
        L.soft_probe_copy.argtypes = [vp, vp, sz, vp]
        L.soft_probe_copy.restype = ctypes.c_int
        L.soft_probe_flops.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp]
        L.soft_probe_flops.restype = ctypes.c_int
        L.soft_probe_flop_count.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.soft_probe_flop_count.restype = ctypes.c_double
        L.soft_status_string.argtypes = [ctypes.c_int]
        L.soft_status_string.restype = ctypes.c_char_p
        for name in ("soft_plan", "soft_plan_uneven", "soft_plan_sizes", "soft_plan_offsets", "soft_plan_describe", "soft_plan_set_dwt_shape", "soft_forward", "soft_inverse", "soft_adjoint",
                     "soft_adjoint_inverse", "soft_plan_destroy", "soft_plan_set_timing", "soft_plan_set_timing_stages",
                     "soft_plan_stage_times"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def status_string(status):
    return lib().soft_status_string(int(status)).decode()


def _check(rc, what):
    if rc != SOFT_OK:
        raise SoftError(rc, what)


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


# ---------------------------------------------------------------------------
# One-to-one wrappers of the C entry points
# ---------------------------------------------------------------------------

def soft_plan(B, batch=1, precision=SOFT_FP64, flags=0):
    """Create a plan on the current device; returns the opaque handle (int)."""
    h = ctypes.c_void_p()
    _check(lib().soft_plan(int(B), int(batch), int(precision), int(flags), ctypes.byref(h)), "soft_plan")
    return h.value


def soft_plan_uneven(B_list, precision=SOFT_FP64, flags=0):
    """Create a plan over functions of the bandwidths in ``B_list`` (in storage order)."""
    Bs = [int(b) for b in B_list]
    arr = (ctypes.c_int * max(1, len(Bs)))(*Bs)
    h = ctypes.c_void_p()
    _check(lib().soft_plan_uneven(arr, len(Bs), int(precision), int(flags), ctypes.byref(h)), "soft_plan_uneven")
    return h.value


def soft_plan_check(B_list, precision=SOFT_FP64, flags=0):
    """Build and check a plan's host side for the bandwidths B_list without a
    device; returns the status code (SOFT_OK when every check holds)."""
    Bs = [int(b) for b in B_list]
    arr = (ctypes.c_int * max(1, len(Bs)))(*Bs)
    return lib().soft_plan_check(arr, len(Bs), int(precision), int(flags))


def soft_plan_offsets(plan, n):
    """(grid_offsets, coeff_offsets), each a list of n+1 element offsets."""
    g = (ctypes.c_size_t * (n + 1))()
    c = (ctypes.c_size_t * (n + 1))()
    _check(lib().soft_plan_offsets(ctypes.c_void_p(plan), g, c), "soft_plan_offsets")
    return list(g), list(c)


def soft_plan_describe(plan):
    """The plan's JSON self-description, parsed."""
    import json
    buf = ctypes.create_string_buffer(1 << 16)
    _check(lib().soft_plan_describe(ctypes.c_void_p(plan), buf, len(buf)), "soft_plan_describe")
    return json.loads(buf.value.decode())


DWT_SHAPES = ((1, 1), (2, 1), (4, 1), (8, 1), (1, 2), (2, 2), (4, 2), (8, 2), (16, 1), (4, 4), (8, 4))
CLENSHAW = (0, 0)  # inverse-DWT "shape" of the Clenshaw kernel (soft_plan_set_dwt_shape)


def soft_plan_set_dwt_shape(plan, launch, direction, waves, subsets):
    _check(lib().soft_plan_set_dwt_shape(ctypes.c_void_p(plan), int(launch), int(direction), int(waves),
                                         int(subsets)), "soft_plan_set_dwt_shape")


def soft_plan_sizes(plan):
    """(grid_elems, coeff_elems, workspace_bytes) of a plan."""
    g, c, w = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib().soft_plan_sizes(ctypes.c_void_p(plan), ctypes.byref(g), ctypes.byref(c), ctypes.byref(w)),
           "soft_plan_sizes")
    return g.value, c.value, w.value


def _ptr(t):
    return ctypes.c_void_p(None if t is None else t.data_ptr())


def soft_forward(plan, grid, coeffs, stream=None):
    _check(lib().soft_forward(ctypes.c_void_p(plan), _ptr(grid), _ptr(coeffs), _stream(stream)), "soft_forward")


def soft_inverse(plan, coeffs, grid, stream=None):
    _check(lib().soft_inverse(ctypes.c_void_p(plan), _ptr(coeffs), _ptr(grid), _stream(stream)), "soft_inverse")


def soft_adjoint(plan, coeffs, grid, stream=None):
    _check(lib().soft_adjoint(ctypes.c_void_p(plan), _ptr(coeffs), _ptr(grid), _stream(stream)), "soft_adjoint")


def soft_adjoint_inverse(plan, grid, coeffs, stream=None):
    _check(lib().soft_adjoint_inverse(ctypes.c_void_p(plan), _ptr(grid), _ptr(coeffs), _stream(stream)),
           "soft_adjoint_inverse")


STAGES = ("fft_gamma_fwd", "fft_alpha_fwd", "dwt_fwd", "dwt_inv", "fft_alpha_inv", "fft_gamma_inv",
          "match_coeffs", "argmax")


def soft_plan_set_timing(plan, enable):
    _check(lib().soft_plan_set_timing(ctypes.c_void_p(plan), int(bool(enable))), "soft_plan_set_timing")


def soft_plan_set_timing_stages(plan, stages):
    """Time only the named stages (names of STAGES) in later calls."""
    mask = 0
    for st in stages:
        mask |= 1 << STAGES.index(st)
    _check(lib().soft_plan_set_timing_stages(ctypes.c_void_p(plan), mask), "soft_plan_set_timing_stages")


def soft_plan_stage_times(plan, reset=False):
    """{stage name: (total ms, launches)} of the HIP-event stage timers."""
    ms = (ctypes.c_double * len(STAGES))()
    n = (ctypes.c_longlong * len(STAGES))()
    _check(lib().soft_plan_stage_times(ctypes.c_void_p(plan), ms, n, int(bool(reset))), "soft_plan_stage_times")
    return {name: (ms[i], n[i]) for i, name in enumerate(STAGES)}


def soft_plan_destroy(plan):
    _check(lib().soft_plan_destroy(ctypes.c_void_p(plan)), "soft_plan_destroy")


def soft_match_plan(B, n, precision=SOFT_FP64, flags=0):
    h = ctypes.c_void_p()
    _check(lib().soft_match_plan(int(B), int(n), int(precision), int(flags), ctypes.byref(h)), "soft_match_plan")
    return h.value


def soft_match_sizes(match):
    """(sh_elems, coeff_elems, grid_elems) of one call."""
    a, c, g = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib().soft_match_sizes(ctypes.c_void_p(match), ctypes.byref(a), ctypes.byref(c), ctypes.byref(g)),
           "soft_match_sizes")
    return a.value, c.value, g.value


def soft_match_plan_soft(match):
    h = ctypes.c_void_p()
    _check(lib().soft_match_plan_soft(ctypes.c_void_p(match), ctypes.byref(h)), "soft_match_plan_soft")
    return h.value


def soft_match_coeffs(match, a, b, coeffs, stream=None):
    _check(lib().soft_match_coeffs(ctypes.c_void_p(match), _ptr(a), _ptr(b), _ptr(coeffs), _stream(stream)),
           "soft_match_coeffs")


def soft_match_coeffs_vjp(match, a, b, g, ga, gb, stream=None):
    _check(lib().soft_match_coeffs_vjp(ctypes.c_void_p(match), _ptr(a), _ptr(b), _ptr(g), _ptr(ga), _ptr(gb),
                                       _stream(stream)), "soft_match_coeffs_vjp")


def soft_match_argmax(match, grid, index, stream=None):
    _check(lib().soft_match_argmax(ctypes.c_void_p(match), _ptr(grid), _ptr(index), _stream(stream)),
           "soft_match_argmax")


def soft_match_argmax_noalloc(B, n, precision, grid, index, stream=None):
    """Argmax of Re over n grids of bandwidth B without a head (no allocation)."""
    _check(lib().soft_match_argmax_noalloc(int(B), int(n), int(precision), _ptr(grid), _ptr(index),
                                           _stream(stream)), "soft_match_argmax_noalloc")


PROBE_FMA64, PROBE_MFMA64, PROBE_MFMA32 = 0, 1, 2


def soft_probe_copy(src, dst, stream=None):
    """Streaming copy of src into dst (device tensors of equal byte size)."""
    nbytes = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() == nbytes
    _check(lib().soft_probe_copy(_ptr(src), _ptr(dst), nbytes, _stream(stream)), "soft_probe_copy")


def soft_probe_flops(kind, blocks, iters, sink, stream=None):
    """Arithmetic loop of `kind` (PROBE_*) on `blocks` blocks; returns its flop count."""
    _check(lib().soft_probe_flops(int(kind), int(blocks), int(iters), _ptr(sink), _stream(stream)),
           "soft_probe_flops")
    return lib().soft_probe_flop_count(int(kind), int(blocks), int(iters))


def soft_sh_forward(B, n, precision, f, a, stream=None):
    """Spherical-harmonic coefficients a (n x B^2) of n sampled functions f (n x 2B x 2B)."""
    _check(lib().soft_sh_forward(int(B), int(n), int(precision), _ptr(f), _ptr(a), _stream(stream)),
           "soft_sh_forward")


def soft_match_refine(match, grid, index, angles, stream=None):
    """Refined rotation (alpha, beta, gamma) of each pair at its grid maximum."""
    _check(lib().soft_match_refine(ctypes.c_void_p(match), _ptr(grid), _ptr(index), _ptr(angles),
                                   _stream(stream)), "soft_match_refine")


def soft_match_polish(match, coeffs, start, iters, angles, value, stream=None):
    """Newton-polished rotation of each pair's correlation maximum, off the grid."""
    _check(lib().soft_match_polish(ctypes.c_void_p(match), _ptr(coeffs), _ptr(start), int(iters), _ptr(angles),
                                   _ptr(value), _stream(stream)), "soft_match_polish")


def soft_match(match, a, b, grid, index, stream=None):
    _check(lib().soft_match(ctypes.c_void_p(match), _ptr(a), _ptr(b), _ptr(grid), _ptr(index), _stream(stream)),
           "soft_match")


def soft_match_destroy(match):
    _check(lib().soft_match_destroy(ctypes.c_void_p(match)), "soft_match_destroy")


# ---------------------------------------------------------------------------
# Convenience wrapper
# ---------------------------------------------------------------------------

def num_coeffs(B):
    return B * (4 * B * B - 1) // 3


def _precision(precision):
    if isinstance(precision, str):
        if precision not in PRECISIONS:
            raise ValueError(f"precision must be one of {sorted(PRECISIONS)}, got {precision!r}")
        return PRECISIONS[precision]
    return int(precision)


def _flags(tune, inplace_ok, graph=False, beta_halves=False, dd=False):
    return (SOFT_PLAN_TUNE if tune else 0) | (SOFT_INPLACE_OK if inplace_ok else 0) | \
        (SOFT_PLAN_GRAPH if graph else 0) | (SOFT_BETA_HALVES if beta_halves else 0) | \
        (SOFT_DD_RECURRENCE if dd else 0)


class _PlanBase:
    """Shape and dtype checks shared by Plan and UnevenPlan."""

    def _init_device(self, device, precision):
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else
                                   torch.device(device).index or 0)
        self.precision = _precision(precision)
        self.dtype = torch.complex128 if self.precision == SOFT_FP64 else torch.complex64

    def _checked(self, t, shape, what):
        if not isinstance(t, torch.Tensor) or t.device != self.device:
            raise ValueError(f"{what} must be a tensor on {self.device}")
        if t.dtype != self.dtype:
            raise ValueError(f"{what} must be {self.dtype}, got {t.dtype}")
        if t.numel() != int(torch.Size(shape).numel()):
            raise ValueError(f"{what} has {t.numel()} elements, expected shape {shape}")
        if not t.is_contiguous():
            raise ValueError(f"{what} must be contiguous")
        return t

    def _out(self, out, shape, what):
        if out is None:
            return torch.empty(shape, dtype=self.dtype, device=self.device)
        return self._checked(out, shape, what)

    # transforms -----------------------------------------------------------
    def forward(self, grid, out=None):
        """FSOFT: coefficients of the sampled function(s).  An ``inplace_ok``
        plan overwrites ``grid`` with scratch."""
        g = self._checked(grid, self.grid_shape(), "grid")
        c = self._out(out, self.coeff_shape(), "out")
        soft_forward(self.handle, g, c)
        return c

    def inverse(self, coeffs, out=None):
        """iFSOFT: grid samples of the band-limited function(s)."""
        c = self._checked(coeffs, self.coeff_shape(), "coeffs")
        g = self._out(out, self.grid_shape(), "out")
        soft_inverse(self.handle, c, g)
        return g

    def adjoint(self, coeffs, out=None):
        """F^H = W I V, adjoint of forward."""
        c = self._checked(coeffs, self.coeff_shape(), "coeffs")
        g = self._out(out, self.grid_shape(), "out")
        soft_adjoint(self.handle, c, g)
        return g

    def adjoint_inverse(self, grid, out=None):
        """I^H = V^-1 F W^-1, adjoint of inverse.  An ``inplace_ok`` plan
        overwrites ``grid`` with scratch."""
        g = self._checked(grid, self.grid_shape(), "grid")
        c = self._out(out, self.coeff_shape(), "out")
        soft_adjoint_inverse(self.handle, g, c)
        return c

    def workspace_bytes(self):
        return soft_plan_sizes(self.handle)[2]

    def describe(self):
        """Bands, DWT launch shapes (tuned or fixed) and workspace of the plan."""
        return soft_plan_describe(self.handle)

    def set_dwt_shape(self, launch, direction, waves, subsets):
        """Pin the (waves, subsets) shape of DWT launch ``launch``; direction
        0 = forward, 1 = inverse."""
        soft_plan_set_dwt_shape(self.handle, launch, direction, waves, subsets)

    def close(self):
        if getattr(self, "handle", None):
            soft_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Plan(_PlanBase):
    @classmethod
    def _borrow(cls, handle, B, batch, device, precision, inplace_ok=False):
        """A Plan over a handle owned elsewhere (closing it does nothing)."""
        self = cls.__new__(cls)
        self._init_device(device, precision)
        self.inplace_ok = inplace_ok
        self.handle = handle
        self._owned = False
        self.B, self.batch, self.N = B, batch, 2 * B
        self.nc = num_coeffs(B)
        return self

    def close(self):
        if getattr(self, "_owned", True):
            super().close()
        else:
            self.handle = None

    """A plan for ``batch`` SO(3) transforms of bandwidth ``B`` on one device.

    Grids are tensors of shape [batch, 2B, 2B, 2B] (or [2B, 2B, 2B] when
    batch == 1); coefficient vectors are [batch, B(4B^2-1)/3] (or flat).
    ``precision`` is "fp64" (complex128), "fp32" or "fp32_split" (complex64).
    ``tune`` times the DWT launch shapes at plan time; ``inplace_ok`` drops
    the plan's FFT intermediate and stages it in the grid tensors instead
    (forward and adjoint_inverse then overwrite their input grid); ``graph``
    replays each call kind as a captured HIP graph (SOFT_PLAN_GRAPH);
    ``beta_halves`` holds the per-order-pair samples for half of the beta
    samples at a time (SOFT_BETA_HALVES, 2B >= 128; always at B = 1024);
    ``dd`` runs the DWT's Wigner-d recurrence in double-double
    (SOFT_DD_RECURRENCE, fp64 only).
    Calls are asynchronous on the current torch stream.
    """

    def __init__(self, B, batch=1, device=None, precision="fp64", tune=False, inplace_ok=False, graph=False,
                 beta_halves=False, dd=False):
        self._init_device(device, precision)
        self.inplace_ok = bool(inplace_ok)
        with torch.cuda.device(self.device):
            self.handle = soft_plan(B, batch, self.precision, _flags(tune, inplace_ok, graph, beta_halves, dd))
        self.B, self.batch, self.N = B, batch, 2 * B
        self.nc = num_coeffs(B)

    def grid_shape(self):
        N = self.N
        return (N, N, N) if self.batch == 1 else (self.batch, N, N, N)

    def coeff_shape(self):
        return (self.nc,) if self.batch == 1 else (self.batch, self.nc)


class UnevenPlan(_PlanBase):
    """One call over functions of mixed bandwidths ``Bs`` (storage order).

    Grids and coefficient vectors are flat 1-D tensors holding the functions
    back to back; ``grid_offsets`` / ``coeff_offsets`` (n+1 entries) give
    where each starts, and ``split_grids`` / ``split_coeffs`` return views.
    """

    def __init__(self, Bs, device=None, precision="fp64", tune=False, inplace_ok=False, graph=False,
                 beta_halves=False, dd=False):
        self._init_device(device, precision)
        self.inplace_ok = bool(inplace_ok)
        self.Bs = [int(b) for b in Bs]
        with torch.cuda.device(self.device):
            self.handle = soft_plan_uneven(self.Bs, self.precision,
                                           _flags(tune, inplace_ok, graph, beta_halves, dd))
        self.grid_offsets, self.coeff_offsets = soft_plan_offsets(self.handle, len(self.Bs))

    def grid_shape(self):
        return (self.grid_offsets[-1],)

    def coeff_shape(self):
        return (self.coeff_offsets[-1],)

    def split_grids(self, flat):
        """Views [2B, 2B, 2B] of each function's grid in a flat grid buffer."""
        return [flat[self.grid_offsets[f]:self.grid_offsets[f + 1]].view(2 * B, 2 * B, 2 * B)
                for f, B in enumerate(self.Bs)]

    def split_coeffs(self, flat):
        """Views of each function's coefficient vector in a flat buffer."""
        return [flat[self.coeff_offsets[f]:self.coeff_offsets[f + 1]] for f in range(len(self.Bs))]


class MatchPlan:
    """Rotational-matching head for ``n`` pairs of functions on the sphere at
    bandwidth ``B``: a, b are [n, B^2] (or [B^2] when n == 1) complex
    tensors, coefficient (l, m) at l^2 + m + l.  ``plan`` is the owned
    soft.Plan of the n correlation functions (for backward passes);
    ``inplace_ok`` makes it a plan without an FFT intermediate of its own."""

    def __init__(self, B, n=1, device=None, precision="fp64", tune=False, inplace_ok=False, beta_halves=False):
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else
                                   torch.device(device).index or 0)
        self.precision = _precision(precision)
        self.dtype = torch.complex128 if self.precision == SOFT_FP64 else torch.complex64
        with torch.cuda.device(self.device):
            self.handle = soft_match_plan(B, n, self.precision, _flags(tune, inplace_ok, False, beta_halves))
        self.B, self.n = B, n
        self.plan = Plan._borrow(soft_match_plan_soft(self.handle), B, n, self.device, self.precision,
                                 bool(inplace_ok))

    def sh_shape(self):
        return (self.B * self.B,) if self.n == 1 else (self.n, self.B * self.B)

    def _chk(self, t, shape, what):
        return self.plan._checked(t, shape, what)

    def coeffs(self, a, b, out=None):
        """f°(l, M, M') = a(l, M) conj(b(l, M')) for every pair."""
        a = self._chk(a, self.sh_shape(), "a")
        b = self._chk(b, self.sh_shape(), "b")
        c = self.plan._out(out, self.plan.coeff_shape(), "out")
        soft_match_coeffs(self.handle, a, b, c)
        return c

    def coeffs_vjp(self, a, b, g):
        """(ga, gb): vector-Jacobian product of ``coeffs`` for g = dL/d conj(f°)."""
        a = self._chk(a, self.sh_shape(), "a")
        b = self._chk(b, self.sh_shape(), "b")
        g = self._chk(g, self.plan.coeff_shape(), "g")
        ga, gb = torch.empty_like(a), torch.empty_like(b)
        soft_match_coeffs_vjp(self.handle, a, b, g, ga, gb)
        return ga, gb

    def argmax(self, grid, out=None):
        """Flat index of the largest real part of each correlation grid (int64)."""
        g = self._chk(grid, self.plan.grid_shape(), "grid")
        idx = out if out is not None else torch.empty(self.n, dtype=torch.int64, device=self.device)
        soft_match_argmax(self.handle, g, idx)
        return idx

    def match(self, a, b, grid=None, index=None):
        """Correlation grids of every pair and the argmax of each: (grid, index)."""
        a = self._chk(a, self.sh_shape(), "a")
        b = self._chk(b, self.sh_shape(), "b")
        g = self.plan._out(grid, self.plan.grid_shape(), "grid")
        idx = index if index is not None else torch.empty(self.n, dtype=torch.int64, device=self.device)
        soft_match(self.handle, a, b, g, idx)
        return g, idx

    def match_index(self, a, b, index=None):
        """The argmax of every pair's correlation grid without the grids: the
        last FFT pass reduces to the argmax instead of storing (same indices
        as ``match``; not for ``inplace_ok`` heads)."""
        a = self._chk(a, self.sh_shape(), "a")
        b = self._chk(b, self.sh_shape(), "b")
        idx = index if index is not None else torch.empty(self.n, dtype=torch.int64, device=self.device)
        soft_match(self.handle, a, b, None, idx)
        return idx

    def sh_forward(self, f):
        """Spherical-harmonic coefficients [n, B^2] (or [B^2]) of functions
        sampled on the sphere, f: [n, 2B, 2B] (or [2B, 2B]) with
        f[j, k] = f(theta_j = (2j+1) pi/(4B), phi_k = k pi/B)."""
        N = 2 * self.B
        shape = (N, N) if self.n == 1 else (self.n, N, N)
        f = self._chk(f, shape, "f")
        a = torch.empty(self.sh_shape(), dtype=self.dtype, device=self.device)
        soft_sh_forward(self.B, self.n, self.precision, f, a)
        return a

    def refine(self, grid, index):
        """Rotation (alpha, beta, gamma) [n, 3] (float64, intrinsic z-y-z) of
        each pair at its grid maximum, refined below the grid spacing."""
        grid = self._chk(grid, self.plan.grid_shape(), "grid")
        if index.dtype != torch.int64 or index.numel() != self.n or index.device != self.device:
            raise ValueError("index: n int64 on the head's device")
        angles = torch.empty(self.n, 3, dtype=torch.float64, device=self.device)
        soft_match_refine(self.handle, grid, index.contiguous(), angles)
        return angles

    def polish(self, coeffs, start, iters=6):
        """Newton steps on the correlation off the grid from ``start``
        (``refine``'s angles [n, 3]); ``coeffs`` the pairs' correlation
        coefficients (``coeffs``).  Returns (angles [n, 3], Re C there [n])."""
        c = self._chk(coeffs, self.plan.coeff_shape(), "coeffs")
        if start.dtype != torch.float64 or start.numel() != 3 * self.n or start.device != self.device:
            raise ValueError("start: n x 3 float64 on the head's device")
        angles = torch.empty(self.n, 3, dtype=torch.float64, device=self.device)
        value = torch.empty(self.n, dtype=torch.float64, device=self.device)
        soft_match_polish(self.handle, c, start.contiguous(), iters, angles, value)
        return angles, value

    def match_rotation(self, f, g, polish_iters=6):
        """The whole matching pipeline for sampled functions on the sphere:
        the rotation R (Euler angles [n, 3], R = Rz(alpha) Ry(beta) Rz(gamma))
        with g(w) ~ f(R^-1 w): the maximum on the SO(3) grid, a parabola
        through its neighbours, then ``polish_iters`` Newton steps off the
        grid (0: none).  Returns (angles, grid index)."""
        a, b = self.sh_forward(f), self.sh_forward(g)
        grid, idx = self.match(a, b)
        angles = self.refine(grid, idx)
        if polish_iters:
            angles, _ = self.polish(self.coeffs(a, b), angles, polish_iters)
        return angles, idx

    def close(self):
        if getattr(self, "handle", None):
            self.plan.close()
            soft_match_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
