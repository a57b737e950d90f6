"""Python binding of the gfx950 star-stencil library (libstencil_mi355x.so).

Argument marshalling only: every cell update runs in the library's HIP
kernels.  Tensors are torch CUDA(HIP) tensors; their data pointers and the
current torch stream are handed to the C ABI declared in include/stencil.h.
There is no fallback: when the shared library is missing or fails to load,
every call raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libstencil_mi355x.so")

OK, EINVAL, ENOMEM, EDEVICE, EUNSUPPORTED, EOVERFLOW = 0, -1, -2, -3, -4, -5
BOUNDARY_CLAMP, BOUNDARY_PADDED = 0, 1
BOUNDARY = {"clamp": BOUNDARY_CLAMP, "padded": BOUNDARY_PADDED}
STORAGE = {"f32": 0, "f16": 1, "bf16": 2, "f16-scaled": 3, "bf16-scaled": 4}

_lib = None

# exported symbols and their signatures, as declared in include/stencil.h
_i64p = ctypes.POINTER(ctypes.c_int64)
_fp = ctypes.POINTER(ctypes.c_float)
_vp = ctypes.c_void_p
SIGNATURES = {
    "stencil_plan": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, _i64p, ctypes.c_int, _fp,
                                    ctypes.c_int, ctypes.c_int]),
    "stencil_plan_ex": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, _i64p, ctypes.c_int, _fp,
                                       ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_char_p]),
    "stencil_plan_symmetric": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, _i64p, ctypes.c_int,
                                              _fp, ctypes.c_int, ctypes.c_int, ctypes.c_char_p]),
    "stencil_coeffs_per_direction": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _fp, _fp]),
    "stencil_run": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int64, _vp]),
    "stencil_run_noalloc": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int64, _vp]),
    "stencil_run_batched": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                           ctypes.POINTER(_vp), _i64p, _vp]),
    "stencil_batch_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, ctypes.POINTER(_vp),
                                            ctypes.POINTER(_vp), ctypes.POINTER(_vp), _i64p,
                                            ctypes.c_char_p]),
    "stencil_batch_launch": (ctypes.c_int, [_vp, _vp]),
    "stencil_batch_autotune": (ctypes.c_int, [_vp, ctypes.c_char_p, ctypes.c_size_t, _vp]),
    "stencil_batch_describe": (ctypes.c_int, [_vp, ctypes.c_char_p, ctypes.c_size_t]),
    "stencil_batch_destroy": (None, [_vp]),
    "stencil_plan_query": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int),
                                          ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                          ctypes.POINTER(ctypes.c_double)]),
    "stencil_plan_describe": (ctypes.c_int, [_vp, ctypes.c_char_p, ctypes.c_size_t]),
    "stencil_plan_autotune": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_char_p, ctypes.c_size_t, _vp]),
    "stencil_plan_model": (ctypes.c_int, [_vp, ctypes.c_char_p, ctypes.POINTER(ctypes.c_double)]),
    "stencil_reduce_f64": (ctypes.c_int, [_vp, _vp, ctypes.c_int64, ctypes.POINTER(ctypes.c_double),
                                          _vp]),
    "stencil_plan_destroy": (None, [_vp]),
    "stencil_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "stencil_last_error": (ctypes.c_char_p, []),
    "stencil_version": (ctypes.c_char_p, []),
}


class StencilError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"[{status}] {message}")
        self.status = status


def load() -> ctypes.CDLL:
    """Loads the shared library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2002_05983_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc: int):
    if rc != OK:
        L = load()
        msg = L.stencil_last_error().decode() or L.stencil_status_string(rc).decode()
        exc = ValueError if rc == EINVAL else StencilError
        if exc is ValueError:
            raise ValueError(f"[{rc}] {msg}")
        raise StencilError(rc, msg)


def _stream_ptr(stream) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _check_grid(t, ncells: int, name: str):
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a GPU tensor")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != ncells:
        raise ValueError(f"{name} has {t.numel()} cells, plan expects {ncells}")


class Plan:
    """A star-stencil plan: grid shape (numpy/torch order, slowest axis first),
    radius and per-point coefficients (centre, then W,E,S,N[,B,A] per distance).

    boundary "padded": `shape` is the interior; the tensors the plan runs on
    hold shape[a] + 2*radius cells per axis (a fixed ghost frame).
    symmetric: coeffs are shared per axis and distance (c_C, then x, y[, z]
    for each distance: stencil_plan_symmetric)."""

    def __init__(self, shape, radius: int, coeffs, storage: str = "f32", anchor_m: int = 0,
                 tune: str | None = None, boundary: str = "clamp", symmetric: bool = False):
        L = load()
        shape = tuple(int(s) for s in shape)
        self.shape = shape
        self.ndim = len(shape)
        self.radius = int(radius)
        pad = self.radius if boundary == "padded" else 0
        self.array_shape = tuple(s + 2 * pad for s in shape)
        self.ncells = 1
        for s in self.array_shape:
            self.ncells *= s
        dims = (ctypes.c_int64 * self.ndim)(*shape[::-1])
        c = [float(v) for v in coeffs]
        carr = (ctypes.c_float * max(1, len(c)))(*c)
        h = _vp()
        if symmetric:
            if storage != "f32" or anchor_m:
                raise ValueError("shared coefficients are built for FP32 storage")
            rc = L.stencil_plan_symmetric(ctypes.byref(h), self.ndim, dims, self.radius, carr,
                                          len(c), BOUNDARY[boundary], tune.encode() if tune else None)
        else:
            rc = L.stencil_plan_ex(ctypes.byref(h), self.ndim, dims, self.radius, carr, len(c),
                                   BOUNDARY[boundary], STORAGE[storage], int(anchor_m),
                                   tune.encode() if tune else None)
        _check(rc)
        self._h = h

    @property
    def handle(self):
        return self._h

    def run(self, inp, out, steps: int, stream=None):
        """Enqueues `steps` time steps from inp into out on the torch stream."""
        _check_grid(inp, self.ncells, "inp")
        _check_grid(out, self.ncells, "out")
        _check(load().stencil_run(self._h, inp.data_ptr(), out.data_ptr(), int(steps),
                                  _stream_ptr(stream)))
        return out

    def run_noalloc(self, inp, out, steps: int, stream=None):
        """run() without device allocation (stencil_run_noalloc): the
        partner grid is the library's static array, shared by every call on
        the device."""
        _check_grid(inp, self.ncells, "inp")
        _check_grid(out, self.ncells, "out")
        _check(load().stencil_run_noalloc(self._h, inp.data_ptr(), out.data_ptr(), int(steps),
                                          _stream_ptr(stream)))
        return out

    def query(self) -> dict:
        K = ctypes.c_int()
        tile = (ctypes.c_int * 3)()
        vec = ctypes.c_int()
        bpc = ctypes.c_double()
        _check(load().stencil_plan_query(self._h, ctypes.byref(K), tile, ctypes.byref(vec),
                                         ctypes.byref(bpc)))
        return {"K": K.value, "tile": tuple(tile), "vec": vec.value,
                "bytes_per_cell_step": bpc.value}

    def autotune(self, inp, out, stream=None):
        """Times every feasible configuration on (inp, out) and keeps the
        fastest; returns [(config, GCell/s), ...], best first.  out is
        overwritten."""
        _check_grid(inp, self.ncells, "inp")
        _check_grid(out, self.ncells, "out")
        buf = ctypes.create_string_buffer(16384)
        _check(load().stencil_plan_autotune(self._h, inp.data_ptr(), out.data_ptr(), buf, 16384,
                                            _stream_ptr(stream)))
        rows = []
        for line in buf.value.decode().splitlines():
            cfg, g = line.rsplit(" ", 1)
            rows.append((cfg, float(g)))
        return rows

    def model(self, config: str | None = None) -> dict:
        """Analytic prediction for the plan's (or the given) configuration."""
        out = (ctypes.c_double * 4)()
        _check(load().stencil_plan_model(self._h, config.encode() if config else None, out))
        return {"GCell/s": out[0], "hbm_us": out[1], "valu_us": out[2], "plane_us": out[3]}

    def describe(self) -> str:
        buf = ctypes.create_string_buffer(512)
        n = load().stencil_plan_describe(self._h, buf, 512)
        if n < 0:
            _check(n)
        return buf.value.decode()

    def close(self):
        if getattr(self, "_h", None):
            load().stencil_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _batch_arrays(plans, ins, outs, steps):
    n = len(plans)
    if not (len(ins) == len(outs) == n):
        raise ValueError("plans, ins and outs must have the same length")
    if isinstance(steps, int):
        steps = [steps] * n
    if len(steps) != n:
        raise ValueError("steps must be an int or have one entry per grid")
    for p, i, o in zip(plans, ins, outs):
        _check_grid(i, p.ncells, "in")
        _check_grid(o, p.ncells, "out")
    hp = (_vp * n)(*[p.handle for p in plans])
    ip = (_vp * n)(*[t.data_ptr() for t in ins])
    op = (_vp * n)(*[t.data_ptr() for t in outs])
    st = (ctypes.c_int64 * n)(*[int(s) for s in steps])
    return n, hp, ip, op, st


def run_batched(plans, ins, outs, steps, stream=None):
    """Runs independent grids as one batch (see stencil_run_batched)."""
    n, hp, ip, op, st = _batch_arrays(plans, ins, outs, steps)
    _check(load().stencil_run_batched(n, hp, ip, op, st, _stream_ptr(stream)))


class Batch:
    """A reusable batch of grids (stencil_batch_create/launch/destroy).

    The plans and tensors must stay alive, and in place, while the batch
    exists; the batch keeps references to them.
    """

    def __init__(self, plans, ins, outs, steps, tune=None):
        n, hp, ip, op, st = _batch_arrays(plans, ins, outs, steps)
        self._keep = (list(plans), list(ins), list(outs))
        h = _vp()
        _check(load().stencil_batch_create(ctypes.byref(h), n, hp, ip, op, st,
                                           tune.encode() if tune else None))
        self._h = h

    def launch(self, stream=None):
        _check(load().stencil_batch_launch(self._h, _stream_ptr(stream)))

    def autotune(self, stream=None) -> str:
        buf = ctypes.create_string_buffer(1 << 16)
        _check(load().stencil_batch_autotune(self._h, buf, len(buf), _stream_ptr(stream)))
        return buf.value.decode()

    def describe(self) -> str:
        n = load().stencil_batch_describe(self._h, None, 0)
        buf = ctypes.create_string_buffer(max(1, n + 1))
        load().stencil_batch_describe(self._h, buf, len(buf))
        return buf.value.decode()

    def close(self):
        if getattr(self, "_h", None):
            load().stencil_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def coeffs_per_direction(ndim: int, radius: int, per_direction):
    """The per-point coefficients of a star whose coefficient is one per
    direction (c_C, c_W, c_E, c_S, c_N[, c_B, c_A]), as stencil_plan takes
    them (stencil_coeffs_per_direction)."""
    src = (ctypes.c_float * (1 + 2 * ndim))(*[float(v) for v in per_direction])
    out = (ctypes.c_float * (1 + 2 * ndim * radius))()
    _check(load().stencil_coeffs_per_direction(int(ndim), int(radius), src, out))
    return [out[k] for k in range(1 + 2 * ndim * radius)]


def reduce_f64(x, ref=None, stream=None):
    """(max|x - ref|, max|ref|, sum x) accumulated in FP64 on the GPU."""
    import torch
    if x.dtype != torch.float32 or not x.is_contiguous():
        raise TypeError("x must be contiguous float32")
    if ref is not None and (ref.dtype != torch.float64 or not ref.is_contiguous()
                            or ref.numel() != x.numel()):
        raise TypeError("ref must be contiguous float64 with x's size")
    out = (ctypes.c_double * 3)()
    _check(load().stencil_reduce_f64(x.data_ptr(), ref.data_ptr() if ref is not None else None,
                                     x.numel(), out, _stream_ptr(stream)))
    return out[0], out[1], out[2]


def version() -> str:
    return load().stencil_version().decode()
