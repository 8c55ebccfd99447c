"""Thin ctypes binding of libooc.so (include/ooc.h): argument marshalling only.

Every step of the path runs inside the HIP library.  PyTorch provides the
device arena (one uint8 tensor) and the three streams; nothing else.  If the
library is missing the import fails loudly -- there is no fallback."""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libooc.so")

OK, E_ARG, E_BUDGET, E_DEVICE, E_STATE, E_FAILED, E_STALE, E_NOMEM = 0, -1, -2, -3, -4, -5, -6, -7
READ, WRITE, RW, INC = 1, 2, 3, 4
RED_MIN, RED_MAX, RED_SUM = 1, 2, 3
ARG_DAT, ARG_RED, ARG_CONST, ARG_DEVSCALAR = 0, 1, 2, 3
FLAG_CYCLIC, FLAG_PREFETCH, FLAG_FP32_STREAM, FLAG_INCORE = 1, 2, 4, 8
FLAG_GRAPH, FLAG_FUSE, FLAG_DEBUG_POISON, FLAG_DEBUG_SYNC, FLAG_PLAN_ONLY = 16, 32, 64, 128, 256
FLAG_KERNEL_COPY = 512
FLAG_RING = 1024
FLAG_MEMCPY_DOWNLOAD = 2048
FIELD_RESIDENT = 1
SCRATCH_DOUBLES = 524288  # OOC_MLP_SCRATCH_DOUBLES: static device scratch of ooc_mlp_predict_noalloc

_ERRNAMES = {E_ARG: "OOC_E_ARG", E_BUDGET: "OOC_E_BUDGET", E_DEVICE: "OOC_E_DEVICE",
             E_STATE: "OOC_E_STATE", E_FAILED: "OOC_E_FAILED", E_STALE: "OOC_E_STALE",
             E_NOMEM: "OOC_E_NOMEM"}


class OocError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (_ERRNAMES.get(code, code), msg))
        self.code = code


class ooc_arg(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("handle", ctypes.c_int32), ("access", ctypes.c_int32),
                ("npts", ctypes.c_int32), ("offsets", ctypes.POINTER(ctypes.c_int32)),
                ("value", ctypes.c_double)]


class ooc_stats(ctypes.Structure):
    _fields_ = [("chains", ctypes.c_uint64), ("tiles", ctypes.c_uint64), ("launches", ctypes.c_uint64),
                ("bytes_h2d", ctypes.c_uint64), ("bytes_d2h", ctypes.c_uint64),
                ("bytes_edge", ctypes.c_uint64), ("bytes_hbm_alg", ctypes.c_uint64),
                ("last_bytes_h2d", ctypes.c_uint64), ("last_bytes_d2h", ctypes.c_uint64),
                ("tile_rows", ctypes.c_int64), ("ntiles_last", ctypes.c_int32),
                ("slots", ctypes.c_int32), ("slot_bytes", ctypes.c_uint64),
                ("last_flush_ms", ctypes.c_double), ("last_kernel_ms", ctypes.c_double),
                ("last_issue_ms", ctypes.c_double), ("max_call_ms", ctypes.c_double),
                ("host_pinned_bytes", ctypes.c_uint64), ("host_pageable_bytes", ctypes.c_uint64),
                ("max_call_kind", ctypes.c_int32), ("max_call_chain", ctypes.c_int32)]


class ooc_tile_time(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int64), ("h2d_begin_us", ctypes.c_float), ("h2d_end_us", ctypes.c_float),
                ("comp_begin_us", ctypes.c_float), ("comp_end_us", ctypes.c_float),
                ("edge_end_us", ctypes.c_float), ("d2h_begin_us", ctypes.c_float), ("d2h_end_us", ctypes.c_float)]


class ooc_plan_info(ctypes.Structure):
    _fields_ = [("ntiles", ctypes.c_int32), ("nloops", ctypes.c_int32), ("nfields", ctypes.c_int32),
                ("slots", ctypes.c_int32), ("tile_rows", ctypes.c_int64), ("slot_bytes", ctypes.c_uint64),
                ("loop_rows", ctypes.POINTER(ctypes.c_int64)), ("resident", ctypes.POINTER(ctypes.c_int64)),
                ("nup", ctypes.c_int32), ("ndown", ctypes.c_int32), ("nedge", ctypes.c_int32),
                ("up", ctypes.POINTER(ctypes.c_int64)), ("down", ctypes.POINTER(ctypes.c_int64)),
                ("edge", ctypes.POINTER(ctypes.c_int64)), ("temporary", ctypes.POINTER(ctypes.c_int32)),
                ("ring", ctypes.c_int32), ("ring_rows", ctypes.POINTER(ctypes.c_int64))]


EXPORTS = ["ooc_create", "ooc_bind_device", "ooc_decl_field", "ooc_decl_reduction", "ooc_set_reduction",
           "ooc_par_loop", "ooc_mark_step", "ooc_discard_queue", "ooc_execute", "ooc_submit", "ooc_reduce", "ooc_fetch_field",
           "ooc_set_field", "ooc_set_flags", "ooc_set_schedule", "ooc_get_stats", "ooc_set_timing", "ooc_set_tile_timing", "ooc_tile_times",
           "ooc_kernel_stats", "ooc_last_error", "ooc_debug_fail_after", "ooc_destroy", "ooc_debug_plan", "ooc_field_shape", "ooc_get_layout",
           "ooc_mlp_create", "ooc_mlp_num_params", "ooc_mlp_get_params", "ooc_mlp_set_params",
           "ooc_mlp_predict", "ooc_mlp_predict_noalloc", "ooc_mlp_gradient", "ooc_mlp_train", "ooc_mlp_destroy"]

_lib = None


def load_library() -> ctypes.CDLL:
    """Load the in-tree libooc.so (built by python -m paper_1709_02125_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libooc.so is not built (%s); run python -m paper_1709_02125_amd.build" % LIB_PATH)
    # PyTorch-ROCm ships its own HIP runtime with the same soname as the system
    # one; load torch first so the library binds to that single runtime instead
    # of bringing a second HIP/HSA runtime into the process.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    P, I, I64, U32, SZ, D = (ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_uint32,
                             ctypes.c_size_t, ctypes.c_double)
    I64P = ctypes.POINTER(ctypes.c_int64)
    I32P = ctypes.POINTER(ctypes.c_int32)
    DP = ctypes.POINTER(ctypes.c_double)
    sig = {
        "ooc_create": [ctypes.POINTER(P), I, I64P, I, SZ, U32],
        "ooc_bind_device": [P, P, SZ, P, P, P],
        "ooc_decl_field": [P, ctypes.c_char_p, I32P, DP, U32, I32P],
        "ooc_decl_reduction": [P, I, I32P],
        "ooc_set_reduction": [P, ctypes.c_int32, D],
        "ooc_par_loop": [P, I, I64P, I, ctypes.POINTER(ooc_arg)],
        "ooc_mark_step": [P],
        "ooc_discard_queue": [P],
        "ooc_execute": [P],
        "ooc_submit": [P],
        "ooc_reduce": [P, ctypes.c_int32, DP],
        "ooc_fetch_field": [P, ctypes.c_int32, DP, SZ],
        "ooc_set_field": [P, ctypes.c_int32, DP, SZ],
        "ooc_set_flags": [P, U32, U32],
        "ooc_set_schedule": [P, I64, I, I],
        "ooc_get_stats": [P, ctypes.POINTER(ooc_stats)],
        "ooc_get_layout": [P, ctypes.POINTER(I64), ctypes.POINTER(I64), ctypes.POINTER(I64)],
        "ooc_set_timing": [P, I],
        "ooc_set_tile_timing": [P, I],
        "ooc_tile_times": [P, ctypes.POINTER(ooc_tile_time), I, ctypes.POINTER(I)],
        "ooc_kernel_stats": [P, I, DP, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64)],
        "ooc_last_error": [P],
        "ooc_debug_fail_after": [P, I64],
        "ooc_destroy": [P],
        "ooc_debug_plan": [P, ctypes.POINTER(ooc_plan_info)],
        "ooc_field_shape": [P, ctypes.c_int32, I64P, I64P],
        "ooc_mlp_create": [ctypes.POINTER(P), I, I, ctypes.c_uint64],
        "ooc_mlp_num_params": [P],
        "ooc_mlp_get_params": [P, DP],
        "ooc_mlp_set_params": [P, DP],
        "ooc_mlp_predict": [P, DP, I, DP],
        "ooc_mlp_predict_noalloc": [P, DP, I, DP],
        "ooc_mlp_gradient": [P, DP, DP, I, DP, DP],
        "ooc_mlp_train": [P, DP, DP, I, I, D, DP],
        "ooc_mlp_destroy": [P],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_char_p if name == "ooc_last_error" else ctypes.c_int
    _lib = lib
    return lib


# ------------------------------------------------------------- arguments
# element of x = 0 within every stored row (ooc_get_layout's x_origin)
X_ORIGIN = 16


def row_pitch(nx: int, halo: int) -> int:
    """Elements per stored row for nx interior points and the given halo:
    x = -halo .. nx + halo (one extra for node-centred fields) from X_ORIGIN,
    rounded up to 32 elements (ooc_get_layout's pitch)."""
    return (X_ORIGIN + nx + halo + 1 + 31) // 32 * 32


class Dat:
    __slots__ = ("field", "access", "offsets")

    def __init__(self, field, access, offsets):
        self.field, self.access, self.offsets = field, access, offsets


def dat(field: int, access: int, *offsets):
    """A field argument; offsets are tuples of ndim ints (default: the point)."""
    return Dat(field, access, offsets or None)


class Const:
    __slots__ = ("value",)

    def __init__(self, v):
        self.value = float(v)


class DevScalar:
    __slots__ = ("red",)

    def __init__(self, r):
        self.red = r


class Red:
    __slots__ = ("red",)

    def __init__(self, r):
        self.red = r


class Context:
    """One grid (ooc_create) with its fields, reductions and lazy loop queue."""

    def __init__(self, ndim: int, dims, halo: int, budget: int, flags: int = 0, bind: bool = True,
                 arena_bytes: int | None = None):
        self.lib = load_library()
        self.ndim = ndim
        self.dims = tuple(dims) + (1,) * (3 - len(dims))
        self.halo = halo
        self._h = ctypes.c_void_p()
        d = (ctypes.c_int64 * 3)(*self.dims)
        self._check(self.lib.ooc_create(ctypes.byref(self._h), ndim, d, halo, int(budget), int(flags)), None)
        self._keep = []
        if bind:
            import torch
            self.streams = [torch.cuda.Stream() for _ in range(3)]
            if flags & FLAG_RING:
                # ring slabs: the library allocates the rings (and the small
                # reduction / resident area) within the budget itself
                self.arena, ptr, nbytes = None, None, 0
            else:
                nbytes = int(arena_bytes if arena_bytes is not None else budget)
                self.arena = torch.empty(max(nbytes, 256), dtype=torch.uint8, device="cuda")
                ptr = self.arena.data_ptr()
            self._check(self.lib.ooc_bind_device(self._h, ctypes.c_void_p(ptr), nbytes,
                                                 ctypes.c_void_p(self.streams[0].cuda_stream),
                                                 ctypes.c_void_p(self.streams[1].cuda_stream),
                                                 ctypes.c_void_p(self.streams[2].cuda_stream)))
        self.field_names = []

    # -- plumbing
    def _check(self, rc, h="self"):
        if rc != OK:
            msg = self.lib.ooc_last_error(self._h if h else None)
            raise OocError(rc, (msg or b"").decode())

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            rc = self.lib.ooc_destroy(self._h)
            self._h = ctypes.c_void_p()
            self.arena = None
            self._check(rc, None)
        self.arena = None

    def debug_fail_after(self, n: int):
        """ooc_debug_fail_after: report the n-th checked runtime call from now
        on as failed (host-side injection; 0 turns it off)."""
        self._check(self.lib.ooc_debug_fail_after(self._h, int(n)))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- declarations
    def decl_field(self, name: str, delta=(0, 0, 0), init: np.ndarray | None = None, resident=False) -> int:
        dl = (ctypes.c_int32 * 3)(*(tuple(delta) + (0,) * (3 - len(delta))))
        out = ctypes.c_int32()
        ptr = None
        if init is not None:
            init = np.ascontiguousarray(init, dtype=np.float64)
            if init.shape != self.field_shape_for(delta):
                raise ValueError("init shape %s != %s" % (init.shape, self.field_shape_for(delta)))
            ptr = init.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        self._check(self.lib.ooc_decl_field(self._h, name.encode(), dl, ptr,
                                            FIELD_RESIDENT if resident else 0, ctypes.byref(out)))
        self.field_names.append(name)
        return out.value

    def field_shape_for(self, delta) -> tuple:
        delta = tuple(delta) + (0,) * (3 - len(delta))
        n = [self.dims[a] + 2 * self.halo + delta[a] for a in range(self.ndim)]
        return tuple(reversed(n))

    def decl_reduction(self, op: int) -> int:
        out = ctypes.c_int32()
        self._check(self.lib.ooc_decl_reduction(self._h, op, ctypes.byref(out)))
        return out.value

    def set_reduction(self, r: int, v: float):
        self._check(self.lib.ooc_set_reduction(self._h, r, float(v)))

    # -- loops
    def par_loop(self, kernel_id: int, rng, args):
        r = [0, 1, 0, 1, 0, 1]
        for a in range(self.ndim):
            r[2 * a], r[2 * a + 1] = int(rng[a][0]), int(rng[a][1])
        rr = (ctypes.c_int64 * 6)(*r)
        arr = (ooc_arg * len(args))()
        keep = []
        for k, g in enumerate(args):
            x = arr[k]
            if isinstance(g, Dat):
                offs = g.offsets or ((0,) * self.ndim,)
                flat = [int(v) for o in offs for v in o]
                if any(len(o) != self.ndim for o in offs):
                    raise ValueError("stencil offsets must have %d components" % self.ndim)
                buf = (ctypes.c_int32 * len(flat))(*flat)
                keep.append(buf)
                x.kind, x.handle, x.access, x.npts = ARG_DAT, g.field, g.access, len(offs)
                x.offsets = ctypes.cast(buf, ctypes.POINTER(ctypes.c_int32))
            elif isinstance(g, Const):
                x.kind, x.value = ARG_CONST, g.value
            elif isinstance(g, DevScalar):
                x.kind, x.handle = ARG_DEVSCALAR, g.red
            elif isinstance(g, Red):
                x.kind, x.handle = ARG_RED, g.red
            else:
                raise TypeError("bad loop argument %r" % (g,))
        self._check(self.lib.ooc_par_loop(self._h, int(kernel_id), rr, len(args), arr))

    def mark_step(self):
        self._check(self.lib.ooc_mark_step(self._h))

    def discard_queue(self):
        self._check(self.lib.ooc_discard_queue(self._h))

    def execute(self):
        self._check(self.lib.ooc_execute(self._h))

    def submit(self):
        self._check(self.lib.ooc_submit(self._h))

    def reduce(self, r: int) -> float:
        v = ctypes.c_double()
        self._check(self.lib.ooc_reduce(self._h, r, ctypes.byref(v)))
        return v.value

    def fetch_field(self, f: int, delta) -> np.ndarray:
        out = np.empty(self.field_shape_for(delta), dtype=np.float64)
        self._check(self.lib.ooc_fetch_field(self._h, f, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                             out.nbytes))
        return out

    def set_field(self, f: int, arr: np.ndarray):
        arr = np.ascontiguousarray(arr, dtype=np.float64)
        self._check(self.lib.ooc_set_field(self._h, f, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                           arr.nbytes))

    def set_flags(self, set_: int = 0, clear: int = 0):
        self._check(self.lib.ooc_set_flags(self._h, set_, clear))

    def set_schedule(self, tile_rows: int = 0, chain_steps: int = 0, slots: int = 0):
        self._check(self.lib.ooc_set_schedule(self._h, int(tile_rows), int(chain_steps), int(slots)))

    def set_timing(self, on: bool, kernel_id: int | None = None):
        """Per-launch hipEvent timing of every loop, or of one kernel id only."""
        mode = 0 if not on else (1 if kernel_id is None else 2 + int(kernel_id))
        self._check(self.lib.ooc_set_timing(self._h, mode))

    def layout(self):
        """(pitch, plane, x_origin) of the storage layout, in elements."""
        v = [ctypes.c_int64() for _ in range(3)]
        self._check(self.lib.ooc_get_layout(self._h, *[ctypes.byref(x) for x in v]))
        return tuple(x.value for x in v)

    def stats(self) -> dict:
        s = ooc_stats()
        self._check(self.lib.ooc_get_stats(self._h, ctypes.byref(s)))
        return {n: getattr(s, n) for n, _ in ooc_stats._fields_}

    def set_tile_timing(self, on: bool = True):
        """Per-tile stage events on the three streams from the next flush on."""
        self._check(self.lib.ooc_set_tile_timing(self._h, 1 if on else 0))

    def tile_times(self) -> list:
        """Stage times (us) of the tiles of the last collected period, one dict
        per tile: tile, h2d_begin/end, comp_begin/end, edge_end, d2h_begin/end."""
        n = ctypes.c_int32()
        self._check(self.lib.ooc_tile_times(self._h, None, 0, ctypes.byref(n)))
        buf = (ooc_tile_time * max(1, n.value))()
        self._check(self.lib.ooc_tile_times(self._h, buf, n.value, ctypes.byref(n)))
        return [{f: getattr(buf[i], f) for f, _ in ooc_tile_time._fields_} for i in range(n.value)]

    def kernel_stats(self, kid: int):
        ms = ctypes.c_double()
        n = ctypes.c_uint64()
        b = ctypes.c_uint64()
        self._check(self.lib.ooc_kernel_stats(self._h, int(kid), ctypes.byref(ms), ctypes.byref(n),
                                              ctypes.byref(b)))
        return ms.value, n.value, b.value

    def debug_plan(self) -> dict:
        p = ooc_plan_info()
        self._check(self.lib.ooc_debug_plan(self._h, ctypes.byref(p)))
        T, n, F = p.ntiles, p.nloops, p.nfields

        def arr(ptr, cnt, shape):
            if cnt == 0:
                return np.zeros(shape, dtype=np.int64)
            return np.ctypeslib.as_array(ptr, shape=(cnt,)).reshape(shape).copy()

        return {
            "ntiles": T, "nloops": n, "nfields": F, "slots": p.slots, "tile_rows": p.tile_rows,
            "slot_bytes": p.slot_bytes,
            "loop_rows": arr(p.loop_rows, n * T * 2, (n, T, 2)),
            "resident": arr(p.resident, F * T * 2, (F, T, 2)),
            "up": arr(p.up, p.nup * 4, (p.nup, 4)),
            "down": arr(p.down, p.ndown * 4, (p.ndown, 4)),
            "edge": arr(p.edge, p.nedge * 4, (p.nedge, 4)),
            "temporary": np.ctypeslib.as_array(p.temporary, shape=(F,)).copy() if F else np.zeros(0),
            "ring": bool(p.ring),
            "ring_rows": np.ctypeslib.as_array(p.ring_rows, shape=(F,)).copy() if F else np.zeros(0, np.int64),
        }

    def field_shape(self, f: int):
        lo = (ctypes.c_int64 * 3)()
        n = (ctypes.c_int64 * 3)()
        self._check(self.lib.ooc_field_shape(self._h, f, lo, n))
        return tuple(lo), tuple(n)


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Mlp:
    """The library's device-trained cost-model network (ooc_mlp_*)."""

    def __init__(self, n_inputs: int, n_hidden: int = 32, seed: int = 1709):
        self.lib = load_library()
        self._h = ctypes.c_void_p()
        rc = self.lib.ooc_mlp_create(ctypes.byref(self._h), n_inputs, n_hidden, seed)
        if rc:
            raise OocError(rc, "ooc_mlp_create failed")
        self.n_inputs, self.n_hidden = n_inputs, n_hidden
        self.n_params = self.lib.ooc_mlp_num_params(self._h)

    def _chk(self, rc, what):
        if rc:
            raise OocError(rc, what)

    def params(self) -> np.ndarray:
        out = np.empty(self.n_params)
        self._chk(self.lib.ooc_mlp_get_params(self._h, _dp(out)), "get_params")
        return out

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float64)
        assert p.size == self.n_params
        self._chk(self.lib.ooc_mlp_set_params(self._h, _dp(p)), "set_params")

    def predict(self, X) -> np.ndarray:
        X = np.ascontiguousarray(X, dtype=np.float64)
        out = np.empty(X.shape[0])
        self._chk(self.lib.ooc_mlp_predict(self._h, _dp(X), X.shape[0], _dp(out)), "predict")
        return out

    def scratch_doubles(self, n: int) -> int:
        """Doubles of the static device scratch a batch of n rows needs in
        predict_noalloc (each part rounded up to 32 doubles)."""
        pad = lambda k: (k + 31) // 32 * 32
        return pad(n * self.n_inputs) + 2 * pad(n * self.n_hidden) + pad(n)

    def predict_noalloc(self, X) -> np.ndarray:
        """predict() without any device allocation (static device scratch)."""
        X = np.ascontiguousarray(X, dtype=np.float64)
        out = np.empty(X.shape[0])
        rc = self.lib.ooc_mlp_predict_noalloc(self._h, _dp(X), X.shape[0], _dp(out))
        if rc == E_ARG and X.shape[0] >= 1 and self.scratch_doubles(X.shape[0]) > SCRATCH_DOUBLES:
            raise OocError(rc, "predict_noalloc: a batch of %d rows needs %d doubles of scratch, the static "
                               "device scratch holds %d" % (X.shape[0], self.scratch_doubles(X.shape[0]),
                                                            SCRATCH_DOUBLES))
        self._chk(rc, "predict_noalloc")
        return out

    def gradient(self, X, y):
        X = np.ascontiguousarray(X, dtype=np.float64)
        y = np.ascontiguousarray(y, dtype=np.float64)
        g = np.empty(self.n_params)
        loss = np.empty(1)
        self._chk(self.lib.ooc_mlp_gradient(self._h, _dp(X), _dp(y), X.shape[0], _dp(g), _dp(loss)), "gradient")
        return g, float(loss[0])

    def train(self, X, y, epochs: int, lr: float) -> float:
        X = np.ascontiguousarray(X, dtype=np.float64)
        y = np.ascontiguousarray(y, dtype=np.float64)
        loss = np.empty(1)
        self._chk(self.lib.ooc_mlp_train(self._h, _dp(X), _dp(y), X.shape[0], int(epochs), float(lr), _dp(loss)),
                  "train")
        return float(loss[0])

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self.lib.ooc_mlp_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
