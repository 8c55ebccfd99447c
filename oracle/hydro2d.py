"""ctypes wrapper of the 2D hydro proxy oracle (oracle/hydro2d.c)."""
import ctypes

import numpy as np

from .build import load

H = 2
FIELDS = ["rho0", "rho1", "e0", "e1", "p", "cs", "q", "vol", "u0", "v0", "u1", "v1",
          "xarea", "vfx", "mfx", "yarea", "vfy", "mfy", "w_pre", "w_post", "w_ef",
          "w_nf", "w_nmpost", "w_nmpre", "w_mf"]
FID = {n: k for k, n in enumerate(FIELDS)}


def _setup(lib):
    if getattr(lib, "_h2d_ready", False):
        return
    lib.h2d_create.restype = ctypes.c_void_p
    lib.h2d_create.argtypes = [ctypes.c_int, ctypes.c_int]
    lib.h2d_destroy.argtypes = [ctypes.c_void_p]
    lib.h2d_field.restype = ctypes.POINTER(ctypes.c_double)
    lib.h2d_field.argtypes = [ctypes.c_void_p, ctypes.c_int]
    lib.h2d_pitch.restype = ctypes.c_long
    lib.h2d_pitch.argtypes = [ctypes.c_void_p]
    lib.h2d_rows.restype = ctypes.c_long
    lib.h2d_rows.argtypes = [ctypes.c_void_p]
    lib.h2d_geometry.argtypes = [ctypes.c_void_p]
    lib.h2d_dt.restype = ctypes.c_double
    lib.h2d_dt.argtypes = [ctypes.c_void_p]
    lib.h2d_step.restype = ctypes.c_double
    lib.h2d_step.argtypes = [ctypes.c_void_p, ctypes.c_double]
    lib.h2d_lagrangian.argtypes = [ctypes.c_void_p, ctypes.c_double]
    lib.h2d_sum_cells.restype = ctypes.c_double
    lib.h2d_sum_cells.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
    lib.h2d_field_summary.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]
    lib._h2d_ready = True


class Hydro2D:
    """Oracle state.  field(name) returns a writable (ny+5, nx+5) numpy view in
    which element [j+2, i+2] is logical index (i, j)."""

    def __init__(self, nx: int, ny: int):
        self.lib = load()
        _setup(self.lib)
        self.nx, self.ny = nx, ny
        self.s = self.lib.h2d_create(nx, ny)
        self.pitch = self.lib.h2d_pitch(self.s)
        self.rows = self.lib.h2d_rows(self.s)
        self.lib.h2d_geometry(self.s)

    def __del__(self):
        if getattr(self, "s", None):
            self.lib.h2d_destroy(self.s)
            self.s = None

    def field(self, name: str) -> np.ndarray:
        p = self.lib.h2d_field(self.s, FID[name])
        return np.ctypeslib.as_array(p, shape=(self.rows, self.pitch))

    def interior(self, name: str, node: bool = False) -> np.ndarray:
        e = 1 if node else 0
        return self.field(name)[H:H + self.ny + e, H:H + self.nx + e]

    def set_state(self, rho: np.ndarray, ene: np.ndarray, u=None, v=None):
        self.interior("rho0")[...] = rho
        self.interior("e0")[...] = ene
        if u is not None:
            self.interior("u0", True)[...] = u
        if v is not None:
            self.interior("v0", True)[...] = v

    def dt(self) -> float:
        return self.lib.h2d_dt(self.s)

    def step(self, dt: float) -> float:
        return self.lib.h2d_step(self.s, dt)

    def lagrangian(self, dt: float):
        self.lib.h2d_lagrangian(self.s, dt)

    def sum_cells(self, name: str, times_rho0: bool = False) -> float:
        return self.lib.h2d_sum_cells(self.s, FID[name], int(times_rho0))

    def field_summary(self) -> np.ndarray:
        """(volume, mass, internal energy, kinetic energy, pressure) of the
        current state; recomputes the pressure field from rho0 and e0."""
        out = np.zeros(5)
        self.lib.h2d_field_summary(self.s, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        return out

    def run(self, steps: int, dt0=None):
        """Advance `steps` steps starting from dt0 (default: the state's own
        bound); returns the list of time steps used and the next one."""
        dt = self.dt() if dt0 is None else dt0
        used = []
        for _ in range(steps):
            used.append(dt)
            dt = self.step(dt)
        return used, dt
