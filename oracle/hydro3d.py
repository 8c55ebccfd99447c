"""ctypes wrapper of the 3D hydro proxy oracle (oracle/hydro3d.c).
Test infrastructure only."""
import ctypes

import numpy as np

from .build import load

H = 2
FIELDS = ["rho0", "rho1", "e0", "e1", "p", "cs", "q", "vol",
          "u0", "v0", "w0", "u1", "v1", "w1",
          "xarea", "vfx", "mfx", "yarea", "vfy", "mfy", "zarea", "vfz", "mfz",
          "w_pre", "w_post", "w_ef", "w_nf", "w_nmpost", "w_nmpre", "w_mf"]
FID = {n: k for k, n in enumerate(FIELDS)}


def _setup(lib):
    if getattr(lib, "_h3d_ready", False):
        return
    P = ctypes.c_void_p
    lib.h3d_create.restype = P
    lib.h3d_create.argtypes = [ctypes.c_int] * 3
    lib.h3d_destroy.argtypes = [P]
    lib.h3d_field.restype = ctypes.POINTER(ctypes.c_double)
    lib.h3d_field.argtypes = [P, ctypes.c_int]
    lib.h3d_extent.restype = ctypes.c_long
    lib.h3d_extent.argtypes = [P, ctypes.c_int]
    lib.h3d_geometry.argtypes = [P]
    lib.h3d_dt.restype = ctypes.c_double
    lib.h3d_dt.argtypes = [P]
    lib.h3d_step.restype = ctypes.c_double
    lib.h3d_step.argtypes = [P, ctypes.c_double]
    lib.h3d_lagrangian.argtypes = [P, ctypes.c_double]
    lib.h3d_sum_cells.restype = ctypes.c_double
    lib.h3d_sum_cells.argtypes = [P, ctypes.c_int, ctypes.c_int]
    lib._h3d_ready = True


class Hydro3D:
    """Oracle state.  field(name) returns a writable (nz+5, ny+5, nx+5) numpy
    view in which element [k+2, j+2, i+2] is logical index (i, j, k)."""

    def __init__(self, nx: int, ny: int, nz: int):
        self.lib = load()
        _setup(self.lib)
        self.n = (nx, ny, nz)
        self.s = self.lib.h3d_create(nx, ny, nz)
        self.shape = tuple(self.lib.h3d_extent(self.s, a) for a in (2, 1, 0))
        self.lib.h3d_geometry(self.s)

    def __del__(self):
        if getattr(self, "s", None):
            self.lib.h3d_destroy(self.s)
            self.s = None

    def field(self, name: str) -> np.ndarray:
        p = self.lib.h3d_field(self.s, FID[name])
        return np.ctypeslib.as_array(p, shape=self.shape)

    def interior(self, name: str, node: bool = False) -> np.ndarray:
        e = 1 if node else 0
        nx, ny, nz = self.n
        return self.field(name)[H:H + nz + e, H:H + ny + e, H:H + nx + e]

    def set_state(self, rho, ene, u=None, v=None, w=None):
        self.interior("rho0")[...] = rho
        self.interior("e0")[...] = ene
        for name, val in (("u0", u), ("v0", v), ("w0", w)):
            if val is not None:
                self.interior(name, True)[...] = val

    def dt(self) -> float:
        return self.lib.h3d_dt(self.s)

    def step(self, dt: float) -> float:
        return self.lib.h3d_step(self.s, dt)

    def lagrangian(self, dt: float):
        self.lib.h3d_lagrangian(self.s, dt)

    def sum_cells(self, name: str, times_rho0: bool = False) -> float:
        return self.lib.h3d_sum_cells(self.s, FID[name], int(times_rho0))

    def run(self, steps: int, dt0=None):
        dt = self.dt() if dt0 is None else dt0
        used = []
        for _ in range(steps):
            used.append(dt)
            dt = self.step(dt)
        return used, dt
