"""ctypes wrapper of the 3D Navier-Stokes proxy oracle (oracle/ns3d.c)."""
import ctypes

import numpy as np

from .build import load

NH = 4
FIELDS = ["q_r", "q_ru", "q_rv", "q_rw", "q_re", "d_r", "d_ru", "d_rv", "d_rw", "d_re",
          "p_r", "p_u", "p_v", "p_w", "p_p",
          "g_ux", "g_uy", "g_uz", "g_vx", "g_vy", "g_vz", "g_wx", "g_wy", "g_wz", "g_tx", "g_ty", "g_tz"]
FID = {n: k for k, n in enumerate(FIELDS)}
Q = FIELDS[:5]


def _setup(lib):
    if getattr(lib, "_ns_ready", False):
        return
    lib.ns_create.restype = ctypes.c_void_p
    lib.ns_create.argtypes = [ctypes.c_int, ctypes.c_double]
    lib.ns_destroy.argtypes = [ctypes.c_void_p]
    lib.ns_field.restype = ctypes.POINTER(ctypes.c_double)
    lib.ns_field.argtypes = [ctypes.c_void_p, ctypes.c_int]
    lib.ns_set_periodic_z.argtypes = [ctypes.c_void_p, ctypes.c_int]
    lib.ns_init.argtypes = [ctypes.c_void_p]
    lib.ns_stage.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double]
    lib.ns_step.argtypes = [ctypes.c_void_p, ctypes.c_double]
    lib.ns_sum.restype = ctypes.c_double
    lib.ns_sum.argtypes = [ctypes.c_void_p, ctypes.c_int]
    lib.ns_kinetic.restype = ctypes.c_double
    lib.ns_kinetic.argtypes = [ctypes.c_void_p]
    lib.ns_mu.restype = ctypes.c_double
    lib.ns_mu.argtypes = [ctypes.c_void_p]
    lib._ns_ready = True


def stable_dt(n: int, cfl: float = 0.5, mach: float = 0.1) -> float:
    """Fixed step of the proxy: cfl * h / (1 + 1/M) (flow speed 1 plus sound speed)."""
    h = 2.0 * np.pi / n
    return cfl * h / (1.0 + 1.0 / mach)


class NS3D:
    """Oracle state; field(name) is a writable (n+8)^3 view indexed [k, j, i]
    with logical index (i, j, k) at [k+4, j+4, i+4]."""

    def __init__(self, n: int, re: float = 1600.0, periodic_z: bool = False):
        self.lib = load()
        _setup(self.lib)
        self.n = n
        self.s = self.lib.ns_create(n, re)
        self.lib.ns_set_periodic_z(self.s, int(periodic_z))

    def __del__(self):
        if getattr(self, "s", None):
            self.lib.ns_destroy(self.s)
            self.s = None

    def field(self, name):
        m = self.n + 2 * NH
        return np.ctypeslib.as_array(self.lib.ns_field(self.s, FID[name]), shape=(m, m, m))

    def interior(self, name):
        return self.field(name)[NH:NH + self.n, NH:NH + self.n, NH:NH + self.n]

    def set_primitives(self, rho, u, v, w, p):
        for name, a in zip(["p_r", "p_u", "p_v", "p_w", "p_p"], (rho, u, v, w, p)):
            self.interior(name)[...] = a
        self.lib.ns_init(self.s)

    def step(self, dt):
        self.lib.ns_step(self.s, dt)

    def sum(self, name):
        return self.lib.ns_sum(self.s, FID[name])

    def kinetic(self):
        return self.lib.ns_kinetic(self.s)
