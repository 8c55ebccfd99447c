"""3D compressible Navier-Stokes proxy as a user of the loop-chain library:
27 fields (5 conserved, 5 Runge-Kutta increments, 5 primitives, 12 stored
gradients), 15 loops per Runge-Kutta stage (12 boundary strips, primitives,
gradients, residual + update), 3 stages per step, no reductions -- so a chain
can span several steps (the paper tiles OpenSBLI over 1, 2 or 3 time steps,
Section 5.3).  Tiled along z; x and y periodic, z mirror walls.

Two fused forms keep 15 fields in the chain: `fused` evaluates the gradients
inside the residual (conserved, increments, primitives; 14 loops per stage),
`fused="q"` the primitives too, reading one copy of the conserved variables
and writing the other (two copies of the conserved variables, increments;
13 loops per stage).  All three forms compute the same values."""
from __future__ import annotations

import math

import numpy as np

from . import ooc
from .ooc import READ, WRITE, RW, Const, dat

NH = 4
GAMMA, MACH, PRANDTL = 1.4, 0.1, 0.71
TWO_PI = 2.0 * math.pi
RK_A = (0.0, -5.0 / 9.0, -153.0 / 128.0)
RK_B = (1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0)
K_MIRROR = 1
K_INIT, K_PRIMS, K_GRADS, K_RHS_FIRST, K_RHS, K_RHS_FUSED_FIRST, K_RHS_FUSED = 200, 201, 202, 203, 204, 205, 206
K_RHS_FUSEDQ_FIRST, K_RHS_FUSEDQ = 207, 208

Q = ["q_r", "q_ru", "q_rv", "q_rw", "q_re"]
D = ["d_r", "d_ru", "d_rv", "d_rw", "d_re"]
P = ["p_r", "p_u", "p_v", "p_w", "p_p"]
G = ["g_ux", "g_uy", "g_uz", "g_vx", "g_vy", "g_vz", "g_wx", "g_wy", "g_wz", "g_tx", "g_ty", "g_tz"]
Q2 = ["q2_r", "q2_ru", "q2_rv", "q2_rw", "q2_re"]  # the other copy of the conserved variables
FIELDS = Q + D + P + G
FIELDS_FUSED = Q + D + P   # gradients evaluated inside the residual kernel
FIELDS_FUSEDQ = Q + D + Q2  # primitives too (P is declared for the initial state only)
STAR = ((1, 0, 0), (-1, 0, 0), (2, 0, 0), (-2, 0, 0), (0, 1, 0), (0, -1, 0), (0, 2, 0), (0, -2, 0),
        (0, 0, 1), (0, 0, -1), (0, 0, 2), (0, 0, -2))


def _fused_stencil():
    """Points of the primitives the fused residual reads: the fluxes at the
    points a e_A (a in 0, +-1, +-2) of the 5-point difference along axis A,
    each from the 5-point differences b e_B of the primitives (73 points)."""
    pts = set()
    for A in range(3):
        for B in range(3):
            for a in (0, 1, -1, 2, -2):
                for b in (0, 1, -1, 2, -2):
                    o = [0, 0, 0]
                    o[A] += a
                    o[B] += b
                    pts.add(tuple(o))
    return tuple(sorted(pts))


FUSED_STENCIL = _fused_stencil()


def stable_dt(n: int, cfl: float = 0.5) -> float:
    """Fixed step: cfl * h / (flow speed 1 + sound speed 1/M)."""
    return cfl * (TWO_PI / n) / (1.0 + 1.0 / MACH)


def _declared(fused) -> list:
    return FIELDS_FUSEDQ + P if fused == "q" else (FIELDS_FUSED if fused else FIELDS)


def footprint_bytes(n: int, fused=False) -> int:
    """Bytes of the fields the step chains stream (the fused forms: 15)."""
    return (15 if fused else len(FIELDS)) * (n + 2 * NH) ** 3 * 8


def device_footprint_bytes(n: int, fused=False) -> int:
    """Device bytes of every declared field resident (in-core runs)."""
    pitch = ooc.row_pitch(n, NH)
    plane = pitch * (n + 2 * NH + 1)
    per = ((n + 2 * NH) * plane * 8 + 255) // 256 * 256
    return len(_declared(fused)) * per + (1 << 20)


class NS3D:
    """prims: interior arrays (rho, u, v, w, p), indexed [z, y, x]."""

    def __init__(self, n: int, prims, budget: int, flags: int = 0, re: float = 1600.0, bind: bool = True,
                 cyclic_after_init: bool = True, plan_only: bool = False, fused=False):
        """plan_only: a context without storage, for planning schedules only;
        fused: the residual evaluates the gradients itself (15 fields, no
        gradient loop) instead of reading the 12 stored gradient fields;
        fused="q": the primitives too (no primitives loop), from one copy of
        the conserved variables into the other."""
        self.n = n
        self.fused = fused
        if plan_only:
            flags |= ooc.FLAG_PLAN_ONLY
            bind = False
        self.ctx = ooc.Context(3, (n, n, n), NH, budget, flags, bind=bind)
        self.h = TWO_PI / n
        self.inv = 1.0 / (12.0 * self.h)
        self.mu = 1.0 / re
        self.kappa = self.mu / (((GAMMA - 1.0) * (MACH * MACH)) * PRANDTL)
        self.gm2 = GAMMA * (MACH * MACH)
        self.dt = stable_dt(n)
        self.f = {}
        self.cur = 0  # fused="q": 0 while Q holds the state, 1 while Q2 does
        m = n + 2 * NH
        for name in _declared(fused):
            init = None
            if name in P and not plan_only:
                init = np.zeros((m, m, m))
                init[NH:NH + n, NH:NH + n, NH:NH + n] = prims[P.index(name)]
            self.f[name] = self.ctx.decl_field(name, (0, 0, 0), init)
        self.cyclic_after_init = cyclic_after_init

    def d(self, name, access=READ, *offs):
        return dat(self.f[name], access, *offs)

    def initialise(self):
        n = self.n
        self.ctx.par_loop(K_INIT, ((0, n), (0, n), (0, n)),
                          [self.d(x) for x in P] + [self.d(x, WRITE) for x in Q])
        self.ctx.execute()
        if self.cyclic_after_init:
            self.ctx.set_flags(ooc.FLAG_CYCLIC, 0)

    def _state(self):
        return Q2 if self.cur else Q

    def _mirror_q(self, rng, off, signs=(1.0,) * 5):
        args = []
        for name in self._state():
            args += [self.d(name, WRITE), self.d(name, READ, off)]
        self.ctx.par_loop(K_MIRROR, rng, args + [Const(s) for s in signs])

    def queue_stage(self, s: int):
        n = self.n
        full = (-NH, n + NH)
        # x and y periodic strips, then z mirror walls (rho w odd) layer by layer
        self._mirror_q(((-NH, 0), (0, n), (0, n)), (n, 0, 0))
        self._mirror_q(((n, n + NH), (0, n), (0, n)), (-n, 0, 0))
        self._mirror_q((full, (-NH, 0), (0, n)), (0, n, 0))
        self._mirror_q((full, (n, n + NH), (0, n)), (0, -n, 0))
        odd = (1.0, 1.0, 1.0, -1.0, 1.0)
        for m in range(NH):
            self._mirror_q((full, full, (-1 - m, -m)), (0, 0, 2 * m + 1), odd)
            self._mirror_q((full, full, (n + m, n + m + 1)), (0, 0, -2 * m - 1), odd)
        first = s == 0
        if self.fused == "q":
            src, dst = self._state(), (Q if self.cur else Q2)
            self.ctx.par_loop(K_RHS_FUSEDQ_FIRST if first else K_RHS_FUSEDQ, ((0, n), (0, n), (0, n)),
                              [self.d(x, READ, *FUSED_STENCIL) for x in src] + [self.d(x, WRITE) for x in dst] +
                              [self.d(x, WRITE if first else RW) for x in D] +
                              [Const(self.inv), Const(self.mu), Const(self.kappa), Const(self.dt), Const(RK_A[s]),
                               Const(RK_B[s]), Const(self.gm2)])
            self.cur ^= 1
            return
        self.ctx.par_loop(K_PRIMS, (full, full, full), [self.d(x) for x in Q] + [self.d(x, WRITE) for x in P])
        if self.fused:
            self.ctx.par_loop(K_RHS_FUSED_FIRST if first else K_RHS_FUSED, ((0, n), (0, n), (0, n)),
                              [self.d(x, READ, *FUSED_STENCIL) for x in P] + [self.d(x, RW) for x in Q] +
                              [self.d(x, WRITE if first else RW) for x in D] +
                              [Const(self.inv), Const(self.mu), Const(self.kappa), Const(self.dt), Const(RK_A[s]),
                               Const(RK_B[s]), Const(self.gm2)])
            return
        g2 = (-2, n + 2)
        self.ctx.par_loop(K_GRADS, (g2, g2, g2), [self.d(x, READ, *STAR) for x in P] +
                          [self.d(x, WRITE) for x in G] + [Const(self.inv), Const(self.gm2)])
        self.ctx.par_loop(K_RHS_FIRST if first else K_RHS, ((0, n), (0, n), (0, n)),
                          [self.d(x, READ, *STAR) for x in P] + [self.d(x, READ, *STAR) for x in G] +
                          [self.d(x, RW) for x in Q] + [self.d(x, WRITE if first else RW) for x in D] +
                          [Const(self.inv), Const(self.mu), Const(self.kappa), Const(self.dt), Const(RK_A[s]),
                           Const(RK_B[s])])

    def queue_step(self):
        for s in range(3):
            self.queue_stage(s)
        self.ctx.mark_step()

    def run(self, steps: int, overlap: bool = True):
        for _ in range(steps):
            self.queue_step()
            if overlap:
                self.ctx.submit()
        self.ctx.execute()

    def interior(self, name: str) -> np.ndarray:
        if self.cur and name in Q:  # the state is in the other copy
            name = Q2[Q.index(name)]
        a = self.ctx.fetch_field(self.f[name], (0, 0, 0))
        n = self.n
        return a[NH:NH + n, NH:NH + n, NH:NH + n]

    def close(self):
        self.ctx.close()
