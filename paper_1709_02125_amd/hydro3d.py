"""3D hydro proxy as a user of the loop-chain library: 30 fields, 82 loops per
time step (24 reflective-wall strips for the state, 6 Lagrangian loops, 3
face fluxes, 46 loops of the x, y and z remap sweeps, 2 copies and the dt
reduction), tiled along z.  The three-dimensional form of the 2D proxy, as the
paper's CloverLeaf 3D is of CloverLeaf 2D (Section 5.1)."""
from __future__ import annotations

import itertools

import numpy as np

from . import ooc
from .ooc import READ, WRITE, RW, Const, DevScalar, Red, dat

H = 2
K_MIRROR, K_FILL, K_SUM_PROD = 1, 2, 3
K_EOS, K_EOS_P = 100, 101
K_VISC, K_PDV_PRED, K_PDV_CORR, K_ACCEL = 300, 301, 302, 303
K_FLUX = (304, 305, 306)
K_ADV_VOL = (307, 308, 309)
K_ADV_FLUX = (310, 311, 312)
K_ADV_CELL = (313, 314, 315)
K_NFLUX = (316, 317, 318)
K_NMASS = (319, 320, 321)
K_MFLUX = (322, 323, 324)
K_VEL = (325, 326, 327)
K_DT = 328

CELL, NODE = (0, 0, 0), (1, 1, 1)
FACE = ((1, 0, 0), (0, 1, 0), (0, 0, 1))
FIELDS = [
    ("rho0", CELL), ("rho1", CELL), ("e0", CELL), ("e1", CELL), ("p", CELL), ("cs", CELL), ("q", CELL),
    ("vol", CELL), ("u0", NODE), ("v0", NODE), ("w0", NODE), ("u1", NODE), ("v1", NODE), ("w1", NODE),
    ("xarea", FACE[0]), ("vfx", FACE[0]), ("mfx", FACE[0]),
    ("yarea", FACE[1]), ("vfy", FACE[1]), ("mfy", FACE[1]),
    ("zarea", FACE[2]), ("vfz", FACE[2]), ("mfz", FACE[2]),
    ("w_pre", NODE), ("w_post", NODE), ("w_ef", NODE), ("w_nf", NODE), ("w_nmpost", NODE),
    ("w_nmpre", NODE), ("w_mf", NODE)]
GEOMETRY = ("vol", "xarea", "yarea", "zarea")
STATE = ("rho0", "e0", "u0", "v0", "w0")     # what persists from step to step
VEL0, VEL1 = ("u0", "v0", "w0"), ("u1", "v1", "w1")
AREA, VF, MF = ("xarea", "yarea", "zarea"), ("vfx", "vfy", "vfz"), ("mfx", "mfy", "mfz")
N8 = tuple(itertools.product((0, 1), repeat=3))          # the 8 nodes of a cell
C8 = tuple(itertools.product((-1, 0), repeat=3))         # the 8 cells of a node


def unit(a, s=1):
    o = [0, 0, 0]
    o[a] = s
    return tuple(o)


def face_nodes(a, e=0):
    """The 4 nodes of a cell's face normal to axis a, at offset e along a."""
    out = []
    for p, q in itertools.product((0, 1), repeat=2):
        o = [p, q]
        o.insert(a, e)
        out.append(tuple(o))
    return tuple(out)


def footprint_bytes(n) -> int:
    tot = 0
    for _, c in FIELDS:
        tot += int(np.prod([n[a] + 2 * H + c[a] for a in range(3)])) * 8
    return tot


def device_footprint_bytes(n) -> int:
    pitch = ooc.row_pitch(n[0], H)
    plane = pitch * (n[1] + 2 * H + 1)
    tot = 0
    for _, c in FIELDS:
        tot += ((n[2] + 2 * H + c[2]) * plane * 8 + 255) // 256 * 256
    # reduction buffers, and the SUM reduction's partials (one per y-z row)
    return tot + 64 * 1024 + ((n[1] + 2 * H + 1) * (n[2] + 2 * H + 1) * 8 + 255) // 256 * 256


def full_extent(n, centring, interior=None):
    a = np.zeros(tuple(n[ax] + 2 * H + centring[ax] for ax in (2, 1, 0)))
    if interior is not None:
        a[H:H + interior.shape[0], H:H + interior.shape[1], H:H + interior.shape[2]] = interior
    return a


class Hydro3D:
    """Drives one 3D hydro run through the library (arguments as the 2D
    proxy's: budget in device bytes, flags ooc.FLAG_*, resident_geometry keeps
    the read-only vol and face areas on the device, resident_state keeps the
    geometry and the state so only the temporaries are tiled)."""

    def __init__(self, n, rho: np.ndarray, ene: np.ndarray, budget: int, flags: int = 0,
                 resident_geometry: bool = False, cyclic_after_init: bool = True, bind: bool = True,
                 arena_bytes: int | None = None, plan_only: bool = False, resident_state: bool = False):
        self.n = tuple(n)
        if plan_only:
            flags |= ooc.FLAG_PLAN_ONLY
            bind = False
        self.ctx = ooc.Context(3, self.n, H, budget, flags, bind=bind, arena_bytes=arena_bytes)
        self.f = {}
        for name, c in FIELDS:
            init = None
            if not plan_only and name == "rho0":
                init = full_extent(self.n, c, rho)
            elif not plan_only and name == "e0":
                init = full_extent(self.n, c, ene)
            res = (resident_geometry and name in GEOMETRY) or (resident_state and name in GEOMETRY + STATE)
            self.f[name] = self.ctx.decl_field(name, c, init, resident=res)
        self.centring = dict(FIELDS)
        self.dt = self.ctx.decl_reduction(ooc.RED_MIN)
        self.mass = self.ctx.decl_reduction(ooc.RED_SUM)
        self.cyclic_after_init = cyclic_after_init

    def d(self, name, access=READ, *offs):
        return dat(self.f[name], access, *offs)

    def _loop(self, kid, rng, *args):
        self.ctx.par_loop(kid, rng, list(args))

    def _mirror(self, pairs, rng):
        """pairs: (dst, src, sign, offset): dst = sign * src(p + offset)."""
        args, consts = [], []
        for dst, src, sign, off in pairs:
            args += [dat(self.f[dst], WRITE), dat(self.f[src], READ, off)]
            consts.append(Const(sign))
        self.ctx.par_loop(K_MIRROR, rng, args + consts)

    def _box(self, lo, hi):
        return tuple((lo[a], hi[a]) for a in range(3))

    # --------------------------------------------------------------- chains
    def queue_init(self):
        n = self.n
        dx, dy, dz = (1.0 / n[0], 1.0 / n[1], 1.0 / n[2])
        for name, val in (("vol", (dx * dy) * dz), ("xarea", dy * dz), ("yarea", dx * dz), ("zarea", dx * dy)):
            c = self.centring[name]
            self._loop(K_FILL, tuple((-H, n[a] + H + c[a]) for a in range(3)), self.d(name, WRITE), Const(val))
        self._queue_dt()

    def initialise(self) -> float:
        self.queue_init()
        dt = self.ctx.reduce(self.dt)
        if self.cyclic_after_init:
            self.ctx.set_flags(ooc.FLAG_CYCLIC, 0)
        return dt

    def _queue_dt(self):
        n = self.n
        self._loop(K_DT, ((0, n[0]), (0, n[1]), (0, n[2])), self.d("e0"),
                   *[self.d(v, READ, *N8) for v in VEL0],
                   Const(1.0 / n[0]), Const(1.0 / n[1]), Const(1.0 / n[2]), Red(self.dt))

    def _walls(self, a, names, signs, node, lo, hi):
        """Reflection of fields about both walls of axis a, layer by layer
        (cell-centred: cell -1-m <- m; node-centred: node -m <- m)."""
        n = self.n[a]
        for m in ((1, 2) if node else (0, 1)):
            for low in (True, False):
                l, h = list(lo), list(hi)
                if low:
                    l[a] = -m if node else -1 - m
                    o = 2 * m if node else 2 * m + 1
                else:
                    l[a] = n + m
                    o = -2 * m if node else -2 * m - 1
                h[a] = l[a] + 1
                self._mirror([(f, f, s, unit(a, o)) for f, s in zip(names, signs)], self._box(l, h))

    def _bc_state(self):
        n = self.n
        for a in range(3):
            lo, hic, hin = [0, 0, 0], list(n), [x + 1 for x in n]
            for b in range(a):
                lo[b], hic[b], hin[b] = -H, n[b] + H, n[b] + H + 1
            self._walls(a, ("rho0", "e0"), (1.0, 1.0), False, lo, hic)
            self._walls(a, VEL0, tuple(-1.0 if c == a else 1.0 for c in range(3)), True, lo, hin)

    def queue_step(self):
        n = self.n
        d, L = self.d, self._loop
        dt = DevScalar(self.dt)
        self._bc_state()
        # ---- Lagrangian phase
        full_c = tuple((-H, n[a] + H) for a in range(3))
        geo = [d("vol")] + [d(AREA[a], READ, (0, 0, 0), unit(a)) for a in range(3)]
        L(K_EOS, full_c, d("rho0"), d("e0"), d("p", WRITE), d("cs", WRITE))
        L(K_VISC, full_c, d("rho0"), d("cs"), *[d(v, READ, *N8) for v in VEL0], d("q", WRITE))
        L(K_PDV_PRED, full_c, d("rho0"), d("e0"), d("p"), d("q"), *geo, *[d(v, READ, *N8) for v in VEL0],
          d("rho1", WRITE), d("e1", WRITE), dt)
        L(K_EOS_P, full_c, d("rho1"), d("e1"), d("p", WRITE))
        nodes_acc = tuple((-1, n[a] + H) for a in range(3))
        face_cells = [tuple(o) for o in itertools.product((-1, 0), repeat=2)]

        def area_st(a):
            out = []
            for p, q in face_cells:
                o = [p, q]
                o.insert(a, 0)
                out.append(tuple(o))
            return tuple(out)
        L(K_ACCEL, nodes_acc, *[d(f, READ, *C8) for f in ("rho0", "vol", "p", "q")],
          *[d(AREA[a], READ, *area_st(a)) for a in range(3)], *[d(v) for v in VEL0],
          *[d(v, WRITE) for v in VEL1], Const(n[0]), Const(n[1]), Const(n[2]), dt)
        L(K_PDV_CORR, tuple((-1, n[a] + 1) for a in range(3)), d("rho0"), d("e0"), d("p"), d("q"), *geo,
          *[d(v, READ, *N8) for v in VEL0], *[d(v, READ, *N8) for v in VEL1], d("rho1", WRITE), d("e1", WRITE), dt)
        for a in range(3):
            hi = [n[b] + 1 for b in range(3)]
            hi[a] = n[a] + 2
            L(K_FLUX[a], self._box((-1, -1, -1), hi), d(AREA[a]), d(VEL0[a], READ, *face_nodes(a)),
              d(VEL1[a], READ, *face_nodes(a)), d(VF[a], WRITE), dt)
        # ---- remap sweeps x, y, z
        ring = self._box((-1, -1, -1), [n[b] + 1 for b in range(3)])
        for s in range(3):
            e, me = unit(s), unit(s, -1)
            if s == 0:
                L(K_ADV_VOL[0], ring, d("vol"), *[d(VF[a], READ, (0, 0, 0), unit(a)) for a in range(3)],
                  d("w_pre", WRITE), d("w_post", WRITE))
            elif s == 1:
                L(K_ADV_VOL[1], ring, d("vol"), *[d(VF[a], READ, (0, 0, 0), unit(a)) for a in (1, 2)],
                  d("w_pre", WRITE), d("w_post", WRITE))
            else:
                L(K_ADV_VOL[2], ring, d("vol"), d(VF[2], READ, (0, 0, 0), unit(2)), d("w_pre", WRITE),
                  d("w_post", WRITE))
            flo, fhi = [-1, -1, -1], [n[b] + 1 for b in range(3)]
            flo[s] = 0
            L(K_ADV_FLUX[s], self._box(flo, fhi), d(VF[s]), d("rho1", READ, me, (0, 0, 0)),
              d("e1", READ, me, (0, 0, 0)), d(MF[s], WRITE), d("w_ef", WRITE))
            clo, chi = [-1, -1, -1], [n[b] + 1 for b in range(3)]
            clo[s], chi[s] = 0, n[s]
            L(K_ADV_CELL[s], self._box(clo, chi), d("rho1", RW), d("e1", RW), d("w_pre"), d("w_post"),
              d(MF[s], READ, (0, 0, 0), e), d("w_ef", READ, (0, 0, 0), e))
            # density of the swept cells beyond the walls normal to s; odd face
            # mass flux beyond them
            lo, hi = [-1, -1, -1], [n[b] + 1 for b in range(3)]
            lo[s], hi[s] = -1, 0
            self._mirror([("rho1", "rho1", 1.0, e), (MF[s], MF[s], -1.0, unit(s, 2))], self._box(lo, hi))
            lo[s], hi[s] = n[s], n[s] + 1
            self._mirror([("rho1", "rho1", 1.0, me)], self._box(lo, hi))
            lo[s], hi[s] = n[s] + 1, n[s] + 2
            self._mirror([(MF[s], MF[s], -1.0, unit(s, -2))], self._box(lo, hi))
            # momentum on the dual mesh
            dlo, dhi = [0, 0, 0], [n[b] + 1 for b in range(3)]
            dlo[s] = -1
            dual = self._box(dlo, dhi)
            B, C = (1, 2) if s == 0 else ((0, 2) if s == 1 else (0, 1))
            nf_st = []
            for ee in (0, 1):
                for y in (0, 1):
                    for x in (0, 1):
                        o = [0, 0, 0]
                        o[s], o[B], o[C] = ee, -(1 - x), -(1 - y)
                        nf_st.append(tuple(o))
            L(K_NFLUX[s], dual, d(MF[s], READ, *nf_st), d("w_nf", WRITE))
            nodes = self._box((0, 0, 0), [n[b] + 1 for b in range(3)])
            L(K_NMASS[s], nodes, d("rho1", READ, *C8), d("w_post", READ, *C8), d("w_nf", READ, me, (0, 0, 0)),
              d("w_nmpost", WRITE), d("w_nmpre", WRITE))
            for vel in VEL1:
                L(K_MFLUX[s], dual, d("w_nf"), d(vel, READ, (0, 0, 0), e), d("w_mf", WRITE))
                L(K_VEL[s], nodes, d(vel, RW), d("w_nmpre"), d("w_nmpost"), d("w_mf", READ, me, (0, 0, 0)))
            if s < 2:
                a = s + 1
                signs = [-1.0 if c == a else 1.0 for c in range(3)]
                lo, hi = [0, 0, 0], [n[b] + 1 for b in range(3)]
                lo[a], hi[a] = -1, 0
                self._mirror([(v, v, sg, unit(a, 2)) for v, sg in zip(VEL1, signs)], self._box(lo, hi))
                lo[a], hi[a] = n[a] + 1, n[a] + 2
                self._mirror([(v, v, sg, unit(a, -2)) for v, sg in zip(VEL1, signs)], self._box(lo, hi))
        # ---- the remapped state becomes the new state; next time step
        cells = self._box((0, 0, 0), n)
        self._mirror([("rho0", "rho1", 1.0, (0, 0, 0)), ("e0", "e1", 1.0, (0, 0, 0))], cells)
        self._mirror([(v0, v1, 1.0, (0, 0, 0)) for v0, v1 in zip(VEL0, VEL1)],
                     self._box((0, 0, 0), [x + 1 for x in n]))
        self._queue_dt()
        self.ctx.mark_step()

    def queue_mass(self):
        """Field summary: order-fixed sum of rho0 * vol over the interior;
        queued after a step, before the flush, it joins that step's chain."""
        n = self.n
        self._loop(K_SUM_PROD, ((0, n[0]), (0, n[1]), (0, n[2])), self.d("rho0"), self.d("vol"), Red(self.mass))

    def run(self, steps: int, overlap: bool = True):
        for _ in range(steps):
            self.queue_step()
            if overlap:
                self.ctx.submit()
        self.ctx.execute()

    def fetch(self, name: str) -> np.ndarray:
        return self.ctx.fetch_field(self.f[name], self.centring[name])

    def interior(self, name: str) -> np.ndarray:
        a = self.fetch(name)
        c = self.centring[name]
        n = self.n
        return a[H:H + n[2] + c[2], H:H + n[1] + c[1], H:H + n[0] + c[0]]

    def close(self):
        self.ctx.close()
