"""2D hydro proxy as a user of the loop-chain library: declares the 25 fields,
queues the 55 loops of one time step (lazy; nothing runs until a flush) and
leaves the time step dt on the device between chains.

Every loop is one ooc_par_loop call with explicit stencils, so the library's
dependency analysis sees exactly what each kernel reads and writes.  The step
follows a staggered-grid Lagrangian predictor-corrector plus donor-cell remap
sweeps in x then y, with reflective walls applied by strip loops (the class of
scheme the paper names for CloverLeaf 2D, Section 5.1)."""
from __future__ import annotations

import numpy as np

from . import ooc
from .ooc import READ, WRITE, RW, Const, DevScalar, Red, dat

H = 2
# kernel ids (include/ooc_kernels.h)
K_MIRROR, K_FILL, K_SUM_PROD = 1, 2, 3
(K_EOS, K_EOS_P, K_VISC, K_PDV_PRED, K_PDV_CORR, K_ACCEL, K_FLUX_X, K_FLUX_Y, K_ADV_VOL_X, K_ADV_VOL_Y,
 K_ADV_FLUX_X, K_ADV_FLUX_Y, K_ADV_CELL_X, K_ADV_CELL_Y, K_NFLUX_X, K_NFLUX_Y, K_NMASS_X, K_NMASS_Y,
 K_MFLUX_X, K_MFLUX_Y, K_VEL_X, K_VEL_Y, K_DT, K_SUMMARY) = range(100, 124)

CELL, NODE, XFACE, YFACE = (0, 0), (1, 1), (1, 0), (0, 1)
FIELDS = [  # name, centring, streamed state?
    ("rho0", CELL), ("rho1", CELL), ("e0", CELL), ("e1", CELL), ("p", CELL), ("cs", CELL), ("q", CELL),
    ("vol", CELL), ("u0", NODE), ("v0", NODE), ("u1", NODE), ("v1", NODE), ("xarea", XFACE),
    ("vfx", XFACE), ("mfx", XFACE), ("yarea", YFACE), ("vfy", YFACE), ("mfy", YFACE),
    ("w_pre", NODE), ("w_post", NODE), ("w_ef", NODE), ("w_nf", NODE), ("w_nmpost", NODE),
    ("w_nmpre", NODE), ("w_mf", NODE)]
GEOMETRY = ("vol", "xarea", "yarea")
STATE = ("rho0", "e0", "u0", "v0")           # what persists from step to step
SUMMARY = ("volume", "mass", "internal_energy", "kinetic_energy", "pressure")  # field summary sums
N4 = ((0, 0), (1, 0), (0, 1), (1, 1))        # the four nodes of a cell
C4 = ((-1, -1), (0, -1), (-1, 0), (0, 0))    # the four cells of a node


def footprint_bytes(nx: int, ny: int) -> int:
    """Bytes of all fields over their full logical extents (halo included)."""
    tot = 0
    for _, (dx, dy) in FIELDS:
        tot += (nx + 2 * H + dx) * (ny + 2 * H + dy) * 8
    return tot


def device_footprint_bytes(nx: int, ny: int, summary: bool = False) -> int:
    """Device bytes to hold every field resident in the library's padded
    layout (ooc.row_pitch elements per row), plus reduction buffers (with
    `summary`, the field summary's five sums too)."""
    pitch = ooc.row_pitch(nx, H)
    tot = 0
    for _, (dx, dy) in FIELDS:
        tot += ((ny + 2 * H + dy) * pitch * 8 + 255) // 256 * 256
    nsum = 1 + (len(SUMMARY) if summary else 0)
    return tot + 64 * 1024 + nsum * (((ny + 2 * H + 1) * 8 + 255) // 256 * 256)


def full_extent(nx, ny, centring, interior=None):
    a = np.zeros((ny + 2 * H + centring[1], nx + 2 * H + centring[0]))
    if interior is not None:
        a[H:H + interior.shape[0], H:H + interior.shape[1]] = interior
    return a


class Hydro2D:
    """Drives one 2D hydro run through the library.

    budget: device bytes for the context; flags: ooc.FLAG_*; resident_geometry
    keeps vol/xarea/yarea on the device (they are read-only after the init
    chain); resident_state keeps the geometry and the state (rho0, e0, u0, v0)
    on the device, so only the temporaries are tiled and nothing crosses the
    host link between steps."""

    def __init__(self, nx: int, ny: int, rho: np.ndarray, ene: np.ndarray, budget: int, flags: int = 0,
                 resident_geometry: bool = False, cyclic_after_init: bool = True, bind: bool = True,
                 arena_bytes: int | None = None, plan_only: bool = False, resident_state: bool = False,
                 summary: bool = False):
        self.nx, self.ny = nx, ny
        if plan_only:
            flags |= ooc.FLAG_PLAN_ONLY
            bind = False
        self.ctx = ooc.Context(2, (nx, ny), H, budget, flags, bind=bind, arena_bytes=arena_bytes)
        self.f = {}
        for name, c in FIELDS:
            init = None
            if plan_only:
                pass
            elif name == "rho0":
                init = full_extent(nx, ny, c, rho)
            elif name == "e0":
                init = full_extent(nx, ny, c, ene)
            self.f[name] = self.ctx.decl_field(name, c + (0,), init,
                                               resident=(resident_geometry and name in GEOMETRY) or
                                               (resident_state and name in GEOMETRY + STATE))
        self.centring = dict(FIELDS)
        self.dt = self.ctx.decl_reduction(ooc.RED_MIN)
        self.mass = self.ctx.decl_reduction(ooc.RED_SUM)
        # the field summary's five order-fixed sums (declared on request)
        self.summary_reds = [self.ctx.decl_reduction(ooc.RED_SUM) for _ in SUMMARY] if summary else []
        self.cyclic_after_init = cyclic_after_init
        self.steps_queued = 0

    # ------------------------------------------------------------- helpers
    def _mirror(self, pairs, rng):
        """pairs: (dst, src, sign, (ox, oy)) -- dst = sign * src(p + o)."""
        args, consts = [], []
        for dst, src, sign, off in pairs:
            args += [dat(self.f[dst], WRITE), dat(self.f[src], READ, off)]
            consts.append(Const(sign))
        self.ctx.par_loop(K_MIRROR, rng, args + consts)

    def _loop(self, kid, rng, *args):
        self.ctx.par_loop(kid, rng, list(args))

    def d(self, name, access=READ, *offs):
        return dat(self.f[name], access, *offs)

    # --------------------------------------------------------------- chains
    def queue_init(self):
        """Init chain: geometry of the uniform mesh, then the first dt."""
        nx, ny = self.nx, self.ny
        dx, dy = 1.0 / nx, 1.0 / ny
        self._loop(K_FILL, ((-H, nx + H), (-H, ny + H)), self.d("vol", WRITE), Const(dx * dy))
        self._loop(K_FILL, ((-H, nx + H + 1), (-H, ny + H)), self.d("xarea", WRITE), Const(dy))
        self._loop(K_FILL, ((-H, nx + H), (-H, ny + H + 1)), self.d("yarea", WRITE), Const(dx))
        self._queue_dt()

    def initialise(self) -> float:
        """Run the init chain; afterwards temporaries may skip downloads."""
        self.queue_init()
        dt = self.ctx.reduce(self.dt)
        if self.cyclic_after_init:
            self.ctx.set_flags(ooc.FLAG_CYCLIC, 0)
        return dt

    def _queue_dt(self):
        nx, ny = self.nx, self.ny
        self._loop(K_DT, ((0, nx), (0, ny)), self.d("e0"), self.d("u0", READ, *N4), self.d("v0", READ, *N4),
                   Const(1.0 / nx), Const(1.0 / ny), Red(self.dt))

    def _bc_state(self):
        nx, ny = self.nx, self.ny
        cells = lambda off: [("rho0", "rho0", 1.0, off), ("e0", "e0", 1.0, off)]
        nodes_y = lambda off: [("u0", "u0", 1.0, off), ("v0", "v0", -1.0, off)]
        nodes_x = lambda off: [("u0", "u0", -1.0, off), ("v0", "v0", 1.0, off)]
        for k in (0, 1):
            self._mirror(cells((0, 2 * k + 1)), ((-H, nx + H), (-1 - k, -k)))
            self._mirror(cells((0, -2 * k - 1)), ((-H, nx + H), (ny + k, ny + k + 1)))
        for k in (1, 2):
            self._mirror(nodes_y((0, 2 * k)), ((-H, nx + H + 1), (-k, -k + 1)))
            self._mirror(nodes_y((0, -2 * k)), ((-H, nx + H + 1), (ny + k, ny + k + 1)))
        for k in (0, 1):
            self._mirror(cells((2 * k + 1, 0)), ((-1 - k, -k), (-H, ny + H)))
            self._mirror(cells((-2 * k - 1, 0)), ((nx + k, nx + k + 1), (-H, ny + H)))
        for k in (1, 2):
            self._mirror(nodes_x((2 * k, 0)), ((-k, -k + 1), (-H, ny + H + 1)))
            self._mirror(nodes_x((-2 * k, 0)), ((nx + k, nx + k + 1), (-H, ny + H + 1)))

    def queue_step(self):
        """Queue one time step (55 loops); the last loop min-reduces the next dt."""
        nx, ny = self.nx, self.ny
        d, L = self.d, self._loop
        dt = DevScalar(self.dt)
        full_c = ((-H, nx + H), (-H, ny + H))
        self._bc_state()
        # ---- Lagrangian phase
        L(K_EOS, full_c, d("rho0"), d("e0"), d("p", WRITE), d("cs", WRITE))
        L(K_VISC, full_c, d("rho0"), d("cs"), d("u0", READ, *N4), d("v0", READ, *N4), d("q", WRITE))
        L(K_PDV_PRED, full_c, d("rho0"), d("e0"), d("p"), d("q"), d("vol"), d("xarea", READ, (0, 0), (1, 0)),
          d("yarea", READ, (0, 0), (0, 1)), d("u0", READ, *N4), d("v0", READ, *N4), d("rho1", WRITE),
          d("e1", WRITE), dt)
        L(K_EOS_P, full_c, d("rho1"), d("e1"), d("p", WRITE))
        L(K_ACCEL, ((-1, nx + H), (-1, ny + H)), d("rho0", READ, *C4), d("vol", READ, *C4), d("p", READ, *C4),
          d("q", READ, *C4), d("xarea", READ, (0, -1), (0, 0)), d("yarea", READ, (-1, 0), (0, 0)), d("u0"),
          d("v0"), d("u1", WRITE), d("v1", WRITE), Const(nx), Const(ny), dt)
        L(K_PDV_CORR, ((-1, nx + 1), (-1, ny + 1)), d("rho0"), d("e0"), d("p"), d("q"), d("vol"),
          d("xarea", READ, (0, 0), (1, 0)), d("yarea", READ, (0, 0), (0, 1)), d("u0", READ, *N4),
          d("v0", READ, *N4), d("u1", READ, *N4), d("v1", READ, *N4), d("rho1", WRITE), d("e1", WRITE), dt)
        L(K_FLUX_X, ((-1, nx + 2), (-1, ny + 1)), d("xarea"), d("u0", READ, (0, 0), (0, 1)),
          d("u1", READ, (0, 0), (0, 1)), d("vfx", WRITE), dt)
        L(K_FLUX_Y, ((-1, nx + 1), (-1, ny + 2)), d("yarea"), d("v0", READ, (0, 0), (1, 0)),
          d("v1", READ, (0, 0), (1, 0)), d("vfy", WRITE), dt)
        # ---- remap, x sweep
        L(K_ADV_VOL_X, ((-1, nx + 1), (-1, ny + 1)), d("vol"), d("vfx", READ, (0, 0), (1, 0)),
          d("vfy", READ, (0, 0), (0, 1)), d("w_pre", WRITE), d("w_post", WRITE))
        L(K_ADV_FLUX_X, ((0, nx + 1), (-1, ny + 1)), d("vfx"), d("rho1", READ, (-1, 0), (0, 0)),
          d("e1", READ, (-1, 0), (0, 0)), d("mfx", WRITE), d("w_ef", WRITE))
        L(K_ADV_CELL_X, ((0, nx), (-1, ny + 1)), d("rho1", RW), d("e1", RW), d("w_pre"), d("w_post"),
          d("mfx", READ, (0, 0), (1, 0)), d("w_ef", READ, (0, 0), (1, 0)))
        self._mirror([("rho1", "rho1", 1.0, (1, 0)), ("e1", "e1", 1.0, (1, 0))], ((-1, 0), (-1, ny + 1)))
        self._mirror([("rho1", "rho1", 1.0, (-1, 0)), ("e1", "e1", 1.0, (-1, 0))], ((nx, nx + 1), (-1, ny + 1)))
        self._mirror([("mfx", "mfx", -1.0, (2, 0))], ((-1, 0), (-1, ny + 1)))
        self._mirror([("mfx", "mfx", -1.0, (-2, 0))], ((nx + 1, nx + 2), (-1, ny + 1)))
        L(K_NFLUX_X, ((-1, nx + 1), (0, ny + 1)), d("mfx", READ, (0, -1), (0, 0), (1, -1), (1, 0)),
          d("w_nf", WRITE))
        nodes = ((0, nx + 1), (0, ny + 1))
        L(K_NMASS_X, nodes, d("rho1", READ, *C4), d("w_post", READ, *C4), d("w_nf", READ, (-1, 0), (0, 0)),
          d("w_nmpost", WRITE), d("w_nmpre", WRITE))
        for vel in ("u1", "v1"):
            L(K_MFLUX_X, ((-1, nx + 1), (0, ny + 1)), d("w_nf"), d(vel, READ, (0, 0), (1, 0)), d("w_mf", WRITE))
            L(K_VEL_X, nodes, d(vel, RW), d("w_nmpre"), d("w_nmpost"), d("w_mf", READ, (-1, 0), (0, 0)))
        self._mirror([("u1", "u1", 1.0, (0, 2)), ("v1", "v1", -1.0, (0, 2))], ((0, nx + 1), (-1, 0)))
        self._mirror([("u1", "u1", 1.0, (0, -2)), ("v1", "v1", -1.0, (0, -2))], ((0, nx + 1), (ny + 1, ny + 2)))
        # ---- remap, y sweep
        L(K_ADV_VOL_Y, ((-1, nx + 1), (-1, ny + 1)), d("vol"), d("vfy", READ, (0, 0), (0, 1)),
          d("w_pre", WRITE), d("w_post", WRITE))
        L(K_ADV_FLUX_Y, ((-1, nx + 1), (0, ny + 1)), d("vfy"), d("rho1", READ, (0, -1), (0, 0)),
          d("e1", READ, (0, -1), (0, 0)), d("mfy", WRITE), d("w_ef", WRITE))
        L(K_ADV_CELL_Y, ((-1, nx + 1), (0, ny)), d("rho1", RW), d("e1", RW), d("w_pre"), d("w_post"),
          d("mfy", READ, (0, 0), (0, 1)), d("w_ef", READ, (0, 0), (0, 1)))
        self._mirror([("rho1", "rho1", 1.0, (0, 1))], ((-1, nx + 1), (-1, 0)))
        self._mirror([("rho1", "rho1", 1.0, (0, -1))], ((-1, nx + 1), (ny, ny + 1)))
        self._mirror([("mfy", "mfy", -1.0, (0, 2))], ((-1, nx + 1), (-1, 0)))
        self._mirror([("mfy", "mfy", -1.0, (0, -2))], ((-1, nx + 1), (ny + 1, ny + 2)))
        L(K_NFLUX_Y, ((0, nx + 1), (-1, ny + 1)), d("mfy", READ, (-1, 0), (0, 0), (-1, 1), (0, 1)),
          d("w_nf", WRITE))
        L(K_NMASS_Y, nodes, d("rho1", READ, *C4), d("w_post", READ, *C4), d("w_nf", READ, (0, -1), (0, 0)),
          d("w_nmpost", WRITE), d("w_nmpre", WRITE))
        for vel in ("u1", "v1"):
            L(K_MFLUX_Y, ((0, nx + 1), (-1, ny + 1)), d("w_nf"), d(vel, READ, (0, 0), (0, 1)), d("w_mf", WRITE))
            L(K_VEL_Y, nodes, d(vel, RW), d("w_nmpre"), d("w_nmpost"), d("w_mf", READ, (0, -1), (0, 0)))
        # ---- the remapped state becomes the new state; next time step
        self._mirror([("rho0", "rho1", 1.0, (0, 0)), ("e0", "e1", 1.0, (0, 0))], ((0, nx), (0, ny)))
        self._mirror([("u0", "u1", 1.0, (0, 0)), ("v0", "v1", 1.0, (0, 0))], nodes)
        self._queue_dt()
        self.ctx.mark_step()
        self.steps_queued += 1

    def queue_mass(self):
        """Field summary: order-fixed sum of rho0 * vol over the interior.
        Queued after a step and before the flush, it joins that step's chain
        (its reduction is not read in the chain) and moves no extra bytes;
        queued alone it is a chain of its own that uploads rho0 and vol."""
        self._loop(K_SUM_PROD, ((0, self.nx), (0, self.ny)), self.d("rho0"), self.d("vol"), Red(self.mass))

    def queue_summary(self):
        """Field summary of the state: volume, mass, internal energy, kinetic
        energy and pressure summed over the interior in one loop (the periodic
        diagnostic whose separate chain the paper names as a cause of its
        CloverLeaf 2D gap, Section 5.3).  Queued after a step and before the
        flush, it joins that step's chain like queue_mass; read the sums with
        summary().  Needs summary=True at construction."""
        if not self.summary_reds:
            raise ValueError("construct with summary=True to queue the field summary")
        self._loop(K_SUMMARY, ((0, self.nx), (0, self.ny)), self.d("vol"), self.d("rho0"), self.d("e0"),
                   self.d("u0", READ, *N4), self.d("v0", READ, *N4), *[Red(r) for r in self.summary_reds])

    def summary(self) -> np.ndarray:
        """The committed field-summary sums, in SUMMARY order (flushes)."""
        return np.array([self.ctx.reduce(r) for r in self.summary_reds])

    # ---------------------------------------------------------------- driver
    def run(self, steps: int, overlap: bool = True):
        """Advance `steps` steps.  With overlap, each step is issued as soon as
        it is queued (ooc_submit), so the host queues step n+1 while the device
        runs step n; the call returns when the device is done."""
        for _ in range(steps):
            self.queue_step()
            if overlap:
                self.ctx.submit()
        self.ctx.execute()

    def fetch(self, name: str) -> np.ndarray:
        return self.ctx.fetch_field(self.f[name], self.centring[name] + (0,))

    def interior(self, name: str) -> np.ndarray:
        a = self.fetch(name)
        c = self.centring[name]
        return a[H:H + self.ny + c[1], H:H + self.nx + c[0]]

    def close(self):
        self.ctx.close()
