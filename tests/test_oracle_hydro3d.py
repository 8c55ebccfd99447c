"""Pins of the 3D hydro oracle against facts that do not come from it: exact
invariants (a gas at rest, conservation, mirror symmetry), the exact Riemann
solution of a shock tube along the tiled axis, and reduction to the pinned 2D
oracle for problems that do not vary along one axis (each pair of axes in
turn, so the x, y and z forms of every loop are checked)."""
import math

import numpy as np
import pytest

import oracle.hydro2d as h2
import oracle.hydro3d as h3
import riemann
from paper_1709_02125_amd.inputs import hydro_initial_state, mirror_symmetrise

H = 2


def _blobs(n):
    o = h3.Hydro3D(*n)
    r, e = hydro_initial_state(n)
    o.set_state(r, e)
    return o


def test_uniform_state_is_preserved_bit_exactly():
    n = (12, 10, 9)
    o = h3.Hydro3D(*n)
    shape = n[::-1]
    o.set_state(np.full(shape, 0.2), np.full(shape, 1.0))
    used, nxt = o.run(6)
    assert np.all(o.interior("rho0") == 0.2)
    assert np.all(o.interior("e0") == 1.0)
    for v in ("u0", "v0", "w0"):
        assert np.all(o.interior(v, True) == 0.0)
    # closed form at rest: CFL * (smallest spacing) / sqrt(gamma (gamma-1) e)
    expect = 0.5 * (1.0 / max(n)) / math.sqrt(1.4 * 0.4 * 1.0)
    assert all(abs(d - expect) <= 1e-15 * expect for d in used + [nxt])


def test_mass_is_conserved_in_reflective_box():
    o = _blobs((20, 18, 16))
    m0 = o.sum_cells("rho0")
    o.run(6)
    assert abs(o.sum_cells("rho0") - m0) <= 1e-13 * m0


def test_internal_energy_total_is_conserved_by_remap():
    # the remap moves rho e between cells in flux form inside a closed box
    n = (16, 14, 12)
    o = _blobs(n)
    o.run(3)
    dt = o.dt()
    o.lagrangian(dt)
    nx, ny, nz = n
    ie_lag = (o.field("rho0") * o.field("vol") * o.field("e1"))[H:H + nz, H:H + ny, H:H + nx].sum()
    o2 = _blobs(n)
    o2.run(3)
    o2.step(dt)
    ie_after = o2.sum_cells("e0", times_rho0=True)
    assert abs(ie_after - ie_lag) <= 1e-12 * ie_lag


def _energies(o, ene, vel):
    nx, ny, nz = o.n
    F = o.field
    rv = F("rho0") * F("vol")
    ie = (rv * F(ene))[H:H + nz, H:H + ny, H:H + nx].sum()
    m = np.zeros((nz + 1, ny + 1, nx + 1))
    for c in (0, 1):
        for b in (0, 1):
            for a in (0, 1):
                m += rv[H - 1 + c:H + nz + c, H - 1 + b:H + ny + b, H - 1 + a:H + nx + a]
    m *= 0.125
    w = np.ones_like(m)
    for ax in range(3):
        sl = [slice(None)] * 3
        sl[ax] = 0
        w[tuple(sl)] *= 0.5
        sl[ax] = -1
        w[tuple(sl)] *= 0.5
    sq = sum(F(v)[H:H + nz + 1, H:H + ny + 1, H:H + nx + 1] ** 2 for v in vel)
    return ie, (w * 0.5 * m * sq).sum()


def test_lagrangian_phase_conserves_total_energy():
    # the node force is the adjoint of the cell volume-change operator, so the
    # PdV work taken from internal energy is the kinetic energy gained (a node
    # on a wall counts half per wall: the box is its own mirror image)
    o = _blobs((16, 14, 12))
    _, dt = o.run(3)
    o.lagrangian(dt)
    ie0, ke0 = _energies(o, "e0", ("u0", "v0", "w0"))
    ie1, ke1 = _energies(o, "e1", ("u1", "v1", "w1"))
    assert abs(ke1 - ke0) > 1e-3 * (ie0 + ke0)
    assert abs((ie1 + ke1) - (ie0 + ke0)) <= 1e-13 * (ie0 + ke0)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_mirror_symmetry(axis):
    n = (18, 16, 14)
    r, e = hydro_initial_state(n)
    flip = 2 - axis   # numpy axis of mesh axis `axis` in [z, y, x] arrays
    r = mirror_symmetrise(r, flip)
    e = mirror_symmetrise(e, flip)
    o = h3.Hydro3D(*n)
    o.set_state(r, e)
    o.run(5)
    rho, ene = o.interior("rho0"), o.interior("e0")
    assert np.abs(rho - np.flip(rho, flip)).max() <= 1e-12 * np.abs(rho).max()
    assert np.abs(ene - np.flip(ene, flip)).max() <= 1e-12 * np.abs(ene).max()
    vel = [o.interior(v, True) for v in ("u0", "v0", "w0")]
    vs = max(np.abs(v).max() for v in vel)
    assert vs > 1e-3
    for c, v in enumerate(vel):
        sign = -1.0 if c == axis else 1.0
        assert np.abs(v - sign * np.flip(v, flip)).max() <= 1e-12 * vs


# plane (a, b) of the 3D mesh that carries the 2D problem; the third axis is
# invariant with 4 cells (a power of two keeps its spacing exact)
PLANES = {"xy": (0, 1), "xz": (0, 2), "yz": (1, 2)}


@pytest.mark.parametrize("plane", list(PLANES))
def test_reduces_to_2d_oracle_on_invariant_axis(plane):
    a, b = PLANES[plane]
    n2 = (24, 20)
    n3 = [4, 4, 4]
    n3[a], n3[b] = n2
    r2, e2 = hydro_initial_state(n2)          # indexed [y2, x2]
    o2 = h2.Hydro2D(*n2)
    o2.set_state(r2, e2)
    o3 = h3.Hydro3D(*n3)
    # 3D arrays are [z, y, x]; put 2D x2 on mesh axis a and y2 on mesh axis b
    def lift(f2):
        f = f2.T                               # [x2, y2]
        shape3 = [1, 1, 1]
        shape3[2 - a], shape3[2 - b] = f.shape
        f = f if (2 - a) < (2 - b) else f.T
        reps = [n3[2], n3[1], n3[0]]
        reps[2 - a] = reps[2 - b] = 1
        return np.tile(f.reshape(shape3), reps)
    o3.set_state(lift(r2), lift(e2))
    vel3 = ("u0", "v0", "w0")
    dt = o2.dt()
    assert abs(o3.dt() - dt) <= 1e-15 * dt
    for _ in range(8):
        nd2 = o2.step(dt)
        nd3 = o3.step(dt)
        assert abs(nd3 - nd2) <= 1e-12 * nd2
        dt = nd2
    for name in ("rho0", "e0"):
        ref = lift(o2.interior(name))
        got = o3.interior(name)
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    def lift_node(f2):
        f = f2.T
        shape3 = [1, 1, 1]
        shape3[2 - a], shape3[2 - b] = f.shape
        f = f if (2 - a) < (2 - b) else f.T
        reps = [n3[2] + 1, n3[1] + 1, n3[0] + 1]
        reps[2 - a] = reps[2 - b] = 1
        return np.tile(f.reshape(shape3), reps)
    u2, v2 = lift_node(o2.interior("u0", True)), lift_node(o2.interior("v0", True))
    vs = max(np.abs(u2).max(), np.abs(v2).max())
    assert vs > 1e-3
    assert np.abs(o3.interior(vel3[a], True) - u2).max() <= 1e-12 * vs
    assert np.abs(o3.interior(vel3[b], True) - v2).max() <= 1e-12 * vs
    third = 3 - a - b
    assert np.abs(o3.interior(vel3[third], True)).max() == 0.0


def test_shock_tube_along_tiled_axis_matches_exact_riemann_solution():
    nz, m, T = 100, 3, 0.2
    o = h3.Hydro3D(m, m, nz)
    z = (np.arange(nz) + 0.5) / nz
    rho = np.where(z < 0.5, 1.0, 0.125)
    pre = np.where(z < 0.5, 1.0, 0.1)
    o.set_state(np.tile(rho[:, None, None], (1, m, m)), np.tile((pre / (0.4 * rho))[:, None, None], (1, m, m)))
    t, dt = 0.0, o.dt()
    while t < T - 1e-14:
        dt = min(dt, T - t)
        nd = o.step(dt)
        t += dt
        dt = nd
    ex = riemann.sample(z, T, 0.5, (1.0, 0.0, 1.0), (0.125, 0.0, 0.1))
    r = o.interior("rho0")
    assert np.abs(r - r[:, :1, :1]).max() == 0.0   # planes of a 1D problem stay uniform
    assert np.abs(r[:, 0, 0] - ex[0]).mean() < 0.02
