"""Pins of the 2D hydro oracle against facts that do not come from the oracle
itself: exact invariants of the discrete scheme, conservation laws, symmetry,
and the exact Riemann solution of a shock tube."""
import math
import os

import numpy as np
import pytest

import oracle.hydro2d as h
import riemann
from paper_1709_02125_amd.inputs import hydro_initial_state, mirror_symmetrise

H = 2


def _blobs(nx, ny):
    o = h.Hydro2D(nx, ny)
    r, e = hydro_initial_state((nx, ny))
    o.set_state(r, e)
    return o


def test_uniform_state_is_preserved_bit_exactly():
    # A gas at rest with uniform density and energy has no pressure gradient,
    # no velocity divergence and no fluxes: every step must return it unchanged.
    nx, ny = 24, 17
    o = h.Hydro2D(nx, ny)
    o.set_state(np.full((ny, nx), 0.2), np.full((ny, nx), 1.0))
    used, nxt = o.run(10)
    assert np.all(o.interior("rho0") == 0.2)
    assert np.all(o.interior("e0") == 1.0)
    assert np.all(o.interior("u0", True) == 0.0)
    assert np.all(o.interior("v0", True) == 0.0)
    # closed form of the time-step bound at rest: CFL * dx / sqrt(gamma (gamma-1) e)
    expect = 0.5 * (1.0 / nx) / math.sqrt(1.4 * 0.4 * 1.0)
    assert all(abs(d - expect) <= 1e-15 * expect for d in used + [nxt])


def test_mass_is_conserved_in_reflective_box():
    o = _blobs(64, 48)
    m0 = o.sum_cells("rho0")
    o.run(10)
    m1 = o.sum_cells("rho0")
    assert abs(m1 - m0) <= 1e-13 * m0


def test_internal_energy_total_is_conserved_by_remap():
    # The remap moves rho*e in flux form between cells of a closed box, so the
    # total internal energy after the full step equals the total after the
    # Lagrangian phase (sum of rho0 V e1, since rho1 V' = rho0 V).
    o = _blobs(40, 36)
    o.run(4)
    dt = o.dt()
    o.lagrangian(dt)
    ie_lag = (o.field("rho0") * o.field("vol") * o.field("e1"))[H:H + 36, H:H + 40].sum()
    o2 = _blobs(40, 36)
    o2.run(4)
    o2.step(dt)
    ie_after = o2.sum_cells("e0", times_rho0=True)
    assert abs(ie_after - ie_lag) <= 1e-12 * ie_lag


def _energies(o, ene, u, v):
    nx, ny = o.nx, o.ny
    F = o.field
    rv = F("rho0") * F("vol")
    ie = (rv * F(ene))[H:H + ny, H:H + nx].sum()
    m = 0.25 * ((rv[H - 1:H + ny, H - 1:H + nx] + rv[H - 1:H + ny, H:H + nx + 1]) +
                (rv[H:H + ny + 1, H - 1:H + nx] + rv[H:H + ny + 1, H:H + nx + 1]))
    w = np.ones((ny + 1, nx + 1))
    w[0, :] *= 0.5
    w[-1, :] *= 0.5
    w[:, 0] *= 0.5
    w[:, -1] *= 0.5
    uu = F(u)[H:H + ny + 1, H:H + nx + 1]
    vv = F(v)[H:H + ny + 1, H:H + nx + 1]
    return ie, (w * 0.5 * m * (uu * uu + vv * vv)).sum()


def test_lagrangian_phase_conserves_total_energy():
    # The node force is the adjoint of the cell volume-change operator, so the
    # PdV work removed from internal energy equals the kinetic energy gained
    # (wall nodes count half, corners a quarter: the box is their mirror).
    o = _blobs(48, 40)
    _, dt = o.run(5)
    o.lagrangian(dt)
    ie0, ke0 = _energies(o, "e0", "u0", "v0")
    ie1, ke1 = _energies(o, "e1", "u1", "v1")
    assert abs(ke1 - ke0) > 1e-3 * (ie0 + ke0)   # the step does real work
    assert abs((ie1 + ke1) - (ie0 + ke0)) <= 1e-13 * (ie0 + ke0)


@pytest.mark.parametrize("axis", [0, 1])
def test_mirror_symmetry(axis):
    nx, ny = 40, 30
    r, e = hydro_initial_state((nx, ny))
    r = mirror_symmetrise(r, 1 - axis)
    e = mirror_symmetrise(e, 1 - axis)
    o = h.Hydro2D(nx, ny)
    o.set_state(r, e)
    o.run(10)
    rho = o.interior("rho0")
    ene = o.interior("e0")
    u = o.interior("u0", True)
    v = o.interior("v0", True)
    flip = 1 - axis
    scale = np.abs(rho).max()
    assert np.abs(rho - np.flip(rho, flip)).max() <= 1e-12 * scale
    assert np.abs(ene - np.flip(ene, flip)).max() <= 1e-12 * np.abs(ene).max()
    normal, tangential = (u, v) if axis == 0 else (v, u)
    vs = max(np.abs(u).max(), np.abs(v).max())
    assert vs > 1e-3
    assert np.abs(normal + np.flip(normal, flip)).max() <= 1e-12 * vs
    assert np.abs(tangential - np.flip(tangential, flip)).max() <= 1e-12 * vs


def test_x_and_y_sweeps_agree_on_transposed_problem():
    # A problem varying only along x, and the same problem along y, must give
    # transposed results: catches any x/y index or area mix-up.
    n, m = 48, 5
    x = (np.arange(n) + 0.5) / n
    rho = np.where(x < 0.4, 1.0, 0.25)
    ene = np.where(x < 0.4, 2.5, 1.5)
    ox = h.Hydro2D(n, m)
    ox.set_state(np.tile(rho, (m, 1)), np.tile(ene, (m, 1)))
    oy = h.Hydro2D(m, n)
    oy.set_state(np.tile(rho[:, None], (1, m)), np.tile(ene[:, None], (1, m)))
    dtx, dty = ox.dt(), oy.dt()
    # dx and dy differ between the two meshes; drive both with the same steps
    dt = min(dtx, dty)
    for _ in range(15):
        ox.step(dt)
        oy.step(dt)
    rx, ry = ox.interior("rho0"), oy.interior("rho0")
    assert np.abs(rx - ry.T).max() <= 1e-12
    ux, vy = ox.interior("u0", True), oy.interior("v0", True)
    assert np.abs(ux - vy.T).max() <= 1e-12 * np.abs(ux).max()
    assert np.abs(ox.interior("v0", True)).max() == 0.0


def _sod(nx, ny=3, T=0.2):
    o = h.Hydro2D(nx, ny)
    x = (np.arange(nx) + 0.5) / nx
    rho = np.where(x < 0.5, 1.0, 0.125)
    pre = np.where(x < 0.5, 1.0, 0.1)
    o.set_state(np.tile(rho, (ny, 1)), np.tile(pre / (0.4 * rho), (ny, 1)))
    t, dt = 0.0, o.dt()
    while t < T - 1e-14:
        dt = min(dt, T - t)
        nd = o.step(dt)
        t += dt
        dt = nd
    ex = riemann.sample(x, T, 0.5, (1.0, 0.0, 1.0), (0.125, 0.0, 0.1))
    r = o.interior("rho0")
    assert np.abs(r - r[0]).max() == 0.0   # rows of a 1D problem stay identical
    return np.abs(r[0] - ex[0]).mean(), o


def test_exact_riemann_helper_matches_published_star_state():
    gold = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", "sod_star_state.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, v = line.split()
                gold[k] = float(v)
    p, u = riemann.star_state(1.0, 0.0, 1.0, 0.125, 0.0, 0.1)
    assert abs(p - gold["p_star"]) < 1e-5 and abs(u - gold["u_star"]) < 1e-5


def test_shock_tube_converges_to_exact_riemann_solution():
    e1, _ = _sod(100)
    e2, _ = _sod(200)
    assert e1 < 0.02
    assert e2 < 0.8 * e1      # first-order scheme: the error falls with dx


# ---- field summary (the periodic diagnostic of Section 5.3)

def test_field_summary_of_a_uniform_gas_at_rest_has_its_closed_form():
    # unit square: volume 1, mass rho, internal energy rho e, no kinetic
    # energy, pressure (gamma - 1) rho e; a stale pressure field is ignored
    nx, ny, rho, e = 30, 22, 0.7, 2.3
    o = h.Hydro2D(nx, ny)
    o.set_state(np.full((ny, nx), rho), np.full((ny, nx), e))
    o.field("p")[...] = 123.0
    vol, mass, ie, ke, press = o.field_summary()
    assert abs(vol - 1.0) <= 1e-13
    assert abs(mass - rho) <= 1e-13 * rho
    assert abs(ie - rho * e) <= 1e-13 * rho * e
    assert ke == 0.0
    assert abs(press - 0.4 * rho * e) <= 1e-13 * rho * e


def test_field_summary_kinetic_energy_of_uniform_and_linear_velocities():
    nx, ny, rho = 24, 20, 1.3
    dx, dy = 1.0 / nx, 1.0 / ny
    # uniform velocity: 0.5 rho |u|^2 over the unit square
    o = h.Hydro2D(nx, ny)
    o.set_state(np.full((ny, nx), rho), np.ones((ny, nx)), np.full((ny + 1, nx + 1), 0.3),
                np.full((ny + 1, nx + 1), -0.4))
    ke = o.field_summary()[3]
    assert abs(ke - 0.5 * rho * (0.09 + 0.16)) <= 1e-13
    # u = x at the nodes: each cell averages x^2 over its two node columns,
    # sum_i (i^2 + (i+1)^2) dx^3 / 4 = (S(n-1) + S(n)) dx^3 / 4, S(m) = sum of squares to m
    S = lambda m: m * (m + 1) * (2 * m + 1) / 6.0
    xs = np.arange(nx + 1) * dx
    o = h.Hydro2D(nx, ny)
    o.set_state(np.full((ny, nx), rho), np.ones((ny, nx)), np.tile(xs, (ny + 1, 1)), np.zeros((ny + 1, nx + 1)))
    assert abs(o.field_summary()[3] - rho * (S(nx - 1) + S(nx)) * dx ** 3 / 4) <= 1e-13
    # v = y at the nodes: the same along y
    ys = np.arange(ny + 1) * dy
    o = h.Hydro2D(nx, ny)
    o.set_state(np.full((ny, nx), rho), np.ones((ny, nx)), np.zeros((ny + 1, nx + 1)),
                np.tile(ys[:, None], (1, nx + 1)))
    assert abs(o.field_summary()[3] - rho * (S(ny - 1) + S(ny)) * dy ** 3 / 4) <= 1e-13
    # u = x y: the mean over a cell's four corners of x^2 y^2 factorises,
    # (x_i^2 + x_i+1^2)(y_j^2 + y_j+1^2) / 4, which only the four true corners give
    o = h.Hydro2D(nx, ny)
    o.set_state(np.full((ny, nx), rho), np.ones((ny, nx)), np.outer(ys, xs), np.zeros((ny + 1, nx + 1)))
    want = rho / 8 * (S(nx - 1) + S(nx)) * dx ** 3 * (S(ny - 1) + S(ny)) * dy ** 3
    assert abs(o.field_summary()[3] - want) <= 1e-13


def test_field_summary_pressure_is_the_equation_of_state_and_mass_is_conserved():
    # for any state the pressure sum is (gamma - 1) times the internal-energy
    # sum; in the closed box the volume and the mass stay as they were
    o = _blobs(48, 40)
    s0 = o.field_summary()
    o.run(6)
    s1 = o.field_summary()
    for s in (s0, s1):
        assert abs(s[4] - 0.4 * s[2]) <= 1e-13 * s[2]
    assert abs(s1[0] - s0[0]) <= 1e-15 and abs(s1[1] - s0[1]) <= 1e-13 * s0[1]
    assert s0[3] == 0.0 and s1[3] > 0.0
