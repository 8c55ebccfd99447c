"""Pins of the 3D Navier-Stokes proxy oracle: exact invariants, conservation,
symmetry, and the closed-form early decay of a viscous Taylor-Green vortex."""
import numpy as np
import pytest

import oracle.ns3d as ns
from paper_1709_02125_amd.inputs import tgv_initial_state


def _run(n, steps, re=1600.0, perturb=1e-3, periodic_z=False, prims=None):
    o = ns.NS3D(n, re=re, periodic_z=periodic_z)
    o.set_primitives(*(prims if prims is not None else tgv_initial_state(n, perturb=perturb)))
    dt = ns.stable_dt(n)
    for _ in range(steps):
        o.step(dt)
    return o


def test_uniform_state_is_preserved_bit_exactly():
    # Central differences of a constant vanish exactly, so a gas at rest with
    # uniform density and pressure has a zero residual and stays unchanged.
    n = 12
    p0 = 1.0 / (1.4 * 0.01)
    one = np.ones((n, n, n))
    o = _run(n, 0, prims=(one, 0 * one, 0 * one, 0 * one, p0 * one))
    q0 = {f: o.interior(f).copy() for f in ns.Q}
    dt = ns.stable_dt(n)
    for _ in range(3):
        o.step(dt)
    for f in ns.Q:
        assert np.array_equal(o.interior(f), q0[f]), f
    assert np.all(q0["q_r"] == 1.0) and np.all(q0["q_ru"] == 0.0)


def test_mass_and_energy_are_conserved():
    # Flux form with periodic x, y and mirror walls in z (where the mass and
    # energy fluxes are odd, so they telescope to zero).
    n = 20
    o = ns.NS3D(n)
    o.set_primitives(*tgv_initial_state(n))
    m0, e0 = o.sum("q_r"), o.sum("q_re")
    dt = ns.stable_dt(n)
    for _ in range(5):
        o.step(dt)
    assert abs(o.sum("q_r") - m0) <= 1e-13 * m0
    assert abs(o.sum("q_re") - e0) <= 1e-13 * e0
    assert np.abs(o.interior("q_rw")).max() > 1e-4  # a real flow


def test_mirror_walls_equal_periodic_for_symmetric_vortex():
    # The unperturbed Taylor-Green vortex is even (w odd) about z = 0 and
    # z = 2 pi, so mirror walls reproduce the periodic solution.
    n = 16
    a = _run(n, 4, perturb=0.0, periodic_z=False)
    b = _run(n, 4, perturb=0.0, periodic_z=True)
    for f in ns.Q:
        scale = max(np.abs(b.interior(f)).max(), 1e-300)
        assert np.abs(a.interior(f) - b.interior(f)).max() <= 1e-12 * scale, f


def test_x_y_transposition_symmetry():
    # Swapping the x and y axes (and u with v) commutes with a step.
    n = 12
    r, u, v, w, p = tgv_initial_state(n)
    T = lambda x: np.swapaxes(x, 1, 2)
    a = _run(n, 3, prims=(r, u, v, w, p))
    b = _run(n, 3, prims=(T(r), T(v), T(u), T(w), T(p)))
    pairs = [("q_r", "q_r"), ("q_ru", "q_rv"), ("q_rv", "q_ru"), ("q_rw", "q_rw"), ("q_re", "q_re")]
    for fa, fb in pairs:
        x, y = a.interior(fa), T(b.interior(fb))
        assert np.abs(x - y).max() <= 1e-12 * np.abs(x).max(), fa


def test_taylor_green_early_decay_matches_closed_form():
    # At t = 0 the incompressible Taylor-Green mode (|k|^2 = 3) loses kinetic
    # energy at rate 2 nu |k|^2 E = 6 nu E with E(0) = 1/8; compressibility at
    # M = 0.1 and truncation at n = 32 keep the rate within 2 %.
    n, re = 32, 10.0
    nu = 1.0 / re
    o = ns.NS3D(n, re=re)
    o.set_primitives(*tgv_initial_state(n, perturb=0.0))
    dt = ns.stable_dt(n)
    ke = [o.kinetic()]
    for _ in range(10):
        o.step(dt)
        ke.append(o.kinetic())
    assert abs(ke[0] - 0.125) < 1e-12
    t = np.arange(len(ke)) * dt
    rate = -np.polyfit(t, np.log(ke), 1)[0]
    assert abs(rate - 6 * nu) <= 0.02 * 6 * nu
    slope = (ke[1] - ke[0]) / dt
    assert abs(slope - (-0.75 * nu)) <= 0.02 * 0.75 * nu


def _rk3_scalar(z, A, B):
    # 2N-storage Runge-Kutta on dq/dt = lambda q with z = lambda dt
    q, d = 1.0 + 0j, 0j
    for a, b in zip(A, B):
        d = a * d + z * q
        q = q + b * d
    return q


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_entropy_wave_amplification_is_the_rk3_polynomial(axis):
    # A density wave carried by a uniform velocity U at uniform pressure is an
    # exact solution of the inviscid semi-discrete equations: momentum and
    # energy follow the mass (rho u = U rho, p unchanged), so the density obeys
    # d rho / dt = -U D rho, a linear system.  The fourth-order difference
    # turns e^{i m x} into i k_h e^{i m x} with k_h = (8 sin mh - sin 2mh)/(6h),
    # and any three-stage third-order Runge-Kutta step multiplies a mode with
    # z = -i U k_h dt by P(z) = 1 + z + z^2/2 + z^3/6.  The amplitude can be
    # large (0.1) because nothing here is linearised; that keeps rounding far
    # below the tolerance.  The z axis runs periodic for this case.
    n, m, eps, U, steps = 16, 3, 0.1, 1.0, 6
    h = 2.0 * np.pi / n
    c = (np.arange(n) + 0.5) * h
    grids = np.meshgrid(c, c, c, indexing="ij")  # z, y, x
    x = grids[2 - axis]
    p0 = 1.0 / (1.4 * 0.01)
    rho = 1.0 + eps * np.cos(m * x)
    vel = [np.zeros_like(rho) for _ in range(3)]
    vel[axis] = np.full_like(rho, U)
    o = ns.NS3D(n, re=float("inf"), periodic_z=True)
    o.set_primitives(rho, vel[0], vel[1], vel[2], np.full_like(rho, p0))
    dt = ns.stable_dt(n)
    for _ in range(steps):
        o.step(dt)
    kh = (8.0 * np.sin(m * h) - np.sin(2.0 * m * h)) / (6.0 * h)
    z = -1j * U * kh * dt
    P = 1.0 + z + z * z / 2.0 + z ** 3 / 6.0
    want = 1.0 + eps * np.real(P ** steps * np.exp(1j * m * x))
    got = o.interior("q_r")
    assert np.abs(got - want).max() <= 1e-12 * eps
    mom = ["q_ru", "q_rv", "q_rw"][axis]
    assert np.abs(o.interior(mom) - U * got).max() <= 1e-13
    # the test is sensitive: the wave moved by a visible amount, and a 1 %
    # change of any Runge-Kutta coefficient (or the second-order difference
    # (f[+1] - f[-1]) / 2h in place of the fourth-order one) moves the answer
    # by far more than the tolerance
    assert np.abs(want - (1.0 + eps * np.cos(m * x))).max() > 1e-3 * eps
    A, B = [0.0, -5.0 / 9.0, -153.0 / 128.0], [1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0]
    assert abs(_rk3_scalar(z, A, B) - P) <= 1e-15
    for k in range(1, 3):
        Ap = list(A)
        Ap[k] *= 1.01
        assert abs(_rk3_scalar(z, Ap, B) ** steps - P ** steps) * eps > 1e3 * 1e-12 * eps
    for k in range(3):
        Bp = list(B)
        Bp[k] *= 1.01
        assert abs(_rk3_scalar(z, A, Bp) ** steps - P ** steps) * eps > 1e3 * 1e-12 * eps
    z2 = -1j * U * (np.sin(m * h) / h) * dt
    P2 = 1.0 + z2 + z2 * z2 / 2.0 + z2 ** 3 / 6.0
    assert abs(P2 ** steps - P ** steps) * eps > 1e3 * 1e-12 * eps
