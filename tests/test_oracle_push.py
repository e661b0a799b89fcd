"""Pins of the oracle's gather and leap-frog push (Sec. 2 steps 3-4):
free streaming, motion in a uniform field, ion sub-cycling, and the cold
plasma oscillation whose leap-frog frequency and stability limit
omega_pe dt <= 2 are the paper's stability law (Sec. 3.5)."""
import numpy as np

from helpers import (EPS0, FIXED_E, IMMOBILE_IONS, ME, MAR, NO_COLL, NO_FIELD, QE, dt_of,
                     params)
from pic_inputs import xsec


def test_free_streaming(ora):
    p = params(gap_m=10.0, n_cells=64, flags=NO_FIELD | NO_COLL, sort_interval=0, ion_subcycle=3)
    sim = ora.Oracle(p, xsec.argon_synthetic())
    rng = np.random.default_rng(1)
    n = 5000
    x0 = rng.uniform(4.0, 6.0, n)
    v = rng.normal(0, 1e5, (3, n))
    vi = rng.normal(0, 1e3, (3, n))
    sim.set_state(0, x0, *v, step=1)
    sim.set_state(1, x0, *vi, step=1)
    sim.step(10)  # steps 1..10; ions move on steps 3, 6, 9 with 3 dt
    dt = dt_of(p)
    x, vx, vy, vz = sim.get_state(0)
    np.testing.assert_allclose(x, x0 + 10 * dt * v[0], rtol=0, atol=1e-13 * 10.0)
    assert np.array_equal(vx, v[0]) and np.array_equal(vy, v[1]) and np.array_equal(vz, v[2])
    xi, *_ = sim.get_state(1)
    np.testing.assert_allclose(xi, x0 + 9 * dt * vi[0], rtol=0, atol=1e-13 * 10.0)


def test_uniform_field_closed_form(ora):
    # x_n = x_0 + n dt v_{-1/2} + a dt^2 n(n+1)/2,  a = qE/m
    p = params(gap_m=10.0, n_cells=32, flags=FIXED_E | NO_COLL, sort_interval=0)
    sim = ora.Oracle(p, xsec.argon_synthetic())
    E0 = 150.0
    sim.set_field(np.full(p["n_cells"] + 1, E0))
    rng = np.random.default_rng(2)
    n = 2000
    x0 = rng.uniform(4.0, 6.0, n)
    v = rng.normal(0, 3e5, (3, n))
    vi = rng.normal(0, 3e2, (3, n))
    sim.set_state(0, x0, *v)
    sim.set_state(1, x0, *vi)
    N = 25
    sim.step(N)
    dt = dt_of(p)
    for sp, (m, q, vv) in enumerate(((ME, -QE, v), (MAR, QE, vi))):
        a = q * E0 / m
        x, vx, _, _ = sim.get_state(sp)
        expect = x0 + N * dt * vv[0] + a * dt * dt * N * (N + 1) / 2
        np.testing.assert_allclose(x, expect, rtol=0, atol=1e-12 * 10.0)
        np.testing.assert_allclose(vx, vv[0] + N * a * dt, rtol=1e-12, atol=1e-9 * abs(N * a * dt))


def _cold_plasma(ora, wpdt, steps, n=12_800):
    # Cold electrons on an immobile ion slab filling [L/4, 3L/4], displaced by
    # xi = a sin(2 pi (x0 - L/4) / (L/2)); the net displacement is zero, so
    # the field outside the slab vanishes and each electron obeys
    # xi'' = -omega_pe^2 xi. (A plasma touching the electrodes is avoided:
    # with the half-cell Gauss-law field at the wall nodes, the discrete
    # system has wall-localized grid-scale modes of negative stiffness.)
    L, ncells, f, Nt = 0.025, 256, 13.56e6, 1000
    dt = 1.0 / (f * Nt)
    n0 = (wpdt / dt) ** 2 * EPS0 * ME / QE**2
    W = n0 * 1e-4 * (L / 2) / n
    p = params(gap_m=L, n_cells=ncells, rf_freq_hz=f, steps_per_cycle=Nt, rf_voltage_v=0.0,
               weight=W, flags=NO_COLL | IMMOBILE_IONS, sort_interval=0, reflection=0.0,
               gamma_see=0.0, capacity=(n, n))
    sim = ora.Oracle(p, xsec.argon_synthetic())
    x0 = L / 4 + (np.arange(n) + 0.5) * (L / 2 / n)
    # small enough that almost no electron crosses a node during the
    # oscillation: node crossings make the CIC force piecewise linear, which
    # couples grid-scale modes at large amplitude near omega_pe dt = 2
    a = 1e-4 * L / ncells
    basis = np.sin(2 * np.pi * (x0 - L / 4) / (L / 2))
    z = np.zeros(n)
    sim.set_state(0, x0 + a * basis, z, z, z)
    sim.set_state(1, x0, z, z, z)
    proj, maxdisp, counts = [], [], []
    for _ in range(steps):
        sim.step(1)
        x, *_ = sim.get_state(0)
        counts.append(x.size)
        if x.size != n:
            break
        d = x - x0
        proj.append(2.0 * np.mean(d * basis))
        maxdisp.append(np.max(np.abs(d)))
    return np.array(proj), np.array(maxdisp), a, counts, dt


def _frequency(series, dt):
    s = series - series.mean()
    idx = np.where(np.sign(s[:-1]) != np.sign(s[1:]))[0]
    t = idx + s[idx] / (s[idx] - s[idx + 1])  # linear interpolation of crossings
    half_period = np.mean(np.diff(t))
    return np.pi / (half_period * dt)


def test_cold_plasma_leapfrog_dispersion(ora):
    for wpdt in (0.5, 1.0):
        proj, _, a, counts, dt = _cold_plasma(ora, wpdt, 240)
        w = _frequency(proj, dt) * dt
        leapfrog = 2 * np.arcsin(wpdt / 2)
        assert abs(w / leapfrog - 1) < 0.01, (wpdt, w, leapfrog)
        if wpdt == 1.0:
            # distinguishable from the continuous frequency (4.7% apart)
            assert abs(w / wpdt - 1) > 0.03


def test_cold_plasma_stability_limit(ora):
    # omega_pe dt = 1.9 < 2 stays bounded; 2.5 > 2 grows (Sec. 3.5)
    # below the limit the leap-frog orbit stays within 1/sqrt(1 - (w dt/2)^2)
    # of the initial displacement (3.2 at 1.9)
    _, maxd, a, counts, _ = _cold_plasma(ora, 1.9, 200)
    assert len(maxd) == 200
    assert np.max(maxd) < 1.1 / np.sqrt(1 - 0.95**2) * a
    _, maxd, a, counts, _ = _cold_plasma(ora, 2.5, 12)
    grew = (counts[-1] < counts[0]) or np.max(maxd) > 100 * a
    assert grew
