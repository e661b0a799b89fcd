"""Pins of the oracle's electrode diagnostics and stability monitors
(Sec. 3.3 and 3.5): arrivals, absorption, impact energies and flux-energy
distributions at each electrode, the particle balance behind the paper's
continuity argument, and the plasma frequency and Debye length against
their textbook constants."""
import numpy as np
import pytest

from helpers import MAR, ME, NO_COLL, NO_FIELD, QE, dt_of, params
from pic_inputs import state, xsec


def _arrivals(ora, R, n=5000, seed=3):
    p = params(gap_m=0.01, n_cells=32, reflection=R, gamma_see=0.0, flags=NO_FIELD | NO_COLL,
               sort_interval=0, capacity=(3 * n, 3 * n), eepf_emax_ev=50.0, eepf_bins=100,
               rf_voltage_v=80.0)
    sim = ora.Oracle(p, xsec.argon_synthetic())
    dt = dt_of(p)
    L = p["gap_m"]
    rng = np.random.default_rng(seed)
    side = rng.integers(0, 2, n)
    # electrons and ions that leave in this step, through the wall on their
    # side, plus as many that stay inside
    out = {}
    for sp, m, vmax in ((0, ME, 4e6), (1, MAR, 2.5e4)):
        v = rng.uniform(0.2, 1.0, n) * vmax
        d = rng.uniform(0, 0.9, n) * v * dt
        x = np.where(side == 0, d, L - d)
        vx = np.where(side == 0, -v, v)
        vy = rng.normal(size=n) * 0.3 * vmax
        vz = rng.normal(size=n) * 0.3 * vmax
        xs = np.concatenate([x, rng.uniform(0.3 * L, 0.7 * L, n)])
        vxs = np.concatenate([vx, np.zeros(n)])
        vys = np.concatenate([vy, vy])
        vzs = np.concatenate([vz, vz])
        sim.set_state(sp, xs, vxs, vys, vzs)
        out[sp] = (m, vx, vy, vz)
    sim.measure(True)
    sim.step(1)
    return sim, p, side, out


@pytest.mark.parametrize("R", [0.0, 1.0])
def test_arrivals_energies_and_histograms_by_hand(ora, R):
    sim, p, side, out = _arrivals(ora, R)
    r = sim.wall_raw()
    nb = p["eepf_bins"]
    emax = (p["eepf_emax_ev"], 1.25 * p["rf_voltage_v"])
    for sp in (0, 1):
        m, vx, vy, vz = out[sp]
        eps = 0.5 * m * (vx * vx + vy * vy + vz * vz) / QE
        for w in (0, 1):
            sel = side == w
            assert r["hits"][sp, w] == sel.sum()
            assert r["esum"][sp, w] == pytest.approx(eps[sel].sum(), rel=1e-12)
            b = np.floor(eps[sel] / (emax[sp] / nb)).astype(int)
            hist = np.bincount(b[b < nb], minlength=nb)
            # a value within rounding of a bin edge may fall either way
            assert np.abs(r["hist"][sp, w] - hist).sum() <= 2
    # electrons are absorbed unless reflected; ions always
    absorbed_e = 0 if R == 1.0 else 1
    assert np.array_equal(r["absorbed"][0], absorbed_e * r["hits"][0])
    assert np.array_equal(r["absorbed"][1], r["hits"][1])
    assert r["steps"] == 1


def test_flux_units_and_normalisation(ora):
    sim, p, side, _ = _arrivals(ora, 0.0)
    wm = sim.wall_moments()
    dt = dt_of(p)
    # one measured step: arrivals x W per electrode area per dt
    expect = np.array([[(side == 0).sum(), (side == 1).sum()]] * 2) * p["weight"] / (p["area_m2"] * dt)
    np.testing.assert_allclose(wm["flux"], expect, rtol=1e-14)
    for sp, emax in ((0, p["eepf_emax_ev"]), (1, 1.25 * p["rf_voltage_v"])):
        de = emax / p["eepf_bins"]
        for w in (0, 1):
            assert wm["fedf"][sp, w].sum() * de == pytest.approx(1.0, rel=1e-12)


def test_ion_balance_is_exact(ora):
    # every ion is born by an ionization and leaves by absorption at an
    # electrode: over any measured window the ion count changes by exactly
    # the ionizations minus the absorbed ions (the continuity balance of
    # Sec. 3.3 before time averaging)
    p = params(ion_subcycle=1, sort_interval=50)
    sim = ora.Oracle(p, xsec.argon_synthetic())
    init = state.initial_state({"params": p, "n_init": (3000, 3000), "t_init_ev": (4.0, 0.03)}, seed=2)
    for sp in (0, 1):
        sim.set_state(sp, *init[sp])
    sim.step(100)
    n0 = sim.count(1)
    sim.measure(True)
    sim.step(300)
    r = sim.wall_raw()
    assert r["ionizations"] > 0 and r["absorbed"][1].sum() > 0
    assert sim.count(1) - n0 == r["ionizations"] - r["absorbed"][1].sum()


def test_monitors_against_textbook_constants(ora):
    # a uniform Maxwellian plasma measured over one step: the electron plasma
    # frequency is 56.41 sqrt(n_e) rad/s and the Debye length
    # 7434 sqrt(T_e[eV] / n_e[m^-3]) m
    import oracle

    n = 200_000
    p = params(n_cells=64, flags=NO_FIELD | NO_COLL, capacity=(2 * n, 2 * n), eepf_emax_ev=40.0)
    sim = ora.Oracle(p, xsec.argon_synthetic())
    init = state.initial_state({"params": p, "n_init": (n, n), "t_init_ev": (3.0, 0.03)}, seed=4)
    for sp in (0, 1):
        sim.set_state(sp, *init[sp])
    sim.measure(True)
    sim.step(1)
    m = sim.moments()
    mon = oracle.monitors(m, p, (0.0, 0.0))
    nc = mon["n_e_center"]
    assert mon["omega_pe_dt"] == pytest.approx(56.41 * np.sqrt(m["n_e"].max()) * dt_of(p), rel=1e-3)
    te = (2.0 / 3.0) * mon["mean_energy_center_ev"]
    assert mon["lambda_d_m"] == pytest.approx(7434.0 * np.sqrt(te / nc), rel=1e-3)
    # and they are those of the loaded plasma, within its sampling noise
    n0 = n * p["weight"] / (p["area_m2"] * p["gap_m"])
    assert nc == pytest.approx(n0, rel=0.1)
    assert te == pytest.approx(3.0, rel=0.1)
    assert mon["n_d"] == pytest.approx(nc * p["area_m2"] * mon["lambda_d_m"] / p["weight"], rel=1e-12)
    dx = p["gap_m"] / p["n_cells"]
    assert mon["dx_over_lambda_d"] == pytest.approx(dx / mon["lambda_d_m"], rel=1e-12)
