"""Pins of the oracle's cell sort (a stable reordering by cell index) and of
the time-averaged moments of Sec. 3.1 (density profiles, EEPF at L/2 with
the normalisation sum sqrt(eps) f d(eps) = 1)."""
import numpy as np

from helpers import ME, NO_COLL, NO_FIELD, QE, params
from pic_inputs import state, xsec


def test_cell_sort_is_stable_argsort(ora):
    K = 5
    p = params(n_cells=64, flags=NO_FIELD | NO_COLL, sort_interval=K, capacity=(50_000, 50_000))
    sim = ora.Oracle(p, xsec.argon_synthetic())
    rng = np.random.default_rng(31)
    n = 30_000
    L = p["gap_m"]
    dx = L / p["n_cells"]
    # many exact ties inside a cell; zero velocity so the push leaves x alone
    x = (rng.integers(0, 64, n) + rng.integers(0, 4, n) / 4.0) * dx
    x = np.minimum(x, L)
    tag = np.arange(n, dtype=np.float64)
    z = np.zeros(n)
    for sp in (0, 1):
        sim.set_state(sp, x, z, tag, z, step=K - 1)
    sim.step(1)  # step K-1 -> K triggers the sort
    # cell index as the method defines it: x times the reciprocal of dx
    key = np.minimum(np.floor(x * (1.0 / dx)).astype(np.int64), p["n_cells"] - 1)
    order = np.argsort(key, kind="stable")
    for sp in (0, 1):
        xs_, _, vy, _ = sim.get_state(sp)
        assert np.array_equal(vy, tag[order])
        assert np.array_equal(xs_, x[order])


def test_initial_eepf_is_maxwellian_and_normalised(ora):
    # A Maxwellian at kT has EEPF (2/sqrt(pi)) (kT)^-3/2 exp(-eps/kT), which
    # satisfies the paper's normalisation exactly.
    T = 2.0
    p = params(n_cells=64, flags=NO_FIELD | NO_COLL, sort_interval=0, eepf_bins=64,
               eepf_emax_ev=16.0, eepf_halfwidth_m=0.5 * 0.025, capacity=(400_000, 8))
    sim = ora.Oracle(p, xsec.argon_synthetic())
    n = 300_000
    x, vx, vy, vz = state.maxwellian_uniform(n, p["gap_m"], T, 0, seed=5)
    sim.set_state(0, x, vx, vy, vz)
    sim.set_state(1, np.zeros(0), np.zeros(0), np.zeros(0), np.zeros(0))
    sim.measure(True)
    sim.step(1)
    m = sim.moments()
    de = 16.0 / 64
    eb = (np.arange(64) + 0.5) * de
    f = m["eepf"]
    assert abs((np.sqrt(eb) * f).sum() * de - 1) < 1e-12
    ref = 2 / np.sqrt(np.pi) * T**-1.5 * np.exp(-eb / T)
    # the histogram stops at 16 eV, which holds all but ~0.1% of a 2 eV gas:
    # renormalise the reference over the window
    ref = ref / ((np.sqrt(eb) * ref).sum() * de)
    counts = f * np.sqrt(eb) * de * n
    sd = np.sqrt(np.maximum(counts, 1)) / (np.sqrt(eb) * de * n)
    ok = np.abs(f - ref) < 5 * sd + 1e-3 * ref
    assert ok.mean() > 0.97
    # CIC-weighted mean energy is 3/2 kT at every node
    em = m["mean_energy_e"]
    assert np.all(np.abs(em[2:-2] / (1.5 * T) - 1) < 0.05)


def test_time_averaged_density_of_uniform_plasma(ora):
    # Uniform particles: n_e = N W / (A L) at interior nodes and, thanks to
    # the half-cell volume, at the wall nodes too.
    p = params(n_cells=32, flags=NO_FIELD | NO_COLL, sort_interval=0, capacity=(200_000, 200_000))
    sim = ora.Oracle(p, xsec.argon_synthetic())
    n = 160_000
    L = p["gap_m"]
    x = (np.arange(n) + 0.5) * (L / n)  # quiet start
    z = np.zeros(n)
    sim.set_state(0, x, z, z, z)
    sim.set_state(1, x, z, z, z)
    sim.measure(True)
    sim.step(3)
    m = sim.moments()
    n0 = n * p["weight"] / (p["area_m2"] * L)
    np.testing.assert_allclose(m["n_e"], n0, rtol=1e-3)
    np.testing.assert_allclose(m["n_i"], n0, rtol=1e-3)
    assert m["steps"] == 3
