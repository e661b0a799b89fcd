"""Pins of the oracle's surface model (Sec. 2 step 5): removal outside
[0, L], electron reflection with probability R, ion-induced secondary
emission with yield gamma; slot order of the rebuilt arrays."""
import numpy as np

from helpers import ME, NO_COLL, NO_FIELD, QE, RECORD, dt_of, params
from pic_inputs import xsec


def _wall_run(ora, R, gamma, n=40_000, seed=21):
    p = params(gap_m=0.01, n_cells=32, reflection=R, gamma_see=gamma, see_temp_ev=1.5,
               flags=NO_FIELD | NO_COLL | RECORD, sort_interval=0, capacity=(3 * n, 3 * n))
    sim = ora.Oracle(p, xsec.argon_synthetic())
    dt = dt_of(p)
    L = p["gap_m"]
    rng = np.random.default_rng(seed)
    # every particle leaves in this step: within |v| dt of its wall, heading out
    side = rng.integers(0, 2, n)
    ve = rng.uniform(1e5, 1e6, n)
    de = rng.uniform(0, 0.9, n) * ve * dt
    xe = np.where(side == 0, de, L - de)
    vxe = np.where(side == 0, -ve, ve)
    vi = rng.uniform(1e3, 1e4, n)
    di = rng.uniform(0, 0.9, n) * vi * dt
    xi = np.where(side == 0, di, L - di)
    vxi = np.where(side == 0, -vi, vi)
    z = np.zeros(n)
    sim.set_state(0, xe, vxe, z, z)
    sim.set_state(1, xi, vxi, z, z)
    sim.step(1)
    return sim, p, dict(xe=xe, vxe=vxe, xi=xi, vxi=vxi, side=side)


def test_reflection_binomial_and_mirror(ora):
    R = 0.3
    sim, p, s = _wall_run(ora, R, 0.0)
    code = sim.decisions(0) & 7
    n = code.size
    refl = code == 2
    k = refl.sum()
    assert abs(k - n * R) < 5 * np.sqrt(n * R * (1 - R))
    assert np.all((code == 1) | (code == 2))
    x, vx, _, _ = sim.get_state(0)
    assert x.size == k
    # specular: pushed position mirrored in the wall, vx reversed
    dt = dt_of(p)
    L = p["gap_m"]
    xp = s["xe"][refl] + s["vxe"][refl] * dt
    mirrored = np.where(xp < 0, -xp, (L + L) - xp)
    assert np.array_equal(x, mirrored)
    assert np.array_equal(vx, -s["vxe"][refl])
    c = sim.counters()
    assert c[4] == k and c[3] == n - k
    # no ion emits with gamma = 0; all ions are absorbed
    assert sim.count(1) == 0 and c[5] == n and c[6] == 0


def test_secondary_emission_binomial_and_half_maxwellian(ora):
    g = 0.25
    sim, p, s = _wall_run(ora, 0.0, g)
    code = sim.decisions(1) & 7
    n = code.size
    emit = code == 3
    assert abs(emit.sum() - n * g) < 5 * np.sqrt(n * g * (1 - g))
    # all electrons absorbed (R = 0); the new electrons are the secondaries,
    # in the order of their parent ions, at the wall their parent hit
    x, vx, vy, vz = sim.get_state(0)
    assert x.size == emit.sum()
    L = p["gap_m"]
    side = s["side"][emit]
    assert np.array_equal(x, np.where(side == 0, 0.0, L))
    # emitted inward, half-Maxwellian at 1.5 eV: <vy^2> = kT/m, vx sign
    assert np.all(np.where(side == 0, vx > 0, vx < 0))
    kt = 1.5 * QE
    for comp in (vx, vy, vz):
        assert abs((comp**2).mean() * ME / kt - 1) < 5 * np.sqrt(2 / comp.size)
    # mean |vx| of a half-Maxwellian: sqrt(2 kT / (pi m))
    assert abs(np.abs(vx).mean() / np.sqrt(2 * kt / (np.pi * ME)) - 1) < 0.03
    c = sim.counters()
    assert c[6] == emit.sum() and c[5] == n


def test_slot_order_after_absorption(ora):
    # survivors keep their relative order (compaction), nothing else moves
    p = params(gap_m=0.01, n_cells=32, reflection=0.0, flags=NO_FIELD | NO_COLL | RECORD,
               sort_interval=0, capacity=(10_000, 10_000))
    sim = ora.Oracle(p, xsec.argon_synthetic())
    dt = dt_of(p)
    rng = np.random.default_rng(22)
    n = 5000
    x = rng.uniform(0, 0.01, n)
    vx = rng.normal(0, 0.004 / dt, n)
    tag = np.arange(n, dtype=np.float64)
    sim.set_state(0, x, vx, tag, np.zeros(n))
    sim.set_state(1, np.zeros(0), np.zeros(0), np.zeros(0), np.zeros(0))
    sim.step(1)
    _, _, vy, _ = sim.get_state(0)
    code = sim.decisions(0) & 7
    assert np.array_equal(vy, tag[code == 0])
    assert 0 < (code == 1).sum() < n
