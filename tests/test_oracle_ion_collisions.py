"""Pins of the oracle's Ar+ - Ar collision branch (Sec. 2 step 6: isotropic
elastic and backward elastic scattering of ions on the background gas).

For each ion candidate the oracle draws a thermal atom velocity v_a, looks
up the cumulative collision frequencies at the relative speed g = |v_i - v_a|
and picks isotropic, backward or null. These tests fix that branch from
outside the oracle: closed forms of the mean relative speed of a thermal
target, conservation laws of a two-body elastic collision, and the exact
atom velocity rebuilt from the published random-number layout (Philox words
of purpose 1 for the atom, Box-Muller normals)."""
import math

import numpy as np
from scipy import special

from helpers import KB, MAR, NO_FIELD, RECORD, dt_of, params, table_for


def _code_coll(c):
    return (c >> 3) & 7


def _sigma_for(p, pcoll, vtop):
    """Constant total cross section giving candidacy probability pcoll for
    a table that ends at vtop."""
    ng = p["pressure_pa"] / (KB * p["gas_temp_k"])
    return -math.log(1.0 - pcoll) / (ng * vtop * dt_of(p))


def _ion_sim(ora, n, sig_iso, sig_back, vtop, seed=1, gas_temp_k=300.0, pressure_pa=100.0):
    nt = 513
    p = params(gap_m=1e3, n_cells=16, pressure_pa=pressure_pa, gas_temp_k=gas_temp_k,
               flags=NO_FIELD | RECORD, sort_interval=0, capacity=(8, n), seed=seed,
               ion_subcycle=1)
    xs = table_for(4e6, vtop, n=nt, sig_i=(sig_iso, sig_back))
    return ora.Oracle(p, xs), p, xs


def _mean_offset_maxwell_speed(V, s):
    """E|V e + s N(0, I_3)| for an offset of length V (closed form of the
    non-central chi distribution with three degrees of freedom)."""
    if V == 0.0:
        return s * math.sqrt(8.0 / math.pi)
    a = V / s
    return s * (math.sqrt(2.0 / math.pi) * math.exp(-0.5 * a * a) + (a + 1.0 / a) * math.erf(a / math.sqrt(2.0)))


def _atom_velocities(ora, p, slots, step=0):
    """The thermal atom drawn for the candidates in `slots`: Philox block
    (step, slot, 16 * 1 + 1, 0) keyed by (seed, run), words mapped to (0, 1)
    as (k + 1/2) 2^-32, two Box-Muller pairs (the fourth normal unused),
    scaled by sqrt(k T_g / M)."""
    ctr = np.zeros((slots.size, 4), np.uint32)
    ctr[:, 0] = step
    ctr[:, 1] = slots
    ctr[:, 2] = 16 * 1 + 1
    key = np.array([p["seed"], p["run"]], np.uint32)
    w = np.array([ora.philox4x32_10(c, key) for c in ctr], dtype=np.float64)
    u = (w + 0.5) * 2.0**-32
    r1 = np.sqrt(-2.0 * np.log(u[:, 0]))
    r2 = np.sqrt(-2.0 * np.log(u[:, 2]))
    n1 = r1 * np.cos(2.0 * np.pi * u[:, 1])
    n2 = r1 * np.sin(2.0 * np.pi * u[:, 1])
    n3 = r2 * np.cos(2.0 * np.pi * u[:, 3])
    sg = math.sqrt(KB * p["gas_temp_k"] / MAR)
    return sg * np.array([n1, n2, n3])


def test_ion_process_selection_uses_relative_speed_and_table_order(ora):
    """Ions at rest and ions drifting at V = 2 sqrt(kT/M), constant
    sigma_iso = 3 sigma_back: a candidate collides for real with probability
    E[g] / v_top (nu = n_g sigma g is linear in speed, so the table's linear
    interpolation is exact), split 3:1 between isotropic and backward.
    Catches: the table read at the ion's lab speed (ions at rest would never
    collide; the drifting group would follow V, not E[g]); isotropic and
    backward swapped (1:3 instead of 3:1); a row of the table skipped."""
    n = 240_000
    vtop = 2500.0
    p0 = params(pressure_pa=100.0)
    st = _sigma_for(p0, 0.5, vtop)
    sim, p, xs = _ion_sim(ora, n, 0.75 * st, 0.25 * st, vtop, seed=3)
    assert abs(sim.derived()["p_coll_i"] - 0.5) < 1e-9
    rng = np.random.default_rng(41)
    sg = math.sqrt(KB * p["gas_temp_k"] / MAR)
    V = 2.0 * sg
    half = n // 2
    # group A at rest, group B drifting with speed V in random directions
    u = rng.uniform(-1, 1, half)
    ph = rng.uniform(0, 2 * np.pi, half)
    s = np.sqrt(1 - u * u)
    vx = np.concatenate([np.zeros(half), V * u])
    vy = np.concatenate([np.zeros(half), V * s * np.cos(ph)])
    vz = np.concatenate([np.zeros(half), V * s * np.sin(ph)])
    sim.set_state(0, np.zeros(0), np.zeros(0), np.zeros(0), np.zeros(0))
    sim.set_state(1, rng.uniform(400, 600, n), vx, vy, vz)
    assert sim.step(1) == 0
    code = _code_coll(sim.decisions(1))
    assert code.size == n
    c = sim.counters()
    assert c[15] == 0  # no relative speed beyond the table (6 sigma margin)
    for grp, Vg in ((slice(0, half), 0.0), (slice(half, n), V)):
        cg = code[grp]
        cand = cg > 0
        obs = np.array([(cg == 2).sum(), (cg == 3).sum(), (cg == 1).sum()], dtype=float)
        preal = _mean_offset_maxwell_speed(Vg, sg) / vtop
        prob = np.array([0.75 * preal, 0.25 * preal, 1 - preal])
        expect = cand.sum() * prob
        chi2 = ((obs - expect) ** 2 / expect).sum()
        assert chi2 < 13.8, (Vg, obs, expect)  # 2 dof, 99.9 %
    # candidacy itself: Binomial(n, 1/2)
    assert abs((code > 0).sum() - 0.5 * n) < 5 * math.sqrt(0.25 * n)


def test_ion_isotropic_collision_conserves_pair_momentum_and_energy(ora):
    """Isotropic scattering only: for every real collision the atom's
    velocity after the collision follows from momentum conservation,
    v_a' = v_i + v_a - v_i'; the pair's kinetic energy must then be
    unchanged to rounding, and the scattering angle in the centre-of-mass
    frame must be isotropic (<cos chi> = 0, <cos^2 chi> = 1/3).
    Catches: a centre-of-mass velocity that drops the atom's share (momentum
    lost, energy identity fails), a relative speed other than |v_i - v_a|,
    a scattering direction tied to the incident one."""
    n = 60_000
    vtop = 8000.0
    p0 = params(pressure_pa=100.0)
    st = _sigma_for(p0, 0.6, vtop)
    sim, p, xs = _ion_sim(ora, n, st, 0.0, vtop, seed=5)
    rng = np.random.default_rng(43)
    sv = math.sqrt(0.5 * 1.602176634e-19 / MAR)  # ions at about 0.5 eV per component
    v = rng.normal(0.0, sv, (3, n))
    sim.set_state(0, np.zeros(0), np.zeros(0), np.zeros(0), np.zeros(0))
    sim.set_state(1, rng.uniform(400, 600, n), *v)
    assert sim.step(1) == 0
    code = _code_coll(sim.decisions(1))
    _, vxo, vyo, vzo = sim.get_state(1)
    assert vxo.size == n
    hit = np.nonzero(code == 2)[0]
    assert hit.size > 5_000
    vi = v[:, hit]
    va = _atom_velocities(ora, p, hit.astype(np.uint32))
    vo = np.array([vxo[hit], vyo[hit], vzo[hit]])
    va_after = vi + va - vo
    e_before = (vi**2).sum(0) + (va**2).sum(0)
    e_after = (vo**2).sum(0) + (va_after**2).sum(0)
    assert np.max(np.abs(e_after / e_before - 1)) < 1e-10
    g = vi - va
    gn = np.sqrt((g**2).sum(0))
    w = vo - 0.5 * (vi + va)
    wn = np.sqrt((w**2).sum(0))
    np.testing.assert_allclose(wn, 0.5 * gn, rtol=1e-10)
    cosx = (w * g).sum(0) / (wn * gn)
    m = hit.size
    assert abs(cosx.mean()) < 5 / math.sqrt(3 * m)
    assert abs((cosx**2).mean() - 1 / 3) < 5 * math.sqrt(4 / 45 / m)
    # particles that were not real collisions keep their velocity
    rest = code != 2
    np.testing.assert_array_equal(vxo[rest], v[0, rest])


def test_ion_backward_collision_returns_the_drawn_atom_velocity(ora):
    """Backward scattering only: the ion leaves with exactly the velocity of
    the atom drawn for it (symmetric charge transfer), rebuilt here from the
    random-number layout; its relative speed to that atom decided the event,
    so the collided ions' pre-collision relative speeds are weighted by g.
    Catches: the ion keeping its own velocity or a reversed one, an atom
    velocity from the wrong Philox purpose or word, a lookup at lab speed."""
    n = 60_000
    vtop = 8000.0
    p0 = params(pressure_pa=100.0)
    st = _sigma_for(p0, 0.6, vtop)
    sim, p, xs = _ion_sim(ora, n, 0.0, st, vtop, seed=7)
    rng = np.random.default_rng(44)
    sv = math.sqrt(0.5 * 1.602176634e-19 / MAR)
    v = rng.normal(0.0, sv, (3, n))
    sim.set_state(0, np.zeros(0), np.zeros(0), np.zeros(0), np.zeros(0))
    sim.set_state(1, rng.uniform(400, 600, n), *v)
    assert sim.step(1) == 0
    code = _code_coll(sim.decisions(1))
    _, vxo, vyo, vzo = sim.get_state(1)
    hit = np.nonzero(code == 3)[0]
    assert hit.size > 5_000
    assert (code == 2).sum() == 0
    va = _atom_velocities(ora, p, hit.astype(np.uint32))
    vo = np.array([vxo[hit], vyo[hit], vzo[hit]])
    sg = math.sqrt(KB * p["gas_temp_k"] / MAR)
    assert np.max(np.abs(vo - va)) < 1e-12 * sg
    # the real/null split among candidates follows g / v_top for each one:
    # sum of g / v_top over candidates is the expected count of real events
    cand = np.nonzero(code > 0)[0]
    vac = _atom_velocities(ora, p, cand.astype(np.uint32))
    gc = np.sqrt(((v[:, cand] - vac) ** 2).sum(0))
    pr = gc / vtop
    expect = pr.sum()
    sd = math.sqrt((pr * (1 - pr)).sum())
    assert abs(hit.size - expect) < 5 * sd, (hit.size, expect, sd)
    # and real events are the ones with larger relative speed: their mean g
    # is <g^2>/<g> of the candidates (size-biased), not <g>
    gh = np.sqrt(((v[:, hit] - va) ** 2).sum(0))
    biased = (gc**2).mean() / gc.mean()
    assert abs(gh.mean() / biased - 1) < 5 * gh.std() / math.sqrt(hit.size) / biased
    assert special.erfc(0) == 1.0  # scipy present (closed forms above)
