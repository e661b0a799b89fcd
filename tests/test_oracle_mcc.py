"""Pins of the oracle's null-collision Monte Carlo step (Sec. 2 step 6,
P_coll = 1 - exp(-nu_max dt) of Sec. 3.5): occurrence rate and free-path
distribution for a constant cross section, process selection, elastic
kinematics, inelastic energy bookkeeping and ion-gas equilibrium."""
import os

import numpy as np

from helpers import (KB, ME, MAR, NO_FIELD, QE, RECORD, dt_of, energy_ev, iso_velocities,
                     params, table_for)
from pic_inputs import xsec


def _code_coll(c):
    return (c >> 3) & 7


def test_collision_rate_and_geometric_free_path(ora):
    # Constant elastic sigma, monoenergetic electrons at half the table's top
    # speed: per step a real collision has probability P_coll * nu/nu_max
    # with nu/nu_max = 1/2, and the step of the first collision is geometric.
    vtop = 4e6
    xs = table_for(vtop, 1e5, n=513, sig_e=(2e-19, 0.0, 0.0))
    p = params(gap_m=1e3, n_cells=16, pressure_pa=50.0, flags=NO_FIELD | RECORD, sort_interval=0,
               capacity=(20_000, 8))
    sim = ora.Oracle(p, xs)
    d = sim.derived()
    n = 20_000
    rng = np.random.default_rng(11)
    v0 = 256 * xs.dv_e  # exactly on a table node
    sim.set_state(0, rng.uniform(400, 600, n), *iso_velocities(n, v0, rng))
    sim.set_state(1, np.zeros(0), np.zeros(0), np.zeros(0), np.zeros(0))
    q = d["p_coll_e"] * (v0 / ((xs.n - 1) * xs.dv_e))
    first = np.full(n, -1)
    K = 40
    for k in range(K):
        sim.step(1)
        hit = _code_coll(sim.decisions(0)) == 2
        newly = hit & (first < 0)
        first[newly] = k
    c = sim.counters()
    trials = n * K
    # elastic energy loss is ~3e-5 per collision, so the speed stays ~v0
    assert abs(c[8] - trials * q) < 5 * np.sqrt(trials * q * (1 - q))
    assert abs(c[7] - trials * d["p_coll_e"]) < 5 * np.sqrt(trials * d["p_coll_e"])
    # geometric first-collision step: P(T = k) = (1 - q)^k q
    ks = np.arange(K)
    expect = n * (1 - q) ** ks * q
    obs = np.bincount(first[first >= 0], minlength=K)
    chi2 = ((obs - expect) ** 2 / expect).sum()
    assert chi2 < 80, chi2  # 40 bins: 99.9% quantile ~ 73
    # the rate tends to n_g sigma v as dt -> 0
    ng = d["gas_density"]
    rate = c[8] / (trials * dt_of(p))
    nu = ng * 2e-19 * v0
    assert abs(rate / nu - 1) < 0.5 * d["nu_max_e"] * dt_of(p) + 5 / np.sqrt(c[8])


def test_process_selection_is_multinomial(ora):
    # At a fixed speed the real processes occur in the ratio of their
    # frequencies and the null event takes the rest of nu_max.
    vtop = 4e6
    sig = (1.0e-19, 0.6e-19, 0.3e-19)
    xs = table_for(vtop, 1e5, n=513, sig_e=sig, exc_threshold_ev=1e-3, ion_threshold_ev=1e-3)
    p = params(gap_m=1e3, n_cells=16, pressure_pa=400.0, flags=NO_FIELD | RECORD, sort_interval=0,
               capacity=(400_000, 400_000))
    sim = ora.Oracle(p, xs)
    n = 150_000
    rng = np.random.default_rng(12)
    frac = 384 / 512.0
    v0 = 384 * xs.dv_e
    sim.set_state(0, rng.uniform(400, 600, n), *iso_velocities(n, v0, rng))
    sim.set_state(1, np.zeros(0), np.zeros(0), np.zeros(0), np.zeros(0))
    sim.step(1)
    code = _code_coll(sim.decisions(0))
    cand = code > 0
    obs = np.array([(code == k).sum() for k in (2, 3, 4, 1)], dtype=float)
    st = sum(sig)
    prob = np.array([sig[0] / st * frac, sig[1] / st * frac, sig[2] / st * frac, 1 - frac])
    expect = cand.sum() * prob
    chi2 = ((obs - expect) ** 2 / expect).sum()
    assert chi2 < 16.3, (obs, expect)  # 3 dof, 99.9%
    # candidates themselves: Binomial(n, P_coll)
    pc = sim.derived()["p_coll_e"]
    assert abs(cand.sum() - n * pc) < 5 * np.sqrt(n * pc * (1 - pc))


def _collide_once(ora, sig_e, thresholds=(11.5, 15.8), n=60_000, speed=3e6, seed=13):
    xs = table_for(6e6, 1e5, n=1025, sig_e=sig_e, exc_threshold_ev=thresholds[0],
                   ion_threshold_ev=thresholds[1])
    p = params(gap_m=1e3, n_cells=16, pressure_pa=2000.0, flags=NO_FIELD | RECORD, sort_interval=0,
               capacity=(3 * n, 3 * n))
    sim = ora.Oracle(p, xs)
    rng = np.random.default_rng(seed)
    v = np.array(iso_velocities(n, speed, rng))
    v *= rng.uniform(0.5, 1.0, n)
    x = rng.uniform(400, 600, n)
    sim.set_state(0, x, *v)
    sim.set_state(1, np.zeros(0), np.zeros(0), np.zeros(0), np.zeros(0))
    sim.step(1)
    return sim, x, v, _code_coll(sim.decisions(0))


def test_elastic_kinematics_conservation_and_mean_loss(ora):
    sim, x, v, code = _collide_once(ora, (2e-19, 0.0, 0.0))
    xo, vx, vy, vz = sim.get_state(0)
    assert xo.size == x.size  # nothing absorbed, nothing born
    hit = code == 2
    assert hit.sum() > 5000
    vin = v[:, hit]
    vout = np.array([vx[hit], vy[hit], vz[hit]])
    m, M = ME, MAR
    # momentum: the atom (at rest before) takes m (v - v') / M; energy is
    # conserved including that recoil
    va = m * (vin - vout) / M
    e_in = 0.5 * m * (vin**2).sum(0)
    e_out = 0.5 * m * (vout**2).sum(0) + 0.5 * M * (va**2).sum(0)
    assert np.max(np.abs(e_out / e_in - 1)) < 1e-9
    # isotropic in the CM frame: <d eps / eps> = -2 m M / (m + M)^2 and the
    # scattering cosine has mean 0 and mean square 1/3
    vcm = m / (m + M) * vin
    u = vout - vcm
    g = np.sqrt((vin**2).sum(0))
    cosx = (u * vin).sum(0) / (np.sqrt((u**2).sum(0)) * g)
    assert abs(cosx.mean()) < 5 / np.sqrt(3 * hit.sum())
    assert abs((cosx**2).mean() - 1 / 3) < 5 * np.sqrt(4 / 45 / hit.sum())
    de = ((vout**2).sum(0) - (vin**2).sum(0)) / (vin**2).sum(0)
    expect = -2 * m * M / (m + M) ** 2
    sd = abs(expect) / np.sqrt(3)
    assert abs(de.mean() - expect) < 5 * sd / np.sqrt(hit.sum())


def test_inelastic_energy_bookkeeping(ora):
    # excitation removes exactly the threshold; ionization shares the rest
    # between the scattered electron (same slot) and the ejected one (the
    # next slot), and a thermal ion is appended in parent order
    sim, x, v, code = _collide_once(ora, (0.0, 1e-19, 1e-19), thresholds=(11.5, 15.8),
                                    speed=4e6)
    xo, vx, vy, vz = sim.get_state(0)
    e_in = energy_ev(ME, *v)
    e_out = energy_ev(ME, vx, vy, vz)
    # map parent slots to output slots: survivors in order, child after parent
    out_idx = np.cumsum(1 + (code == 4)) - 1 - (code == 4)
    exc = code == 3
    ion = code == 4
    assert exc.sum() > 1000 and ion.sum() > 1000
    np.testing.assert_allclose(e_out[out_idx[exc]], np.maximum(e_in[exc] - 11.5, 0), rtol=1e-12,
                               atol=1e-12)
    pair = e_out[out_idx[ion]] + e_out[out_idx[ion] + 1]
    np.testing.assert_allclose(pair, np.maximum(e_in[ion] - 15.8, 0), rtol=1e-12, atol=1e-12)
    # children sit at their parent's position
    assert np.array_equal(xo[out_idx[ion] + 1], xo[out_idx[ion]])
    xi, vix, viy, viz = sim.get_state(1)
    assert xi.size == ion.sum()
    assert np.array_equal(xi, xo[out_idx[ion]])
    # ions born thermal at 300 K: <1/2 M v^2> = 3/2 k T
    ei = 0.5 * MAR * (vix**2 + viy**2 + viz**2)
    assert abs(ei.mean() / (1.5 * KB * 300.0) - 1) < 5 * np.sqrt(2 / 3 / xi.size)
    c = sim.counters()
    # P_{n+1} = P_n - absorbed + born
    assert xo.size == x.size + c[10]
    assert c[9] == exc.sum() and c[10] == ion.sum()


def test_ion_gas_relaxation_to_maxwellian(ora):
    # With E = 0, ions loaded hot relax through isotropic and backward
    # collisions with a 300 K gas to a Maxwellian at T_g (detailed balance).
    xs = xsec.argon_synthetic()
    p = params(gap_m=100.0, n_cells=16, pressure_pa=100.0, steps_per_cycle=20,
               flags=NO_FIELD, sort_interval=0, capacity=(8, 40_000))
    sim = ora.Oracle(p, xs)
    n = 20_000
    rng = np.random.default_rng(14)
    s = np.sqrt(0.3 * QE / MAR)
    sim.set_state(1, rng.uniform(40, 60, n), *rng.normal(0, s, (3, n)))
    sim.set_state(0, np.zeros(0), np.zeros(0), np.zeros(0), np.zeros(0))
    sim.step(300)
    _, vx, vy, vz = sim.get_state(1)
    v2 = vx**2 + vy**2 + vz**2
    kt = KB * 300.0
    assert abs(0.5 * MAR * v2.mean() / (1.5 * kt) - 1) < 0.03
    # Maxwellian speed-squared moments: <v^4>/<v^2>^2 = 5/3
    assert abs((v2**2).mean() / v2.mean() ** 2 / (5 / 3) - 1) < 0.05
    # each velocity component is Gaussian: kurtosis 3
    k = (vx**4).mean() / (vx**2).mean() ** 2
    assert abs(k - 3) < 0.15


def test_cross_section_scale_matches_paper_collision_probabilities(ora):
    # Sec. 3.5 prints the electron collision probability of the 10 Pa base
    # cases at their lowest stable N_t (tests/golden fixture); the synthetic
    # cross sections must give comparable values.
    xs = xsec.argon_synthetic()
    path = os.path.join(os.path.dirname(__file__), "golden", "paper_sec35_collision_probability.txt")
    rows = np.loadtxt(path, comments="#", ndmin=2)
    assert len(rows) == 2
    for pa, Nt, target, tol in rows:
        sim = ora.Oracle(params(pressure_pa=float(pa), steps_per_cycle=int(Nt)), xs)
        pc = sim.derived()["p_coll_e"]
        assert abs(pc / target - 1) < tol, (Nt, pc)


def test_speed_beyond_table_uses_last_entry(ora):
    # Candidates faster than the last table speed collide with the last
    # tabulated frequency (<= nu_max, so the null-collision bound holds) and
    # are counted. With a constant sigma, nu(v_last) = nu_max: every
    # candidate is a real collision.
    vtop = 1e6
    xs = table_for(vtop, 1e5, n=65, sig_e=(1e-19, 0.0, 0.0))
    p = params(gap_m=1e3, n_cells=16, pressure_pa=300.0, flags=NO_FIELD | RECORD, sort_interval=0,
               capacity=(20_000, 8))
    sim = ora.Oracle(p, xs)
    n = 20_000
    rng = np.random.default_rng(15)
    sim.set_state(0, rng.uniform(400, 600, n), *iso_velocities(n, 3 * vtop, rng))
    sim.set_state(1, np.zeros(0), np.zeros(0), np.zeros(0), np.zeros(0))
    assert sim.step(1) == 0
    code = _code_coll(sim.decisions(0))
    c = sim.counters()
    assert c[15] == (code > 0).sum() > 0      # every candidate was beyond the table
    assert (code == 1).sum() == 0             # and none was a null event
    assert c[8] == (code == 2).sum()


def test_candidacy_draws_are_independent_within_a_block(ora):
    # Four consecutive slots share one Philox block for their candidacy
    # uniforms (one word each). With P_coll = 1/2 the 16 candidacy patterns
    # of a group of four slots must be equally likely: a reused or shifted
    # word would concentrate them (e.g. on 0000 and 1111).
    vtop = 4e6
    p = params(gap_m=1e3, n_cells=16, pressure_pa=50.0, flags=NO_FIELD | RECORD, sort_interval=0,
               capacity=(40_000, 8))
    ng = p["pressure_pa"] / (KB * p["gas_temp_k"])
    sigma = np.log(2.0) / (ng * vtop * dt_of(p))
    xs = table_for(vtop, 1e5, n=513, sig_e=(sigma, 0.0, 0.0))
    sim = ora.Oracle(p, xs)
    assert abs(sim.derived()["p_coll_e"] - 0.5) < 1e-9
    n = 40_000
    rng = np.random.default_rng(5)
    sim.set_state(0, rng.uniform(400, 600, n), *iso_velocities(n, 0.5 * vtop, rng))
    sim.set_state(1, np.zeros(0), np.zeros(0), np.zeros(0), np.zeros(0))
    chi2 = []
    for _ in range(3):
        sim.step(1)
        cand = (_code_coll(sim.decisions(0)) != 0).astype(int).reshape(-1, 4)
        assert abs(cand.mean() - 0.5) < 5 * np.sqrt(0.25 / n)
        pattern = cand @ np.array([1, 2, 4, 8])
        obs = np.bincount(pattern, minlength=16)
        expect = n / 4 / 16
        chi2.append(((obs - expect) ** 2 / expect).sum())
    assert max(chi2) < 45, chi2  # 15 dof: 99.9% quantile ~ 37.7
