"""GPU (libpic through the C ABI) against the CPU oracle.

Single steps from a shared state must agree exactly in every decision
(absorption, reflection, emission, collision process), in particle counts,
slot order and integer deposits, and within 1e-12 relative in positions and
velocities (only the scattering transcendentals may differ by ulps).
"""
import numpy as np
import pytest

from gpu_common import assert_state_close, assert_state_equal, near_wall_state, need_gpu, pair
from helpers import FIXED_E, NO_COLL, RECORD, THOMAS, ME, MAR, QE, params
from pic_inputs import state, workloads, xsec

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _vth(T_ev, m):
    return np.sqrt(T_ev * QE / m)


def test_philox_matches_oracle():
    import oracle
    from paper_2109_04469_amd import selftest_philox

    rng = np.random.default_rng(1)
    n = 4096
    ctr = rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    key = np.array([123456789, 987654321], dtype=np.uint32)
    got = selftest_philox(ctr, key)
    for i in range(0, n, 37):
        assert np.array_equal(got[i], oracle.philox4x32_10(ctr[i], key)), i


def test_sqrt_correctly_rounded():
    from paper_2109_04469_amd import selftest_sqrt

    rng = np.random.default_rng(2)
    x = np.concatenate([
        rng.uniform(0, 1, 400_000),
        np.exp(rng.uniform(-700, 700, 400_000)),
        rng.uniform(0, 1e14, 200_000),  # squared speeds of the method
        np.array([0.0, 1.0, 2.0, 4.0, np.finfo(float).tiny, np.finfo(float).max]),
    ])
    # numpy's sqrt is the IEEE correctly rounded square root
    assert np.array_equal(selftest_sqrt(x), np.sqrt(x))


@pytest.mark.parametrize("n", [1, 1023, 1024, 5000, 37_001])
def test_deposit_exact(n):
    p = params(n_cells=128, capacity=(40_000, 40_000))
    xs = xsec.argon_synthetic()
    L = p["gap_m"]
    rng = np.random.default_rng(n)
    x = rng.uniform(0, L, n)
    x[: min(n, 3)] = [0.0, L, 0.5 * L][: min(n, 3)]
    z = np.zeros(n)
    init = {0: (x, z, z, z), 1: (x[::-1].copy(), z, z, z)}
    gpu, ora = pair(p, xs, init)
    ora.deposit()
    fg, fo = gpu.get_field(), ora.get_field()
    assert np.array_equal(fg["dep_e"], fo["dep_e"])
    assert np.array_equal(fg["dep_i"], fo["dep_i"])
    assert int(fg["dep_e"].sum()) == n * 2**32


def _field_case(mode_flags, n_cells, seed):
    p = params(n_cells=n_cells, flags=NO_COLL | mode_flags, capacity=(60_000, 60_000), sort_interval=0)
    xs = xsec.argon_synthetic()
    rng = np.random.default_rng(seed)
    L = p["gap_m"]
    # non-uniform charge: electrons depleted near the walls (sheath-like)
    xe = rng.uniform(0.1 * L, 0.9 * L, 20_000)
    xi = rng.uniform(0, L, 21_000)
    init = {0: (xe, *np.zeros((3, xe.size))), 1: (xi, *np.zeros((3, xi.size)))}
    gpu, ora = pair(p, xs, init, step=7)
    gpu.step(1)
    ora.step(1)
    return gpu.get_field(), ora.get_field(), p


@pytest.mark.parametrize("n_cells", [128, 512, 2048, 4096])
def test_field_thomas_bitwise(n_cells):
    fg, fo, _ = _field_case(THOMAS, n_cells, 5)
    assert np.array_equal(fg["rho"], fo["rho"])
    assert np.array_equal(fg["phi"], fo["phi"])
    assert np.array_equal(fg["E"], fo["E"])


@pytest.mark.parametrize("n_cells", [128, 512, 2048, 4096])
def test_field_exact_solver_within_rounding(n_cells):
    # The default solver sums the integer deposits exactly and rounds a few
    # times per node; the oracle's Thomas recurrence accumulates rounding over
    # the grid. Both are within a few hundred ulps of max|phi| (max|E| dx).
    fg, fo, p = _field_case(0, n_cells, 6)
    assert np.array_equal(fg["rho"], fo["rho"])
    eps = np.finfo(float).eps
    nx = n_cells + 1
    phis = np.max(np.abs(fo["phi"]))
    assert np.max(np.abs(fg["phi"] - fo["phi"])) < 8 * nx * eps * phis
    dx = p["gap_m"] / n_cells
    Es = max(np.max(np.abs(fo["E"])), phis / dx)
    assert np.max(np.abs(fg["E"] - fo["E"])) < 8 * nx * eps * Es


def _single_step_case(n, seed, step, subcycle, flags, R=0.3, gamma=0.25, n_cells=128):
    p = params(n_cells=n_cells, reflection=R, gamma_see=gamma, ion_subcycle=subcycle,
               flags=flags | RECORD, capacity=(3 * n + 64, 3 * n + 64), sort_interval=0,
               pressure_pa=30.0)
    xs = xsec.argon_synthetic()
    L = p["gap_m"]
    dt = 1.0 / (p["rf_freq_hz"] * p["steps_per_cycle"])
    ve = _vth(3.0, ME)
    vi = _vth(50.0, MAR)
    e = near_wall_state(n, L, ve, ve * dt, seed, 0)
    i = near_wall_state(n + 17, L, vi, vi * dt * subcycle, seed, 1)
    rng = np.random.default_rng(seed + 1)
    E = rng.normal(0, 3e4, n_cells + 1) if flags & FIXED_E else None
    return p, xs, {0: e, 1: i}, E, L, ve, vi


@pytest.mark.parametrize("n,seed,step,subcycle,n_cells", [
    (5000, 1, 0, 1, 128), (20_011, 2, 3, 1, 128), (7_777, 3, 10, 5, 128), (7_777, 4, 11, 5, 128),
    (1, 5, 0, 1, 128), (30_001, 6, 2, 1, 4096)])
def test_single_step_fixed_field(n, seed, step, subcycle, n_cells):
    # the last case uses the largest grid (4096 cells, 4097 nodes)
    p, xs, init, E, L, ve, vi = _single_step_case(n, seed, step, subcycle, FIXED_E, n_cells=n_cells)
    gpu, ora = pair(p, xs, init, step=step, fixed_E=E)
    gpu.step(1)
    ora.step(1)
    for sp, vs in ((0, ve), (1, vi)):
        assert np.array_equal(gpu.decisions(sp), ora.decisions(sp)), f"decisions species {sp}"
        assert_state_close(gpu.get_state(sp), ora.get_state(sp), L, vs, what=f"species {sp}")
    assert np.array_equal(gpu.counters(), ora.counters())
    fg, fo = gpu.get_field(), (ora.deposit() or ora.get_field())
    assert np.array_equal(fg["dep_e"], fo["dep_e"])
    assert np.array_equal(fg["dep_i"], fo["dep_i"])


@pytest.mark.parametrize("empty", [0, 1, 2])
def test_empty_species_steps_match_oracle(empty):
    # no electrons (ion impacts emit the first ones), no ions (ionizations
    # make the first ones) or neither: three steps, each from the state the
    # last one left, against the oracle stepped alongside
    p, xs, init, E, L, ve, vi = _single_step_case(4000, 8, 0, 1, FIXED_E, R=0.2, gamma=0.4)
    z = np.zeros(0)
    for sp in ((0,) if empty == 0 else (1,) if empty == 1 else (0, 1)):
        init[sp] = (z, z, z, z)
    gpu, ora = pair(p, xs, init, step=0, fixed_E=E)
    for k in range(3):
        # the GPU's counters restart with each set_state; the oracle's run on
        oc0 = np.asarray(ora.counters()).copy()
        gpu.step(1)
        assert ora.step(1) == 0
        assert gpu.sync() == 0
        assert np.array_equal(gpu.counters(), np.asarray(ora.counters()) - oc0), f"step {k}"
        for sp, vs in ((0, ve), (1, vi)):
            assert np.array_equal(gpu.decisions(sp), ora.decisions(sp)), f"step {k} decisions {sp}"
            assert_state_close(gpu.get_state(sp), ora.get_state(sp), L, vs, what=f"step {k} sp {sp}")
        # the next step starts from the oracle's state on both sides
        for sp in (0, 1):
            gpu.set_state(sp, *ora.get_state(sp), step=k + 1)
    if empty == 2:
        assert gpu.count(0) == 0 and gpu.count(1) == 0


def test_single_step_with_field_solve_thomas():
    # the whole step including deposit and Thomas solve, from an evolved state
    w = workloads.scaled(workloads.get("c1_small"), 6000)
    p = dict(w["params"], flags=RECORD | THOMAS, gamma_see=0.2, reflection=0.3, sort_interval=10)
    xs = xsec.argon_synthetic()
    import oracle as O

    warm = O.Oracle(p, xs)
    init = state.initial_state(w, seed=9)
    for sp in (0, 1):
        warm.set_state(sp, *init[sp], step=0)
    assert warm.step(40) == 0
    st = {sp: warm.get_state(sp) for sp in (0, 1)}
    gpu, ora = pair(p, xs, st, step=40)
    gpu.step(1)
    ora.step(1)
    assert np.array_equal(gpu.get_field()["E"], ora.get_field()["E"])
    for sp, vs in ((0, _vth(2.0, ME)), (1, _vth(0.03, MAR))):
        assert np.array_equal(gpu.decisions(sp), ora.decisions(sp))
        assert_state_close(gpu.get_state(sp), ora.get_state(sp), p["gap_m"], vs, what=f"sp {sp}")


def test_multi_step_bitwise_without_collisions():
    # No transcendental enters a collisionless step with R > 0 and gamma = 0:
    # 300 steps with Thomas solves, wall reflections, compaction and cell sorts
    # must reproduce the oracle bit for bit.
    w = workloads.scaled(workloads.get("c1_small"), 8000)
    p = dict(w["params"], flags=NO_COLL | THOMAS, reflection=0.4, gamma_see=0.0, sort_interval=25)
    xs = xsec.argon_synthetic()
    init = state.initial_state(w, seed=4)
    gpu, ora = pair(p, xs, init)
    for _ in range(3):
        gpu.step(100)
        assert ora.step(100) == 0
        for sp in (0, 1):
            assert_state_equal(gpu.get_state(sp), ora.get_state(sp), what=f"species {sp}")
    assert np.array_equal(gpu.counters(), ora.counters())


def test_multi_step_default_solver_close():
    # Same run with the default (exact-integer) Poisson solver: states agree
    # to rounding level after 60 steps, counts and wall events exactly.
    w = workloads.scaled(workloads.get("c1_small"), 8000)
    p = dict(w["params"], flags=NO_COLL, reflection=0.4, gamma_see=0.0, sort_interval=25)
    xs = xsec.argon_synthetic()
    init = state.initial_state(w, seed=4)
    gpu, ora = pair(p, xs, init)
    gpu.step(60)
    assert ora.step(60) == 0
    for sp, vs in ((0, _vth(2.0, ME)), (1, _vth(0.03, MAR))):
        assert_state_close(gpu.get_state(sp), ora.get_state(sp), p["gap_m"], vs, rtol=1e-9,
                           what=f"species {sp}")
    assert np.array_equal(gpu.counters(), ora.counters())


def test_determinism_and_exact_resume():
    w = workloads.scaled(workloads.get("c1_small"), 6000)
    p = dict(w["params"], sort_interval=20)
    xs = xsec.argon_synthetic()
    init = state.initial_state(w, seed=8)
    from paper_2109_04469_amd import Discharge

    def run(split):
        d = Discharge(p, xs)
        for sp in (0, 1):
            d.set_state(sp, *init[sp], step=0)
        if split:
            d.step(50)
            st = {sp: d.get_state(sp) for sp in (0, 1)}
            s = d.step_index
            d = Discharge(p, xs)
            for sp in (0, 1):
                d.set_state(sp, *st[sp], step=s)
            d.step(50)
        else:
            d.step(100)
        return [d.get_state(sp) for sp in (0, 1)]

    a, b, c = run(False), run(False), run(True)
    for sp in (0, 1):
        assert_state_equal(a[sp], b[sp], what="rerun")
        assert_state_equal(a[sp], c[sp], what="resume")


def test_full_size_c3_steps_match_oracle():
    # The large workload at its full size (4M electrons + 4M ions, 2049
    # nodes) in the library's default launch configuration, the one bench.py
    # times, with the default solver. The oracle runs the same steps (about a
    # second each on one core); every decision, count and counter must agree
    # and states within rounding. Step 0 moves both species (ion
    # sub-cycling x10), steps 1-2 the electrons; a cell sort after step 2.
    w = workloads.get("c3_large_lowp")
    p = dict(w["params"], flags=RECORD, sort_interval=2)
    xs = xsec.argon_synthetic()
    init = state.initial_state(w)
    gpu, ora = pair(p, xs, init)
    L = p["gap_m"]
    for k in range(3):
        gpu.step(1)
        assert ora.step(1) == 0
        for sp, vs in ((0, _vth(2.0, ME)), (1, _vth(0.03, MAR))):
            dg, do = gpu.decisions(sp), ora.decisions(sp)
            assert dg.size == do.size, (k, sp)
            assert np.array_equal(dg, do), f"step {k} species {sp}: decisions"
            assert_state_close(gpu.get_state(sp), ora.get_state(sp), L, vs, rtol=1e-10,
                               what=f"step {k} species {sp}")
        assert np.array_equal(gpu.counters(), ora.counters()), f"step {k}"
    # the integer deposit of the GPU's own positions is exact at any size;
    # against the oracle's positions (other Poisson solver, rounding-level
    # differences) only a few fixed-point weights may move by one unit
    import oracle as O

    f = gpu.get_field()
    o = ora.deposit() or ora.get_field()
    nx = p["n_cells"] + 1
    inv_dx = 1.0 / (L / p["n_cells"])  # as both sides compute it
    for sp, key in ((0, "dep_e"), (1, "dep_i")):
        xg = gpu.get_state(sp)[0]
        assert np.array_equal(f[key], O.deposit_array(nx, inv_dx, xg)), key
        assert np.max(np.abs(f[key] - o[key])) <= 64, key


def test_measured_moments_match_oracle():
    # Time-averaged densities, CIC mean energy and the mid-gap EEPF over 30
    # measured steps (Sec. 3): the histogram counts are integers and must be
    # equal; the FP64 sums agree to rounding.
    w = workloads.scaled(workloads.get("c1_small"), 8000)
    p = dict(w["params"], flags=THOMAS, reflection=0.2, gamma_see=0.1)
    xs = xsec.argon_synthetic()
    init = state.initial_state(w, seed=12)
    gpu, ora = pair(p, xs, init)
    gpu.step(20)
    assert ora.step(20) == 0
    gpu.measure(True)
    ora.measure(True)
    gpu.step(30)
    assert ora.step(30) == 0
    mg, mo = gpu.moments(), ora.moments()
    assert mg["steps"] == mo["steps"] == 30
    for k in ("n_e", "n_i", "mean_energy_e", "eepf"):
        g, o = mg[k], mo[k]
        scale = max(np.max(np.abs(o)), 1e-300)
        assert np.max(np.abs(g - o)) <= 1e-9 * scale, k
    assert np.sum(mg["eepf"] > 0) == np.sum(mo["eepf"] > 0)


def test_capacity_overflow_is_reported():
    # Births beyond the output capacity are an error, not a silent drop:
    # 50 eV electrons at 300 Pa ionize in the first step, and the electron
    # arrays have no room beyond the initial count.
    w = workloads.scaled(workloads.get("c1_small"), 2000)
    p = dict(w["params"], capacity=(2000, 4000), pressure_pa=300.0)
    xs = xsec.argon_synthetic()
    L = p["gap_m"]
    e = state.maxwellian_uniform(2000, L, 50.0, 0, 3)
    i = state.maxwellian_uniform(2000, L, 0.03, 1, 3)
    from paper_2109_04469_amd import Discharge

    d = Discharge(p, xs)
    d.set_state(0, *e, step=0)
    d.set_state(1, *i, step=0)
    d.step(1)
    assert d.sync() == -3


@pytest.mark.parametrize("pipeline", [True, False])
def test_capacity_overflow_in_multi_step_calls_is_reported(pipeline):
    # The same overflow inside a call of several steps with sub-cycled ions,
    # so that (pipelined) the fused emit-and-decide kernel and the queued
    # slots it runs meet outputs, births and pool entries beyond the
    # capacities on every step after the first: the writes past them are
    # dropped and the error stays latched, so the state is not handed out.
    w = workloads.scaled(workloads.get("c1_small"), 2000)
    p = dict(w["params"], capacity=(2000, 4000), pressure_pa=300.0, ion_subcycle=4,
             sort_interval=0)
    xs = xsec.argon_synthetic()
    L = p["gap_m"]
    e = state.maxwellian_uniform(2000, L, 50.0, 0, 3)
    i = state.maxwellian_uniform(2000, L, 0.03, 1, 3)
    from paper_2109_04469_amd import Discharge, PicError

    d = Discharge(p, xs)
    d.set_pipeline(pipeline)
    d.set_state(0, *e, step=0)
    d.set_state(1, *i, step=0)
    d.step(7)
    assert d.sync() == -3
    with pytest.raises(PicError):
        d.get_state(0)
    assert d.sync() == -3


def test_timing_levels():
    w = workloads.scaled(workloads.get("c1_small"), 4000)
    p = dict(w["params"], ion_subcycle=5)
    xs = xsec.argon_synthetic()
    init = state.initial_state(w, seed=2)
    from paper_2109_04469_amd import Discharge, PicError

    d = Discharge(p, xs)
    for sp in (0, 1):
        d.set_state(sp, *init[sp], step=0)
    with pytest.raises(PicError):
        d.timing(3)
    d.set_pipeline(False)
    d.timing(1)
    d.step(10)
    t = d.get_timing(reset=True)
    assert t["electron"][1] == 10 and t["ion"][1] == 2 and t["field"][1] == 1
    assert t["e_decide"][1] == 0
    d.timing(2)
    d.step(10)
    t = d.get_timing(reset=True)
    assert t["e_decide"][1] == 10 and t["e_emit"][1] == 10 and t["i_decide"][1] == 2
    # pipelined steps have no decide pass of their own
    d.set_pipeline(True)
    d.step(10)
    t = d.get_timing(reset=True)
    assert 1 <= t["e_decide"][1] < 10 and t["e_emit"][1] == 10 and t["i_decide"][1] == 2
    assert all(v[0] > 0 for k, v in t.items() if v[1])
    d.timing(0)
    d.step(5)
    assert all(v[1] == 0 for v in d.get_timing().values())


def test_batched_sweep_equals_single_runs():
    # Independent discharges advanced together on their own streams compute
    # exactly what each computes alone.
    import torch

    from paper_2109_04469_amd import Discharge, step_many
    from pic_inputs import sweep

    sw = sweep.draw(6, seed=3, particles=(2_000, 20_000))
    init = sweep.initial_states(sw, seed=5)
    xs = xsec.argon_synthetic()
    streams = [torch.cuda.Stream() for _ in sw]
    batch = [Discharge(w["params"], xs, stream=s) for w, s in zip(sw, streams)]
    for d, st in zip(batch, init):
        for sp in (0, 1):
            d.set_state(sp, *st[sp], step=0)
    step_many(batch, 60, chunk=7)
    torch.cuda.synchronize()
    for w, st, d in zip(sw, init, batch):
        assert d.sync() == 0
        alone = Discharge(w["params"], xs)
        for sp in (0, 1):
            alone.set_state(sp, *st[sp], step=0)
        alone.step(60)
        assert alone.sync() == 0
        for sp in (0, 1):
            assert_state_equal(d.get_state(sp), alone.get_state(sp), what=f"{w['name']} sp {sp}")
        assert np.array_equal(d.counters(), alone.counters())


def test_batched_launches_equal_single_runs():
    # One launch per pass for all discharges of a batch: each discharge
    # computes exactly what it computes alone, across calls and upload
    # chunks, with mixed ion sub-cycling, sort intervals and measurement.
    import torch

    from paper_2109_04469_amd import Batch, Discharge
    from pic_inputs import sweep

    sw = sweep.draw(6, seed=11, particles=(2_000, 20_000))
    sw[1]["params"]["ion_subcycle"] = 3
    sw[4]["params"]["ion_subcycle"] = 4
    sw[2]["params"]["sort_interval"] = 20
    sw[3]["params"]["sort_interval"] = 0
    init = sweep.initial_states(sw, seed=7)
    xs = xsec.argon_synthetic()
    stream = torch.cuda.Stream()
    ds = [Discharge(w["params"], xs, stream=stream) for w in sw]
    for d, st in zip(ds, init):
        for sp in (0, 1):
            d.set_state(sp, *st[sp], step=0)
    for k in (0, 5):
        ds[k].measure(True)
    b = Batch(ds)
    b.step(100)   # two upload chunks
    b.step(1)
    b.step(29)
    torch.cuda.synchronize()
    for k, (w, st, d) in enumerate(zip(sw, init, ds)):
        assert d.sync() == 0
        alone = Discharge(w["params"], xs)
        for sp in (0, 1):
            alone.set_state(sp, *st[sp], step=0)
        if k in (0, 5):
            alone.measure(True)
        alone.step(130)
        assert alone.sync() == 0
        assert alone.step_index == d.step_index == 130
        for sp in (0, 1):
            assert_state_equal(d.get_state(sp), alone.get_state(sp), what=f"{w['name']} sp {sp}")
        assert np.array_equal(d.counters(), alone.counters())
        f1, f2 = d.get_field(), alone.get_field()
        for key in ("E", "dep_e", "dep_i"):
            assert np.array_equal(f1[key], f2[key]), key
        if k in (0, 5):
            m1, m2 = d.moments(), alone.moments()
            # densities and EEPF come from integer counts; the energy weights
            # are FP64 atomic sums whose order is not fixed
            for key in ("n_e", "n_i", "eepf"):
                assert np.array_equal(m1[key], m2[key]), key
            np.testing.assert_allclose(m1["mean_energy_e"], m2["mean_energy_e"], rtol=1e-12)
    # a single discharge may still step alone after batch steps
    ds[2].step(3)
    assert ds[2].sync() == 0
    b.close()


def test_alternating_single_and_batched_steps():
    # the tile-total buffers alternate between the passes of a species
    # whichever launch path runs them: single steps, batch steps and single
    # steps again give the bits of single steps throughout
    import torch

    from paper_2109_04469_amd import Batch, Discharge
    from pic_inputs import sweep

    sw = sweep.draw(3, seed=12, particles=(3_000, 30_000))
    sw[1]["params"]["ion_subcycle"] = 3
    init = sweep.initial_states(sw, seed=8)
    xs = xsec.argon_synthetic()
    stream = torch.cuda.Stream()
    ds = [Discharge(w["params"], xs, stream=stream) for w in sw]
    for d, st in zip(ds, init):
        for sp in (0, 1):
            d.set_state(sp, *st[sp], step=0)
    b = Batch(ds)
    for d in ds:
        d.step(7)
    b.step(11)
    ds[0].step(4)
    ds[1].step(4)
    ds[2].step(4)
    b.step(9)
    for d in ds:
        d.step(5)
    torch.cuda.synchronize()
    for w, st, d in zip(sw, init, ds):
        assert d.sync() == 0
        alone = Discharge(w["params"], xs)
        for sp in (0, 1):
            alone.set_state(sp, *st[sp], step=0)
        alone.step(36)
        assert alone.sync() == 0
        for sp in (0, 1):
            assert_state_equal(d.get_state(sp), alone.get_state(sp), what=f"{w['name']} sp {sp}")
        assert np.array_equal(d.counters(), alone.counters())
    b.close()


def test_batch_with_empty_populations():
    # a batch in which one discharge has no electrons and another no ions
    # at the start equals the same discharges stepped alone
    import torch

    from paper_2109_04469_amd import Batch, Discharge
    from pic_inputs import sweep

    sw = sweep.draw(3, seed=13, particles=(2_000, 8_000))
    init = sweep.initial_states(sw, seed=9)
    z = np.zeros(0)
    init[0][0] = (z, z, z, z)
    init[1][1] = (z, z, z, z)
    xs = xsec.argon_synthetic()
    stream = torch.cuda.Stream()
    ds = [Discharge(w["params"], xs, stream=stream) for w in sw]
    for d, st in zip(ds, init):
        for sp in (0, 1):
            d.set_state(sp, *st[sp], step=0)
    b = Batch(ds)
    b.step(25)
    torch.cuda.synchronize()
    for w, st, d in zip(sw, init, ds):
        assert d.sync() == 0
        alone = Discharge(w["params"], xs)
        for sp in (0, 1):
            alone.set_state(sp, *st[sp], step=0)
        alone.step(25)
        assert alone.sync() == 0
        for sp in (0, 1):
            assert_state_equal(d.get_state(sp), alone.get_state(sp), what=f"{w['name']} sp {sp}")
        assert np.array_equal(d.counters(), alone.counters())
    b.close()


def test_electrode_diagnostics_match_oracle():
    # Sec. 3.3 diagnostics over 40 measured steps of an evolving discharge
    # with reflection, emission and collisions: arrivals, absorptions and
    # ionizations are decisions (equal), the impact-energy sums FP64 (to
    # rounding), the flux-energy histograms integers (equal).
    import oracle

    w = workloads.scaled(workloads.get("c1_small"), 8000)
    p = dict(w["params"], flags=THOMAS, reflection=0.3, gamma_see=0.2, ion_subcycle=1,
             rf_voltage_v=150.0)
    xs = xsec.argon_synthetic()
    init = state.initial_state(w, seed=13)
    gpu, ora = pair(p, xs, init)
    gpu.step(30)
    assert ora.step(30) == 0
    gpu.measure(True)
    ora.measure(True)
    n0 = (gpu.count(1), ora.count(1))
    gpu.step(40)
    assert ora.step(40) == 0
    wg = gpu.wall_moments()
    wo = ora.wall_moments()
    r = wo["raw"]
    assert wg["steps"] == r["steps"] == 40
    assert np.array_equal(wg["arrivals"], r["hits"]) and r["hits"].sum() > 0
    assert np.array_equal(wg["absorbed"], r["absorbed"])
    assert wg["ionizations"] == r["ionizations"]
    np.testing.assert_allclose(wg["mean_energy_ev"], wo["mean_energy_ev"], rtol=1e-9)
    np.testing.assert_allclose(wg["flux"], wo["flux"], rtol=1e-14)
    assert wg["ionization_rate"] == pytest.approx(wo["ionization_rate"], rel=1e-14)
    np.testing.assert_allclose(wg["fedf_emax_ev"], r["emax"], rtol=0)
    assert np.array_equal(wg["fedf"], wo["fedf"])
    # the ion balance holds exactly on the GPU as well
    assert gpu.count(1) - n0[0] == wg["ionizations"] - wg["absorbed"][1].sum()
    # monitors from the time averages
    mg = gpu.monitors()
    mo = oracle.monitors(ora.moments(), p, (gpu.derived()["p_coll_e"], gpu.derived()["p_coll_i"]))
    for k in ("omega_pe_dt", "n_e_max", "n_e_center", "mean_energy_center_ev", "lambda_d_m",
              "dx_over_lambda_d", "n_d"):
        assert mg[k] == pytest.approx(mo[k], rel=1e-9), k
    assert mg["p_coll"] == pytest.approx(mo["p_coll"], rel=1e-15)
    # a moments reset clears the electrode diagnostics too
    gpu.moments(reset=True)
    assert gpu.wall_moments()["arrivals"].sum() == 0


def test_method_variants_single_step_match_oracle():
    # anisotropic elastic scattering and Opal sharing (flags): one step of a
    # hot, collisional state, as the default single-step cases. The forward
    # deflections put the pow() of cos chi through sqrt(1 - cos^2 chi), which
    # can amplify a last-bit difference of the two libm's by ~1e3, hence the
    # looser velocity bound (decisions are still exact).
    from helpers import ANISO, OPAL

    w = workloads.scaled(workloads.get("c1_small"), 12000)
    p = dict(w["params"], flags=RECORD | THOMAS | ANISO | OPAL, pressure_pa=80.0, gamma_see=0.1)
    xs = xsec.argon_synthetic()
    rng = np.random.default_rng(17)
    L = p["gap_m"]
    init = {}
    for sp, T, m in ((0, 25.0, ME), (1, 0.05, MAR)):
        n = 12000
        v = rng.normal(size=(3, n)) * _vth(T, m)
        init[sp] = (rng.uniform(0.05, 0.95, n) * L, v[0].copy(), v[1].copy(), v[2].copy())
    gpu, ora = pair(p, xs, init)
    gpu.step(1)
    ora.step(1)
    for sp, vs in ((0, _vth(25.0, ME)), (1, _vth(0.05, MAR))):
        dg, do = gpu.decisions(sp), ora.decisions(sp)
        assert np.array_equal(dg, do), f"decisions species {sp}"
        if sp == 0:
            assert np.sum(((dg >> 3) & 7) == 2) > 100 and np.sum(((dg >> 3) & 7) == 4) > 20
        assert_state_close(gpu.get_state(sp), ora.get_state(sp), L, vs, rtol=1e-10, what=f"species {sp}")
    assert np.array_equal(gpu.counters(), ora.counters())


def test_launch_shape_does_not_change_results():
    # grid sizes and the decide kernels' compiled workgroup size (512 or 256
    # threads) change which workgroup and thread take which slots, never a
    # result; 30,001 slots per species make 15 tiles, the last one ragged
    from paper_2109_04469_amd import Discharge, PicError

    w = workloads.scaled(workloads.get("c1_small"), 30_001)
    p = dict(w["params"], reflection=0.3, gamma_see=0.2, sort_interval=20)
    xs = xsec.argon_synthetic()
    init = state.initial_state(w, seed=21)
    ds = []
    for block, kd, ke in ((512, 1, 1), (512, 3, 4), (512, 2, 3), (256, 1, 2), (256, 8, 4)):
        d = Discharge(p, xs)
        for sp in (0, 1):
            d.set_state(sp, *init[sp], step=0)
        d.set_decide_block(block)
        d.set_launch(kd, ke)
        d.step(60)
        assert d.sync() == 0
        ds.append(d)
    for d in ds[1:]:
        for sp in (0, 1):
            assert_state_equal(d.get_state(sp), ds[0].get_state(sp), what=f"species {sp}")
        assert np.array_equal(d.counters(), ds[0].counters())
    kd, ke = ds[0].tune(10)
    assert kd >= 1 and ke >= 1 and ds[0].sync() == 0
    for bad in (0, 128, 384, 1024):
        with pytest.raises(PicError):
            ds[0].set_decide_block(bad)


def test_pass_tuner_keeps_results_and_reports_candidates():
    # the pass tuner times pipelined and unpipelined candidates on the
    # discharge itself; the steps it takes are ordinary steps, so a discharge
    # tuned along the way equals one stepped with the default schedule
    from paper_2109_04469_amd import Discharge

    w = workloads.scaled(workloads.get("c1_small"), 9000)
    p = dict(w["params"], reflection=0.3, gamma_see=0.2, sort_interval=20)
    xs = xsec.argon_synthetic()
    init = state.initial_state(w, seed=22)
    a, b = Discharge(p, xs), Discharge(p, xs)
    for d in (a, b):
        for sp in (0, 1):
            d.set_state(sp, *init[sp], step=0)
    res = a.tune_pass(steps_per_trial=12)
    n = len(res["trials"])
    assert n >= 4 and 0 <= res["best"] < n
    assert {t["pipeline"] for t in res["trials"]} == {True, False}
    assert {t["decide_block"] for t in res["trials"] if not t["pipeline"]} == {512, 256}
    assert all(t["us_per_step"] > 0.0 for t in res["trials"])
    best = res["trials"][res["best"]]
    assert best["us_per_step"] == min(t["us_per_step"] for t in res["trials"])
    b.step(12 * n)
    a.step(30)
    b.step(30)
    assert a.sync() == 0 and b.sync() == 0
    for sp in (0, 1):
        assert_state_equal(a.get_state(sp), b.get_state(sp), what=f"species {sp}")
    assert np.array_equal(a.counters(), b.counters())


@pytest.mark.parametrize("decide_block", [512, 256])
def test_workgroups_taking_several_tiles_match_oracle(decide_block):
    # More tiles than workgroups: 700,001 slots per species make 342 tiles of
    # 2048, against 256 workgroups at one per CU, so a workgroup takes two
    # tiles (the ion emit carries its prefix over the tiles in between), and
    # the last tile is ragged. The default shape (one tile per workgroup) and
    # the oracle must agree with it, with the decide kernels compiled for
    # either workgroup size.
    from paper_2109_04469_amd import Discharge

    w = workloads.scaled(workloads.get("c1_small"), 700_001)
    p = dict(w["params"], flags=RECORD, reflection=0.3, gamma_see=0.2)
    xs = xsec.argon_synthetic()
    init = state.initial_state(w, seed=33)
    L = p["gap_m"]
    gpu, ora = pair(p, xs, init)
    gpu.set_decide_block(decide_block)
    gpu.set_launch(1, 1)
    ref = Discharge(p, xs, "cuda:0")
    for sp in (0, 1):
        ref.set_state(sp, *init[sp], step=0)
    for k in range(3):
        gpu.step(1)
        ref.step(1)
        assert ora.step(1) == 0
        for sp, vs in ((0, _vth(2.0, ME)), (1, _vth(0.03, MAR))):
            assert np.array_equal(gpu.decisions(sp), ora.decisions(sp)), f"step {k} species {sp}"
            assert_state_close(gpu.get_state(sp), ora.get_state(sp), L, vs, rtol=1e-10,
                               what=f"step {k} species {sp}")
            assert_state_equal(ref.get_state(sp), gpu.get_state(sp), what=f"default shape, step {k}")
        assert np.array_equal(gpu.counters(), ora.counters()), f"step {k}"
        assert np.array_equal(ref.counters(), gpu.counters()), f"step {k}"


def test_batch_rejects_bad_handle_lists():
    import torch

    from paper_2109_04469_amd import Batch, Discharge, PicError

    w = workloads.scaled(workloads.get("c1_small"), 500)
    xs = xsec.argon_synthetic()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    a = Discharge(w["params"], xs, stream=s1)
    b = Discharge(w["params"], xs, stream=s2)
    c = Discharge(w["params"], xs, stream=s1)
    for bad in ([a, b], [a, a], []):
        with pytest.raises(PicError):
            Batch(bad)
    Batch([a, c]).close()
