"""Pipelined electron steps against unpipelined ones. With the pipeline on
(pic_set_pipeline; the default), within one call of pic_step the electron emit of a step
also decides the next step (its push,
candidacy, wall and collision decisions, deposit and tile totals), so the
next step has no decide pass; a call of one step never does this. The
arithmetic is the same, so runs of many steps in one call must equal the
same steps taken one call at a time bit for bit: states, decisions, event
counters, deposits and fields. The one-step path is the one the
single-step parity tests hold against the oracle."""
import numpy as np
import pytest

from gpu_common import assert_state_equal, near_wall_state, need_gpu
from helpers import ANISO, MAR, ME, OPAL, QE, RECORD, THOMAS
from pic_inputs import state, workloads, xsec

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _vth(T_ev, m):
    return np.sqrt(T_ev * QE / m)


def _pair(p, xs, init, step=0):
    from paper_2109_04469_amd import Discharge

    ds = []
    for _ in range(2):
        d = Discharge(p, xs, "cuda:0")
        for sp in (0, 1):
            d.set_state(sp, *init[sp], step=step)
        ds.append(d)
    return ds


def _same(a, b, what):
    assert a.sync() == 0 and b.sync() == 0, what
    for sp in (0, 1):
        assert_state_equal(a.get_state(sp), b.get_state(sp), what=f"{what} species {sp}")
        assert np.array_equal(a.decisions(sp), b.decisions(sp)), f"{what}: decisions {sp}"
    assert np.array_equal(a.counters(), b.counters()), f"{what}: counters"
    fa, fb = a.get_field(), b.get_field()
    for k in ("dep_e", "dep_i", "E"):
        assert np.array_equal(fa[k], fb[k]), f"{what}: {k}"


CASES = {
    # collisions, reflection, emission, sub-cycled ions, sorts
    "small_collisional": dict(base="c1_small", n=9000, over=dict(
        reflection=0.3, gamma_see=0.3, ion_subcycle=3, sort_interval=7, pressure_pa=40.0,
        rf_voltage_v=250.0, flags=RECORD)),
    # the Thomas solver, no sorting (pool repacks every 256 steps)
    "thomas_no_sort": dict(base="c1_small", n=6000, over=dict(
        reflection=0.5, gamma_see=0.1, ion_subcycle=1, sort_interval=0, flags=RECORD | THOMAS)),
    # the method variants (the queued-slot kernels with their paths)
    "variants": dict(base="c1_small", n=7000, over=dict(
        reflection=0.2, gamma_see=0.2, ion_subcycle=2, sort_interval=11, pressure_pa=80.0,
        flags=RECORD | ANISO | OPAL)),
    # the production-shaped discharge (512 cells, 50 Pa, 300 V, gamma 0.1)
    "production_shape": dict(base="c2_production", n=20_000, over=dict(
        sort_interval=13, flags=RECORD)),
    # the largest grid (4096 cells): the fused kernel stages the field of
    # both steps and its deposit histogram over 4097 nodes
    "largest_grid": dict(base="c1_small", n=12_000, over=dict(
        n_cells=4096, reflection=0.3, gamma_see=0.2, ion_subcycle=4, sort_interval=17,
        pressure_pa=30.0, flags=RECORD)),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_pipelined_steps_equal_single_steps(name):
    c = CASES[name]
    w = workloads.scaled(workloads.get(c["base"]), c["n"])
    p = dict(w["params"], **c["over"])
    xs = xsec.argon_synthetic()
    L = p["gap_m"]
    dt = 1.0 / (p["rf_freq_hz"] * p["steps_per_cycle"])
    ve, vi = _vth(8.0, ME), _vth(20.0, MAR)
    init = {0: near_wall_state(w["n_init"][0], L, ve, ve * dt, 3, 0),
            1: near_wall_state(w["n_init"][1], L, vi, vi * dt * p["ion_subcycle"], 3, 1)}
    many, single = _pair(p, xs, init)
    off = _pair(p, xs, init)[0]
    many.set_pipeline(True)
    off.set_pipeline(False)
    for k, n in enumerate((1, 2, 37, 9, 300)):
        print(f"[pipeline] {name}: call {k} of {n} steps", flush=True)
        many.step(n)
        off.step(n)
        for _ in range(n):
            single.step(1)
        _same(many, single, f"{name} after call {k}")
        _same(off, single, f"{name} unpipelined, after call {k}")


def test_pipelined_steps_with_measurement_switching():
    # measuring steps are not pipelined; switching between calls
    w = workloads.scaled(workloads.get("c1_small"), 8000)
    p = dict(w["params"], reflection=0.3, gamma_see=0.2, flags=RECORD)
    xs = xsec.argon_synthetic()
    init = state.initial_state(w, seed=12)
    many, single = _pair(p, xs, init)
    many.set_pipeline(True)
    for k, (n, meas) in enumerate(((20, False), (15, True), (30, False), (12, True))):
        for d in (many, single):
            d.measure(meas)
        many.step(n)
        for _ in range(n):
            single.step(1)
        _same(many, single, f"measure call {k}")
        if meas:
            ma, mb = many.moments(reset=True), single.moments(reset=True)
            for key in ("n_e", "n_i", "eepf"):
                assert np.array_equal(ma[key], mb[key]), key
            np.testing.assert_allclose(ma["mean_energy_e"], mb["mean_energy_e"], rtol=1e-12)


def test_pipelined_large_workload_equals_single_steps():
    # the large low-pressure workload at full size (4M + 4M), ions sub-cycled
    # x10: 23 steps in one call against 23 calls of one step
    w = workloads.get("c3_large_lowp")
    p = dict(w["params"], flags=RECORD)
    xs = xsec.argon_synthetic()
    init = state.initial_state(w)
    many, single = _pair(p, xs, init)
    many.set_pipeline(True)
    many.step(23)
    for _ in range(23):
        single.step(1)
    _same(many, single, "c3 23 steps")


@pytest.mark.parametrize("empty", [0, 1])
def test_pipelined_steps_from_an_empty_species(empty):
    # no electrons at the start (ion impacts emit the first ones) or no ions
    # (ionizations make the first ones): the fused kernel and the candidacy
    # draw meet empty passes and then the first particles of a species;
    # calls of several steps against single steps, bit for bit. (Without
    # ions the electrons' own space charge heats them within tens of steps;
    # the pressure, the step count and the capacities keep the ionization
    # growth inside the arrays.)
    w = workloads.scaled(workloads.get("c1_small"), 6000, capacity_factor=8)
    p = dict(w["params"], reflection=0.2, gamma_see=0.4, ion_subcycle=3, sort_interval=0,
             pressure_pa=20.0, rf_voltage_v=150.0, flags=RECORD)
    xs = xsec.argon_synthetic()
    L = p["gap_m"]
    dt = 1.0 / (p["rf_freq_hz"] * p["steps_per_cycle"])
    ve, vi = _vth(8.0, ME), _vth(20.0, MAR)
    init = {0: near_wall_state(6000, L, ve, ve * dt, 5, 0),
            1: near_wall_state(6000, L, vi, vi * dt * p["ion_subcycle"], 5, 1)}
    z = np.zeros(0)
    init[empty] = (z, z, z, z)
    many, single = _pair(p, xs, init)
    many.set_pipeline(True)
    for k, n in enumerate((1, 7, 22)):
        print(f"[pipeline] empty species {empty}: call {k} of {n} steps", flush=True)
        many.step(n)
        for _ in range(n):
            single.step(1)
        _same(many, single, f"empty species {empty}, after call {k}")
    assert many.count(empty) > 0, "the empty species gained particles"


def test_pipelined_steps_with_the_smaller_decide_workgroups():
    # the decide kernels compiled for 256 threads feed the fused kernel on
    # the steps that cannot be pipelined (the first of a call, after ion
    # steps); against single steps with the default 512-thread decide
    w = workloads.scaled(workloads.get("c1_small"), 30_001)
    p = dict(w["params"], reflection=0.3, gamma_see=0.2, ion_subcycle=4, sort_interval=19,
             pressure_pa=30.0, flags=RECORD)
    xs = xsec.argon_synthetic()
    init = state.initial_state(w, seed=14)
    many, single = _pair(p, xs, init)
    many.set_pipeline(True)
    many.set_decide_block(256)
    for k, n in enumerate((3, 41)):
        print(f"[pipeline] 256-thread decide: call {k} of {n} steps", flush=True)
        many.step(n)
        for _ in range(n):
            single.step(1)
        _same(many, single, f"256-thread decide, after call {k}")
