"""The OpenMP build of the oracle (used only to time the oracle on several
cores) computes what the plain build computes: a pass split into
slot-ordered runs, one per thread, joined in slot order, with integer
deposits summed over threads, gives the same states, decisions, counters
and time averages bit for bit."""
import numpy as np

from pic_inputs import state, workloads, xsec


def _run(ora, openmp):
    w = workloads.scaled(workloads.get("c1_small"), 6000)
    p = dict(w["params"], reflection=0.3, gamma_see=0.2, flags=16, sort_interval=25,
             rf_voltage_v=200.0, ion_subcycle=2)
    o = ora.Oracle(p, xsec.argon_synthetic(), openmp=openmp)
    init = state.initial_state(w, seed=5)
    for sp in (0, 1):
        o.set_state(sp, *init[sp], step=0)
    assert o.step(120) == 0
    o.measure(True)
    assert o.step(80) == 0
    m = o.moments()
    r = o.wall_raw()
    return ([*o.get_state(0), *o.get_state(1), o.counters(), o.decisions(0), o.decisions(1),
             m["n_e"], m["n_i"], m["eepf"], r["hits"], r["absorbed"], r["hist"]])


def test_openmp_build_equals_plain_build(ora):
    assert ora.threads(openmp=False) == 1
    assert ora.threads(openmp=True) >= 1
    a, b = _run(ora, False), _run(ora, True)
    for k, (x, y) in enumerate(zip(a, b)):
        assert np.array_equal(np.asarray(x), np.asarray(y)), k
