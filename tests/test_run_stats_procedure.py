"""The run-level statistical comparison (tests/run_stats.py) on the CPU: its
false-alarm rate on synthetic ensembles drawn from one distribution, its
power against a shifted distribution, and the whole procedure on the oracle
against itself with independent seeds, with and without a mistake planted
in the oracle's inputs (electron cross sections doubled, as a factor-2 slip
in a table's units would do)."""
import numpy as np

import run_stats
from pic_inputs import workloads

NX, NB = 129, 128


def _synthetic_runs(rng, n, shift=0.0):
    """n runs of profile-like data: a common amplitude per run (the particle
    count fluctuates between seeds), smooth noise along the profile and
    white noise per node; EEPF-like bins with Poisson counts."""
    x = np.linspace(0, 1, NX)
    base = np.sin(np.pi * x) + 0.05
    runs = []
    for _ in range(n):
        amp = 1.0 + 0.03 * rng.normal()
        smooth = 0.01 * rng.normal() * np.cos(np.pi * x) + 0.01 * rng.normal() * np.sin(2 * np.pi * x)
        prof = (1.0 + shift * np.exp(-((x - 0.5) / 0.15) ** 2)) * base
        ne = 1e15 * (amp * prof + smooth + 0.01 * rng.normal(size=NX))
        ni = 1e15 * (amp * prof + smooth + 0.01 * rng.normal(size=NX)) * 1.1
        em = 3.0 + 0.05 * rng.normal(size=NX) + 0.02 * rng.normal()
        lam = 2000.0 * np.exp(-np.arange(NB) / 12.0)
        ep = rng.poisson(lam) / 1000.0
        runs.append({"n_e": ne, "n_i": ni, "mean_energy_e": em, "eepf": ep,
                     "ne": 10_000 * amp + 50 * rng.normal(), "ni": 11_000 * amp + 50 * rng.normal()})
    return runs


def test_false_alarm_rate_on_one_distribution():
    rng = np.random.default_rng(7)
    trials = 300
    fails = sum(not run_stats.compare(_synthetic_runs(rng, 8), _synthetic_runs(rng, 8))["ok"]
                for _ in range(trials))
    # 5 Hotelling tests at 0.1 % each plus the 99 % node rule
    assert fails / trials < 0.03, fails


def test_power_against_a_shifted_profile():
    rng = np.random.default_rng(8)
    trials = 50
    hits = sum(not run_stats.compare(_synthetic_runs(rng, 8), _synthetic_runs(rng, 8, shift=0.08))["ok"]
               for _ in range(trials))
    assert hits / trials > 0.9, hits


def test_node_rule_with_flat_columns():
    a = np.zeros((8, 3))
    b = np.zeros((8, 3))
    b[:, 2] = 1.0
    ok = run_stats.node_test(a, b)
    assert ok.tolist() == [True, True, False]


def test_hotelling_matches_univariate_t_squared():
    # with one band Hotelling's T^2 is the pooled two-sample t squared
    rng = np.random.default_rng(9)
    a, b = rng.normal(0, 1, (8, 1)), rng.normal(0.3, 1, (8, 1))
    f, df = run_stats.hotelling_f(a, b)
    from scipy import stats

    t = stats.ttest_ind(a[:, 0], b[:, 0], equal_var=True).statistic
    assert df == (1, 14)
    assert abs(f - t * t) < 1e-10 * max(1.0, t * t)


def _small_c1():
    w = workloads.scaled(workloads.get("c1_small"), 3000)
    return w


def test_oracle_against_itself_and_a_planted_mistake():
    w = _small_c1()
    warm, measured = 500, 1500
    a = run_stats.oracle_ensemble_async(w, range(1, 9), warm, measured).get()
    b = run_stats.oracle_ensemble_async(w, range(101, 109), warm, measured).get()
    c = run_stats.oracle_ensemble_async(w, range(201, 209), warm, measured, xs_scale=2.0).get()
    same = run_stats.compare(a, b)
    assert same["ok"], same
    planted = run_stats.compare(a, c)
    assert not planted["ok"], planted
