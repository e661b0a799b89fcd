"""Run-level statistical parity (the paper's Sec. 3.1 diagnostics of a run:
time-averaged density profiles, mean electron energy profile and the EEPF at
mid-gap) between two independent ensembles of runs of one discharge.

Each run gives one time average per node or bin. Two ensembles of n1 and n2
seeds (different seeds on the two sides, so the samples are independent)
agree when

* per node or bin, |mean_1 - mean_2| <= c * se with se the standard error
  of the difference (Welch); "3 sigma" is read as the two-sided 0.27 % tail,
  so c is the Student-t quantile of that tail at the Welch degrees of
  freedom (the standard deviations are estimated from a few seeds); at least
  99 % of the nodes and bins must pass, and
* per quantity, Hotelling's two-sample T^2 over a few coarse bands (the
  multivariate form of the chi-squared of the mean differences, with the
  band covariance estimated from the pooled samples), converted to its
  F(k, n1 + n2 - k - 1) statistic, is below the F distribution's 99.9th
  percentile.

The oracle side runs in worker processes (one per seed); nothing here uses
the GPU. Only tests import this module.
"""
from __future__ import annotations

import multiprocessing as mp
import os

import numpy as np
from scipy import stats

TAIL_3SIGMA = 2.0 * stats.norm.sf(3.0)  # 0.0027, two-sided


def node_test(a, b, tail=TAIL_3SIGMA):
    """a [n1, m], b [n2, m]: per-column pass flags of the Welch comparison;
    columns with no spread on either side pass iff their means are equal."""
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    n1, n2 = a.shape[0], b.shape[0]
    va = a.var(axis=0, ddof=1) / n1
    vb = b.var(axis=0, ddof=1) / n2
    se2 = va + vb
    d = np.abs(a.mean(axis=0) - b.mean(axis=0))
    ok = np.ones(a.shape[1], bool)
    flat = se2 <= 0.0
    ok[flat] = d[flat] <= 1e-12 * np.maximum(np.abs(a.mean(axis=0)[flat]), 1e-300)
    live = ~flat
    if live.any():
        nu = se2[live] ** 2 / (va[live] ** 2 / (n1 - 1) + vb[live] ** 2 / (n2 - 1))
        c = stats.t.isf(0.5 * tail, nu)
        ok[live] = d[live] <= c * np.sqrt(se2[live])
    return ok


def bands(x, k, lo=0, hi=None):
    """Sums of k equal bands of the columns [lo, hi)."""
    x = np.asarray(x, float)[..., lo:hi]
    n = x.shape[-1] // k * k
    return x[..., :n].reshape(x.shape[:-1] + (k, n // k)).sum(-1)


def hotelling_f(a, b):
    """Two-sample Hotelling T^2 of a [n1, k] and b [n2, k] as its F
    statistic and degrees of freedom (pooled covariance)."""
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    n1, n2, k = a.shape[0], b.shape[0], a.shape[1]
    assert n1 + n2 - k - 1 >= 1
    d = a.mean(0) - b.mean(0)
    S = ((n1 - 1) * np.cov(a, rowvar=False) + (n2 - 1) * np.cov(b, rowvar=False)) / (n1 + n2 - 2)
    S = np.atleast_2d(S)
    t2 = n1 * n2 / (n1 + n2) * float(d @ np.linalg.solve(S, d))
    f = t2 * (n1 + n2 - k - 1) / (k * (n1 + n2 - 2))
    return f, (k, n1 + n2 - k - 1)


def quantities(runs, eepf_hi):
    """Per-run vectors compared node by node, and the band vectors of the
    Hotelling test, from a list of moment dictionaries."""
    ne = np.array([r["n_e"] for r in runs])
    ni = np.array([r["n_i"] for r in runs])
    em = np.array([r["mean_energy_e"] for r in runs])
    ep = np.array([r["eepf"] for r in runs])
    cnt = np.array([[r["ne"], r["ni"]] for r in runs], float)
    nodes = {"n_e": ne, "n_i": ni, "mean_energy_e": em, "eepf": ep, "counts": cnt}
    nb = {"n_e": bands(ne, 6), "n_i": bands(ni, 6), "mean_energy_e": bands(em, 4),
          "eepf": bands(ep, 6, 0, eepf_hi), "counts": cnt}
    return nodes, nb


def compare(runs_a, runs_b, eepf_hi=64, min_frac=0.99, f_quantile=0.999):
    """The outcome of comparing two ensembles: a report dictionary with
    'ok' and, per quantity, the failing nodes and the Hotelling F against
    its percentile. eepf_hi: EEPF bins [0, eepf_hi) enter the bands (the
    populated part of the distribution)."""
    na, ba = quantities(runs_a, eepf_hi)
    nb_, bb = quantities(runs_b, eepf_hi)
    rep = {"ok": True}
    total = passed = 0
    for key in na:
        okn = node_test(na[key], nb_[key])
        total += okn.size
        passed += int(okn.sum())
        f, df = hotelling_f(ba[key], bb[key])
        lim = float(stats.f.ppf(f_quantile, *df))
        rep[key] = {"nodes": int(okn.size), "failed_nodes": np.flatnonzero(~okn).tolist(),
                    "hotelling_f": f, "f_limit": lim, "df": df}
        if f > lim:
            rep["ok"] = False
    rep["node_fraction"] = passed / total
    if passed < min_frac * total:
        rep["ok"] = False
    return rep


def run_oracle(job):
    """One oracle run: job = (params, n_init, t_init, seed, warm, measured).
    Returns its moments and final counts."""
    import oracle
    from pic_inputs import state, xsec

    p, n_init, t_init, seed, warm, measured, xs_scale = job
    w = {"params": dict(p, seed=seed), "n_init": n_init, "t_init_ev": t_init}
    xs = xsec.argon_synthetic()
    if xs_scale != 1.0:
        xs = xsec.XsecTables(xs.n, xs.dv_e, xs.dv_i, [s * xs_scale for s in xs.sigma_e],
                             list(xs.sigma_i), xs.exc_threshold_ev, xs.ion_threshold_ev)
    o = oracle.Oracle(w["params"], xs)
    init = state.initial_state(w, seed=seed)
    for sp in (0, 1):
        o.set_state(sp, *init[sp], step=0)
    assert o.step(warm) == 0
    o.measure(True)
    assert o.step(measured) == 0
    m = o.moments()
    return dict(m, ne=o.count(0), ni=o.count(1))


def oracle_ensemble_async(workload, seeds, warm, measured, processes=None, xs_scale=1.0):
    """Starts the oracle runs of `seeds` in worker processes; returns an
    object whose .get() gives the list of results in seed order. xs_scale
    multiplies the electron cross sections (tests that plant a mistake in
    the oracle's inputs)."""
    jobs = [(dict(workload["params"]), tuple(workload["n_init"]), tuple(workload["t_init_ev"]), s,
             warm, measured, float(xs_scale)) for s in seeds]
    n = processes or min(len(jobs), 8, os.cpu_count() or 1)
    ctx = mp.get_context("spawn")
    pool = ctx.Pool(n)

    class _Pending:
        def __init__(self):
            self.r = pool.map_async(run_oracle, jobs)

        def get(self, timeout=None):
            try:
                return self.r.get(timeout)
            finally:
                pool.close()
                pool.join()

    return _Pending()
