"""Learned warm start of RF discharge runs.

A run of the explicit PIC/MCC method (arXiv:2109.04469, Sec. 2) started from
a uniform plasma needs many RF cycles before its time-averaged profiles
settle. Here a network trained on the converged averages of a batched sweep
of discharges (their density profiles of both species, mean electron energy
profile and EEPF, the diagnostics of Sec. 3) predicts those averages from the
six discharge parameters, and a new discharge is loaded from the prediction
(pic_load_profile) instead of from a uniform plasma. The plain cold start
remains both the fallback (when a prediction is unusable) and the yardstick: the
converged averages of a long cold run are the reference the warm run is
measured against.

Everything here is orchestration: the particle steps, the sweep, the
network's training and inference and the particle loading run in libpic.

    python -m paper_2109_04469_amd.warmstart generate OUT.npz   # cold runs
    python -m paper_2109_04469_amd.warmstart evaluate IN.npz OUT.json
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from .discharge import Batch, Discharge, Mlp

NPTS = 128          # profile points (grid points of the family's 127 cells)
NBINS = 128         # EEPF bins
N_OUT = 3 * NPTS + NBINS
DENS_FLOOR = 1e12   # m^-3, floor of the log-density targets
EEPF_FLOOR = 1e-6   # eV^-3/2
WINDOW_CYCLES = 10  # cycles per time-averaging window
KB_EV = 8.617333262e-5  # Boltzmann constant in eV/K


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ---- features and targets ------------------------------------------------------

def features(params_list):
    """Network inputs in [-1, 1]: log pressure, voltage, gap, frequency,
    gamma and R scaled over the family's ranges."""
    from pic_inputs.warm import RANGES

    x = np.zeros((len(params_list), len(RANGES)), np.float32)
    for i, p in enumerate(params_list):
        for j, (name, lo, hi, is_log) in enumerate(RANGES):
            v, a, b = (np.log(p[name]), np.log(lo), np.log(hi)) if is_log else (p[name], lo, hi)
            x[i, j] = 2.0 * (v - a) / (b - a) - 1.0
    return x


def to_targets(prof):
    """Raw averages {n_e, n_i, mean_energy_e, eepf} [N, 128] -> [N, 512]."""
    return np.concatenate([
        np.log10(np.maximum(prof["n_e"], DENS_FLOOR)),
        np.log10(np.maximum(prof["n_i"], DENS_FLOOR)),
        np.maximum(prof["mean_energy_e"], 0.0),
        np.log10(np.maximum(prof["eepf"], EEPF_FLOOR)),
    ], axis=1).astype(np.float32)


def from_targets(t):
    t = np.asarray(t, dtype=np.float64)
    return {
        "n_e": 10.0 ** t[:, :NPTS],
        "n_i": 10.0 ** t[:, NPTS:2 * NPTS],
        "mean_energy_e": np.maximum(t[:, 2 * NPTS:3 * NPTS], 0.0),
        "eepf": 10.0 ** t[:, 3 * NPTS:],
    }


# ---- cold runs -----------------------------------------------------------------

def start_cold(d, w, seed):
    from pic_inputs import state

    init = state.initial_state(w, seed=seed)
    for sp in (0, 1):
        d.set_state(sp, *init[sp], step=0)


def run_windows(ds, cycles, steps_per_cycle, on_window=None):
    """Advances the discharges (one batch) by `cycles` RF cycles in windows of
    WINDOW_CYCLES, measuring through each window; returns per-window
    averages {n_e, n_i, mean_energy_e, eepf: [W, N, 128]} and counts [W, N, 2]."""
    b = Batch(ds)
    for d in ds:
        d.measure(True)
        d.moments(reset=True)
    nwin = cycles // WINDOW_CYCLES
    out = {k: np.zeros((nwin, len(ds), NPTS)) for k in ("n_e", "n_i", "mean_energy_e")}
    out["eepf"] = np.zeros((nwin, len(ds), NBINS))
    counts = np.zeros((nwin, len(ds), 2), np.int64)
    failed = np.zeros(len(ds), bool)
    t0 = time.time()
    for wi in range(nwin):
        b.step(WINDOW_CYCLES * steps_per_cycle)
        for i, d in enumerate(ds):
            if not failed[i] and d.sync() != 0:
                # a latched error (a species outgrew its capacity, or a
                # non-finite state): the discharge keeps stepping harmlessly
                # in the batch but is left out of every result
                failed[i] = True
                log(f"[warmstart] discharge {i} failed in window {wi}")
            if failed[i]:
                for k in out:
                    out[k][wi, i] = np.nan
                continue
            m = d.moments(reset=True)
            for k in ("n_e", "n_i", "mean_energy_e", "eepf"):
                out[k][wi, i] = m[k]
            counts[wi, i] = (d.count(0), d.count(1))
        if on_window:
            on_window(wi, nwin, time.time() - t0, counts[wi])
    b.close()
    return out, counts, failed


def final_average(win, last):
    return {k: v[-last:].mean(axis=0) for k, v in win.items()}


def generate(n_train=96, n_test=16, cycles=2000, avg_windows=20, seed=0):
    """Cold runs of the family's discharges in one batch; returns arrays for
    training (converged averages) and for judging (per-window trajectories)."""
    from pic_inputs import warm, xsec

    ws = warm.draw(n_train + n_test, seed=seed, capacity_factor=40)
    xs = xsec.argon_synthetic()
    stream = torch.cuda.Stream()
    ds = [Discharge(w["params"], xs, stream=stream) for w in ws]
    for k, (d, w) in enumerate(zip(ds, ws)):
        start_cold(d, w, seed=k)

    def progress(wi, nwin, el, counts):
        if wi % 10 == 0 or wi == nwin - 1:
            log(f"[warmstart] cold window {wi + 1}/{nwin} ({el:.0f} s), "
                f"particles e {int(counts[:, 0].sum())} i {int(counts[:, 1].sum())}")

    win, counts, failed = run_windows(ds, cycles, warm.STEPS_PER_CYCLE, progress)
    ref = final_average(win, avg_windows)
    params = [w["params"] for w in ws]
    return {
        "x": features(params),
        "y": to_targets(ref),
        "n_train": n_train,
        "cycles": cycles,
        "avg_windows": avg_windows,
        "seed": seed,
        "params": np.array([[p[name] for name, *_ in warm.RANGES] for p in params]),
        "ref_n_e": ref["n_e"], "ref_n_i": ref["n_i"],
        "ref_mean_energy_e": ref["mean_energy_e"], "ref_eepf": ref["eepf"],
        "win_n_i": win["n_i"].astype(np.float32), "win_n_e": win["n_e"].astype(np.float32),
        "counts": counts,
        "failed": failed,
    }


def run_to_convergence(ds, steps_per_cycle, delta=0.01, block_windows=10, max_cycles=5000,
                       on_block=None):
    """Advances discharges (one batch) until each is steady: its ion density
    profile averaged over the last block of `block_windows` windows of
    WINDOW_CYCLES cycles differs from the previous block's by at most delta
    (relative L2). A discharge that is steady leaves the batch; returns the
    RF cycles each needed (None if max_cycles passed first) and the last
    block averages {n_e, n_i, mean_energy_e, eepf} of each."""
    n = len(ds)
    done = [None] * n
    last = [None] * n
    prev = [None] * n
    active = list(range(n))
    cycles = 0
    block = block_windows * WINDOW_CYCLES
    while active and cycles < max_cycles:
        win, _, failed = run_windows([ds[i] for i in active], block, steps_per_cycle)
        cycles += block
        avg = final_average(win, block_windows)
        still = []
        for k, i in enumerate(active):
            if failed[k]:
                continue  # dropped: never steady
            cur = {key: v[k] for key, v in avg.items()}
            if prev[i] is not None and rel_l2(cur["n_i"], prev[i]["n_i"]) <= delta:
                done[i] = cycles
            else:
                still.append(i)
            prev[i] = cur
            last[i] = cur
        active = still
        if on_block:
            on_block(cycles, len(active))
    return done, last


# ---- the network -----------------------------------------------------------------

class Surrogate:
    """The network with its target standardisation."""

    def __init__(self, width=256, depth=4, seed=0, max_batch=1024):
        self.net = Mlp(6, width, depth, N_OUT, max_batch)
        rng = np.random.default_rng([seed, 13])
        # He initialisation of the weights, zero biases
        p = np.zeros(self.net.num_params, np.float32)
        o = 0
        dims = [6] + [width] * depth + [N_OUT]
        for i in range(len(dims) - 1):
            n = dims[i] * dims[i + 1]
            p[o:o + n] = rng.normal(scale=np.sqrt(2.0 / dims[i]), size=n)
            o += n + dims[i + 1]
        self.net.set_params(p)
        self.mu = np.zeros(N_OUT, np.float32)
        self.sd = np.ones(N_OUT, np.float32)

    def fit(self, x, y, steps=3000, lr=1e-3, weight_decay=1e-4):
        self.mu = y.mean(axis=0)
        self.sd = np.maximum(y.std(axis=0), 1e-3).astype(np.float32)
        xd = torch.as_tensor(x, dtype=torch.float32).cuda().contiguous()
        yd = torch.as_tensor((y - self.mu) / self.sd, dtype=torch.float32).cuda().contiguous()
        torch.cuda.synchronize()
        losses = []
        t0 = time.time()
        for s in range(steps):
            cur_lr = lr * 0.5 * (1.0 + np.cos(np.pi * s / steps))  # cosine decay
            self.net.train_step(xd, yd, float(cur_lr), weight_decay=weight_decay)
            if s % 500 == 0 or s == steps - 1:
                self.net.grad(xd, yd)
                losses.append((s, self.net.loss()))
        torch.cuda.synchronize()
        return losses, time.time() - t0

    def predict(self, x):
        y = self.net.forward(np.asarray(x, dtype=np.float32)).cpu().numpy()
        return y * self.sd + self.mu


# ---- warm start ------------------------------------------------------------------

def start_warm(d, w, prof, i):
    """Loads discharge d from predicted profiles (row i); False when the
    prediction is unusable (then the caller starts cold)."""
    p = w["params"]
    L = p["gap_m"]
    x = np.linspace(0.0, L, NPTS)
    ne, ni = prof["n_e"][i], prof["n_i"][i]
    te = (2.0 / 3.0) * prof["mean_energy_e"][i]
    counts = []
    for dens in (ne, ni):
        if not np.all(np.isfinite(dens)):
            return False
        counts.append(int(round(np.trapezoid(dens, x) * p["area_m2"] / p["weight"])))
    if min(counts) < 100 or max(counts) > p["capacity"][0] or not np.all(np.isfinite(te)):
        return False
    ti = np.full(NPTS, KB_EV * p["gas_temp_k"])
    d.load_profile(0, counts[0], ne, te, step=0)
    d.load_profile(1, counts[1], ni, ti, step=0)
    return True


def rel_l2(a, b):
    return np.linalg.norm(a - b, axis=-1) / np.linalg.norm(b, axis=-1)


def cycles_to(dist, delta):
    """RF cycles until the window-averaged profile first comes within delta
    (relative L2) of the reference and every later window stays within
    2 delta; None if it never does."""
    n = len(dist)
    for k in range(n):
        if dist[k] <= delta and np.all(dist[k:] <= 2 * delta):
            return (k + 1) * WINDOW_CYCLES
    return None


def evaluate(data, warm_cycles=600, deltas=(0.05, 0.10), train_steps=3000, seed=0):
    """Trains the network on the training discharges, warm-starts the held-out
    ones from its predictions and compares RF cycles to convergence with the
    cold runs of the same discharges."""
    from pic_inputs import warm, xsec

    ntr = int(data["n_train"])
    x, y = data["x"], data["y"]
    failed = data["failed"].astype(bool)
    train = [i for i in range(ntr) if not failed[i]]
    sur = Surrogate(seed=seed)
    losses, t_train = sur.fit(x[train], y[train], steps=train_steps)
    log(f"[warmstart] trained {train_steps} steps in {t_train:.1f} s, loss {losses[-1][1]:.4g}")
    ws = warm.draw(len(x), seed=int(data["seed"]), capacity_factor=40)
    test = [i for i in range(ntr, len(x)) if not failed[i]]
    pred = from_targets(sur.predict(x[test]))
    ref_ni = data["ref_n_i"][test]
    err_pred = rel_l2(pred["n_i"], ref_ni)
    xs = xsec.argon_synthetic()
    stream = torch.cuda.Stream()
    ds = [Discharge(ws[i]["params"], xs, stream=stream) for i in test]
    warm_ok = []
    for k, (d, i) in enumerate(zip(ds, test)):
        ok = start_warm(d, ws[i], pred, k)
        if not ok:
            start_cold(d, ws[i], seed=i)  # fallback: the plain cold start
        warm_ok.append(bool(ok))

    def progress(wi, nwin, el, counts):
        if wi % 10 == 0 or wi == nwin - 1:
            log(f"[warmstart] warm window {wi + 1}/{nwin} ({el:.0f} s)")

    t0 = time.time()
    win, _, wfailed = run_windows(ds, warm_cycles, warm.STEPS_PER_CYCLE, progress)
    t_warm = time.time() - t0
    dist_warm = rel_l2(win["n_i"], ref_ni[None, :, :])          # [W, T]
    dist_cold = rel_l2(data["win_n_i"][:, test], ref_ni[None])  # [W, T]
    res = {"n_train": len(train), "n_test": len(test), "cold_cycles": int(data["cycles"]),
           "failed_cold": np.flatnonzero(failed).tolist(),
           "failed_warm": [test[k] for k in np.flatnonzero(wfailed)],
           "reference": (f"mean of the last {int(data['avg_windows'])} windows of "
                         f"{WINDOW_CYCLES} cycles of the {int(data['cycles'])}-cycle cold run"),
           "train_loss": losses, "train_seconds": t_train, "warm_run_seconds": t_warm,
           "warm_loaded": warm_ok,
           "prediction_rel_l2_n_i": err_pred.tolist(),
           "initial_rel_l2_n_i": {"cold": dist_cold[0].tolist(), "warm": dist_warm[0].tolist()}}
    for delta in deltas:
        cold = [cycles_to(dist_cold[:, k], delta) for k in range(len(test))]
        wrm = [cycles_to(dist_warm[:, k], delta) for k in range(len(test))]
        res[f"delta_{delta:g}"] = compare_cycles(cold, wrm, int(data["cycles"]), warm_cycles)
    return res


def compare_cycles(cold, warm, cold_cap, warm_cap):
    """Cycles to convergence of the same discharges started cold and warm. A
    run that never converged counts at the cycles it ran (cold_cap,
    warm_cap: a lower bound on what it needs, so runs should be equally
    long for a fair mean), and no run drops out of the means and medians.
    A warm run is faster than its cold twin only if it converged first; one
    that did not converge is never counted as faster."""
    c = np.array([x if x is not None else cold_cap for x in cold], dtype=float)
    w = np.array([x if x is not None else warm_cap for x in warm], dtype=float)
    faster = sum(1 for a, b in zip(cold, warm) if b is not None and (a is None or b < a))
    slower = sum(1 for a, b in zip(cold, warm) if a is not None and (b is None or b > a))
    out = {"cold_cycles": cold, "warm_cycles": warm,
           "converged_cold": sum(x is not None for x in cold),
           "converged_warm": sum(x is not None for x in warm),
           "unconverged_counted_at": {"cold": cold_cap, "warm": warm_cap},
           "warm_faster": faster, "warm_slower": slower}
    if len(c):
        out.update({"mean_cold": float(c.mean()), "mean_warm": float(w.mean()),
                    "median_cold": float(np.median(c)), "median_warm": float(np.median(w)),
                    "speedup_mean": float(c.mean() / w.mean()),
                    "speedup_median": float(np.median(c) / np.median(w))})
    return out


# The study at the size a test or a benchmark line can afford (about two
# GPU-minutes) and at the size of the full study.
REDUCED_STUDY = dict(n_train=40, n_test=6, cycles=1000, avg_windows=20, warm_cycles=1000,
                     train_steps=2000, seed=3)
FULL_STUDY = dict(n_train=96, n_test=16, cycles=2000, avg_windows=20, warm_cycles=2000,
                  train_steps=3000, seed=0)


def study(n_train, n_test, cycles, avg_windows, warm_cycles, deltas=(0.05, 0.10),
          train_steps=3000, seed=0):
    """The whole study at a chosen size: cold runs of n_train + n_test
    discharges (their converged averages train the network and judge the
    held-out runs), then the held-out discharges started from the network's
    predictions. Returns evaluate()'s result with the cold-run time."""
    t0 = time.time()
    data = generate(n_train, n_test, cycles, avg_windows, seed)
    t_cold = time.time() - t0
    res = evaluate(data, warm_cycles=warm_cycles, deltas=deltas, train_steps=train_steps,
                   seed=seed)
    res["cold_run_seconds"] = t_cold
    return res

    return res


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    g = sub.add_parser("generate")
    g.add_argument("out")
    g.add_argument("--train", type=int, default=96)
    g.add_argument("--test", type=int, default=16)
    g.add_argument("--cycles", type=int, default=2000)
    g.add_argument("--avg-windows", type=int, default=20)
    g.add_argument("--seed", type=int, default=0)
    e = sub.add_parser("evaluate")
    e.add_argument("data")
    e.add_argument("out")
    e.add_argument("--warm-cycles", type=int, default=600)
    e.add_argument("--train-steps", type=int, default=3000)
    a = ap.parse_args(argv)
    assert torch.cuda.is_available(), "the warm-start study needs a GPU"
    if a.cmd == "generate":
        data = generate(a.train, a.test, a.cycles, a.avg_windows, a.seed)
        np.savez_compressed(a.out, **data)
        log(f"[warmstart] wrote {a.out}")
    else:
        data = dict(np.load(a.data))
        res = evaluate(data, warm_cycles=a.warm_cycles, train_steps=a.train_steps)
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)
        log(f"[warmstart] wrote {a.out}")


if __name__ == "__main__":
    main()
