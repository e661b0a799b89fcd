#!/usr/bin/env python3
"""Throughput of the explicit 1D3V PIC/MCC step (arXiv:2109.04469, Sec. 2) on
one MI355X.

A step is one pass of the whole hot path: field solve, electron particle
kernel, the sub-cycled ion kernel on its steps and the periodic cell sort.
The default workload is the large low-pressure discharge: 6.7 cm gap, 2048
cells, dt = T_RF/8000, 2 Pa, 500 V, gamma = 0.2, R = 0.5, 4M electrons + 4M
Ar+ in FP64, ions sub-cycled x10, synthetic argon-shaped cross sections,
starting from a uniform Maxwellian plasma listed in position order. After `--warmup` steps (default
two RF cycles) `--steps` steps (default one RF cycle) are timed with inputs
resident in HBM.

value = particle-steps per second over the timed region (electrons every
step, ions on their sub-cycled steps), from the library's own push counters.
roofline: the electron particle pass (its decide and emit kernels and the
kernel that takes its queued slots, launched back to back on the library's
stream; on most steps that last kernel also solves the next step's field
on one CU, which this figure charges to the pass), algorithmic traffic 64 B per
particle-step (x, vx, vy, vz read and written in FP64) divided by the pass's
mean duration from HIP events recorded on that stream, over a second window
of the same length right after the timed one (event records slow a step by a
few percent, so the timed window itself has none). copy_ref is the
library's plain streaming copy on 2 x 256 MiB, the achievable-bandwidth
reference on the same GPU.
sort: the periodic cell sort's cost per sort and amortised per step (the
timed window may hold no sort), and the throughput with it included.
cpu_baseline: the CPU oracle (single thread, and the OpenMP build of the same
source on all host cores) on a bounded sample of the same workload, with the
host's CPU model and core count.
c1_full: the small discharge for its full 10 RF cycles on the GPU and on the
oracle.
sweep: the batched-sweep workload (64 seeded independent discharges of
uneven size), advanced one discharge after the other, on one stream each,
and as one batch with one launch per pass for all; throughputs, speedups
over the one-after-the-other run, and whether all three agree bitwise.
warm_start (default: a reduced study, about 2 GPU-minutes; --warm-start full
for the 10-minute one): RF cycles to convergence of held-out discharges
started from the network's predicted profiles vs from a uniform plasma
(paper_2109_04469_amd.warmstart).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/s (push+MCC+CIC) vs HBM roofline; batched & warm-start speedup"
HBM_PEAK_GBS = 8000.0
BYTES_PER_PARTICLE_STEP = 64
# HBM bytes the electron pass moves per electron particle-step, read with
# rocprofv3 FETCH_SIZE (x2, the factor a plain copy of known size gives)
# and WRITE_SIZE (x1) at c3; a constant taken from the profile named below,
# to be re-measured whenever the pass's kernels change (None when not
# measured for the current kernels)
PASS_TRAFFIC_BYTES_PER_PARTICLE = 47.4
PASS_TRAFFIC_SOURCE = ("constant per electron particle-step of the pipelined pass from "
                       "profiles/particle_pass_c3_first_steps_hbm_traffic.md and "
                       "profiles/particle_pass_c3_large_lowp_hbm_traffic.md (rocprofv3 FETCH_SIZE x2 + "
                       "WRITE_SIZE over 20 steps, after 5 steps and after two RF cycles), "
                       "times this window's particles")
# the same for the unpipelined pass (--pipeline off)
PASS_TRAFFIC_BYTES_UNPIPELINED = 60.15
PASS_TRAFFIC_SOURCE_UNPIPELINED = ("constant per electron particle-step of the unpipelined pass "
                                   "(k_decide + k_emit + k_tail; rocprofv3 FETCH_SIZE x2 + WRITE_SIZE "
                                   "over 20 steps after two RF cycles), times this window's particles")

# the kernels the electron pass timer covers (per step, in launch order)
PASS_KERNELS = ("electron particle pass: k_decide<0> + k_emit<0> + k_tail<0> (its queued slots, "
                "overlapped with the next step's field); k_rare<0> instead of k_tail on ion steps")
PASS_KERNELS_PIPELINED = (
    "electron particle pass, pipelined: k_field_cand (next step's field and candidacy bits) + "
    "k_emit_decide<2> (this step's emit, the next step's decisions, this step's queued slots); "
    "on ion steps k_emit<0, 1> + k_rare<0>, on the step after one and the first of a call "
    "k_decide<0> + k_field_cand + k_emit_decide<3> (the emit pushes again)")

DESCRIPTIONS = {
    "c3_large_lowp": ("gap 6.7 cm, 2048 cells, dt=T_RF/8000, 13.56 MHz, 500 V, 2 Pa, gamma 0.2, R 0.5, "
                      "4M e + 4M Ar+ fp64, ions sub-cycled x10, synthetic argon cross sections"),
    "c2_production": ("gap 2.5 cm, 512 cells, dt=T_RF/4000, 13.56 MHz, 300 V, 50 Pa, gamma 0.1, R 0, "
                      "400k e + 400k Ar+ fp64, synthetic argon cross sections"),
    "c1_small": ("gap 2.5 cm, 128 cells, dt=T_RF/1000, 13.56 MHz, 100 V, 10 Pa, gamma 0, R 0.2, "
                 "10k e + 10k Ar+ fp64"),
}


def host_cpu():
    """Host CPU model and the cores this process may run on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "nproc": len(os.sched_getaffinity(0)), "os_cpu_count": os.cpu_count()}


def _oracle_run(workload, init, xs, nsteps, openmp):
    import oracle

    o = oracle.Oracle(dict(workload["params"]), xs, openmp=openmp)
    for sp in (0, 1):
        o.set_state(sp, *init[sp], step=0)
    c0 = o.counters()
    t0 = time.perf_counter()
    st = o.step(nsteps)
    t1 = time.perf_counter()
    c1 = o.counters()
    ps = int((c1[1] - c0[1]) + (c1[2] - c0[2]))
    return ps, t1 - t0, st


def cpu_baseline(workload, init, xs, nsteps):
    """The oracle on this host: the plain single-threaded build (the
    checker) and the OpenMP build of the same source on all the host's
    cores, both on the first nsteps steps of the workload."""
    import oracle

    ps, sec, st = _oracle_run(workload, init, xs, nsteps, False)
    ps_m, sec_m, st_m = _oracle_run(workload, init, xs, nsteps, True)
    cpu = host_cpu()
    return {
        "value": ps / sec,
        "unit": "particle-steps/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"first {nsteps} steps of {workload['name']} from its synthetic initial state "
                  f"({ps} particle-steps, {sec:.1f} s, status {st})",
        "openmp": {"value": ps_m / sec_m, "unit": "particle-steps/s",
                   "cores": oracle.threads(openmp=True), "seconds": sec_m, "status": st_m,
                   "note": "same oracle source built with -fopenmp: each pass split into one "
                           "slot-ordered run per thread (bit-identical results)"},
        "host": cpu,
    }


def c1_full(torch, log):
    """The small discharge in full (10 RF cycles, 10k + 10k particles) on the
    GPU and on the oracle (plain and OpenMP builds), from the same state."""
    from paper_2109_04469_amd import Discharge
    from pic_inputs import state, workloads, xsec

    w = workloads.get("c1_small")
    p = dict(w["params"])
    xs = xsec.argon_synthetic()
    init = state.initial_state(w)
    nsteps = w["cycles"] * p["steps_per_cycle"]
    d = Discharge(p, xs, "cuda:0")
    for sp in (0, 1):
        d.set_state(sp, *init[sp], step=0)
    torch.cuda.synchronize()
    c0 = d.counters()
    t0 = time.perf_counter()
    d.step(nsteps)
    st = d.sync()
    t1 = time.perf_counter()
    assert st == 0, f"c1 run failed: status {st}"
    c1 = d.counters()
    ps = int((c1[1] - c0[1]) + (c1[2] - c0[2]))
    log(f"[bench] c1 in full: GPU {t1 - t0:.2f} s; oracle (plain, then OpenMP)")
    ops, osec, ost = _oracle_run(w, init, xs, nsteps, False)
    mps, msec, mst = _oracle_run(w, init, xs, nsteps, True)
    import oracle

    return {
        "workload": f"c1_small in full: {DESCRIPTIONS['c1_small']}, {w['cycles']} RF cycles "
                    f"({nsteps} steps) from the synthetic initial state",
        "unit": "particle-steps/s",
        "gpu": {"value": ps / (t1 - t0), "seconds": t1 - t0, "particle_steps": ps},
        "oracle_1_core": {"value": ops / osec, "seconds": osec, "particle_steps": ops, "status": ost},
        "oracle_openmp": {"value": mps / msec, "seconds": msec, "particle_steps": mps, "status": mst,
                          "cores": oracle.threads(openmp=True)},
        "note": "c1 is launch- and latency-bound on the GPU (20k particles); it is the parity case",
    }


def copy_reference(torch, nbytes=1 << 28, reps=20):
    """Read+write bandwidth of the library's plain streaming copy."""
    from paper_2109_04469_amd import selftest_copy

    n = nbytes // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        selftest_copy(a, b)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        selftest_copy(a, b)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    assert torch.equal(a, b)
    return {"GBs": 2 * nbytes / (ms * 1e-3) / 1e9, "bytes_read": nbytes, "bytes_written": nbytes,
            "us_per_copy": ms * 1e3, "kernel": "k_selftest_copy"}


def sweep_measurement(torch, steps, n=64, log=print):
    """The batched-sweep workload: n seeded independent discharges (N_t in
    [500, 8000], 64-1024 cells, 20k-2M particles per species, R, gamma,
    pressure and voltage drawn), each advanced by `steps` steps from its
    initial state three ways on the same GPU: one after the other with
    pic_step (the plain single-run method), all at once on their own streams
    (pic_step_many), and as one batch with one launch per pass for all
    (pic_batch_step). The three compute the same particle-steps bitwise."""
    from paper_2109_04469_amd import Batch, Discharge, step_many
    from pic_inputs import sweep, xsec

    sw = sweep.draw(n, seed=0, capacity_factor=4)
    init = sweep.initial_states(sw, seed=0)
    xs = xsec.argon_synthetic()

    def reset(ds):
        for d, st in zip(ds, init):
            for sp in (0, 1):
                d.set_state(sp, *st[sp], step=0)
        torch.cuda.synchronize()

    def timed(ds, fn):
        reset(ds)
        c0 = [d.counters() for d in ds]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for d in ds:
            st = d.sync()
            assert st == 0, f"sweep discharge failed: status {st}"
        c1 = [d.counters() for d in ds]
        ps = sum(int((b[1] - a[1]) + (b[2] - a[2])) for a, b in zip(c0, c1))
        return {"value": ps / (t1 - t0), "seconds": t1 - t0}, ps, [b - a for a, b in zip(c0, c1)]

    def snapshot(ds):
        return [tuple(t.clone() for t in d.get_state(sp, to_numpy=False)) for d in ds for sp in (0, 1)]

    def same(a, b):
        return all(all(torch.equal(x, y) for x, y in zip(p, q)) for p, q in zip(a, b))

    one = torch.cuda.Stream()
    ds = [Discharge(w["params"], xs, stream=one) for w in sw]

    def sequential():
        for d in ds:
            d.step(steps)

    log(f"[bench] sweep: {n} discharges x {steps} steps, sequential")
    seq, ps, cnt_seq = timed(ds, sequential)
    ref = snapshot(ds)
    batch = Batch(ds)
    log("[bench] sweep: batched launches")
    bat, ps_b, cnt_b = timed(ds, lambda: batch.step(steps))
    equal = ps_b == ps and same(ref, snapshot(ds)) and all(
        (a == b).all() for a, b in zip(cnt_seq, cnt_b))
    batch.close()
    del batch, ds
    torch.cuda.empty_cache()

    log("[bench] sweep: one stream per discharge")
    streams = [torch.cuda.Stream() for _ in sw]
    ds = [Discharge(w["params"], xs, stream=s_) for w, s_ in zip(sw, streams)]
    mst, ps_m, cnt_m = timed(ds, lambda: step_many(ds, steps, chunk=50))
    equal = equal and ps_m == ps and same(ref, snapshot(ds))
    del ds
    torch.cuda.empty_cache()
    sizes = [w["n_init"][0] for w in sw]
    return {
        "workload": (f"{n} seeded discharges (sweep seed 0): N_t in [500, 8000], 64-1024 cells, "
                     f"{min(sizes)}-{max(sizes)} particles per species ({sum(sizes)} in all), "
                     "R in [0, 0.7], gamma in [0, 0.4], 2-100 Pa, 100-500 V, ion_subcycle 1, "
                     "sort every 50 steps; each advanced from its initial state"),
        "steps": steps,
        "particle_steps": ps,
        "unit": "particle-steps/s",
        "sequential": seq,
        "streams": mst,
        "batched": bat,
        "speedup_batched_vs_sequential": bat["value"] / seq["value"],
        "speedup_streams_vs_sequential": mst["value"] / seq["value"],
        "bitwise_equal": bool(equal),
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default: one RF cycle)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed steps (default: two RF cycles)")
    ap.add_argument("--workload", default="c3_large_lowp", choices=sorted(DESCRIPTIONS))
    ap.add_argument("--cpu-steps", type=int, default=50, help="oracle steps for cpu_baseline")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle timing")
    ap.add_argument("--no-timing", action="store_true", help="do not record per-kernel events")
    ap.add_argument("--sweep-steps", type=int, default=200, help="steps of the batched-sweep workload")
    ap.add_argument("--no-sweep", action="store_true", help="skip the batched-sweep workload")
    ap.add_argument("--sweep-only", action="store_true",
                    help="run only the batched-sweep workload and print its JSON object")
    ap.add_argument("--warm-start", choices=("reduced", "full", "none"), default="reduced",
                    help="warm-start study: reduced (default, about 2 GPU-minutes: 46 cold runs of "
                         "1000 RF cycles, training on 40, 6 warm runs of 1000 cycles), full (about 10 "
                         "GPU-minutes: 112 cold runs of 2000 cycles, 16 warm runs of 2000) or none")
    ap.add_argument("--no-c1", action="store_true", help="skip the small discharge in full")
    ap.add_argument("--tune-steps", type=int, default=40,
                    help="steps per candidate of the particle-pass tuner (with the sweep)")
    ap.add_argument("--pipeline", choices=("on", "off"), default="on",
                    help="pipelined electron steps (pic_set_pipeline) for the timed workload")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs one discharge on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU design is described, not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.sweep_only:
        assert torch.cuda.is_available(), "bench.py needs a GPU"
        print(json.dumps({"sweep": sweep_measurement(
            torch, args.sweep_steps, log=lambda *a: print(*a, file=sys.stderr, flush=True))}))
        return

    from paper_2109_04469_amd import Discharge
    from pic_inputs import state, workloads, xsec

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    w = workloads.get(args.workload)
    p = dict(w["params"])
    nt = p["steps_per_cycle"]
    steps = args.steps if args.steps is not None else nt
    warmup = args.warmup if args.warmup is not None else 2 * nt
    xs = xsec.argon_synthetic()
    init = state.initial_state(w)

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    log(f"[bench] {w['name']}: init {w['n_init']} particles")
    d = Discharge(p, xs, "cuda:0")
    for sp in (0, 1):
        d.set_state(sp, *init[sp], step=0)
    d.set_pipeline(args.pipeline == "on")
    chunk = max(1, nt // 4)
    done = 0
    while done < warmup:
        k = min(chunk, warmup - done)
        d.step(k)
        st = d.sync()
        assert st == 0, f"warm-up step failed: status {st}"
        done += k
        log(f"[bench] warm-up {done}/{warmup} steps, e={d.count(0)} i={d.count(1)}")

    # timed region: no event records inside it
    c0 = d.counters()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    d.step(steps)
    st = d.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    assert st == 0, f"timed steps failed: status {st}"
    c1 = d.counters()
    elapsed = t1 - t0
    pe = int(c1[1] - c0[1])
    pi = int(c1[2] - c0[2])
    value = (pe + pi) / elapsed
    log(f"[bench] timed {steps} steps in {elapsed:.3f} s")

    roof = None
    kernels = None
    sort_block = None
    if not args.no_timing:
        # the same number of steps again with HIP events around the field
        # kernel, each species' particle pass and each sort (event records
        # add a few microseconds per step, so they stay out of `value`)
        d.timing(1)
        d.get_timing(reset=True)
        e0 = d.counters()
        d.step(steps)
        assert d.sync() == 0
        e1 = d.counters()
        tm = d.get_timing(reset=True)
        pe_w = int(e1[1] - e0[1])
        # a shorter window with events around every particle kernel too
        d.timing(2)
        d.step(min(steps, 400))
        assert d.sync() == 0
        tk = d.get_timing(reset=True)
        d.timing(0)
        kernels = {k: {"launches": v[1], "us_per_launch": (1e3 * v[0] / v[1]) if v[1] else None}
                   for k, v in tm.items() if v[1] and k in ("field", "electron", "ion", "sort")}
        kernels.update({k: {"launches": v[1], "us_per_launch": 1e3 * v[0] / v[1],
                            "note": "events around each kernel"}
                        for k, v in tk.items() if v[1] and k.split("_")[0] in ("e", "i")})
        if tk.get("field", (0.0, 0))[1]:
            # the next step's field inside the pass (k_field_cand on
            # pipelined steps), events around each launch
            v = tk["field"]
            kernels["field_in_pass"] = {"launches": v[1], "us_per_launch": 1e3 * v[0] / v[1],
                                        "note": "events around each kernel"}
        # the periodic cell sort: when the windows above hold none, step on
        # to the next sort with events around it, so its cost per step can
        # be stated (it is part of every step in the mean over a sort
        # interval)
        si = p["sort_interval"]
        sort_ms = tm.get("sort", (0.0, 0))
        sort_ms = (sort_ms[0] + tk.get("sort", (0.0, 0))[0], sort_ms[1] + tk.get("sort", (0.0, 0))[1])
        if si > 0 and sort_ms[1] == 0:
            d.timing(1)
            d.get_timing(reset=True)
            d.step(si - d.step_index % si)
            assert d.sync() == 0
            ts = d.get_timing(reset=True)
            d.timing(0)
            sort_ms = ts.get("sort", (0.0, 0))
        if si > 0 and sort_ms[1]:
            us_sort = 1e3 * sort_ms[0] / sort_ms[1]
            sort_block = {"interval_steps": si, "us_per_sort": us_sort,
                          "sorts_timed": sort_ms[1], "us_per_step_amortised": us_sort / si,
                          "value_with_sort_amortised": (pe + pi) / (elapsed + steps * us_sort / si * 1e-6),
                          "note": "both species' stable cell sorts, HIP events around them"}
        ems, en = tm["electron"]
        if en:
            avg_s = ems / en * 1e-3
            bytes_per_launch = BYTES_PER_PARTICLE_STEP * pe_w / en
            achieved = bytes_per_launch / avg_s / 1e9
            piped = args.pipeline == "on"
            tb = PASS_TRAFFIC_BYTES_PER_PARTICLE if piped else PASS_TRAFFIC_BYTES_UNPIPELINED
            traffic = tb * pe_w / en if tb is not None else None
            roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                    "traffic_unit": "HBM bytes per launch", "traffic_source": (PASS_TRAFFIC_SOURCE if piped else PASS_TRAFFIC_SOURCE_UNPIPELINED),
                    "kernel": (PASS_KERNELS_PIPELINED if args.pipeline == "on" else PASS_KERNELS),
                    "bytes_per_launch": bytes_per_launch, "avg_launch_us": avg_s * 1e6,
                    "particles_per_launch": pe_w / en, "window_steps": steps}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": 1e3 * elapsed / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{w['name']}: {DESCRIPTIONS[w['name']]}",
            "particles_e": d.count(0), "particles_i": d.count(1),
            "particle_steps_e": pe, "particle_steps_i": pi,
            "n_cells": p["n_cells"], "steps_per_cycle": nt, "ion_subcycle": p["ion_subcycle"],
            "sort_interval": p["sort_interval"], "parallelism": "single GPU",
            "pipeline": args.pipeline,
            "collision_candidates": int((c1[7] - c0[7]) + (c1[11] - c0[11])),
            "beyond_table": int(c1[15] - c0[15]),
        },
        "roofline": roof,
        "kernels": kernels,
        "sort": sort_block,
        "cpu_baseline": None,
        "copy_ref": copy_reference(torch),
    }
    out["sweep"] = None
    if not args.no_sweep:
        # the per-discharge tuner on the timed workload (after the timed
        # windows): every candidate schedule and launch shape of the particle
        # passes, timed on the discharge itself, and the one it keeps
        log("[bench] tuner: particle-pass candidates on the timed workload")
        tuned = d.tune_pass(steps_per_trial=args.tune_steps)
        del d
        torch.cuda.empty_cache()
        out["sweep"] = sweep_measurement(torch, args.sweep_steps, log=log)
        out["sweep"]["tuner"] = {
            "workload": w["name"], "steps_per_trial": args.tune_steps,
            "unit": "us of particle passes (electron + ion) per step, events around the passes",
            "trials": tuned["trials"], "choice": tuned["trials"][tuned["best"]],
            "note": "pipelined: fused emit-and-decide kernel at 1..3 workgroups per CU; unpipelined: "
                    "separate decide and emit kernels, the decide compiled for 512 and for 256 "
                    "threads per workgroup at each of its shapes, then each emit shape",
        }
    out["warm_start"] = None
    if args.warm_start != "none":
        from paper_2109_04469_amd import warmstart

        size = warmstart.REDUCED_STUDY if args.warm_start == "reduced" else warmstart.FULL_STUDY
        log(f"[bench] warm-start study ({args.warm_start}): cold runs, training, warm runs")
        res = warmstart.study(**size)
        out["warm_start"] = {
            "workload": (f"warm-start family (seed {size['seed']}): {size['n_train']} training + "
                         f"{size['n_test']} held-out discharges, cold runs of {size['cycles']} RF "
                         f"cycles (reference: mean of the last {size['avg_windows'] * 10}), warm runs "
                         f"of {size['warm_cycles']}"),
            "metric": "RF cycles until the 10-cycle-averaged ion density stays within delta of the "
                      "cold-run reference (runs that never converge counted at the cycles they ran)",
            "delta_0.1": res["delta_0.1"], "delta_0.05": res["delta_0.05"],
            "prediction_rel_l2_n_i": res["prediction_rel_l2_n_i"],
            "initial_rel_l2_n_i": res["initial_rel_l2_n_i"],
            "cold_run_seconds": res["cold_run_seconds"],
            "train_seconds": res["train_seconds"], "warm_run_seconds": res["warm_run_seconds"],
        }
    if not args.no_c1:
        out["c1_full"] = c1_full(torch, log)
    if not args.no_cpu:
        log(f"[bench] cpu baseline: oracle, {args.cpu_steps} steps")
        out["cpu_baseline"] = cpu_baseline(w, init, xs, args.cpu_steps)
    _ = np
    print(json.dumps(out))


if __name__ == "__main__":
    main()
