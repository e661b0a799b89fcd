"""Seeded discharge family of the warm-start study (synthetic inputs only).

Six varied parameters, the network's inputs: pressure 10-50 Pa
(log-uniform), RF voltage 100-250 V, gap 2.0-3.0 cm, RF frequency 10-20 MHz,
secondary emission coefficient gamma 0-0.3 and electron reflection
coefficient R 0-0.5, around the kind of base case Sec. 3 of the paper varies
(argon, 300 K gas, one RF electrode, the other grounded). Fixed: 127 cells
(128 grid points, one per network output point), 1000 steps per RF cycle,
ions sub-cycled x5, a cell sort every 100 steps, and a cold start of
10,000 particles per species (uniform plasma of 1e15 m^-3, Maxwellian
electrons at 2 eV and ions at 0.03 eV). This module only produces parameter
dictionaries; it holds none of the simulation's arithmetic.
"""
from __future__ import annotations

import copy

import numpy as np

from . import workloads

N0 = 1e15          # cold-start plasma density, m^-3
N_PER_SPECIES = 10_000
N_CELLS = 127
STEPS_PER_CYCLE = 1000

# (name, low, high, log-uniform)
RANGES = (
    ("pressure_pa", 10.0, 50.0, True),
    ("rf_voltage_v", 100.0, 250.0, False),
    ("gap_m", 0.020, 0.030, False),
    ("rf_freq_hz", 10e6, 20e6, False),
    ("gamma_see", 0.0, 0.3, False),
    ("reflection", 0.0, 0.5, False),
)


def draw(n, seed=0, capacity_factor=12):
    """n workload dictionaries (layout of workloads.get) of the family."""
    rng = np.random.default_rng([int(seed), 5])
    base = workloads.get("c1_small")
    out = []
    for k in range(n):
        w = copy.deepcopy(base)
        p = w["params"]
        for name, lo, hi, log in RANGES:
            p[name] = float(np.exp(rng.uniform(np.log(lo), np.log(hi))) if log else rng.uniform(lo, hi))
        L = p["gap_m"]
        p.update(
            steps_per_cycle=STEPS_PER_CYCLE,
            n_cells=N_CELLS,
            weight=N0 * p["area_m2"] * L / N_PER_SPECIES,
            capacity=(capacity_factor * N_PER_SPECIES, capacity_factor * N_PER_SPECIES),
            ion_subcycle=5,
            sort_interval=100,
            eepf_bins=128,
            eepf_emax_ev=40.0,
            eepf_halfwidth_m=0.1 * L,
            seed=2000 + k,
            run=7,
        )
        w["name"] = f"warm{k:03d}"
        w["n_init"] = (N_PER_SPECIES, N_PER_SPECIES)
        out.append(w)
    return out
