"""Seeded parameter sweep of independent discharges (synthetic inputs only).

A sweep of the kind the paper runs in Sec. 3 (time step, grid, weight,
reflection and emission coefficients, pressure and voltage varied around
base cases), drawn at random: each discharge takes N_t in [500, 8000]
(dt = T_RF / N_t), 64 to 1024 cells, a superparticle weight that puts 20k to
2M particles per species in its initial uniform plasma, R in [0, 0.7],
gamma in [0, 0.4], 2 to 100 Pa and 100 to 500 V, on the 2.5 cm gap at
13.56 MHz. This module only produces parameter dictionaries and initial
states; it holds none of the simulation's arithmetic.
"""
from __future__ import annotations

import copy

import numpy as np

from . import state, workloads

N0 = 1e15  # initial plasma density, m^-3


def draw(n=64, seed=0, particles=(20_000, 2_000_000), capacity_factor=3):
    """n workload dictionaries (same layout as workloads.get) with seeded
    parameters; particle counts and pressures are log-uniform."""
    rng = np.random.default_rng([int(seed), 4])
    out = []
    base = workloads.get("c1_small")
    for k in range(n):
        w = copy.deepcopy(base)
        p = w["params"]
        L = p["gap_m"]
        npart = int(np.exp(rng.uniform(np.log(particles[0]), np.log(particles[1]))))
        p.update(
            steps_per_cycle=int(rng.integers(500, 8001)),
            n_cells=int(rng.integers(64, 1025)),
            reflection=float(rng.uniform(0.0, 0.7)),
            gamma_see=float(rng.uniform(0.0, 0.4)),
            pressure_pa=float(np.exp(rng.uniform(np.log(2.0), np.log(100.0)))),
            rf_voltage_v=float(rng.uniform(100.0, 500.0)),
            weight=N0 * p["area_m2"] * L / npart,
            capacity=(capacity_factor * npart, capacity_factor * npart),
            ion_subcycle=1,
            sort_interval=50,
            seed=1000 + k,
            run=4,
        )
        p["eepf_halfwidth_m"] = 0.05 * L
        w["name"] = f"sweep{k:02d}"
        w["n_init"] = (npart, npart)
        out.append(w)
    return out


def initial_states(sweep, seed=0):
    return [state.initial_state(w, seed=seed + k) for k, w in enumerate(sweep)]
