"""Seeded synthetic particle states (inputs only).

The paper (arXiv:2109.04469, Sec. 2) starts every run from some initial
plasma and iterates to convergence; it does not prescribe the initial load.
Here initial states are drawn with numpy's PCG64 from a seed: positions
uniform on (0, L), velocities from an isotropic Maxwellian at the given
temperature. The same arrays are handed to the library and to the oracle.
"""
from __future__ import annotations

import numpy as np

from .xsec import E_CHARGE, M_ARGON, M_ELECTRON

MASS = (M_ELECTRON, M_ARGON)


def maxwellian_uniform(n, gap_m, temp_ev, species, seed, ordered=False):
    """n particles uniform in (0, L) with Maxwellian velocities; returns
    float64 arrays (x, vx, vy, vz). ordered: the positions are listed in
    increasing order (the same draws, relabelled), the slot order a cell
    sort of the uniform load would give."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), int(species), 7])))
    x = rng.uniform(0.0, gap_m, size=n)
    if ordered:
        x = np.sort(x, kind="stable")
    sig = np.sqrt(temp_ev * E_CHARGE / MASS[species])
    v = rng.normal(0.0, sig, size=(3, n))
    return (np.ascontiguousarray(x), np.ascontiguousarray(v[0]),
            np.ascontiguousarray(v[1]), np.ascontiguousarray(v[2]))


def initial_state(workload, seed=None, ordered=None):
    """Both species of a named workload: {species: (x, vx, vy, vz)}.
    ordered (default: the workload's "ordered_load"): positions listed in
    increasing order."""
    p = workload["params"]
    s = p["seed"] if seed is None else seed
    o = workload.get("ordered_load", False) if ordered is None else ordered
    return {
        sp: maxwellian_uniform(workload["n_init"][sp], p["gap_m"], workload["t_init_ev"][sp], sp, s,
                               ordered=o)
        for sp in (0, 1)
    }


def random_state(n, gap_m, v_scale, species, seed, wall_fraction=0.0):
    """A state for single-step tests: uniform positions, Gaussian velocities
    of scale v_scale, and optionally a fraction of particles placed within one
    step's flight of either wall so the wall step is exercised."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), int(species), 11])))
    x = rng.uniform(0.0, gap_m, size=n)
    v = rng.normal(0.0, v_scale, size=(3, n))
    if wall_fraction > 0.0:
        k = int(wall_fraction * n)
        idx = rng.choice(n, size=k, replace=False)
        side = rng.integers(0, 2, size=k)
        d = rng.uniform(0.0, 1e-3 * gap_m, size=k)
        x[idx] = np.where(side == 0, d, gap_m - d)
        v[0, idx] = np.where(side == 0, -np.abs(v[0, idx]), np.abs(v[0, idx]))
    return (np.ascontiguousarray(x), np.ascontiguousarray(v[0]),
            np.ascontiguousarray(v[1]), np.ascontiguousarray(v[2]))
