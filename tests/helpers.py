"""Shared test helpers: parameter dictionaries and physical constants."""
import copy

import numpy as np

from pic_inputs import workloads, xsec

QE = 1.602176634e-19
ME = 9.1093837015e-31
MAR = 39.948 * 1.66053906660e-27
EPS0 = 8.8541878128e-12
KB = 1.380649e-23

NO_FIELD, FIXED_E, NO_COLL, IMMOBILE_IONS, RECORD, THOMAS = 1, 2, 4, 8, 16, 32
ANISO, OPAL = 64, 128


def params(base="c1_small", **over):
    p = copy.deepcopy(workloads.get(base)["params"])
    p.update(over)
    if "capacity" in over:
        p["capacity"] = tuple(int(c) for c in over["capacity"])
    return p


def dt_of(p):
    return 1.0 / (p["rf_freq_hz"] * p["steps_per_cycle"])


def table_for(vmax_e, vmax_i, n=2048, sig_e=(1e-19, 0.0, 0.0), sig_i=(1e-18, 0.0), **kw):
    """Constant cross sections on tables reaching vmax."""
    return xsec.constant(n, vmax_e / (n - 1), vmax_i / (n - 1), sig_e, sig_i, **kw)


def energy_ev(m, vx, vy, vz):
    return 0.5 * m * (vx * vx + vy * vy + vz * vz) / QE


def iso_velocities(n, speed, rng):
    u = rng.uniform(-1, 1, n)
    ph = rng.uniform(0, 2 * np.pi, n)
    s = np.sqrt(1 - u * u)
    return speed * u, speed * s * np.cos(ph), speed * s * np.sin(ph)
