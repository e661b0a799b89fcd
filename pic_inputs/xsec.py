"""Synthetic argon-shaped collision cross sections, tabulated on speed grids.

The discharge model of arXiv:2109.04469 (Sec. 2, step 6) uses Phelps'
e-Ar (elastic, excitation, ionization) and Ar+-Ar (isotropic elastic,
symmetric charge transfer) data, which are not available here. These
analytic forms stand in for them: they have the Ramsauer-like elastic
minimum, an 11.5 eV excitation and a 15.8 eV ionization threshold, and an
electron max(sigma_T v) of 3.3-3.4e-13 m^3/s, close to the value implied by
the collision probabilities quoted in Sec. 3.5 (P_coll = 0.2 at N_t = 300
and 0.1 at N_t = 600, 10 Pa).

This module only produces input data (sigma in m^2 at table speeds); it
holds none of the simulation's arithmetic. Both the simulation library and
the test oracle receive the same arrays.
"""
from __future__ import annotations

import numpy as np

# Physical constants (CODATA 2018) used to map table speeds to energies.
E_CHARGE = 1.602176634e-19
M_ELECTRON = 9.1093837015e-31
M_ARGON = 39.948 * 1.66053906660e-27

EXC_THRESHOLD_EV = 11.5
ION_THRESHOLD_EV = 15.8
A2 = 1e-20  # the forms below are in units of 1e-20 m^2


def _g(u):
    """Inelastic shape: 0 below threshold (u <= 1), peak 1 at u = 3."""
    u = np.asarray(u, dtype=np.float64)
    out = np.zeros_like(u)
    m = u > 1.0
    out[m] = 2.598 * (u[m] - 1.0) / u[m] ** 1.5
    return out


def sigma_e_elastic(eps_ev):
    eps = np.asarray(eps_ev, dtype=np.float64)
    x = eps / 12.0
    return A2 * (6.0 * np.exp(-eps / 0.06) + 0.3 + 12.0 * x ** 1.5 / (1.0 + x ** 2.5))


def sigma_e_excitation(eps_ev):
    return A2 * 1.5 * _g(np.asarray(eps_ev, dtype=np.float64) / EXC_THRESHOLD_EV)


def sigma_e_ionization(eps_ev):
    return A2 * 3.0 * _g(np.asarray(eps_ev, dtype=np.float64) / ION_THRESHOLD_EV)


def sigma_i_isotropic(eps_ev):
    eps = np.asarray(eps_ev, dtype=np.float64)
    return A2 * (30.0 / np.sqrt(eps + 0.1) + 10.0 / (1.0 + eps / 10.0))


def sigma_i_backward(eps_ev):
    eps = np.asarray(eps_ev, dtype=np.float64)
    return A2 * (7.5 - 0.35 * np.log(np.maximum(eps, 1e-3))) ** 2


class XsecTables:
    """Cross sections at speeds k*dv (k = 0..n-1), the layout the library
    and the oracle both take: electron tables by electron speed, ion tables
    by ion-atom relative speed with lab energy 1/2 M g^2."""

    def __init__(self, n, dv_e, dv_i, sigma_e, sigma_i,
                 exc_threshold_ev=EXC_THRESHOLD_EV, ion_threshold_ev=ION_THRESHOLD_EV):
        self.n = int(n)
        self.dv_e = float(dv_e)
        self.dv_i = float(dv_i)
        self.sigma_e = [np.ascontiguousarray(s, dtype=np.float64) for s in sigma_e]
        self.sigma_i = [np.ascontiguousarray(s, dtype=np.float64) for s in sigma_i]
        self.exc_threshold_ev = float(exc_threshold_ev)
        self.ion_threshold_ev = float(ion_threshold_ev)
        assert len(self.sigma_e) == 3 and len(self.sigma_i) == 2
        for s in self.sigma_e + self.sigma_i:
            assert s.shape == (self.n,)


def argon_synthetic(n=8192, emax_e_ev=3000.0, emax_i_ev=3000.0):
    """The synthetic argon set on n-point speed grids reaching emax. Over
    0-3 keV the electron max(sigma_T v) is 3.74e-13 m^3/s, so at 10 Pa the
    collision probability is 0.199 at N_t = 300 and 0.105 at N_t = 600."""
    vmax_e = np.sqrt(2.0 * emax_e_ev * E_CHARGE / M_ELECTRON)
    vmax_i = np.sqrt(2.0 * emax_i_ev * E_CHARGE / M_ARGON)
    dv_e = vmax_e / (n - 1)
    dv_i = vmax_i / (n - 1)
    k = np.arange(n, dtype=np.float64)
    eps_e = 0.5 * M_ELECTRON * (k * dv_e) ** 2 / E_CHARGE
    eps_i = 0.5 * M_ARGON * (k * dv_i) ** 2 / E_CHARGE
    return XsecTables(
        n, dv_e, dv_i,
        [sigma_e_elastic(eps_e), sigma_e_excitation(eps_e), sigma_e_ionization(eps_e)],
        [sigma_i_isotropic(eps_i), sigma_i_backward(eps_i)],
    )


def constant(n, dv_e, dv_i, sig_e=(1e-19, 0.0, 0.0), sig_i=(1e-18, 0.0),
             exc_threshold_ev=EXC_THRESHOLD_EV, ion_threshold_ev=ION_THRESHOLD_EV):
    """Energy-independent cross sections (test cases with closed forms)."""
    return XsecTables(
        n, dv_e, dv_i,
        [np.full(n, float(s)) for s in sig_e],
        [np.full(n, float(s)) for s in sig_i],
        exc_threshold_ev, ion_threshold_ev,
    )


def read_two_column(path):
    """A cross section as two whitespace-separated columns, energy in eV and
    sigma in m^2 (lines starting with '#' skipped), as tabulated data sets
    (e.g. from LXCat) are commonly exported."""
    a = np.loadtxt(path, comments="#", dtype=np.float64, ndmin=2)
    e, s = a[:, 0], a[:, 1]
    if not np.all(np.diff(e) > 0):
        raise ValueError(f"{path}: energies must increase")
    return e, s


def from_energy_tables(electron, ion, n=8192, emax_e_ev=3000.0, emax_i_ev=3000.0,
                       exc_threshold_ev=EXC_THRESHOLD_EV, ion_threshold_ev=ION_THRESHOLD_EV):
    """Tables in the library's layout from cross sections given on energy
    grids: electron = [(eV, m^2) for elastic, excitation, ionization], ion =
    [(eV, m^2) for isotropic, backward] (ion energies in the lab frame of
    1/2 M g^2). Each is interpolated linearly in energy at the table speeds;
    inelastic processes are zero below their thresholds, and beyond its last
    energy a table keeps its last value."""
    vmax_e = np.sqrt(2.0 * emax_e_ev * E_CHARGE / M_ELECTRON)
    vmax_i = np.sqrt(2.0 * emax_i_ev * E_CHARGE / M_ARGON)
    dv_e = vmax_e / (n - 1)
    dv_i = vmax_i / (n - 1)
    k = np.arange(n, dtype=np.float64)
    eps_e = 0.5 * M_ELECTRON * (k * dv_e) ** 2 / E_CHARGE
    eps_i = 0.5 * M_ARGON * (k * dv_i) ** 2 / E_CHARGE
    if len(electron) != 3 or len(ion) != 2:
        raise ValueError("need three electron and two ion processes")
    se = []
    for p, (e, s) in enumerate(electron):
        t = np.interp(eps_e, e, s)
        thr = (None, exc_threshold_ev, ion_threshold_ev)[p]
        if thr is not None:
            t[eps_e < thr] = 0.0
        se.append(np.maximum(t, 0.0))
    si = [np.maximum(np.interp(eps_i, e, s), 0.0) for e, s in ion]
    return XsecTables(n, dv_e, dv_i, se, si, exc_threshold_ev, ion_threshold_ev)
