"""Pins of the oracle's method variants (not in the paper): the
screened-Coulomb angular distribution of electron elastic scattering and the
Opal ionization energy sharing, against their cumulative distributions, and
the default uniform sharing for contrast."""
import numpy as np
from scipy import stats

from helpers import ANISO, ME, NO_FIELD, OPAL, QE, RECORD, params, table_for

W_OPAL = 10.0


def _beam(ora, flags, sig_e, eps0, direction, n=60_000, seed=1):
    v0 = np.sqrt(2 * eps0 * QE / ME)
    p = params(flags=NO_FIELD | RECORD | flags, capacity=(3 * n, 3 * n), sort_interval=0)
    xs = table_for(2.0 * v0, 1e4, sig_e=sig_e, sig_i=(0.0, 0.0))
    sim = ora.Oracle(p, xs)
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.4, 0.6, n) * p["gap_m"]
    d = np.asarray(direction, dtype=np.float64)
    d = d / np.linalg.norm(d)
    sim.set_state(0, x, np.full(n, v0 * d[0]), np.full(n, v0 * d[1]), np.full(n, v0 * d[2]))
    sim.set_state(1, np.zeros(0), np.zeros(0), np.zeros(0), np.zeros(0))
    sim.step(1)
    code = sim.decisions(0)
    proc = (code >> 3) & 7
    out = sim.get_state(0)
    # survivors keep slot order, an ionization electron follows its parent
    births_before = np.concatenate([[0], np.cumsum(proc == 4)[:-1]])
    idx = np.arange(n) + births_before
    return proc, out, idx, v0, d


def _two_body_dir(v_out, v_in, ):
    mr = ME / (ME + 39.948 * 1.66053906660e-27)
    mm = 1.0 - mr
    speed = np.linalg.norm(v_in, axis=0)
    return (v_out - mr * v_in) / (mm * speed)


def _check_screened_coulomb(ora, direction, eps0=8.0):
    proc, out, idx, v0, d = _beam(ora, ANISO, (1e-18, 0.0, 0.0), eps0, direction)
    el = proc == 2
    assert el.sum() > 10_000
    k = idx[el]
    v_out = np.stack([out[1][k], out[2][k], out[3][k]])
    v_in = (v0 * d)[:, None] * np.ones((1, k.size))
    n = _two_body_dir(v_out, v_in)
    np.testing.assert_allclose(np.linalg.norm(n, axis=0), 1.0, rtol=1e-9)
    c = np.clip(d @ n, -1.0, 1.0)
    # the cumulative distribution of cos chi: u = ln(1 + eps (1 - c) / 2) / ln(1 + eps)
    u = np.log1p(eps0 * (1.0 - c) / 2.0) / np.log1p(eps0)
    assert stats.kstest(u, "uniform").pvalue > 1e-3
    # forward peaked: mean cos chi well above the isotropic 0
    assert c.mean() > 0.3
    # azimuth uniform about the incident direction
    a = np.array([0.0, 1.0, 0.0]) if abs(d[0]) >= 0.9 else np.array([1.0, 0.0, 0.0])
    b1 = np.cross(d, a)
    b1 /= np.linalg.norm(b1)
    b2 = np.cross(d, b1)
    ph = np.mod(np.arctan2(b2 @ n, b1 @ n), 2 * np.pi) / (2 * np.pi)
    assert stats.kstest(ph, "uniform").pvalue > 1e-3
    # energy kept up to the two-body loss
    e_in = 0.5 * ME * v0 ** 2 / QE
    e_out = 0.5 * ME * (v_out ** 2).sum(axis=0) / QE
    assert np.all(e_out <= e_in * (1 + 1e-12)) and np.all(e_out >= e_in * (1 - 4 * 2.8e-5))


def test_screened_coulomb_off_axis(ora):
    _check_screened_coulomb(ora, (0.2, 1.0, -0.5))


def test_screened_coulomb_along_x(ora):
    _check_screened_coulomb(ora, (1.0, 0.05, 0.0))


def _ionization_split(ora, flags, eps0=60.0):
    proc, out, idx, v0, d = _beam(ora, flags, (0.0, 0.0, 3e-19), eps0, (0.0, 1.0, 0.0))
    ion = proc == 4
    assert ion.sum() > 3_000
    k = idx[ion]
    e = lambda j: 0.5 * ME * (out[1][j] ** 2 + out[2][j] ** 2 + out[3][j] ** 2) / QE  # noqa: E731
    e_sc, e_ej = e(k), e(k + 1)
    avail = eps0 - 15.8
    np.testing.assert_allclose(e_sc + e_ej, avail, rtol=1e-12)
    return e_ej, avail


def test_opal_sharing_distribution(ora):
    e_ej, avail = _ionization_split(ora, OPAL)
    assert np.all(e_ej <= avail / 2 * (1 + 1e-12))
    cdf = lambda e: np.arctan(e / W_OPAL) / np.arctan(avail / (2 * W_OPAL))  # noqa: E731
    assert stats.kstest(e_ej, cdf).pvalue > 1e-3


def test_uniform_sharing_distribution(ora):
    e_ej, avail = _ionization_split(ora, 0)
    assert stats.kstest(e_ej / avail, "uniform").pvalue > 1e-3
