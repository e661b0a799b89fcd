"""Tabulated cross sections given on energy grids (two-column text files)
resampled onto the library's speed tables."""
import numpy as np

from pic_inputs import xsec


def _write(tmp_path, name, e, s):
    p = tmp_path / name
    np.savetxt(p, np.column_stack([e, s]), header="energy_eV sigma_m2")
    return p


def test_energy_tables_reproduce_the_analytic_set(tmp_path):
    # the synthetic argon set written out on a fine log grid and read back
    e = np.concatenate([[0.0], np.geomspace(1e-3, 3000.0, 4000)])
    forms = [xsec.sigma_e_elastic, xsec.sigma_e_excitation, xsec.sigma_e_ionization]
    iforms = [xsec.sigma_i_isotropic, xsec.sigma_i_backward]
    el = [xsec.read_two_column(_write(tmp_path, f"e{k}.txt", e, f(e))) for k, f in enumerate(forms)]
    io = [xsec.read_two_column(_write(tmp_path, f"i{k}.txt", e, f(e))) for k, f in enumerate(iforms)]
    t = xsec.from_energy_tables(el, io, n=2048)
    ref = xsec.argon_synthetic(n=2048)
    assert t.dv_e == ref.dv_e and t.dv_i == ref.dv_i
    for a, b in zip(t.sigma_e + t.sigma_i, ref.sigma_e + ref.sigma_i):
        # linear interpolation between log-spaced points: well under 1 %
        # of the scale except at the very first table points
        scale = np.abs(b).max()
        assert np.max(np.abs(a[4:] - b[4:])) <= 1e-2 * scale


def test_thresholds_and_extrapolation():
    e = np.array([10.0, 20.0, 30.0])
    s = np.array([1e-20, 2e-20, 3e-20])
    flat = (np.array([0.0, 1e4]), np.array([1e-19, 1e-19]))
    t = xsec.from_energy_tables([flat, (e, s), (e, s)], [flat, flat], n=512, emax_e_ev=100.0)
    eps = 0.5 * xsec.M_ELECTRON * (np.arange(512) * t.dv_e) ** 2 / xsec.E_CHARGE
    assert np.all(t.sigma_e[1][eps < xsec.EXC_THRESHOLD_EV] == 0.0)
    assert np.all(t.sigma_e[2][eps < xsec.ION_THRESHOLD_EV] == 0.0)
    # beyond the last energy the last value holds
    assert np.all(t.sigma_e[1][eps > 30.0] == 3e-20)
    mid = (eps > 20.0) & (eps < 30.0)
    np.testing.assert_allclose(t.sigma_e[1][mid], 1e-20 * (1 + eps[mid] / 10.0 - 1), rtol=1e-12)


def test_tables_drive_the_oracle(ora):
    from helpers import params

    e = np.geomspace(1e-3, 3000.0, 2000)
    el = [(e, f(e)) for f in (xsec.sigma_e_elastic, xsec.sigma_e_excitation, xsec.sigma_e_ionization)]
    io = [(e, f(e)) for f in (xsec.sigma_i_isotropic, xsec.sigma_i_backward)]
    t = xsec.from_energy_tables(el, io, n=4096)
    sim = ora.Oracle(params(), t)
    d = sim.derived()
    assert 0.0 < d["p_coll_e"] < 1.0 and 0.0 < d["p_coll_i"] < 1.0
