"""Pins of the oracle's grid steps: linear (CIC) charge assignment (Sec. 2
step 1), the finite-difference Poisson solve by the Thomas algorithm and the
field by numerical differentiation (Sec. 2 step 2)."""
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg

from pic_inputs import workloads, xsec

EPS0 = 8.8541878128e-12
QE = 1.602176634e-19
TWO32 = 2**32


# --------------------------------------------------------------- deposit ---

def test_deposit_hand_cases(ora):
    nx, L = 9, 0.008
    dx = L / (nx - 1)
    inv = 1.0 / dx
    # a particle exactly on node 3 puts all its weight there
    j, f, w1 = ora.cell(nx, inv, 3 * dx)
    assert (j, w1) == (3, 0) or (j, w1) == (2, TWO32)
    # mid-cell: half each
    j, f, w1 = ora.cell(nx, inv, 2.5 * dx)
    assert j == 2 and w1 == TWO32 // 2
    # x = 0 and x = L: all weight on the wall node
    dep = ora.deposit_array(nx, inv, np.array([0.0]))
    assert dep[0] == TWO32 and dep[1:].sum() == 0
    dep = ora.deposit_array(nx, inv, np.array([L]))
    assert dep[-1] == TWO32 and dep[:-1].sum() == 0
    # a quarter of the way into cell 5
    dep = ora.deposit_array(nx, inv, np.array([5.25 * dx]))
    assert dep[5] == 3 * TWO32 // 4 and dep[6] == TWO32 // 4


def test_deposit_partition_of_unity_and_dipole(ora):
    rng = np.random.default_rng(3)
    nx, L = 129, 0.025
    dx = L / (nx - 1)
    x = rng.uniform(0, L, size=100_000)
    dep = ora.deposit_array(nx, 1.0 / dx, x)
    # each particle deposits exactly 2^32 units
    assert int(dep.sum()) == x.size * TWO32
    # linear weighting conserves the first moment: sum_j j dx w_j = x
    # (per particle up to the 2^-33 rounding of the weight)
    first = float((np.arange(nx) * dep.astype(np.float64)).sum()) * dx / TWO32
    assert abs(first - x.sum()) < x.size * dx * 2.0**-32 + 1e-9 * x.sum()


def test_deposit_linear_weights_per_particle(ora):
    rng = np.random.default_rng(4)
    nx, L = 33, 1.0
    dx = L / (nx - 1)
    for x in rng.uniform(0, L, size=300):
        j, f, w1 = ora.cell(nx, 1.0 / dx, x)
        # node j+1 gets (x - x_j)/dx, node j the rest (shape of width 2 dx)
        assert j == min(int(x / dx), nx - 2)
        assert abs(w1 / TWO32 - (x - j * dx) / dx) < 1e-9


# --------------------------------------------------------------- Poisson ---

def test_thomas_matches_dense_solve(ora):
    rng = np.random.default_rng(5)
    n = 50
    a = rng.uniform(-1, 1, n)
    c = rng.uniform(-1, 1, n)
    b = 3.0 + rng.uniform(0, 1, n)
    d = rng.normal(size=n)
    A = np.diag(b) + np.diag(a[1:], -1) + np.diag(c[:-1], 1)
    y = ora.thomas(a, b, c, d)
    np.testing.assert_allclose(y, np.linalg.solve(A, d), rtol=1e-12, atol=1e-13)


def test_poisson_uniform_charge_closed_form(ora):
    # For uniform rho0 the second-order stencil is exact on the quadratic
    # phi = V (1 - x/L) + rho0 x (L - x) / (2 eps0).
    nx, L, V, rho0 = 257, 0.025, 250.0, 3e-4
    dx = L / (nx - 1)
    x = np.arange(nx) * dx
    phi = ora.poisson(nx, dx, V, np.full(nx, rho0))
    exact = V * (1 - x / L) + rho0 * x * (L - x) / (2 * EPS0)
    assert np.max(np.abs(phi - exact)) < 1e-12 * np.max(np.abs(exact))


def test_poisson_matches_banded_solver(ora):
    rng = np.random.default_rng(6)
    nx, L, V = 513, 0.025, -120.0
    dx = L / (nx - 1)
    rho = rng.normal(0, 1e-3, nx)
    phi = ora.poisson(nx, dx, V, rho)
    n = nx - 2
    ab = np.zeros((3, n))
    ab[0, 1:] = 1.0
    ab[1, :] = -2.0
    ab[2, :-1] = 1.0
    rhs = -dx * dx * rho[1:-1] / EPS0
    rhs[0] -= V
    ref = scipy.linalg.solve_banded((1, 1), ab, rhs)
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(phi[1:-1] - ref)) < 1e-12 * scale
    assert phi[0] == V and phi[-1] == 0.0


def test_poisson_against_exact_rationals(ora):
    # The discrete solution computed exactly in rational arithmetic; the
    # oracle's FP64 Thomas result must agree to a few ulps of max|phi|.
    rng = np.random.default_rng(7)
    nx, L, V = 65, 0.025, 100.0
    dx = L / (nx - 1)
    rho = rng.normal(0, 1e-3, nx)
    phi = ora.poisson(nx, dx, V, rho)
    n = nx - 2
    d = [Fraction(float(-(dx * dx) * rho[i + 1] / EPS0)) for i in range(n)]
    d[0] -= Fraction(V)
    # exact Thomas in rationals
    cp = [Fraction(0)] * n
    dp = [Fraction(0)] * n
    cp[0] = Fraction(1, -2)
    dp[0] = d[0] / -2
    for i in range(1, n):
        m = -2 - cp[i - 1]
        cp[i] = 1 / m
        dp[i] = (d[i] - dp[i - 1]) / m
    y = [Fraction(0)] * n
    y[-1] = dp[-1]
    for i in range(n - 2, -1, -1):
        y[i] = dp[i] - cp[i] * y[i + 1]
    exact = np.array([float(v) for v in y])
    assert np.max(np.abs(phi[1:-1] - exact)) < 64 * np.finfo(float).eps * np.max(np.abs(exact))


def test_poisson_second_order_convergence(ora):
    # rho = rho0 sin(pi x / L): phi = V(1 - x/L) + rho0 L^2/(pi^2 eps0) sin(pi x/L)
    L, V, rho0 = 0.02, 0.0, 1e-5
    errs = []
    for nx in (17, 33, 65, 129):
        dx = L / (nx - 1)
        x = np.arange(nx) * dx
        phi = ora.poisson(nx, dx, V, rho0 * np.sin(np.pi * x / L))
        exact = V * (1 - x / L) + rho0 * L**2 / (np.pi**2 * EPS0) * np.sin(np.pi * x / L)
        errs.append(np.max(np.abs(phi - exact)))
    ratios = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    for r in ratios:
        assert 3.8 < r < 4.2, ratios


# ----------------------------------------------------------------- field ---

def test_field_zero_charge_is_uniform(ora):
    nx, L, V = 129, 0.025, 77.0
    dx = L / (nx - 1)
    rho = np.zeros(nx)
    E = ora.efield(nx, dx, rho, ora.poisson(nx, dx, V, rho))
    np.testing.assert_allclose(E, V / L, rtol=1e-12)


def test_field_discrete_gauss_law(ora):
    # eps0 (E_{N-1} - E_0) = e W (P_i - P_e) / A for the deposit of any
    # particle set: charge assignment, Poisson and the wall half-cell field
    # together conserve the total charge.
    w = workloads.get("c1_small")
    p = dict(w["params"])
    xs = xsec.argon_synthetic()
    sim = ora.Oracle(p, xs)
    rng = np.random.default_rng(8)
    ne, ni = 3000, 3400
    L = p["gap_m"]
    z = np.zeros(ne)
    sim.set_state(0, rng.uniform(0, L, ne), z, z, z, step=5)
    z = np.zeros(ni)
    sim.set_state(1, rng.uniform(0, L, ni), z, z, z, step=5)
    sim.solve_field()
    f = sim.get_field()
    lhs = EPS0 * (f["E"][-1] - f["E"][0])
    rhs = QE * p["weight"] * (ni - ne) / p["area_m2"]
    assert abs(lhs - rhs) < 1e-9 * abs(rhs)
    # rho integrates (trapezoid with half cells) to the net charge per area
    dx = L / p["n_cells"]
    total = (f["rho"][1:-1].sum() + 0.5 * (f["rho"][0] + f["rho"][-1])) * dx
    assert abs(total - rhs) < 1e-9 * abs(rhs)
    # phi carries the drive V(t) at x = 0 of step 5 and 0 at x = L
    Nt = p["steps_per_cycle"]
    assert f["phi"][0] == pytest.approx(p["rf_voltage_v"] * np.cos(2 * np.pi * 5 / Nt), rel=1e-14)
    assert f["phi"][-1] == 0.0
