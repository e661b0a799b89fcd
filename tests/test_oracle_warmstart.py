"""Pins of the warm-start oracles (CPU only): the network's BFloat16
rounding, forward and backward pass and AdamW step, and the particle loader
that draws positions and velocities from profiles."""
import numpy as np
import pytest

import oracle
from oracle import mlp

QE = 1.602176634e-19
ME = 9.1093837015e-31


# ---- BFloat16 rounding ------------------------------------------------------

def test_bf16_round_matches_torch_round_to_nearest_even():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1)
    vals = np.concatenate([
        rng.normal(size=20000).astype(np.float32) * np.float32(10.0) ** rng.integers(-30, 30, 20000),
        np.array([0.0, -0.0, 1.0, -1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -9,
                  65504.0, 3.389e38, 1e-40, -1e-42, np.inf, -np.inf], dtype=np.float32),
    ]).astype(np.float32)
    ref = torch.from_numpy(vals).to(torch.bfloat16).to(torch.float32).numpy()
    got = mlp.bf16_round(vals)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


def test_bf16_round_ties_go_to_even():
    # 1 + 2^-8 lies halfway between 1 and 1 + 2^-7: the even neighbour is 1
    assert mlp.bf16_round(np.float32(1.0 + 2.0 ** -8)) == np.float32(1.0)
    # 1 + 3 * 2^-8 lies halfway between 1 + 2^-7 and 1 + 2^-6: even is 1 + 2^-6
    assert mlp.bf16_round(np.float32(1.0 + 3 * 2.0 ** -8)) == np.float32(1.0 + 2.0 ** -6)


# ---- network ----------------------------------------------------------------

def test_gelu_known_values():
    # gelu(z) = z Phi(z): Phi(1) = 0.8413447460685429, Phi(-1) = 1 - Phi(1)
    assert mlp.gelu(np.array(1.0)) == pytest.approx(0.8413447460685429, rel=1e-15)
    assert mlp.gelu(np.array(-1.0)) == pytest.approx(-(1 - 0.8413447460685429), rel=1e-13)
    assert mlp.gelu(np.array(0.0)) == 0.0
    assert mlp.gelu(np.array(12.0)) == pytest.approx(12.0, rel=1e-15)
    z = np.linspace(-4, 4, 41)
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    np.testing.assert_allclose(mlp.gelu_grad(z), fd, rtol=1e-8, atol=1e-9)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(2)
    dims = mlp.dims_of(3, 5, 2, 4)
    p = rng.normal(scale=0.5, size=mlp.num_params(dims))
    x = rng.normal(size=(3, 3))
    t = rng.normal(size=(3, 4))
    loss, g = mlp.loss_and_grad(p, x, t, dims, exact=True)
    h = 1e-6
    fd = np.zeros_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        fd[i] = (mlp.loss_and_grad(p + e, x, t, dims, exact=True)[0]
                 - mlp.loss_and_grad(p - e, x, t, dims, exact=True)[0]) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-9)
    y, _ = mlp.forward(p, x, dims, exact=True)
    assert loss == pytest.approx(np.mean((y - t) ** 2), rel=1e-15)


def test_single_linear_layer_is_least_squares():
    # depth 0: y = x W^T + b, and the gradient of the mean squared error is
    # the normal-equation residual
    rng = np.random.default_rng(3)
    dims = mlp.dims_of(4, 8, 0, 2)
    p = rng.normal(size=mlp.num_params(dims))
    x = rng.normal(size=(6, 4))
    t = rng.normal(size=(6, 2))
    W = p[:8].reshape(2, 4)
    b = p[8:10]
    r = x @ W.T + b - t
    _, g = mlp.loss_and_grad(p, x, t, dims, exact=True)
    np.testing.assert_allclose(g[:8].reshape(2, 4), 2 * r.T @ x / r.size, rtol=1e-13)
    np.testing.assert_allclose(g[8:10], 2 * r.sum(axis=0) / r.size, rtol=1e-13)


def test_bf16_products_stay_close_to_exact():
    rng = np.random.default_rng(4)
    dims = mlp.dims_of(6, 64, 3, 32)
    p = rng.normal(scale=0.2, size=mlp.num_params(dims))
    x = rng.normal(size=(16, 6))
    ye, _ = mlp.forward(p, x, dims, exact=True)
    yq, _ = mlp.forward(p, x, dims, exact=False)
    # every operand carries at most 2^-9 relative rounding
    assert np.abs(yq - ye).max() <= 0.05 * np.abs(ye).max()
    assert not np.array_equal(yq, ye)


def test_adamw_first_step_closed_form():
    # at t = 1 the bias-corrected moments are g and g^2
    w = np.array([0.5, -1.0, 2.0, 0.0])
    g = np.array([0.1, -3.0, 0.0, 1e-3])
    lr, eps, wd = 1e-2, 1e-8, 0.01
    w1, m1, v1 = mlp.adamw(w, np.zeros(4), np.zeros(4), g, 1, lr, 0.9, 0.999, eps, wd)
    np.testing.assert_allclose(w1, w - lr * (g / (np.abs(g) + eps) + wd * w), rtol=1e-12)
    np.testing.assert_allclose(m1, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v1, 0.001 * g * g, rtol=1e-12)


# ---- particle loader ----------------------------------------------------------

def _uniforms(seed, run, species, n, purpose=0, word=0):
    r = np.array([oracle.philox4x32_10((0xFFFFFFFE, i, 16 * species + purpose, 0), (seed, run))[word]
                  for i in range(n)], dtype=np.float64)
    return (r + 0.5) * 2.0 ** -32


def test_loader_uniform_profile_is_uniform():
    L = 0.025
    x, *_ = oracle.load_profile(np.full(33, 7.0), np.full(33, 1.0), L, QE / ME, 5, 6, 0, 4000)
    u = _uniforms(5, 6, 0, 4000)
    np.testing.assert_allclose(x, u * L, rtol=0, atol=1e-12 * L)


def test_loader_linear_profile_inverts_exactly():
    # density proportional to x: cumulative (x / L)^2, so x = L sqrt(u); the
    # piecewise-linear representation is exact for a linear profile
    L = 0.03
    pts = np.linspace(0.0, 1.0, 9)
    x, *_ = oracle.load_profile(pts, np.full(9, 1.0), L, QE / ME, 9, 1, 1, 5000)
    u = _uniforms(9, 1, 1, 5000)
    np.testing.assert_allclose(x, L * np.sqrt(u), rtol=0, atol=1e-12 * L)


def test_loader_step_profile_masses_and_velocities():
    # two plateaus joined over one interval: each interval's share of the
    # particles follows its trapezoid mass, and each velocity component has
    # variance e T / m (electrons, T = 3 eV)
    L = 0.02
    dens = np.array([1.0, 1.0, 1.0, 4.0, 4.0, 4.0])
    n = 200000
    x, vx, vy, vz = oracle.load_profile(dens, np.full(6, 3.0), L, QE / ME, 3, 3, 0, n)
    h = L / 5
    mass = np.array([(dens[k] + dens[k + 1]) / 2 for k in range(5)])
    share = mass / mass.sum()
    counts = np.histogram(x, bins=np.linspace(0, L, 6))[0] / n
    sig = np.sqrt(share * (1 - share) / n)
    assert np.all(np.abs(counts - share) < 4 * sig)
    # within the rising interval the density grows linearly: mean position
    # (1/h) int t (a + (b-a) t/h) dt / mass = h (a/2 + (b-a)/3) / ((a+b)/2)
    sel = (x >= 2 * h) & (x < 3 * h)
    t = x[sel] - 2 * h
    mean_t = h * (0.5 + 3.0 / 3.0) / 2.5
    assert abs(t.mean() - mean_t) < 4 * h / np.sqrt(12 * sel.sum())
    var = QE * 3.0 / ME
    for v in (vx, vy, vz):
        assert abs(v.mean()) < 4 * np.sqrt(var / n)
        assert abs(v.var() / var - 1) < 4 * np.sqrt(2.0 / n)


def test_loader_temperature_follows_profile():
    L = 0.025
    n = 100000
    temp = np.array([1.0, 9.0])  # linear from 1 eV to 9 eV
    x, vx, _, _ = oracle.load_profile(np.ones(2), temp, L, QE / ME, 4, 4, 0, n)
    T = 1.0 + 8.0 * x / L
    # vx / sqrt(e T(x) / m) is standard normal
    z = vx / np.sqrt(QE * T / ME)
    assert abs(z.var() - 1) < 4 * np.sqrt(2.0 / n)


def test_loader_zero_mass_and_negative_values():
    L = 0.01
    x, vx, _, _ = oracle.load_profile(np.zeros(5), np.ones(5), L, QE / ME, 1, 1, 0, 10)
    assert np.all(x == 3 * L / 4)
    # negative densities count as zero: all mass in the last interval
    x, *_ = oracle.load_profile(np.array([-1.0, -2.0, 0.0, 2.0]), np.ones(4), L, QE / ME, 1, 2, 0, 1000)
    assert np.all(x >= 2 * L / 3) and np.all(x <= L)
