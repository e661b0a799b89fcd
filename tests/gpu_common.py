"""Helpers for the GPU-vs-oracle parity tests."""
import numpy as np
import pytest

RTOL = 1e-12  # single step from a shared state: positions and velocities


def need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def assert_state_close(gpu, ora, L, vscale, rtol=RTOL, what=""):
    """Element-wise |g - o| <= rtol * max(|o|, floor), floors rtol*L for x
    and rtol*vscale for v."""
    assert gpu[0].size == ora[0].size, f"{what}: count {gpu[0].size} != {ora[0].size}"
    floors = (L, vscale, vscale, vscale)
    for k, (g, o, fl) in enumerate(zip(gpu, ora, floors)):
        tol = rtol * np.maximum(np.abs(o), fl)
        bad = np.abs(g - o) > tol
        if bad.any():
            i = int(np.argmax(bad))
            raise AssertionError(f"{what}: component {k} differs at {int(bad.sum())} slots, "
                                 f"first {i}: {g[i]!r} vs {o[i]!r}")


def assert_state_equal(gpu, ora, what=""):
    assert gpu[0].size == ora[0].size, f"{what}: count {gpu[0].size} != {ora[0].size}"
    for k, (g, o) in enumerate(zip(gpu, ora)):
        if not np.array_equal(g, o):
            bad = g != o
            i = int(np.argmax(bad))
            raise AssertionError(f"{what}: component {k} differs at {int(bad.sum())} slots, "
                                 f"first {i}: {g[i]!r} vs {o[i]!r}")


def pair(params, xs, init, step=0, fixed_E=None):
    """A GPU discharge and an oracle with the same parameters and state."""
    import oracle
    from paper_2109_04469_amd import Discharge

    gpu = Discharge(params, xs, "cuda:0")
    ora = oracle.Oracle(params, xs)
    if fixed_E is not None:
        gpu.set_field(fixed_E)
        ora.set_field(fixed_E)
    for sp in (0, 1):
        gpu.set_state(sp, *init[sp], step=step)
        ora.set_state(sp, *init[sp], step=step)
    return gpu, ora


def near_wall_state(n, L, vscale, reach, seed, species, frac=0.05):
    """Uniform particles with Gaussian velocities; a fraction sits within
    `reach` of a wall and moves towards it."""
    rng = np.random.default_rng([seed, species, 5])
    x = rng.uniform(0, L, n)
    v = rng.normal(0, vscale, (3, n))
    k = int(frac * n)
    idx = rng.choice(n, size=k, replace=False)
    side = rng.integers(0, 2, k)
    d = rng.uniform(0, reach, k)
    x[idx] = np.where(side == 0, d, L - d)
    v[0, idx] = np.where(side == 0, -1, 1) * np.abs(v[0, idx])
    return (x, v[0].copy(), v[1].copy(), v[2].copy())
