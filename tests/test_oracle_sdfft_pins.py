"""Pins of the Fourier-accelerated steepest-descent oracle (oracle/sdfft.py)."""
import numpy as np
import pytest

from oracle import sdfft

LANDAU, COULOMB = 0, 1


def lattice_laplacian(f, axes):
    """-d^2 f by nearest-neighbour differences along the given axes."""
    out = np.zeros_like(f)
    for ax in axes:
        out += 2 * f - np.roll(f, 1, axis=ax) - np.roll(f, -1, axis=ax)
    return out


@pytest.mark.parametrize("gauge", [LANDAU, COULOMB])
def test_p2_are_the_laplacian_eigenvalues(gauge):
    shape = (4, 6, 2, 8)
    p2 = sdfft.lattice_p2(shape, gauge)
    axes = sdfft.fft_axes(gauge)
    rng = np.random.default_rng(0)
    grids = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    for _ in range(10):
        k = [int(rng.integers(n)) if ax in axes else 0 for ax, n in enumerate(shape)]
        wave = np.exp(2j * np.pi * sum(k[ax] * grids[ax] / shape[ax] for ax in range(4)))
        lap = lattice_laplacian(wave, axes)
        np.testing.assert_allclose(lap, p2[tuple(k)] * wave, atol=1e-12)
    assert np.isclose(p2.max(), 4 * len(axes))


@pytest.mark.parametrize("gauge", [LANDAU, COULOMB])
def test_acceleration_scales_each_mode(gauge):
    """A single Fourier mode of an anti-hermitian field is multiplied by
    p^2_max / p^2(k); the zero mode is removed."""
    shape = (4, 4, 6, 2)
    axes = sdfft.fft_axes(gauge)
    grids = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    k = (1, 2, 1, 1) if gauge == LANDAU else (0, 1, 3, 1)
    phase = 2 * np.pi * sum(k[ax] * grids[ax] / shape[ax] for ax in range(4))
    H = np.array([[0, 1 - 2j, 0.5], [1 + 2j, 0.3, -1j], [0.5, 1j, -0.3]])
    X = 1j * np.cos(phase)[..., None, None] * H  # anti-hermitian, real amplitude
    p2 = sdfft.lattice_p2(shape, gauge)[k]
    out = sdfft.accelerate(X, gauge)
    np.testing.assert_allclose(out, (4 * len(axes) / p2) * X, atol=1e-13)
    const = np.broadcast_to(1j * H, shape + (3, 3))
    np.testing.assert_allclose(sdfft.accelerate(const, gauge), 0, atol=1e-13)


@pytest.mark.parametrize("gauge", [LANDAU, COULOMB])
def test_sd_fft_steps_increase_F_and_keep_unitarity(oracle_lib, field_cache, gauge):
    dims = (4, 4, 4, 4)
    U = field_cache(dims, 0.5, 60)
    F = [oracle_lib.quality(U, dims, gauge)[0]]
    for _ in range(20):
        U = sdfft.sd_step(U, 0.08, gauge)
        F.append(oracle_lib.quality(U, dims, gauge)[0])
    assert np.all(np.diff(F) > -1e-15)
    L = U.reshape(-1, 3, 3)
    assert np.abs(L @ np.swapaxes(L, -1, -2).conj() - np.eye(3)).max() < 1e-13


def test_sd_fft_fixes_a_pure_gauge(oracle_lib, field_cache):
    dims = (4, 4, 4, 4)
    U = field_cache(dims, 0.0, 61)
    U, r = sdfft.sd_fix(U, dims, 0.08, 1e-12, 3000)
    assert r["converged"] and abs(r["F"] - 1) < 1e-12


def test_gauge_step_is_the_accelerated_exponent_to_first_order(field_cache):
    """Before reunitarisation, g = 1 + (alpha/2) F^-1 (p2max/p2) F Delta; the
    reunitarised g differs from it at second order in alpha."""
    dims = (4, 2, 4, 2)
    U = field_cache(dims, 0.4, 62)
    X = sdfft.accelerate(sdfft.sd_direction(U, LANDAU), LANDAU)
    for alpha in (1e-3, 1e-4):
        g = sdfft.gauge_step(U, alpha)
        lin = np.eye(3) + (alpha / 2) * X
        assert np.abs(g - lin).max() < 5 * (alpha * np.abs(X).max()) ** 2
