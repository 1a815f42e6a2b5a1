"""FP64 oracle for steepest descent with Fourier acceleration (Alg. 2, eqs. 7-9).
Test infrastructure only.

One step, as Alg. 2 orders it:
1. Delta(x) = sum_nu Delta_{-nu}[U_nu(x) - U_nu(x)^+] - trace, the argument of
   eqs. (7)/(8) (equal to Delta of eq. 3), over the functional's directions.
2. Every matrix element of Delta is Fourier transformed over the lattice
   (4D for Landau; 3D over x, y, z in each time slice for Coulomb),
   multiplied by p^2_max / p^2 with p^2(k) = sum_mu 4 sin^2(pi k_mu / L_mu)
   the eigenvalues of -d^2 on the lattice (p^2_max = 4 x number of
   transformed axes; the zero mode, where Delta vanishes, gets factor 0),
   transformed back and normalised.
3. g(x) = exp[(alpha/2) X(x)] to first order, 1 + (alpha/2) X, then
   reunitarised (Gram-Schmidt of rows 0, 1; row 2 = conj(row0 x row1)).
4. U_mu(x) <- g(x) U_mu(x) g(x + mu)^+ for all four mu.
Alg. 2 then recomputes Delta, F and theta; the loop stops at theta < eps.

Fields are numpy arrays in the canonical layout (nt, nz, ny, nx, 4, 3, 3).
"""
from __future__ import annotations

import numpy as np

from . import core
from .diff import sd_direction, transform

LANDAU, COULOMB = 0, 1


def fft_axes(gauge):
    """Lattice axes of the array (t, z, y, x, ...) that are transformed."""
    return (0, 1, 2, 3) if gauge == LANDAU else (1, 2, 3)


def lattice_p2(shape_tzyx, gauge):
    """p^2(k) = sum over transformed axes of 4 sin^2(pi k / L), shape (nt, nz, ny, nx)."""
    p2 = np.zeros(shape_tzyx)
    for ax in fft_axes(gauge):
        L = shape_tzyx[ax]
        k = np.arange(L)
        s = 4 * np.sin(np.pi * k / L) ** 2
        bshape = [1, 1, 1, 1]
        bshape[ax] = L
        p2 = p2 + s.reshape(bshape)
    return p2


def accelerate(X, gauge):
    """F^{-1} (p^2_max / p^2) F applied to every matrix element of X (..., 3, 3)."""
    axes = fft_axes(gauge)
    p2 = lattice_p2(X.shape[:4], gauge)
    p2max = 4.0 * len(axes)
    with np.errstate(divide="ignore"):
        factor = np.where(p2 > 0, p2max / np.where(p2 > 0, p2, 1.0), 0.0)
    spec = np.fft.fftn(X, axes=axes)
    return np.fft.ifftn(spec * factor[..., None, None], axes=axes)


def gauge_step(U, alpha, gauge=LANDAU):
    """g(x) of one Fourier-accelerated steepest-descent step."""
    X = (alpha / 2) * accelerate(sd_direction(U, gauge), gauge)
    g = np.ascontiguousarray(np.eye(3) + X)
    core.reunit(g)
    return g


def sd_step(U, alpha, gauge=LANDAU):
    return np.ascontiguousarray(transform(U, gauge_step(U, alpha, gauge)))


def sd_fix(U, dims, alpha, eps, max_iter, gauge=LANDAU, check_every=1):
    """Alg. 2: returns (U, dict(converged, iters, F, theta))."""
    F, th = core.quality(U, dims, gauge)
    it, fresh = 0, True
    while it < max_iter:
        if fresh and th < eps:
            break
        U = sd_step(U, alpha, gauge)
        it += 1
        fresh = it % check_every == 0 or it == max_iter
        if fresh:
            F, th = core.quality(U, dims, gauge)
    return U, dict(converged=th < eps, iters=it, F=F, theta=th)
