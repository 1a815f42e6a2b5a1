"""FP64 oracle for F_U[g] as a function of a gauge transformation, its
gradient, and the steepest-descent step of eq. (7). Test infrastructure only.

g(x) = exp(S(x)), S(x) = i sum_a s_a(x) lambda_a / 2. With the hermitian
H = sum_a s_a lambda_a / 2 diagonalised as H = W diag(t) W^+, every function
of S is evaluated through the eigenvalues i t_j:

* exp(S) = W diag(e^{i t_j}) W^+.
* d exp(S) / d s_a = W [(W^+ (i lambda_a / 2) W) o Phi] W^+ with the
  divided differences Phi_jk = (e^{i t_j} - e^{i t_k}) / (i t_j - i t_k),
  Phi_jj = e^{i t_j} (the derivative of a matrix function along a
  direction, taken in the eigenbasis).
* F_U[g] (eq. 1) = sum_x sum_{mu in D} Re Tr[g(x) U_mu(x) g(x+mu)^+] / (d N_c V),
  d = 4 (Landau) or 3 (Coulomb, mu = 0..2).
* dF/ds_a(x) = Re Tr[(dg(x)/ds_a) K(x)] / (d N_c V) with K of eq. (5):
  K(x) = sum_{mu in D} [U_mu(x) g(x+mu)^+ + U_mu(x-mu)^+ g(x-mu)^+].
* eq. (7): g(x) = exp[(alpha/2) (sum_nu Delta_{-nu}[U_nu(x) - U_nu(x)^+] - trace)]
  with the backward difference Delta_{-nu} f(x) = f(x - nu) - f(x) of eq. (9),
  applied as U_mu(x) <- g(x) U_mu(x) g(x+mu)^+ for all mu.

Fields are numpy arrays in the canonical layout (nt, nz, ny, nx, 4, 3, 3);
algebra fields s have shape (nt, nz, ny, nx, 8).
"""
from __future__ import annotations

import numpy as np

LANDAU, COULOMB = 0, 1


def gell_mann():
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1], lam[1][1, 0] = -1j, 1j
    lam[2][0, 0], lam[2][1, 1] = 1, -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2], lam[4][2, 0] = -1j, 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2], lam[6][2, 1] = -1j, 1j
    lam[7] = np.diag([1.0, 1.0, -2.0]) / np.sqrt(3.0)
    return lam


LAMBDA = gell_mann()


def _dag(m):
    return np.swapaxes(m, -1, -2).conj()


def _fwd(a, mu):
    """a(x + mu) for arrays shaped (nt, nz, ny, nx, ...)."""
    return np.roll(a, -1, axis=3 - mu)


def _bwd(a, mu):
    """a(x - mu)."""
    return np.roll(a, 1, axis=3 - mu)


def _ndirs(gauge):
    return 3 if gauge == COULOMB else 4


def hermitian_generator(s):
    """H = sum_a s_a lambda_a / 2, shape (..., 3, 3)."""
    return np.einsum("...a,aij->...ij", s, LAMBDA) / 2


def expi_eig(H):
    """exp(i H) for hermitian H via eigendecomposition; returns (E, t, W)."""
    t, W = np.linalg.eigh(H)
    E = np.einsum("...ij,...j,...kj->...ik", W, np.exp(1j * t), W.conj())
    return E, t, W


def gauge_fields(s):
    return expi_eig(hermitian_generator(s))[0]


def transform(U, g):
    """U_mu(x) <- g(x) U_mu(x) g(x+mu)^+ for all four mu."""
    out = np.empty_like(U)
    for mu in range(4):
        out[..., mu, :, :] = g @ U[..., mu, :, :] @ _dag(_fwd(g, mu))
    return out


def functional(U, s, gauge=LANDAU):
    """F_U[g] of eq. (1) for g = exp(S(s))."""
    g = gauge_fields(s)
    nd = _ndirs(gauge)
    V = U.shape[0] * U.shape[1] * U.shape[2] * U.shape[3]
    tot = 0.0
    for mu in range(nd):
        tot += np.einsum("...ij,...ji->...", g @ U[..., mu, :, :], _dag(_fwd(g, mu))).real.sum()
    return tot / (nd * 3 * V)


def staple(U, g, gauge=LANDAU):
    """K(x) of eq. (5) for the transformation g (all sites)."""
    nd = _ndirs(gauge)
    K = np.zeros(U.shape[:4] + (3, 3), dtype=np.complex128)
    for mu in range(nd):
        K += U[..., mu, :, :] @ _dag(_fwd(g, mu))
        K += _dag(_bwd(U[..., mu, :, :], mu)) @ _dag(_bwd(g, mu))
    return K


def dexp_directions(t, W):
    """d exp(S)/d s_a for a = 1..8 at every site, shape (..., 8, 3, 3)."""
    ej = np.exp(1j * t)
    dt = t[..., :, None] - t[..., None, :]
    mid = np.exp(1j * (t[..., :, None] + t[..., None, :]) / 2)
    # (e^{i tj} - e^{i tk}) / (i (tj - tk)) = e^{i (tj+tk)/2} sinc((tj - tk)/2)
    half = dt / 2
    with np.errstate(invalid="ignore", divide="ignore"):
        sinc = np.where(np.abs(half) > 1e-8, np.sin(half) / np.where(half == 0, 1, half),
                        1 - half ** 2 / 6)
    Phi = mid * sinc
    Xa = 1j * LAMBDA / 2
    Wd = _dag(W)
    A = np.einsum("...ij,ajk,...kl->...ail", Wd, Xa, W)     # W^+ X_a W
    return np.einsum("...ij,...ajk,...lk->...ail", W, A * Phi[..., None, :, :], W.conj())


def gradient(U, s, gauge=LANDAU):
    """dF_U[g]/ds_a(x), shape (nt, nz, ny, nx, 8)."""
    E, t, W = expi_eig(hermitian_generator(s))
    K = staple(U, E, gauge)
    D = dexp_directions(t, W)
    nd = _ndirs(gauge)
    V = U.shape[0] * U.shape[1] * U.shape[2] * U.shape[3]
    return np.einsum("...aij,...ji->...a", D, K).real / (nd * 3 * V)


def sd_direction(U, gauge=LANDAU):
    """sum_nu Delta_{-nu}[U_nu(x) - U_nu(x)^+] - trace (the argument of eq. 7
    without alpha/2), shape (nt, nz, ny, nx, 3, 3)."""
    nd = _ndirs(gauge)
    X = np.zeros(U.shape[:4] + (3, 3), dtype=np.complex128)
    for nu in range(nd):
        A = U[..., nu, :, :] - _dag(U[..., nu, :, :])
        X += _bwd(A, nu) - A
    tr = np.trace(X, axis1=-2, axis2=-1) / 3
    X -= tr[..., None, None] * np.eye(3)
    return X


def sd_step(U, alpha, gauge=LANDAU):
    """One naive steepest-descent step, eq. (7), applied to U (returns new U)."""
    X = (alpha / 2) * sd_direction(U, gauge)   # anti-hermitian
    g = expi_eig(-1j * X)[0]                    # exp(X) = exp(i (-i X))
    return transform(U, g)
