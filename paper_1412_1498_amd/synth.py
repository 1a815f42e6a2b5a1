"""Seeded synthetic SU(3) gauge fields for tests and benchmarks.

This module only *creates inputs*; it holds none of the gauge-fixing
arithmetic (no functional, no quality measure, no local update). Both the
FP64 CPU oracle and the HIP path are fed from it, so it deliberately has its
own small SU(3) helpers (Gell-Mann table, Haar sampler, matrix exponential)
that nothing else imports.

Recipe (the paper's MILC lattices are not available; these stand in):

    U_mu(x) = h(x) . exp(i * amp * sum_a r_a lambda_a / 2) . h(x + mu)^dagger

* ``h(x)`` is Haar-distributed on SU(3): two rows drawn from a complex
  Ginibre ensemble are Gram-Schmidt orthonormalised, the third row is the
  complex-conjugated cross product of the first two (this fixes det = 1 and
  keeps the measure right-invariant, hence Haar).
* ``r_a ~ N(0, 1)`` per link and generator, ``lambda_a`` the Gell-Mann
  matrices (Tr lambda_a lambda_b = 2 delta_ab).
* With ``amp = 0`` the field is a pure gauge: a gauge transform of the unit
  field, whose Landau/Coulomb-fixed form is U = 1 everywhere.

Random numbers come from ``numpy.random.Generator(PCG64(seed))`` in a fixed
draw order: the Ginibre rows of every h(x) in site order (t slowest, x
fastest; shape [V][2][3] complex as (re, im) pairs), then r with shape
[t][z][y][x][mu][a]. The arithmetic runs in float64 with torch on the
requested device (CPU for parity fixtures, the GPU only to make large
benchmark inputs quickly); results agree across devices to rounding.

Canonical ("AoS") layout of a field: complex tensor of shape
(nt, nz, ny, nx, 4, 3, 3), i.e. [t][z][y][x][mu][row][col] with x fastest and
mu = 0, 1, 2, 3 along x, y, z, t.
"""
from __future__ import annotations

import numpy as np
import torch

__all__ = [
    "gell_mann",
    "haar_su3",
    "su3_expi",
    "random_gauge_field",
    "random_gauge_transform",
    "random_algebra_field",
    "sun_generators",
    "haar_sun",
    "random_sun_field",
]


def gell_mann(dtype=torch.complex128, device="cpu") -> torch.Tensor:
    """The eight Gell-Mann matrices, shape (8, 3, 3)."""
    s3 = 1.0 / np.sqrt(3.0)
    m = np.zeros((8, 3, 3), dtype=np.complex128)
    m[0, 0, 1] = m[0, 1, 0] = 1
    m[1, 0, 1], m[1, 1, 0] = -1j, 1j
    m[2, 0, 0], m[2, 1, 1] = 1, -1
    m[3, 0, 2] = m[3, 2, 0] = 1
    m[4, 0, 2], m[4, 2, 0] = -1j, 1j
    m[5, 1, 2] = m[5, 2, 1] = 1
    m[6, 1, 2], m[6, 2, 1] = -1j, 1j
    m[7, 0, 0] = m[7, 1, 1] = s3
    m[7, 2, 2] = -2 * s3
    return torch.from_numpy(m).to(device=device, dtype=dtype)


def haar_su3(rows: torch.Tensor) -> torch.Tensor:
    """Map Ginibre rows (..., 2, 3) complex to Haar SU(3) matrices (..., 3, 3)."""
    z0, z1 = rows[..., 0, :], rows[..., 1, :]
    r0 = z0 / torch.linalg.vector_norm(z0, dim=-1, keepdim=True)
    proj = (r0.conj() * z1).sum(-1, keepdim=True)
    r1 = z1 - proj * r0
    r1 = r1 / torch.linalg.vector_norm(r1, dim=-1, keepdim=True)
    r2 = torch.linalg.cross(r0, r1, dim=-1).conj()
    return torch.stack([r0, r1, r2], dim=-2)


def su3_expi(H: torch.Tensor) -> torch.Tensor:
    """exp(i H) for Hermitian H (..., n, n) by scaling and squaring of a
    degree-18 Taylor polynomial (every scaled argument has norm <= 1/2)."""
    X = 1j * H
    if X.numel() == 0:
        return X.clone()
    norm = torch.linalg.matrix_norm(X, ord="fro").max().item()
    s = max(0, int(np.ceil(np.log2(max(norm, 1e-300) / 0.5))))
    Y = X / (2.0 ** s)
    eye = torch.eye(X.shape[-1], dtype=X.dtype, device=X.device).expand_as(X)
    E = eye.clone()
    for k in range(18, 0, -1):  # Horner: I + Y/1 (I + Y/2 (I + ...))
        E = eye + torch.matmul(Y, E) / k
    for _ in range(s):
        E = torch.matmul(E, E)
    return E


def _shift_fwd(a: torch.Tensor, mu: int) -> torch.Tensor:
    """a(x + mu_hat) for a field shaped (nt, nz, ny, nx, ...)."""
    axis = 3 - mu
    return torch.roll(a, shifts=-1, dims=axis)


def _haar_field(dims, rng, device) -> torch.Tensor:
    nx, ny, nz, nt = (int(d) for d in dims)
    V = nx * ny * nz * nt
    g = torch.from_numpy(rng.standard_normal((V, 2, 3, 2))).to(device)
    rows = torch.complex(g[..., 0], g[..., 1])
    return haar_su3(rows).reshape(nt, nz, ny, nx, 3, 3)


def random_gauge_transform(dims, seed: int, device="cpu") -> torch.Tensor:
    """Haar-random h(x), shape (nt, nz, ny, nx, 3, 3) complex128."""
    return _haar_field(dims, np.random.Generator(np.random.PCG64(seed)), device)


def random_gauge_field(dims, amp: float, seed: int, device="cpu",
                       chunk_sites: int = 1 << 18) -> torch.Tensor:
    """Seeded synthetic SU(3) link field in the canonical layout.

    dims = (nx, ny, nz, nt). Returns complex128, shape (nt, nz, ny, nx, 4, 3, 3).
    """
    nx, ny, nz, nt = (int(d) for d in dims)
    V = nx * ny * nz * nt
    rng = np.random.Generator(np.random.PCG64(seed))
    h = _haar_field(dims, rng, device)
    r = rng.standard_normal((V, 4, 8))
    lam = gell_mann(device=device).reshape(8, 9)
    hflat = h.reshape(V, 3, 3)
    hfwd = [_shift_fwd(h, mu).reshape(V, 3, 3) for mu in range(4)]
    U = torch.empty((V, 4, 3, 3), dtype=torch.complex128, device=device)
    for s0 in range(0, V, chunk_sites):
        s1 = min(V, s0 + chunk_sites)
        rc = torch.from_numpy(r[s0:s1]).to(device=device, dtype=torch.complex128)
        H = (0.5 * amp) * torch.matmul(rc, lam).reshape(s1 - s0, 4, 3, 3)
        E = su3_expi(H)
        for mu in range(4):
            U[s0:s1, mu] = torch.matmul(torch.matmul(hflat[s0:s1], E[:, mu]),
                                        hfwd[mu][s0:s1].transpose(-1, -2).conj())
    return U.reshape(nt, nz, ny, nx, 4, 3, 3)


def random_algebra_field(dims, sigma: float, seed: int) -> torch.Tensor:
    """s_a(x) ~ N(0, sigma^2), shape (nt, nz, ny, nx, 8) float64 (CPU)."""
    nx, ny, nz, nt = (int(d) for d in dims)
    rng = np.random.Generator(np.random.PCG64(seed))
    s = rng.standard_normal((nt, nz, ny, nx, 8)) * sigma
    return torch.from_numpy(s)


def ensemble_members(n_landau: int = 64, seed: int = 0, amp: float = 0.6):
    """The uneven ensemble: one Coulomb-gauge 48^3 x 96 lattice (field seed 0)
    and n_landau Landau-gauge lattices whose sides are drawn uniformly from
    {8, 12, 16, 20, 24} with numpy PCG64(seed); member i uses field seed
    1 + i. Returns [(dims (nx, ny, nz, nt), gauge 0 Landau / 1 Coulomb, amp,
    field seed)]."""
    rng = np.random.default_rng(seed)
    sides = rng.choice([8, 12, 16, 20, 24], size=n_landau)
    return [((48, 48, 48, 96), 1, amp, 0)] + \
           [((int(L),) * 4, 0, amp, 1 + i) for i, L in enumerate(sides)]


# ---- SU(N), N != 3 ----------------------------------------------------------


def sun_generators(n: int, dtype=torch.complex128, device="cpu") -> torch.Tensor:
    """Generalised Gell-Mann matrices of SU(n), shape (n*n - 1, n, n), with
    Tr T_a T_b = 2 delta_ab: for j < k the symmetric E_jk + E_kj and the
    antisymmetric -i E_jk + i E_kj, then for l = 1..n-1 the diagonal
    sqrt(2 / (l (l + 1))) diag(1, ..., 1, -l, 0, ..., 0) (l ones)."""
    m = []
    for j in range(n):
        for k in range(j + 1, n):
            a = np.zeros((n, n), dtype=np.complex128)
            a[j, k] = a[k, j] = 1
            m.append(a)
            b = np.zeros((n, n), dtype=np.complex128)
            b[j, k], b[k, j] = -1j, 1j
            m.append(b)
    for l in range(1, n):
        c = np.zeros((n, n), dtype=np.complex128)
        c[range(l), range(l)] = 1
        c[l, l] = -l
        m.append(c * np.sqrt(2.0 / (l * (l + 1))))
    return torch.from_numpy(np.stack(m)).to(device=device, dtype=dtype)


def haar_sun(rows: torch.Tensor) -> torch.Tensor:
    """Map Ginibre rows (..., n-1, n) complex to Haar SU(n) matrices
    (..., n, n): Gram-Schmidt of the n-1 rows, last row the complex
    conjugate of its cofactors (det = 1). For n = 3 this is haar_su3."""
    n = rows.shape[-1]
    out = []
    for r in range(n - 1):
        v = rows[..., r, :]
        for q in out:
            v = v - (q.conj() * v).sum(-1, keepdim=True) * q
        out.append(v / torch.linalg.vector_norm(v, dim=-1, keepdim=True))
    top = torch.stack(out, dim=-2)  # (..., n-1, n)
    last = []
    for j in range(n):
        sub = torch.cat([top[..., :, :j], top[..., :, j + 1:]], dim=-1)
        c = torch.linalg.det(sub)
        last.append((-c if (n - 1 + j) % 2 else c).conj())
    return torch.cat([top, torch.stack(last, dim=-1).unsqueeze(-2)], dim=-2)


def random_sun_field(dims, n: int, amp: float, seed: int, device="cpu",
                     chunk_sites: int = 1 << 16) -> torch.Tensor:
    """Seeded synthetic SU(n) link field, the SU(3) recipe with n colours:
    U_mu(x) = h(x) exp(i amp sum_a r_a T_a / 2) h(x + mu)^dagger, h Haar on
    SU(n) (Ginibre rows (V, n-1, n) as (re, im) pairs drawn first, in site
    order), r ~ N(0, 1) with shape [t][z][y][x][mu][a], a < n*n - 1.
    Returns complex128, shape (nt, nz, ny, nx, 4, n, n)."""
    nx, ny, nz, nt = (int(d) for d in dims)
    V = nx * ny * nz * nt
    rng = np.random.Generator(np.random.PCG64(seed))
    g = torch.from_numpy(rng.standard_normal((V, n - 1, n, 2))).to(device)
    h = haar_sun(torch.complex(g[..., 0], g[..., 1])).reshape(nt, nz, ny, nx, n, n)
    na = n * n - 1
    r = rng.standard_normal((V, 4, na))
    T = sun_generators(n, device=device).reshape(na, n * n)
    hflat = h.reshape(V, n, n)
    hfwd = [_shift_fwd(h, mu).reshape(V, n, n) for mu in range(4)]
    U = torch.empty((V, 4, n, n), dtype=torch.complex128, device=device)
    for s0 in range(0, V, chunk_sites):
        s1 = min(V, s0 + chunk_sites)
        rc = torch.from_numpy(r[s0:s1]).to(device=device, dtype=torch.complex128)
        H = (0.5 * amp) * torch.matmul(rc, T).reshape(s1 - s0, 4, n, n)
        E = su3_expi(H)
        for mu in range(4):
            U[s0:s1, mu] = torch.matmul(torch.matmul(hflat[s0:s1], E[:, mu]),
                                        hfwd[mu][s0:s1].transpose(-1, -2).conj())
    return U.reshape(nt, nz, ny, nx, 4, n, n)
