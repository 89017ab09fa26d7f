"""Seeded synthetic inputs for the even-odd Wilson operator.

This module only draws and shapes random fields.  It contains none of the
operator's arithmetic (no hopping term, no projector, no solver), so both the
CPU oracle's tests and the GPU path's tests and benchmarks can consume the very
same FP64 arrays.

Canonical host layouts (complex128, x fastest):

* gauge field ``U[mu][t][z][y][x][a][b]``: one SU(3) matrix per link, mu = 0..3
  for the x, y, z, t directions (the link joins x and x + mu-hat, paper Sec. 2);
* full-lattice spinor ``psi[t][z][y][x][s][c]``: 4 spin x 3 colour components
  per site (paper Sec. 2, footnote to Eq. (1));
* one-parity spinor ``psi[t][z][y][x//2][s][c]``: the sites of one parity
  compacted along x (paper Sec. 3.3, Fig. 4).  The site with half index
  ``xh`` in row (y, z, t) of parity p sits at ``x = 2*xh + ((y+z+t+p) & 1)``.

Recipes (all normal draws are i.i.d. N(0, 1) from ``numpy.random.PCG64``):

* links: for each link draw a complex 3x3 matrix A (real and imaginary parts
  from one array of shape ``(4, Lt, Lz, Ly, Lx, 3, 3, 2)`` drawn in that
  order), set ``H = (A + A^dagger)/2`` minus its trace part, and take
  ``U = exp(i eps H)``; the rows are then re-orthonormalised and the third
  row is rebuilt as the conjugated cross product of the first two so that
  ``det U = 1`` to rounding.  The matrix exponential uses the closed
  Cayley-Hamilton form of Morningstar and Peardon (Phys. Rev. D 69, 054501,
  2004), which is exact for 3x3 Hermitian arguments.
* spinors: real and imaginary parts of every component drawn independently,
  directly on the one-parity lattice.
* point + noise sources: ``e_(s,c)`` at the origin (an even site) plus Gaussian
  noise of standard deviation ``(24 * V/2) ** -0.5`` per real component.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "seed_for", "rng", "gen_gauge", "gen_spinor_half", "gen_spinor_full",
    "gen_point_noise_sources", "gen_su3_random", "gen_traceless_hermitian",
    "check_dims", "half_volume",
]

# Config numbers used to derive seeds: 1 = 4^4 FP64, 2 = 32^3x64 FP32,
# 3 = 48^3x96 mixed precision, 4 = 32^3x64 with 12 sources, 5 = 16^3x32
# gradients.  Roles: 1 gauge, 2 source/psi, 3 eta, 4 phi, 5 directions,
# 6 noise.
def seed_for(config: int, role: int) -> int:
    return 100 * int(config) + int(role)


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def check_dims(dims) -> tuple:
    d = tuple(int(v) for v in dims)
    if len(d) != 4 or any(v < 2 or v % 2 for v in d):
        raise ValueError(f"lattice dims must be 4 even extents >= 2, got {dims}")
    return d


def half_volume(dims) -> int:
    lx, ly, lz, lt = check_dims(dims)
    return lx * ly * lz * lt // 2


def _complex_normal(g: np.random.Generator, shape) -> np.ndarray:
    a = g.standard_normal(tuple(shape) + (2,))
    return a[..., 0] + 1j * a[..., 1]


def _traceless_hermitian_from(a: np.ndarray) -> np.ndarray:
    h = 0.5 * (a + np.conj(np.swapaxes(a, -1, -2)))
    tr = (h[..., 0, 0] + h[..., 1, 1] + h[..., 2, 2]).real / 3.0
    for i in range(3):
        h[..., i, i] -= tr
    return h


def gen_traceless_hermitian(g: np.random.Generator, n: int) -> np.ndarray:
    """n random traceless Hermitian 3x3 matrices (Gaussian entries)."""
    return _traceless_hermitian_from(_complex_normal(g, (n, 3, 3)))


def _det3(q: np.ndarray) -> np.ndarray:
    return (q[:, 0, 0] * (q[:, 1, 1] * q[:, 2, 2] - q[:, 1, 2] * q[:, 2, 1])
            - q[:, 0, 1] * (q[:, 1, 0] * q[:, 2, 2] - q[:, 1, 2] * q[:, 2, 0])
            + q[:, 0, 2] * (q[:, 1, 0] * q[:, 2, 1] - q[:, 1, 1] * q[:, 2, 0]))


def _expi_traceless_hermitian(q: np.ndarray) -> np.ndarray:
    """exp(iQ) for a stack (N,3,3) of traceless Hermitian Q.

    Cayley-Hamilton: exp(iQ) = f0 + f1 Q + f2 Q^2 with the coefficients of
    Morningstar and Peardon (2004), evaluated for |det Q| and mapped back with
    f_j(-c0) = (-1)^j conj(f_j(c0)).
    """
    c0 = _det3(q).real
    q2 = q @ q
    c1 = 0.5 * (q2[:, 0, 0] + q2[:, 1, 1] + q2[:, 2, 2]).real
    c1 = np.maximum(c1, 0.0)
    c0max = 2.0 * (c1 / 3.0) ** 1.5
    neg = c0 < 0
    safe = c0max > 0
    ratio = np.where(safe, np.abs(c0) / np.where(safe, c0max, 1.0), 0.0)
    theta = np.arccos(np.clip(ratio, 0.0, 1.0))
    u = np.sqrt(c1 / 3.0) * np.cos(theta / 3.0)
    w = np.sqrt(c1) * np.sin(theta / 3.0)
    w2 = w * w
    small = np.abs(w) < 0.05
    xi0 = np.where(small, 1.0 - w2 / 6.0 * (1.0 - w2 / 20.0 * (1.0 - w2 / 42.0)),
                   np.sin(w) / np.where(small, 1.0, w))
    e2iu = np.exp(2j * u)
    emiu = np.exp(-1j * u)
    cw = np.cos(w)
    uu = u * u
    h0 = (uu - w2) * e2iu + emiu * (8.0 * uu * cw + 2j * u * (3.0 * uu + w2) * xi0)
    h1 = 2.0 * u * e2iu - emiu * (2.0 * u * cw - 1j * (3.0 * uu - w2) * xi0)
    h2 = e2iu - emiu * (cw + 3j * u * xi0)
    den = 9.0 * uu - w2
    zero = den <= 0.0          # only Q == 0 reaches this
    den = np.where(zero, 1.0, den)
    f0 = np.where(zero, 1.0, h0 / den)
    f1 = np.where(zero, 0.0, h1 / den)
    f2 = np.where(zero, 0.0, h2 / den)
    f0 = np.where(neg, np.conj(f0), f0)
    f1 = np.where(neg, -np.conj(f1), f1)
    f2 = np.where(neg, np.conj(f2), f2)
    out = f1[:, None, None] * q + f2[:, None, None] * q2
    for i in range(3):
        out[:, i, i] += f0
    return out


def _reunitarise(u: np.ndarray) -> np.ndarray:
    """Gram-Schmidt on rows 0 and 1, row 2 = conj(row0 x row1): det = 1."""
    r0 = u[:, 0, :]
    r0 = r0 / np.sqrt(np.sum(np.abs(r0) ** 2, axis=1))[:, None]
    r1 = u[:, 1, :]
    r1 = r1 - np.sum(np.conj(r0) * r1, axis=1)[:, None] * r0
    r1 = r1 / np.sqrt(np.sum(np.abs(r1) ** 2, axis=1))[:, None]
    r2 = np.conj(np.stack([r0[:, 1] * r1[:, 2] - r0[:, 2] * r1[:, 1],
                           r0[:, 2] * r1[:, 0] - r0[:, 0] * r1[:, 2],
                           r0[:, 0] * r1[:, 1] - r0[:, 1] * r1[:, 0]], axis=1))
    return np.stack([r0, r1, r2], axis=1)


def gen_su3_near_unit(g: np.random.Generator, n: int, eps: float,
                      chunk: int = 1 << 20) -> np.ndarray:
    """n links exp(i eps H), H Gaussian traceless Hermitian, re-unitarised.

    Normals are drawn sequentially chunk by chunk; the result does not depend
    on ``chunk`` because the generator's normal stream is sequential.
    """
    out = np.empty((n, 3, 3), dtype=np.complex128)
    for s in range(0, n, chunk):
        m = min(chunk, n - s)
        h = _traceless_hermitian_from(_complex_normal(g, (m, 3, 3)))
        out[s:s + m] = _reunitarise(_expi_traceless_hermitian(eps * h))
    return out


def gen_gauge(dims, eps: float, seed: int) -> np.ndarray:
    """Near-unit random SU(3) gauge field, complex128 [4][Lt][Lz][Ly][Lx][3][3]."""
    lx, ly, lz, lt = check_dims(dims)
    n = 4 * lt * lz * ly * lx
    u = gen_su3_near_unit(rng(seed), n, float(eps))
    return u.reshape(4, lt, lz, ly, lx, 3, 3)


def gen_unit_gauge(dims) -> np.ndarray:
    lx, ly, lz, lt = check_dims(dims)
    u = np.zeros((4, lt, lz, ly, lx, 3, 3), dtype=np.complex128)
    for i in range(3):
        u[..., i, i] = 1.0
    return u


def gen_su3_random(dims, seed: int) -> np.ndarray:
    """Haar-like random SU(3) per site, complex128 [Lt][Lz][Ly][Lx][3][3].

    QR of a complex Gaussian matrix with the phases of R's diagonal moved into
    Q, then divided by a cube root of the determinant.  Used as a gauge
    transformation in covariance tests.
    """
    lx, ly, lz, lt = check_dims(dims)
    n = lx * ly * lz * lt
    a = _complex_normal(rng(seed), (n, 3, 3))
    q, r = np.linalg.qr(a)
    d = np.diagonal(r, axis1=1, axis2=2)
    q = q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(q)
    q = q / (det ** (1.0 / 3.0))[:, None, None]
    return q.reshape(lt, lz, ly, lx, 3, 3)


def gen_spinor_half(dims, seed: int, nrhs: int | None = None) -> np.ndarray:
    """Gaussian one-parity spinor, complex128 [(nrhs)][Lt][Lz][Ly][Lx/2][4][3]."""
    lx, ly, lz, lt = check_dims(dims)
    shape = (lt, lz, ly, lx // 2, 4, 3)
    if nrhs is not None:
        shape = (int(nrhs),) + shape
    return _complex_normal(rng(seed), shape)


def gen_spinor_full(dims, seed: int) -> np.ndarray:
    """Gaussian full-lattice spinor, complex128 [Lt][Lz][Ly][Lx][4][3]."""
    lx, ly, lz, lt = check_dims(dims)
    return _complex_normal(rng(seed), (lt, lz, ly, lx, 4, 3))


def gen_site_blocks(dims, eps: float, seed: int) -> np.ndarray:
    """Site-local diagonal blocks of a clover-type operator: per site two 6 x 6
    Hermitian matrices 1 + eps * X, X with Gaussian entries (X = (G + G^dag) / 2
    scaled by 6^-1/2), complex128 [Lt][Lz][Ly][Lx][2][6][6].  Near the identity
    (invertible for eps well below 1), like 1 + c sigma.F on smooth links."""
    lx, ly, lz, lt = check_dims(dims)
    g = _complex_normal(rng(seed), (lt, lz, ly, lx, 2, 6, 6))
    x = 0.5 * (g + np.conj(np.swapaxes(g, -1, -2))) / np.sqrt(6.0)
    return np.eye(6, dtype=np.complex128) + eps * x


def gen_point_noise_sources(dims, seed: int, sigma: float | None = None) -> np.ndarray:
    """12 sources (one per spin x colour) on the even sublattice.

    Source k = 3*s + c is the unit vector e_(s,c) at the origin (half index 0,
    an even site) plus i.i.d. Gaussian noise of standard deviation ``sigma``
    per real component (default ``(24 * V/2) ** -0.5``, so the noise norm is
    about 1, the norm of the point part).
    """
    lx, ly, lz, lt = check_dims(dims)
    vh = lx * ly * lz * lt // 2
    if sigma is None:
        sigma = (24.0 * vh) ** -0.5
    b = sigma * _complex_normal(rng(seed), (12, lt, lz, ly, lx // 2, 4, 3))
    for k in range(12):
        b[k, 0, 0, 0, 0, k // 3, k % 3] += 1.0
    return b
