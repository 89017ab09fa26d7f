"""Site-local diagonal blocks D_ee, D_oo (clover-type operator) for the oracle.

Sec. 2 states the even-odd system for a general fermion matrix: Eq. (4),
(1 - D_ee^-1 D_eo D_oo^-1 D_oe) xi_e = D_ee^-1 (eta_e - D_eo D_oo^-1 eta_o),
and Eq. (5), xi_o = D_oo^-1 (eta_o - D_oe xi_e); with a clover term its
diagonal blocks act site by site, and for Wilson they are the unit matrix.  Here D = A - kappa H with A(x) a site-local 12 x 12
matrix (spin x colour) that commutes with gamma5, as a clover term
1 + c sigma_mu_nu F_mu_nu does.  D_eo = -kappa P_e H P_o, D_oe = -kappa P_o H P_e.

The site matrix is given as two 6 x 6 blocks in the gamma5 eigenbasis of the
Dirac representation, where gamma5 = -[[0, 1], [1, 0]] in 2 x 2 spin blocks:
    psi_A = (psi_up + psi_dn) / sqrt2   (gamma5 = -1),
    psi_B = (psi_up - psi_dn) / sqrt2   (gamma5 = +1),
with up = spins 0, 1 and dn = spins 2, 3, each 6-vector ordered (spin, colour).
A acts as psi_A -> B0 psi_A, psi_B -> B1 psi_B.  Plain FP64 NumPy; test
infrastructure only.
"""
import numpy as np

from .wilson import hop_eo

_S = 1.0 / np.sqrt(2.0)


def blocks_to_dirac(blocks):
    """[..., 2, 6, 6] chiral blocks -> [..., 12, 12] matrices acting on the
    Dirac-representation (spin, colour) index s * 3 + c."""
    b0, b1 = blocks[..., 0, :, :], blocks[..., 1, :, :]
    # T maps (up, dn) -> (A, B): A = (up + dn)/sqrt2, B = (up - dn)/sqrt2
    t = _S * np.block([[np.eye(6), np.eye(6)], [np.eye(6), -np.eye(6)]])
    z = np.zeros_like(b0)
    bd = np.concatenate([np.concatenate([b0, z], axis=-1), np.concatenate([z, b1], axis=-1)], axis=-2)
    return np.conj(t.T) @ bd @ t


def apply_sites(a12, psi):
    """out(x) = A(x) psi(x) for site matrices [..., 12, 12] and spinors [..., 4, 3]."""
    shp = psi.shape
    v = psi.reshape(shp[:-2] + (12,))
    return np.einsum("...ij,...j->...i", a12, v).reshape(shp)


def half_blocks(blocks_full, parity):
    """Canonical full-lattice blocks [Lt][Lz][Ly][Lx][2][6][6] -> the sites of
    one parity in half-lattice order [Lt][Lz][Ly][Lx/2][2][6][6]."""
    from .lattice import full_to_half
    return full_to_half(blocks_full, parity)


def apply_m_clover(u, psi_e, kappa, phases, ainv_e, ainv_o, dagger=False):
    """M psi_e = psi_e - D_ee^-1 D_eo D_oo^-1 D_oe psi_e
               = psi_e - kappa^2 A_ee^-1 H_eo A_oo^-1 H_oe psi_e   (Eq. (4))
    with ainv_e / ainv_o the inverse site matrices [..., 12, 12] of each
    parity in half-lattice order.  With dagger the adjoint,
    psi_e - kappa^2 H_eo^dag A_oo^-dag H_oe^dag A_ee^-dag psi_e."""
    if not dagger:
        t = apply_sites(ainv_o, hop_eo(u, psi_e, 0, phases))
        return psi_e - kappa * kappa * apply_sites(ainv_e, hop_eo(u, t, 1, phases))
    ah_e = np.conj(np.swapaxes(ainv_e, -1, -2))
    ah_o = np.conj(np.swapaxes(ainv_o, -1, -2))
    t = apply_sites(ah_o, hop_eo(u, apply_sites(ah_e, psi_e), 0, phases, dagger=True))
    return psi_e - kappa * kappa * hop_eo(u, t, 1, phases, dagger=True)


def apply_m_clover_at_sites(u, psi_e, kappa, phases, ainv_at, half_indices, dagger=False):
    """(M psi_e) of ``apply_m_clover`` at the listed even half indices, for
    lattices where whole-lattice site matrices are inconvenient: ``ainv_at(x,
    y, z, t)`` returns the inverse site matrix [12, 12] of one site.  Each
    output is psi_e(x) - kappa^2 A^-1(x) sum over the neighbours y of x of
    H(x, y) A^-1(y) (H psi_e)(y) (the adjoint takes A^-dag and the adjoint
    hops in the reverse order).  Returns (n, 4, 3)."""
    from .lattice import half_index_coords
    from .wilson import _half_getter, hop_at_site
    lt, lz, ly, lxh = psi_e.shape[:4]
    dims = (2 * lxh, ly, lz, lt)
    get_e = _half_getter(psi_e, 0, dims)

    def site_mat(site, v):
        a = ainv_at(*site)
        if dagger:
            a = np.conj(a.T)
        return (a @ v.reshape(12)).reshape(4, 3)

    if dagger:
        def get_src(x, y, z, t):
            return site_mat((x, y, z, t), get_e(x, y, z, t))
    else:
        get_src = get_e

    def get_mid(x, y, z, t):
        return site_mat((x, y, z, t), hop_at_site(u, get_src, (x, y, z, t), phases, dims, dagger))

    out = []
    for ih in half_indices:
        site = half_index_coords(dims, 0, int(ih))
        x, y, z, t = site
        hh = hop_at_site(u, get_mid, site, phases, dims, dagger)
        if not dagger:
            hh = site_mat(site, hh)
        out.append(psi_e[t, z, y, x >> 1] - kappa * kappa * hh)
    return np.array(out)


def dense_sites(a12_full):
    """Block-diagonal dense matrix of full-lattice site matrices [Lt][Lz][Ly][Lx][12][12]
    in the oracle's dense ordering (site-major, then spin, colour)."""
    n = a12_full.shape[:-2]
    v = int(np.prod(n))
    flat = a12_full.reshape(v, 12, 12)
    d = np.zeros((12 * v, 12 * v), dtype=np.complex128)
    for i in range(v):
        d[12 * i:12 * i + 12, 12 * i:12 * i + 12] = flat[i]
    return d
