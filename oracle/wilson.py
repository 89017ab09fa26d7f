"""Wilson hopping term, Wilson matrix and the even-odd Schur operator (oracle).

Conventions (paper Sec. 2):

* Eq. (1):  D_W(x, y) = delta_xy - kappa * H(x, y) with the hopping term
      H(x, y) = sum_mu [ (1 - gamma_mu) U_mu(x) delta_{x+mu, y}
                        + (1 + gamma_mu) U_mu(x - mu)^dag delta_{x-mu, y} ].
  The forward neighbour carries (1 - gamma_mu) as in Eq. (1); the serial
  pseudo-code of Fig. 2 writes the opposite signs, which is the same operator
  in the representation gamma -> -gamma.  The oracle follows Eq. (1).
* Boundary conditions are a U(1) phase per direction: a hop that crosses the
  lattice edge forward picks up phases[mu], a hop that crosses it backward
  picks up conj(phases[mu]).  Periodic is 1, antiperiodic is -1.
* Eqs. (3)-(4) with D_ee = D_oo = 1 (Wilson, Sec. 2): D_eo = -kappa P_e H P_o,
  D_oe = -kappa P_o H P_e, and the operator on the even sublattice is
      M = 1 - kappa^2 (P_e H P_o)(P_o H P_e).
  ``hop_eo`` returns the hopping block without the -kappa factor.
* "dagger" is the Hermitian conjugate of the operator; for H it swaps the
  two projectors and keeps the phases, so H^dag = gamma5 H gamma5.

Spinor layout [t][z][y][x][spin][colour]; links U[mu][t][z][y][x][a][b].
"""
import numpy as np

from .gamma import GAMMA5, proj_minus, proj_plus
from .lattice import dims_of, full_to_half, half_to_full, half_index_coords


def _axis(mu: int) -> int:
    # arrays are [t][z][y][x]: x is axis 3, t is axis 0
    return 3 - mu


def _slice_at(ndim: int, axis: int, index: int):
    s = [slice(None)] * ndim
    s[axis] = index
    return tuple(s)


def _colour(u: np.ndarray, v: np.ndarray) -> np.ndarray:
    """(U v)_sa = sum_b U_ab v_sb at every site."""
    return np.einsum("...ab,...sb->...sa", u, v)


def _colour_dag(u: np.ndarray, v: np.ndarray) -> np.ndarray:
    """(U^dag v)_sa = sum_b conj(U_ba) v_sb at every site."""
    return np.einsum("...ba,...sb->...sa", np.conj(u), v)


def _spin(p: np.ndarray, v: np.ndarray) -> np.ndarray:
    return np.einsum("st,...ta->...sa", p, v)


def hop(u, psi, phases, dagger=False, dirs=(0, 1, 2, 3)):
    """Full-lattice hopping term H psi (Eq. (1) without delta and -kappa).

    ``dirs`` restricts the sum over mu (used to test one direction alone).
    """
    psi = np.asarray(psi, dtype=np.complex128)
    out = np.zeros_like(psi)
    for mu in dirs:
        ax = _axis(mu)
        length = psi.shape[ax]
        pf, pb = proj_minus(mu), proj_plus(mu)
        if dagger:
            pf, pb = pb, pf
        # forward: psi(x + mu); the site at x_mu = L-1 reads the wrapped value
        fwd = np.roll(psi, -1, axis=ax)
        fwd[_slice_at(psi.ndim, ax, length - 1)] *= phases[mu]
        out += _spin(pf, _colour(u[mu], fwd))
        # backward: U(x - mu)^dag psi(x - mu); the site at x_mu = 0 wraps
        bwd = np.roll(psi, 1, axis=ax)
        bwd[_slice_at(psi.ndim, ax, 0)] *= np.conj(phases[mu])
        ub = np.roll(u[mu], 1, axis=ax)
        out += _spin(pb, _colour_dag(ub, bwd))
    return out


def dirac_wilson(u, psi, kappa, phases, dagger=False):
    """D_W psi = psi - kappa H psi (Eq. (1)); dagger gives D_W^dag psi."""
    return psi - kappa * hop(u, psi, phases, dagger=dagger)


def hop_eo(u, psi_half, in_parity, phases, dagger=False):
    """Hopping block from parity ``in_parity`` to the other parity.

    in_parity 0 gives P_o H P_e (the hop inside D_oe), 1 gives P_e H P_o.
    Input and output are one-parity arrays [t][z][y][x/2][4][3].
    """
    lt, lz, ly, lxh = psi_half.shape[:4]
    dims = (2 * lxh, ly, lz, lt)
    full = half_to_full(psi_half, in_parity, dims)
    return full_to_half(hop(u, full, phases, dagger=dagger), 1 - in_parity)


def apply_m(u, psi_e, kappa, phases, dagger=False):
    """M psi_e = psi_e - kappa^2 P_e H P_o H psi_e (Eq. (4) left-hand side).

    With dagger, M^dag = 1 - kappa^2 P_e H^dag P_o H^dag P_e.
    """
    tmp_o = hop_eo(u, psi_e, 0, phases, dagger=dagger)
    return psi_e - kappa * kappa * hop_eo(u, tmp_o, 1, phases, dagger=dagger)


def apply_mdagm(u, psi_e, kappa, phases):
    return apply_m(u, apply_m(u, psi_e, kappa, phases), kappa, phases, dagger=True)


def gamma5_half(psi):
    """gamma5 acting on the spin index of any spinor array."""
    return np.einsum("st,...ta->...sa", GAMMA5, psi)


# ---------------------------------------------------------------------------
# Dense second route: the component formula of the footnote to Eq. (1),
# assembled site by site with explicit index arithmetic (no np.roll).
# ---------------------------------------------------------------------------

def site_index(x, y, z, t, dims):
    lx, ly, lz, _ = dims
    return x + lx * (y + ly * (z + lz * t))


def dense_hop(u, phases):
    """Dense 12V x 12V matrix of H; row (site, spin i, colour a) = 12n+3i+a."""
    lt, lz, ly, lx = u.shape[1:5]
    dims = (lx, ly, lz, lt)
    vol = lx * ly * lz * lt
    h = np.zeros((12 * vol, 12 * vol), dtype=np.complex128)
    extent = dims
    for t in range(lt):
        for z in range(lz):
            for y in range(ly):
                for x in range(lx):
                    c = [x, y, z, t]
                    n = site_index(x, y, z, t, dims)
                    for mu in range(4):
                        # forward neighbour y = x + mu
                        f = list(c)
                        f[mu] += 1
                        ph = 1.0
                        if f[mu] == extent[mu]:
                            f[mu] = 0
                            ph = phases[mu]
                        m = site_index(*f, dims)
                        link = u[mu, t, z, y, x]
                        h[12 * n:12 * n + 12, 12 * m:12 * m + 12] += \
                            np.kron(proj_minus(mu), ph * link)
                        # backward neighbour y = x - mu
                        b = list(c)
                        b[mu] -= 1
                        ph = 1.0
                        if b[mu] < 0:
                            b[mu] = extent[mu] - 1
                            ph = np.conj(phases[mu])
                        m = site_index(*b, dims)
                        bx, by, bz, bt = b
                        link = u[mu, bt, bz, by, bx]
                        # (U^dag)_ab = conj(U_ba)
                        h[12 * n:12 * n + 12, 12 * m:12 * m + 12] += \
                            np.kron(proj_plus(mu), ph * np.conj(link.T))
    return h


def dense_dirac_wilson(u, kappa, phases):
    h = dense_hop(u, phases)
    return np.eye(h.shape[0], dtype=np.complex128) - kappa * h


def dense_parity_rows(dims, parity):
    """Row indices of the dense matrix that belong to sites of one parity,
    in the order of the one-parity compaction (x/2 fastest)."""
    lx, ly, lz, lt = dims
    rows = []
    for ih in range(lx * ly * lz * lt // 2):
        x, y, z, t = half_index_coords(dims, parity, ih)
        n = site_index(x, y, z, t, dims)
        rows.extend(range(12 * n, 12 * n + 12))
    return np.array(rows)


def flatten_half(psi_half):
    """One-parity array -> vector in the order of ``dense_parity_rows``."""
    return np.asarray(psi_half).reshape(-1)


# ---------------------------------------------------------------------------
# Per-site evaluation: used to check sampled outputs on lattices too large for
# the full-lattice routines to be convenient.
# ---------------------------------------------------------------------------

def _half_getter(field_half, parity, dims):
    lx, ly, lz, lt = dims

    def get(x, y, z, t):
        assert (x + y + z + t) % 2 == parity
        return field_half[t, z, y, x >> 1]
    return get


def hop_at_site(u, get, site, phases, dims, dagger=False):
    """(H psi)(site) for a field given by ``get(x, y, z, t) -> (4, 3)``."""
    out = np.zeros((4, 3), dtype=np.complex128)
    for mu in range(4):
        pf, pb = proj_minus(mu), proj_plus(mu)
        if dagger:
            pf, pb = pb, pf
        f = list(site)
        f[mu] += 1
        ph = 1.0
        if f[mu] == dims[mu]:
            f[mu] = 0
            ph = phases[mu]
        x, y, z, t = site
        link = u[mu, t, z, y, x]
        out += ph * (pf @ (get(*f) @ link.T))
        b = list(site)
        b[mu] -= 1
        ph = 1.0
        if b[mu] < 0:
            b[mu] = dims[mu] - 1
            ph = np.conj(phases[mu])
        bx, by, bz, bt = b
        link = u[mu, bt, bz, by, bx]
        out += ph * (pb @ (get(*b) @ np.conj(link)))
    return out


def apply_m_at_sites(u, psi_e, kappa, phases, half_indices, dagger=False):
    """(M psi_e) at the listed even half indices; returns (n, 4, 3)."""
    lt, lz, ly, lxh = psi_e.shape[:4]
    dims = (2 * lxh, ly, lz, lt)
    get_e = _half_getter(psi_e, 0, dims)

    def get_tmp(x, y, z, t):
        return hop_at_site(u, get_e, (x, y, z, t), phases, dims, dagger)

    out = []
    for ih in half_indices:
        site = half_index_coords(dims, 0, int(ih))
        x, y, z, t = site
        hh = hop_at_site(u, get_tmp, site, phases, dims, dagger)
        out.append(psi_e[t, z, y, x >> 1] - kappa * kappa * hh)
    return np.array(out)


def hop_at_sites(u, psi_half, in_parity, phases, half_indices, dagger=False):
    """(P_{1-p} H P_p psi)(site) at listed half indices of the output parity."""
    lt, lz, ly, lxh = psi_half.shape[:4]
    dims = (2 * lxh, ly, lz, lt)
    get = _half_getter(psi_half, in_parity, dims)
    out = []
    for ih in half_indices:
        site = half_index_coords(dims, 1 - in_parity, int(ih))
        out.append(hop_at_site(u, get, site, phases, dims, dagger))
    return np.array(out)
