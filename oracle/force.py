"""Derivatives of the even-odd Wilson operator (oracle).

Convention: for a real function L of complex fields the gradient g of a
field z is defined by dL = Re sum conj(g) dz (torch's convention for complex
tensors: L = |z|^2 gives g = 2 z).  For links, g_U is that gradient with every
matrix entry taken as free, and the su(3) force along the left-multiplied
variation U -> exp(i eps X) U (X traceless Hermitian) is

    dL/d eps |_0 = tr(X F),   F = TH(i U g_U^dag),
    TH(Y) = (Y + Y^dag)/2 - tr((Y + Y^dag)/2)/3.

L1 = Re <eta, M psi> with M = 1 - kappa^2 H_eo H_oe (paper Eq. (4), Sec. 2).
Its variation under a change of links is -kappa^2 Re <Lambda, dH R> on the
full lattice, where Lambda = (eta_e, H_eo^dag eta_e) and R = (psi_e,
H_oe psi_e) (even part, odd part).  The link U_mu(x) enters H twice: in the
forward term at x (projector 1 - gamma_mu, phase b) and in the backward term at
x + mu (projector 1 + gamma_mu, phase conj(b)), where b is the boundary phase
of that link (phases[mu] when x_mu = L_mu - 1, else 1).  Collecting the
coefficients of dU gives

    g_U = -kappa^2 conj(b) [ sum_s w_s v_s^dag + sum_s v'_s w'_s^dag ],
    w = (1 - gamma_mu) Lambda(x), v = R(x + mu), v' = R(x),
    w' = (1 + gamma_mu) Lambda(x + mu),

with the outer products over colour and the sums over spin.

L2 = <phi, (M^dag M)^-1 phi> (the pseudofermion action behind the
determinant of paper Sec. 2): with chi = (M^dag M)^-1 phi, g_phi = 2 chi and
dL2 = -2 Re <M chi, dM chi>, so the link gradient is -2 times that of L1 with
eta = M chi and psi = chi.
"""
import numpy as np

from .gamma import proj_minus, proj_plus
from .lattice import half_to_full
from .wilson import apply_m, hop_eo


def grad_psi_l1(u, eta_e, kappa, phases):
    """dL1/dpsi for L1 = Re<eta, M psi>: g = M^dag eta."""
    return apply_m(u, eta_e, kappa, phases, dagger=True)


def grad_eta_l1(u, psi_e, kappa, phases):
    """dL1/deta: g = M psi."""
    return apply_m(u, psi_e, kappa, phases)


def boundary_factor(dims, mu, phase):
    """b_mu(x) on the full lattice: phase where x_mu = L_mu - 1, else 1."""
    lx, ly, lz, lt = dims
    b = np.ones((lt, lz, ly, lx), dtype=np.complex128)
    s = [slice(None)] * 4
    s[3 - mu] = dims[mu] - 1
    b[tuple(s)] = phase
    return b


def link_grad_bilinear(u, lam_full, r_full, coeff, phases):
    """g_U of coeff * Re <Lambda, H R> with respect to the links."""
    lt, lz, ly, lx = u.shape[1:5]
    dims = (lx, ly, lz, lt)
    g = np.zeros_like(u)
    for mu in range(4):
        ax = 3 - mu
        b = boundary_factor(dims, mu, phases[mu])
        w = np.einsum("st,...ta->...sa", proj_minus(mu), lam_full)
        v = np.roll(r_full, -1, axis=ax)                    # R(x + mu)
        vp = r_full                                          # R(x)
        wp = np.roll(np.einsum("st,...ta->...sa", proj_plus(mu), lam_full),
                     -1, axis=ax)                            # (1+g)Lambda(x+mu)
        outer = (np.einsum("...sa,...sb->...ab", w, np.conj(v))
                 + np.einsum("...sa,...sb->...ab", vp, np.conj(wp)))
        g[mu] = coeff * np.conj(b)[..., None, None] * outer
    return g


def link_grad_l1(u, psi_e, eta_e, kappa, phases):
    """g_U for L1 = Re<eta, M psi> (even-sublattice M)."""
    lt, lz, ly, lx = u.shape[1:5]
    dims = (lx, ly, lz, lt)
    lam_o = hop_eo(u, eta_e, 0, phases, dagger=True)       # H_eo^dag eta_e
    r_o = hop_eo(u, psi_e, 0, phases)                        # H_oe psi_e
    lam = half_to_full(eta_e, 0, dims) + half_to_full(lam_o, 1, dims)
    r = half_to_full(psi_e, 0, dims) + half_to_full(r_o, 1, dims)
    return link_grad_bilinear(u, lam, r, -kappa * kappa, phases)


def traceless_hermitian(y):
    h = 0.5 * (y + np.conj(np.swapaxes(y, -1, -2)))
    tr = np.trace(h, axis1=-2, axis2=-1) / 3.0
    return h - tr[..., None, None] * np.eye(3)


def force_from_grad(u, g):
    """F = TH(i U g^dag): the su(3) force of a link gradient."""
    return traceless_hermitian(1j * u @ np.conj(np.swapaxes(g, -1, -2)))


def link_force_l1(u, psi_e, eta_e, kappa, phases):
    return force_from_grad(u, link_grad_l1(u, psi_e, eta_e, kappa, phases))


def l2_value(phi_e, chi_e):
    """L2 = <phi, chi> with chi = (M^dag M)^-1 phi (real for exact chi)."""
    return float(np.vdot(phi_e.reshape(-1), chi_e.reshape(-1)).real)


def link_grad_l2(u, chi_e, kappa, phases):
    """g_U for L2 given chi = (M^dag M)^-1 phi."""
    m_chi = apply_m(u, chi_e, kappa, phases)
    return -2.0 * link_grad_l1(u, chi_e, m_chi, kappa, phases)


def grad_phi_l2(chi_e):
    return 2.0 * chi_e
