"""Pins of the oracle's clover-type operator (site-local D_ee, D_oo, Sec. 2):
the chiral-block convention against gamma5, the spectrum of the site matrix,
the even-odd Schur complement (Eqs. (3)-(5)) against dense solves and
determinants, the reduction to the Wilson operator for scalar blocks, the
adjoint, and gamma5-hermiticity of the full matrix."""
import numpy as np
import pytest

from oracle import clover as CL
from oracle import wilson as W
from oracle.gamma import GAMMA5
from oracle.lattice import full_to_half, half_to_full
from paper_2303_08609_amd import inputs

PH = np.array([1, 1, 1, -1], dtype=np.complex128)
G5 = np.kron(GAMMA5, np.eye(3))


def _match(a, b):
    a = np.sort_complex(np.round(a, 9))
    b = np.sort_complex(np.round(b, 9))
    return np.abs(a - b).max()


def test_blocks_commute_with_gamma5_and_keep_spectrum():
    blocks = inputs.gen_site_blocks((2, 2, 2, 2), 0.4, 11)[0, 0, 0, 0]
    a = CL.blocks_to_dirac(blocks)
    assert np.abs(a @ G5 - G5 @ a).max() < 1e-14
    assert np.abs(a - np.conj(a.T)).max() < 1e-14             # Hermitian blocks -> Hermitian A
    ev = np.linalg.eigvalsh(a)
    want = np.concatenate([np.linalg.eigvalsh(blocks[0]), np.linalg.eigvalsh(blocks[1])])
    assert np.abs(np.sort(ev) - np.sort(want)).max() < 1e-13
    # block 0 acts on gamma5 = -1, block 1 on gamma5 = +1
    b = np.zeros((2, 6, 6), dtype=complex)
    b[0] = np.eye(6)
    a0 = CL.blocks_to_dirac(b)
    assert np.abs(a0 - 0.5 * (np.eye(12) - G5)).max() < 1e-15
    assert np.abs(CL.blocks_to_dirac(np.stack([np.eye(6)] * 2)) - np.eye(12)).max() < 1e-15


def test_scalar_blocks_reduce_to_wilson():
    dims = (4, 2, 2, 4)
    u = inputs.gen_gauge(dims, 0.5, 21)
    psi = inputs.gen_spinor_half(dims, 22)
    a = 1.3
    ainv = np.broadcast_to(np.eye(12) / a, psi.shape[:4] + (12, 12))
    for dag in (False, True):
        got = CL.apply_m_clover(u, psi, 0.13, PH, ainv, ainv, dagger=dag)
        want = W.apply_m(u, psi, 0.13 / a, PH, dagger=dag)
        assert np.abs(got - want).max() < 1e-13


def _setup(dims, kappa=0.13, eps=0.3, seed=31):
    u = inputs.gen_gauge(dims, 0.5, seed)
    blocks = inputs.gen_site_blocks(dims, eps, seed + 1)
    a_full = CL.blocks_to_dirac(blocks)
    ainv_full = np.linalg.inv(a_full)
    return u, a_full, ainv_full


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 2, 2, 4)])
def test_schur_complement_with_site_blocks(dims):
    kappa = 0.13
    u, a_full, ainv_full = _setup(dims, kappa)
    d = CL.dense_sites(a_full) - kappa * W.dense_hop(u, PH)
    re, ro = W.dense_parity_rows(dims, 0), W.dense_parity_rows(dims, 1)
    ai_e, ai_o = full_to_half(ainv_full, 0), full_to_half(ainv_full, 1)
    # dense M from the oracle's apply, column by column
    shape = full_to_half(np.zeros((dims[3], dims[2], dims[1], dims[0], 4, 3)), 0).shape
    n = 12 * int(np.prod(shape[:4]))
    m = np.array([CL.apply_m_clover(u, np.eye(1, n, j).reshape(shape), kappa, PH, ai_e, ai_o).reshape(-1)
                  for j in range(n)]).T
    # det D = det A_ee det A_oo det M  (block LDU of Eq. (3))
    s_d, l_d = np.linalg.slogdet(d)
    s_ae, l_ae = np.linalg.slogdet(d[np.ix_(re, re)])
    s_ao, l_ao = np.linalg.slogdet(d[np.ix_(ro, ro)])
    s_m, l_m = np.linalg.slogdet(m)
    assert abs(l_d - (l_ae + l_ao + l_m)) < 1e-9
    assert abs(s_d - s_ae * s_ao * s_m) < 1e-9
    # D xi = eta through Eq. (4) and Eq. (5)
    eta = inputs.gen_spinor_full(dims, 33)
    xi = np.linalg.solve(d, eta.reshape(-1)).reshape(eta.shape)
    eta_e, eta_o = full_to_half(eta, 0), full_to_half(eta, 1)
    b_e = CL.apply_sites(ai_e, eta_e + kappa * W.hop_eo(u, CL.apply_sites(ai_o, eta_o), 1, PH))
    xi_e = np.linalg.solve(m, b_e.reshape(-1)).reshape(b_e.shape)
    xi_o = CL.apply_sites(ai_o, eta_o + kappa * W.hop_eo(u, xi_e, 0, PH))
    assert np.abs(xi_e - full_to_half(xi, 0)).max() < 1e-11
    assert np.abs(xi_o - full_to_half(xi, 1)).max() < 1e-11


def test_adjoint_and_gamma5_hermiticity():
    dims = (4, 2, 2, 4)
    kappa = 0.13
    u, a_full, ainv_full = _setup(dims, kappa)
    ai_e, ai_o = full_to_half(ainv_full, 0), full_to_half(ainv_full, 1)
    psi = inputs.gen_spinor_half(dims, 41)
    chi = inputs.gen_spinor_half(dims, 42)
    lhs = np.vdot(chi, CL.apply_m_clover(u, psi, kappa, PH, ai_e, ai_o))
    rhs = np.vdot(CL.apply_m_clover(u, chi, kappa, PH, ai_e, ai_o, dagger=True), psi)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    d = CL.dense_sites(a_full) - kappa * W.dense_hop(u, PH)
    g5 = np.kron(np.eye(d.shape[0] // 12), G5)
    assert np.abs(g5 @ d @ g5 - np.conj(d.T)).max() < 1e-13


def test_site_evaluation_matches_full_lattice():
    """apply_m_clover_at_sites (used for sampled checks on big lattices)
    equals the full-lattice routine at every listed site, with complex
    phases, for M and M^dag."""
    dims = (4, 6, 2, 8)
    u = inputs.gen_gauge(dims, 0.5, 61)
    blocks = inputs.gen_site_blocks(dims, 0.3, 62)
    psi = inputs.gen_spinor_half(dims, 63)
    ph = np.exp(1j * np.array([0.3, -0.9, 1.7, 2.6]))
    a = CL.blocks_to_dirac(blocks)
    ainv = np.linalg.inv(a)
    ai_e, ai_o = full_to_half(ainv, 0), full_to_half(ainv, 1)
    vh = 4 * 6 * 2 * 8 // 2
    idx = [0, 1, 7, vh // 3, vh - 1]
    at = lambda x, y, z, t: ainv[t, z, y, x]
    for dag in (False, True):
        full = CL.apply_m_clover(u, psi, 0.126, ph, ai_e, ai_o, dagger=dag).reshape(vh, 4, 3)
        got = CL.apply_m_clover_at_sites(u, psi, 0.126, ph, at, idx, dagger=dag)
        assert np.abs(got - full[idx]).max() < 1e-13, dag
