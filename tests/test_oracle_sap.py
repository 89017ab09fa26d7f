"""Pins of the oracle's Schwarz alternating procedure and flexible GCR
(``oracle/sap.py``) against what the mathematics fixes: one block spanning
the lattice with exact block solves is the exact inverse; a colour sweep with
exact block solves leaves no residual on that colour's blocks (checked with
the full Wilson matrix, which knows nothing of blocks); many MR steps reach
the exact block solution and each block keeps its own scalars; SAP cycles
converge to the dense solution; GCR without preconditioning attains the
minimal residual over the Krylov space (a dense least-squares problem), and
GCR-SAP, with and without restarts, reaches the dense solution."""
import numpy as np
import pytest

from oracle import sap as SAP
from oracle import wilson as W
from paper_2303_08609_amd import inputs

AP = np.array([1, 1, 1, -1], dtype=np.complex128)


def _setup(dims, seed, eps=0.5):
    u = inputs.gen_gauge(dims, eps, seed)
    eta = inputs.gen_spinor_full(dims, seed + 1)
    return u, eta


def _dense_solve(u, eta, kappa, ph):
    d = np.eye(eta.size) - kappa * W.dense_hop(u, ph)
    return np.linalg.solve(d, eta.reshape(-1)).reshape(eta.shape)


def test_block_layout():
    assert SAP.check_blocks((8, 4, 4, 8), (4, 2, 4, 2)) == (2, 2, 1, 4)
    with pytest.raises(ValueError):
        SAP.check_blocks((6, 4, 4, 4), (2, 2, 2, 2))          # 3 blocks along x
    with pytest.raises(ValueError):
        SAP.check_blocks((8, 4, 4, 4), (3, 2, 2, 2))
    bid, col = SAP.block_ids((4, 4, 2, 2), (2, 2, 2, 2))
    assert bid.max() == 3 and col[0, 0, 0, 0] == 0 and col[0, 0, 0, 2] == 1 and col[0, 0, 2, 2] == 0
    # neighbouring blocks always differ in colour (across the wrap too)
    for ax in range(4):
        diff = bid != np.roll(bid, 1, axis=ax)
        assert np.all(col[diff] != np.roll(col, 1, axis=ax)[diff])


@pytest.mark.parametrize("dims", [(2, 2, 2, 4), (4, 2, 2, 4)])
def test_one_block_over_the_lattice_is_the_exact_inverse(dims):
    kappa = 0.124
    ph = np.exp(1j * np.array([0.3, -0.8, 1.1, np.pi]))
    u, eta = _setup(dims, 10)
    got = SAP.sap(u, eta, kappa, ph, dims, ncy=1, nmr=None)
    assert np.abs(got - _dense_solve(u, eta, kappa, ph)).max() < 1e-12 * np.abs(got).max()
    # and the block operator is then D_W itself (hops across the edge kept)
    psi = inputs.gen_spinor_full(dims, 12)
    assert np.abs(SAP.d_blocks(u, psi, kappa, ph, dims) - W.dirac_wilson(u, psi, kappa, ph)).max() < 1e-14


def test_block_matrix_is_the_masked_dense_hop():
    """D_blk built from ``hop_blocks`` equals 1 - kappa H with H from the
    dense component formula of Eq. (1) and every entry between sites of
    different blocks removed (an independent route)."""
    dims, bsize, kappa = (4, 2, 2, 4), (2, 2, 2, 2), 0.125
    ph = np.exp(1j * np.array([0.3, -0.8, 1.1, 2.9]))
    u, eta = _setup(dims, 15)
    dblk = SAP.block_matrix(u, kappa, ph, bsize, eta.shape)
    bid, _ = SAP.block_ids(dims, bsize)
    site_block = np.repeat(bid.reshape(-1), 12)
    same = site_block[:, None] == site_block[None, :]
    want = np.eye(eta.size) - kappa * W.dense_hop(u, ph) * same
    assert np.abs(dblk - want).max() < 1e-14


def test_colour_sweep_leaves_no_residual_on_its_blocks():
    dims, bsize, kappa = (4, 4, 2, 4), (2, 2, 2, 2), 0.125
    u, eta = _setup(dims, 20)
    _, col = SAP.block_ids(dims, bsize)
    dblk = SAP.block_matrix(u, kappa, AP, bsize, eta.shape)
    for c in (0, 1):
        e = SAP.block_exact(u, eta, kappa, AP, bsize, c, dblk)
        assert np.all(e[col != c] == 0)
        rho = eta - W.dirac_wilson(u, e, kappa, AP)
        assert np.abs(rho[col == c]).max() < 1e-12
        # the other colour's blocks feel only the hops out of the solved blocks
        assert np.abs(rho[col != c] - eta[col != c]).max() > 1e-3


def test_block_mr_reaches_the_exact_block_solution():
    dims, bsize, kappa = (4, 4, 2, 4), (2, 2, 2, 2), 0.125
    u, rho = _setup(dims, 30)
    dblk = SAP.block_matrix(u, kappa, AP, bsize, rho.shape)
    for c in (0, 1):
        e, r = SAP.block_mr(u, rho, kappa, AP, bsize, c, 80)
        ex = SAP.block_exact(u, rho, kappa, AP, bsize, c, dblk)
        assert np.abs(e - ex).max() < 1e-10 * np.abs(ex).max()
        # the MR recurrence carries the block residual rho_L - D_L e_L
        _, col = SAP.block_ids(dims, bsize)
        on = (col == c)[..., None, None]
        want = np.where(on, rho - SAP.d_blocks(u, e, kappa, AP, bsize), 0)
        assert np.abs(r - want).max() < 1e-12


def test_block_mr_scalars_are_per_block():
    """MR on all blocks of a colour together equals MR on each block alone
    (a residual 1000x larger on one block does not change the others)."""
    dims, bsize, kappa = (4, 4, 2, 2), (2, 2, 2, 2), 0.125
    u, rho = _setup(dims, 40)
    bid, col = SAP.block_ids(dims, bsize)
    rho = np.where((bid == 0)[..., None, None], 1e3 * rho, rho)
    e, _ = SAP.block_mr(u, rho, kappa, AP, bsize, 0, 3)
    tot = np.zeros_like(e)
    for b in np.unique(bid[col == 0]):
        only = np.where((bid == b)[..., None, None], rho, 0)
        eb, _ = SAP.block_mr(u, only, kappa, AP, bsize, 0, 3)
        tot += eb
    assert np.abs(e - tot).max() < 1e-12 * np.abs(e).max()


def test_sap_cycles_converge_to_the_dense_solution():
    dims, bsize, kappa = (4, 4, 2, 4), (2, 2, 2, 2), 0.124
    u, eta = _setup(dims, 50)
    x = _dense_solve(u, eta, kappa, AP)
    dblk = SAP.block_matrix(u, kappa, AP, bsize, eta.shape)
    errs = [np.linalg.norm(SAP.sap(u, eta, kappa, AP, bsize, ncy=k, nmr=None, dblk=dblk) - x) / np.linalg.norm(x)
            for k in (1, 2, 4)]
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 0.01
    # MR block solves approximate the exact ones
    e_mr = np.linalg.norm(SAP.sap(u, eta, kappa, AP, bsize, ncy=4, nmr=6) - x) / np.linalg.norm(x)
    assert e_mr < 0.05


def test_gcr_unpreconditioned_attains_the_minimal_residual():
    dims, kappa = (2, 2, 2, 4), 0.124
    u, b = _setup(dims, 60)
    d = np.eye(b.size) - kappa * W.dense_hop(u, AP)
    apply_d = lambda v: (d @ v.reshape(-1)).reshape(v.shape)
    bv = b.reshape(-1)
    kry = [bv]
    for k in range(1, 6):
        x, it, hist = SAP.fgcr(apply_d, lambda r: r, b, 0.0, k, nkv=8)
        assert it == k
        basis = np.array(kry).T
        y, *_ = np.linalg.lstsq(d @ basis, bv, rcond=None)
        rmin = np.linalg.norm(bv - d @ basis @ y) / np.linalg.norm(bv)
        assert abs(hist[-1] - rmin) < 1e-12, (k, hist[-1], rmin)
        assert np.linalg.norm(bv - d @ x.reshape(-1)) / np.linalg.norm(bv) == pytest.approx(rmin, abs=1e-12)
        kry.append(d @ kry[-1])


@pytest.mark.parametrize("nkv", [2, 8])
def test_gcr_sap_reaches_the_dense_solution(nkv):
    dims, bsize, kappa = (4, 4, 4, 4), (2, 2, 2, 2), 0.124
    u, b = _setup(dims, 70)
    apply_d = lambda v: W.dirac_wilson(u, v, kappa, AP)
    pre = lambda r: SAP.sap(u, r, kappa, AP, bsize, ncy=2, nmr=4)
    x, it, hist = SAP.fgcr(apply_d, pre, b, 1e-12, 200, nkv)
    assert hist[-1] <= 1e-12
    xd = _dense_solve(u, b, kappa, AP)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-10
    # the preconditioner pays: plain GCR needs more iterations
    _, it0, _ = SAP.fgcr(apply_d, lambda r: r, b, 1e-12, 400, nkv)
    assert it < it0
