"""Schwarz alternating procedure (SAP) and flexible GCR for the Wilson matrix
(oracle; test infrastructure only).

The solver library the paper builds on (QWS, Sec. 1 and Sec. 2) solves the
fermion system with a Krylov method preconditioned by the Schwarz
alternating procedure on a domain-decomposed matrix: the lattice is cut into
blocks, and the preconditioner solves the blocks' own small systems, which
need no communication.  The paper names the method and gives no details; the
definitions below follow Luescher's SAP (Comput. Phys. Commun. 156 (2004)
209; 165 (2005) 199), written out from the mathematics.

* Blocks.  Boxes of extent b = (bx, by, bz, bt), each b_mu dividing L_mu;
  n_mu = L_mu / b_mu blocks along mu, each n_mu 1 or even.  Block coordinates
  c_mu = x_mu // b_mu, colour = sum_mu c_mu mod 2: a checkerboard of blocks,
  so blocks of one colour share no face (n_mu even keeps the alternation
  across the periodic wrap).
* Block operator D_L: the Wilson matrix D_W = 1 - kappa H of Eq. (1)
  restricted to the sites of block L, every hop that leaves L dropped (zero
  Dirichlet boundary).  Where n_mu = 1 the block spans the whole direction
  and the hop across the lattice edge (with its boundary phase) stays inside.
  D_blk is the block-diagonal part of D_W (all blocks together).
* Block solve.  Either exact (a dense solve of D_L), or nmr steps of the
  minimal residual iteration on D_L started from zero, every block with its
  own scalars:  e = 0, r = rho_L;  repeat nmr times:  q = D_L r,
  alpha = <q, r> / <q, q>,  e += alpha r,  r -= alpha q.
* SAP with ncy cycles, an approximation K eta of D_W^-1 eta from psi = 0:
      rho = eta;  repeat ncy times, for colour 0 then colour 1:
          psi_L += (block solve of D_L e = rho_L) on every block L of the colour
          rho = eta - D_W psi
  (multiplicative Schwarz over the two colours).  With MR block solves K is
  not linear, hence:
* flexible GCR with restart length nkv, solving D_W x = b with right
  preconditioner K (the preconditioned directions phi_k are kept):
      r = b - D_W x
      for k = 0 .. nkv-1:
          phi_k = K r;  chi = D_W phi_k
          a_lk = <chi_l, chi> for l < k;  chi -= sum_l a_lk chi_l  (classical
          Gram-Schmidt against the normalised chi_l); a_kk = ||chi||;
          chi_k = chi / a_kk;  c_k = <chi_k, r>;  r -= c_k chi_k
          stop the cycle when ||r|| <= tol ||b||
      x += sum_k alpha_k phi_k with sum_{k >= l} a_lk alpha_k = c_l
      (then D_W sum alpha_k phi_k = sum c_l chi_l); restart from r = b - D_W x.
  GCR minimises ||r|| over the span of the chi_k.

Full-lattice spinors are [t][z][y][x][4][3] as in ``wilson``.
"""
import numpy as np

from .gamma import proj_minus, proj_plus
from .lattice import coords
from .wilson import _axis, _colour, _colour_dag, _slice_at, _spin, dirac_wilson


def check_blocks(dims, bsize):
    """Number of blocks per direction; raises for an unusable block size."""
    n = []
    for L, b in zip(dims, bsize):
        if b < 1 or L % b:
            raise ValueError(f"block extent {b} does not divide {L}")
        k = L // b
        if k != 1 and k % 2:
            raise ValueError(f"{k} blocks along a direction: must be 1 or even")
        n.append(k)
    return tuple(n)


def block_ids(dims, bsize):
    """(block id, colour) of every site, arrays [t][z][y][x]."""
    n = check_blocks(dims, bsize)
    x, y, z, t = coords(dims)
    c = [x // bsize[0], y // bsize[1], z // bsize[2], t // bsize[3]]
    bid = c[0] + n[0] * (c[1] + n[1] * (c[2] + n[2] * c[3]))
    colour = (c[0] + c[1] + c[2] + c[3]) % 2
    return bid, colour


def hop_blocks(u, psi, phases, bsize, dagger=False):
    """The block-diagonal part of the hopping term: H psi with every term
    between sites of different blocks dropped."""
    dims = (psi.shape[3], psi.shape[2], psi.shape[1], psi.shape[0])
    bid, _ = block_ids(dims, bsize)
    out = np.zeros_like(psi)
    for mu in range(4):
        ax = _axis(mu)
        length = psi.shape[ax]
        pf, pb = proj_minus(mu), proj_plus(mu)
        if dagger:
            pf, pb = pb, pf
        keep_f = (bid == np.roll(bid, -1, axis=ax))[..., None, None]
        keep_b = (bid == np.roll(bid, 1, axis=ax))[..., None, None]
        fwd = np.roll(psi, -1, axis=ax)
        fwd[_slice_at(psi.ndim, ax, length - 1)] *= phases[mu]
        out += keep_f * _spin(pf, _colour(u[mu], fwd))
        bwd = np.roll(psi, 1, axis=ax)
        bwd[_slice_at(psi.ndim, ax, 0)] *= np.conj(phases[mu])
        ub = np.roll(u[mu], 1, axis=ax)
        out += keep_b * _spin(pb, _colour_dag(ub, bwd))
    return out


def d_blocks(u, psi, kappa, phases, bsize):
    """D_blk psi = psi - kappa H_blk psi."""
    return psi - kappa * hop_blocks(u, psi, phases, bsize)


def _per_block_sum(bid, nblk, v):
    return np.bincount(bid.reshape(-1), weights=v.reshape(-1), minlength=nblk)


def block_mr(u, rho, kappa, phases, bsize, colour, nmr):
    """nmr MR steps on D_L for every block L of the given colour, from zero,
    each block with its own alpha.  rho: full-lattice residual (only the
    colour's blocks are read).  Returns (e, r): the block solutions and the
    block residuals rho_L - D_L e_L, zero outside the colour's blocks."""
    dims = (rho.shape[3], rho.shape[2], rho.shape[1], rho.shape[0])
    bid, col = block_ids(dims, bsize)
    nblk = int(bid.max()) + 1
    on = (col == colour)[..., None, None]
    r = np.where(on, rho, 0)
    e = np.zeros_like(rho)
    for _ in range(nmr):
        q = np.where(on, d_blocks(u, r, kappa, phases, bsize), 0)
        qr = np.sum(np.conj(q) * r, axis=(-2, -1))
        qq = np.sum(np.abs(q) ** 2, axis=(-2, -1))
        num = _per_block_sum(bid, nblk, qr.real) + 1j * _per_block_sum(bid, nblk, qr.imag)
        den = _per_block_sum(bid, nblk, qq)
        alpha = np.where(den > 0, num / np.where(den > 0, den, 1), 0)[bid][..., None, None]
        e = e + alpha * r
        r = r - alpha * q
    return e, r


def block_matrix(u, kappa, phases, bsize, shape):
    """Dense matrix of D_blk on full-lattice spinors of the given shape,
    built column by column from ``d_blocks`` (small lattices only)."""
    n = int(np.prod(shape))
    cols = [d_blocks(u, np.eye(1, n, j, dtype=np.complex128).reshape(shape), kappa, phases, bsize).reshape(-1)
            for j in range(n)]
    return np.array(cols).T


def block_exact(u, rho, kappa, phases, bsize, colour, dblk=None):
    """Exact block solves D_L e_L = rho_L on every block of the colour, from
    the dense D_blk (``dblk``, built here when not given)."""
    dims = (rho.shape[3], rho.shape[2], rho.shape[1], rho.shape[0])
    _, col = block_ids(dims, bsize)
    shape = rho.shape
    if dblk is None:
        dblk = block_matrix(u, kappa, phases, bsize, shape)
    sel = np.broadcast_to((col == colour)[..., None, None], shape).reshape(-1)
    e = np.zeros(rho.size, dtype=np.complex128)
    idx = np.nonzero(sel)[0]
    if idx.size:
        e[idx] = np.linalg.solve(dblk[np.ix_(idx, idx)], rho.reshape(-1)[idx])
    return e.reshape(shape)


def sap(u, eta, kappa, phases, bsize, ncy, nmr=None, dblk=None):
    """K eta: ncy SAP cycles from zero; nmr=None takes exact block solves
    (from the dense D_blk ``dblk`` if given), else nmr MR steps per block.
    Returns psi."""
    dims = (eta.shape[3], eta.shape[2], eta.shape[1], eta.shape[0])
    n = check_blocks(dims, bsize)
    colours = (0, 1) if any(k > 1 for k in n) else (0,)
    psi = np.zeros_like(eta)
    rho = eta.copy()
    for _ in range(ncy):
        for c in colours:
            if nmr is None:
                if dblk is None:
                    dblk = block_matrix(u, kappa, phases, bsize, eta.shape)
                e = block_exact(u, rho, kappa, phases, bsize, c, dblk)
            else:
                e, _ = block_mr(u, rho, kappa, phases, bsize, c, nmr)
            psi = psi + e
            rho = eta - dirac_wilson(u, psi, kappa, phases)
    return psi


def _vdot(a, b):
    return np.vdot(a.reshape(-1), b.reshape(-1))


def fgcr(apply_d, precond, b, tol, maxiter, nkv):
    """Flexible GCR with restart nkv for D x = b from x = 0, right
    preconditioner ``precond`` (any map, e.g. SAP).  Returns (x, iterations,
    history of ||r|| / ||b|| after every iteration)."""
    bnorm = np.sqrt(_vdot(b, b).real)
    x = np.zeros_like(b)
    r = b.copy()
    hist = [1.0]
    it = 0
    while hist[-1] > tol and it < maxiter:
        phis, chis = [], []
        a = np.zeros((nkv, nkv), dtype=np.complex128)
        c = np.zeros(nkv, dtype=np.complex128)
        k = 0
        while k < nkv and it < maxiter:
            phi = precond(r)
            chi = apply_d(phi)
            for l in range(k):
                a[l, k] = _vdot(chis[l], chi)
            for l in range(k):
                chi = chi - a[l, k] * chis[l]
            a[k, k] = np.sqrt(_vdot(chi, chi).real)
            chi = chi / a[k, k]
            c[k] = _vdot(chi, r)
            r = r - c[k] * chi
            phis.append(phi)
            chis.append(chi)
            k += 1
            it += 1
            hist.append(np.sqrt(_vdot(r, r).real) / bnorm)
            if hist[-1] <= tol:
                break
        alpha = np.zeros(k, dtype=np.complex128)
        for l in range(k - 1, -1, -1):
            alpha[l] = (c[l] - np.dot(a[l, l + 1:k], alpha[l + 1:k])) / a[l, l]
        for l in range(k):
            x = x + alpha[l] * phis[l]
        r = b - apply_d(x)
        hist[-1] = np.sqrt(_vdot(r, r).real) / bnorm
    return x, it, hist
