"""Textbook FP64 solvers for the even-odd system (oracle).

The paper (Sec. 2) only says that iterative Krylov solvers are used and that
their cost is dominated by multiplications by the fermion matrix; it names no
algorithm.  The oracle uses the standard ones:

* CGLS (conjugate gradients on the normal equations M^dag M x = M^dag b,
  carrying the residual s = b - M x of the original system) to solve M x = b;
* CG on the Hermitian positive definite operator A = M^dag M to solve A x = b;
* BiCGStab (van der Vorst, SIAM J. Sci. Stat. Comput. 13 (1992) 631) on M
  itself, for non-Hermitian M;
* block CG for several right-hand sides at once (O'Leary, Linear Algebra
  Appl. 29 (1980) 293) in the QR-retooled form of Dubrulle (Electron. Trans.
  Numer. Anal. 12 (2001) 216), on A = M^dag M directly or, for M x = b, on the
  normal equations while carrying S = B - M X;
* defect correction (iterative refinement): x += solve(b - M x) with the inner
  solve run to a loose relative tolerance;
* dense ``numpy.linalg.solve`` on tiny lattices.

Each solver takes the operators as callables on one-parity arrays.  Residuals
are ||b - M x||_2 / ||b||_2 recomputed from scratch at the end.
"""
import numpy as np


def vdot(a, b):
    return np.vdot(a.reshape(-1), b.reshape(-1))


def norm2(a):
    return float(np.vdot(a.reshape(-1), a.reshape(-1)).real)


def rel_resid(apply_op, x, b):
    r = b - apply_op(x)
    return np.sqrt(norm2(r) / norm2(b))


def cgls(apply_m, apply_mdag, b, tol, maxiter, x0=None):
    """Solve M x = b by CG on M^dag M x = M^dag b.

    Stops when the recursive residual ||s|| <= tol * ||b|| (s = b - M x).
    Returns (x, iterations, history of ||s||/||b||).
    """
    x = np.zeros_like(b) if x0 is None else x0.copy()
    s = b - apply_m(x) if x0 is not None else b.copy()
    r = apply_mdag(s)
    p = r.copy()
    gamma = norm2(r)
    bnorm = np.sqrt(norm2(b))
    hist = [np.sqrt(norm2(s)) / bnorm]
    it = 0
    while hist[-1] > tol and it < maxiter:
        q = apply_m(p)
        alpha = gamma / norm2(q)
        x = x + alpha * p
        s = s - alpha * q
        r = apply_mdag(s)
        gamma_new = norm2(r)
        beta = gamma_new / gamma
        gamma = gamma_new
        p = r + beta * p
        it += 1
        hist.append(np.sqrt(norm2(s)) / bnorm)
    return x, it, hist


def cg(apply_a, b, tol, maxiter, x0=None):
    """Solve A x = b for Hermitian positive definite A by plain CG."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - apply_a(x) if x0 is not None else b.copy()
    p = r.copy()
    rr = norm2(r)
    bnorm = np.sqrt(norm2(b))
    hist = [np.sqrt(rr) / bnorm]
    it = 0
    while hist[-1] > tol and it < maxiter:
        q = apply_a(p)
        alpha = rr / float(vdot(p, q).real)
        x = x + alpha * p
        r = r - alpha * q
        rr_new = norm2(r)
        beta = rr_new / rr
        rr = rr_new
        p = r + beta * p
        it += 1
        hist.append(np.sqrt(rr) / bnorm)
    return x, it, hist


def bicgstab(apply_a, b, tol, maxiter, x0=None):
    """Solve A x = b for a general (non-Hermitian) A by BiCGStab.

    Shadow residual r^ = r_0; per iteration two products with A:
      rho = <r^, r>;  beta = (rho / rho_prev) (alpha / omega)
      p = r + beta (p - omega v);  v = A p;  alpha = rho / <r^, v>
      s = r - alpha v;  t = A s;  omega = <t, s> / <t, t>
      x += alpha p + omega s;  r = s - omega t
    Stops when the recursive residual ||r|| <= tol ||b||.  Returns (x,
    iterations, history of ||r||/||b||).
    """
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - apply_a(x) if x0 is not None else b.copy()
    rh = r.copy()
    bnorm = np.sqrt(norm2(b))
    hist = [np.sqrt(norm2(r)) / bnorm]
    rho_prev = alpha = omega = 1.0
    v = np.zeros_like(b)
    p = np.zeros_like(b)
    it = 0
    while hist[-1] > tol and it < maxiter:
        rho = vdot(rh, r)
        beta = (rho / rho_prev) * (alpha / omega)
        p = r + beta * (p - omega * v)
        v = apply_a(p)
        alpha = rho / vdot(rh, v)
        s = r - alpha * v
        t = apply_a(s)
        tt = norm2(t)
        omega = vdot(t, s) / tt if tt > 0 else 0.0
        x = x + alpha * p + omega * s
        r = s - omega * t
        rho_prev = rho
        it += 1
        hist.append(np.sqrt(norm2(r)) / bnorm)
    return x, it, hist


RANK_EPS = 64 * 2.0 ** -53


def _block_qr(z, rank_eps=RANK_EPS):
    """Thin QR of the n x s block z with deflation: z = Q psi, Q (n x r)
    orthonormal over the columns that are independent, psi (r x s) the
    coefficients of every column of z in that basis.  The columns are taken
    in order; column j is dropped when the part of it orthogonal to the
    columns kept before it has squared norm <= rank_eps ||z_j||^2 (it is
    then, to that accuracy, a combination of them).  Q is the Householder QR
    of the kept columns."""
    kept = []
    for j in range(z.shape[1]):
        nj = np.linalg.norm(z[:, j]) ** 2
        if kept:
            qk, _ = np.linalg.qr(z[:, kept], mode="reduced")
            perp = z[:, j] - qk @ (qk.conj().T @ z[:, j])
        else:
            perp = z[:, j]
        if np.linalg.norm(perp) ** 2 > rank_eps * nj:
            kept.append(j)
    if not kept:
        return np.zeros((z.shape[0], 0), dtype=z.dtype), np.zeros((0, z.shape[1]), dtype=z.dtype)
    q, _ = np.linalg.qr(z[:, kept], mode="reduced")
    return q, q.conj().T @ z


def block_cg(apply_a, b, tol, maxiter, apply_m=None, apply_mdag=None):
    """Block CG for s right-hand sides, Dubrulle's QR form.

    ``b`` is a list of s one-parity arrays.  Without ``apply_m`` it solves
    A X = B for Hermitian positive definite ``apply_a``.  With ``apply_m`` and
    ``apply_mdag`` it solves M X = B through A = M^dag M, M^dag B and also
    carries S = B - M X.

    The residual block of the system solved is kept as R = Q C with Q
    orthonormal (n x r) and C (r x s), r <= s the rank of the block (columns
    that become dependent are deflated by ``_block_qr``: the block shrinks
    and the dropped directions' coefficients stay in C); the search block P
    (n x r) satisfies P^H Q = I:
        start   Q C = R_0 (QR),  P = Q
        repeat  W = A P,  delta = (P^H W)^-1
                X += P delta C       (S -= (M P) delta C)
                Q' psi = Q - W delta (QR),  C = psi C
                P = Q' + P psi^H,    Q = Q'
    X_k is the Galerkin solution over the block Krylov space of R_0.  Stops
    when every column meets ||r_j|| <= tol ||b_j|| (r = S for M x = b, else
    the recurrence ||r_j|| = ||C[:, j]||).  Returns (X as a list, iterations,
    history of the largest relative residual).
    """
    shape = b[0].shape
    s = len(b)
    bm = np.stack([v.reshape(-1) for v in b], axis=1)
    bnorm = np.linalg.norm(bm, axis=0)
    normal = apply_m is not None

    def blk(f, m):
        return np.stack([f(m[:, j].reshape(shape)).reshape(-1) for j in range(m.shape[1])], axis=1)

    x = np.zeros_like(bm)
    sres = bm.copy()
    r0 = blk(apply_mdag, bm) if normal else bm.copy()
    q, c = _block_qr(r0)
    p = q.copy()

    def rel():
        res = np.linalg.norm(sres, axis=0) if normal else np.linalg.norm(c, axis=0)
        return float(np.max(res / bnorm))

    hist = [rel()]
    it = 0
    while hist[-1] > tol and it < maxiter and q.shape[1] > 0:
        if normal:
            mp = blk(apply_m, p)
            w = blk(apply_mdag, mp)
        else:
            w = blk(apply_a, p)
        delta = np.linalg.inv(p.conj().T @ w)
        x = x + p @ (delta @ c)
        if normal:
            sres = sres - mp @ (delta @ c)
        q_new, psi = _block_qr(q - w @ delta)
        c = psi @ c
        p = q_new + p @ psi.conj().T
        q = q_new
        it += 1
        hist.append(rel())
    return [x[:, j].reshape(shape) for j in range(s)], it, hist


def defect_correction(apply_m, inner_solve, b, tol, max_outer, x0=None):
    """Iterative refinement: r = b - M x; x += inner_solve(r); repeat.

    ``inner_solve(r)`` returns an approximate solution of M e = r.  Stops when
    the true relative residual is <= tol.  Returns (x, outer iterations,
    history of true relative residuals).
    """
    x = np.zeros_like(b) if x0 is None else x0.copy()
    bnorm = np.sqrt(norm2(b))
    r = b - apply_m(x)
    hist = [np.sqrt(norm2(r)) / bnorm]
    k = 0
    while hist[-1] > tol and k < max_outer:
        x = x + inner_solve(r)
        r = b - apply_m(x)
        k += 1
        hist.append(np.sqrt(norm2(r)) / bnorm)
    return x, k, hist


def dense_solve(d, rhs):
    return np.linalg.solve(d, rhs)
