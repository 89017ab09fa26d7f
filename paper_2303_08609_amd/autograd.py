"""torch.autograd Functions over the C ABI.

Gradients follow torch's convention for complex tensors: for a real loss L,
the gradient g of z satisfies dL = Re sum conj(g) dz.

* ``wilson_apply(U, psi, lat)`` returns M psi (even sublattice).  Backward:
  g_psi = M^dag g_out = gamma5 M gamma5 g_out (one adjoint apply) and
  g_U from the link-gradient kernel with Lambda = (g_out, H_eo^dag g_out),
  R = (psi, H_oe psi) and coefficient -kappa^2.
* ``wilson_solve(U, phi, lat)`` returns chi = (M^dag M)^-1 phi (with
  mixed = True by FP64 defect correction around FP32 inner solves, also for
  complex64 fields).  Backward:
  lambda = (M^dag M)^-1 g_chi (adjoint solve through the same CG), g_phi =
  lambda, and g_U = g[Re<-M lambda, M chi>] + g[Re<-M chi, M lambda>], each
  term a link-gradient kernel call.
* ``link_force_l1(U, psi, eta, lat)`` is the su(3) force TH(i U g_U^dag) of
  Re<eta, M psi>, projected inside the kernel.

Fields are canonical complex tensors on the GPU: links [4][Lt][Lz][Ly][Lx][3][3],
one-parity spinors [Lt][Lz][Ly][Lx/2][4][3].  complex128 computes in FP64,
complex64 in FP32 (18-real links).
"""
from __future__ import annotations

import warnings

import torch

from . import wilson_eo as W
from .ops import Format, Lattice, _ptr, _stream
from .solve import cg


def _fmt_for(t: torch.Tensor) -> Format:
    if t.dtype == torch.complex128:
        return Format("f64", "f64", 18)
    if t.dtype == torch.complex64:
        return Format("f32", "f32", 18)
    raise TypeError(f"expected complex128 or complex64, got {t.dtype}")


def _canon_prec(t):
    return W.WEO_F64 if t.dtype == torch.complex128 else W.WEO_F32


def _link_grad_into(lat, fmt, u_packed, eta_p, psi_p, coeff, out, accumulate, project=False):
    """out (+)= link gradient of coeff * Re<Lambda, H R> with
    Lambda = (eta, H_eo^dag eta), R = (psi, H_oe psi); with project, the
    su(3) force TH(i U g^dag) instead."""
    lam_o = lat.hop(u_packed, eta_p, fmt, out_parity=1, dagger=True)
    r_o = lat.hop(u_packed, psi_p, fmt, out_parity=1, dagger=False)
    flags = (W.WEO_FORCE_ACCUMULATE if accumulate else 0) | (W.WEO_FORCE_PROJECT if project else 0)
    W.check(W.wilson_eo_force(lat.c, fmt.c, _ptr(u_packed), _ptr(eta_p), _ptr(lam_o), _ptr(psi_p),
                              _ptr(r_o), float(coeff), flags, _ptr(out), _canon_prec(out),
                              _stream()), "wilson_eo_force")


class WilsonApply(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u, psi, lat: Lattice, dagger: bool = False):
        fmt = _fmt_for(psi)
        u_p = lat.pack_gauge(u.contiguous(), fmt)
        x_p = lat.pack_spinor(psi.contiguous(), fmt)
        out_p = lat.apply(u_p, x_p, fmt, dagger=dagger)
        ctx.save_for_backward(u, psi)
        ctx.lat, ctx.fmt, ctx.dagger = lat, fmt, dagger
        return lat.unpack_spinor(out_p, fmt, dtype=psi.dtype)

    @staticmethod
    def backward(ctx, g_out):
        u, psi = ctx.saved_tensors
        lat, fmt, dagger = ctx.lat, ctx.fmt, ctx.dagger
        g_out = g_out.contiguous()
        u_p = lat.pack_gauge(u.contiguous(), fmt)
        g_p = lat.pack_spinor(g_out, fmt)
        g_u = g_psi = None
        if ctx.needs_input_grad[1]:
            g_psi = lat.unpack_spinor(lat.apply(u_p, g_p, fmt, dagger=not dagger), fmt,
                                      dtype=psi.dtype)
        if ctx.needs_input_grad[0]:
            if dagger:
                raise NotImplementedError("link gradient of M^dag is not provided")
            x_p = lat.pack_spinor(psi.contiguous(), fmt)
            g_u = torch.empty(lat.gauge_shape(), dtype=u.dtype, device=u.device)
            _link_grad_into(lat, fmt, u_p, g_p, x_p, -lat.kappa ** 2, g_u, False)
        return g_u, g_psi, None, None


class WilsonSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u, phi, lat: Lattice, tol: float = 1e-12, mixed: bool = False):
        fmt = _fmt_for(phi)
        chi, info = _solve_canon(lat, u, phi, tol, mixed)
        ctx.save_for_backward(u, chi)
        ctx.lat, ctx.fmt, ctx.tol, ctx.mixed = lat, fmt, tol, mixed
        ctx.info = info
        return chi

    @staticmethod
    def backward(ctx, g_chi):
        u, chi = ctx.saved_tensors
        lat, fmt = ctx.lat, ctx.fmt
        lam, _ = _solve_canon(lat, u, g_chi.to(chi.dtype), ctx.tol, ctx.mixed)
        g_u = g_phi = None
        if ctx.needs_input_grad[1]:
            g_phi = lam
        if ctx.needs_input_grad[0]:
            u_p = lat.pack_gauge(u.contiguous(), fmt)
            lam_p = lat.pack_spinor(lam, fmt)
            chi_p = lat.pack_spinor(chi.contiguous(), fmt)
            m_lam = lat.apply(u_p, lam_p, fmt)
            m_chi = lat.apply(u_p, chi_p, fmt)
            g_u = torch.empty(lat.gauge_shape(), dtype=u.dtype, device=u.device)
            # dL = -Re<M lam, dM chi> - Re<M chi, dM lam> with dM = -kappa^2 d(H_eo H_oe):
            # two bilinear terms, each with coefficient +kappa^2
            _link_grad_into(lat, fmt, u_p, m_lam, chi_p, lat.kappa ** 2, g_u, False)
            _link_grad_into(lat, fmt, u_p, m_chi, lam_p, lat.kappa ** 2, g_u, True)
        return g_u, g_phi, None, None, None


def _solve_canon(lat, u, b, tol, mixed, maxiter=100000):
    """chi = (M^dag M)^-1 b for canonical fields; chi has b's dtype.
    mixed = False: CG in the fields' own precision.  mixed = True: FP64 defect
    correction around FP32 inner solves, whatever the fields' precision (FP32
    fields are widened exactly), so that FP32 gradients rest on a solve
    accurate to tol.  Raises WilsonEOError unless the solve reports WEO_OK: an
    unconverged forward or adjoint solve would otherwise turn into silently
    wrong values and gradients."""
    fmt = Format("f64", "f64", 18) if mixed else _fmt_for(b)
    u_p = lat.pack_gauge(u.contiguous(), fmt)
    b_p = lat.pack_spinor(b.contiguous(), fmt)
    x_p, info = _solve_normal(lat, fmt, u, u_p, b_p, tol, mixed, maxiter)
    return lat.unpack_spinor(x_p, fmt, dtype=b.dtype), info


def _solve_normal(lat, fmt, u_canon, u_p, b_p, tol, mixed, maxiter=100000):
    """Packed chi = (M^dag M)^-1 b in format fmt (FP64 defect correction
    around FP32 inner solves when mixed and fmt is FP64).  Raises
    WilsonEOError unless the solve reports WEO_OK."""
    with warnings.catch_warnings():
        warnings.simplefilter("ignore", W.SolverWarning)
        if mixed and fmt.spinor == "f64":
            inner = Format("f32", "f32", 18)
            u_in = lat.pack_gauge(u_canon.contiguous(), inner)
            x, info = cg(lat, fmt, u_p, b_p, op="MdagM", tol=tol, inner=inner, u_inner=u_in,
                         inner_tol=1e-5, maxiter=maxiter)
        else:
            x, info = cg(lat, fmt, u_p, b_p, op="MdagM", tol=tol, maxiter=maxiter)
    if info["status"] != W.WEO_OK:
        raise W.WilsonEOError(info["status"], f"wilson_solve (true residual {info['true_rel_resid'][0]:.3e}, "
                                              f"tolerance {tol:.1e})")
    return x, info


def wilson_apply(u, psi, lat: Lattice, dagger=False):
    return WilsonApply.apply(u, psi, lat, dagger)


def wilson_solve(u, phi, lat: Lattice, tol=1e-12, mixed=False):
    return WilsonSolve.apply(u, phi, lat, tol, mixed)


def link_force_l1(u, psi, eta, lat: Lattice):
    """su(3) force of L1 = Re<eta, M psi>: F_mu(x) = TH(i U g_U^dag), so that
    dL1/d eps = tr(X F) for U_mu(x) -> exp(i eps X) U_mu(x)."""
    fmt = _fmt_for(psi)
    u_p = lat.pack_gauge(u.contiguous(), fmt)
    x_p = lat.pack_spinor(psi.contiguous(), fmt)
    e_p = lat.pack_spinor(eta.contiguous(), fmt)
    f = torch.empty(lat.gauge_shape(), dtype=u.dtype, device=u.device)
    _link_grad_into(lat, fmt, u_p, e_p, x_p, -lat.kappa ** 2, f, False, project=True)
    return f
