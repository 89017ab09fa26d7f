"""Derivatives on the GPU: the link-gradient kernel and the autograd Functions
against the oracle's gradients, and central finite differences (step 1e-6)
on 20 link and 20 site directions at 16^3x32 (kappa = 0.125, eps = 0.5)."""
import numpy as np
import pytest
import torch

from oracle import force as F
from oracle import wilson as W
from paper_2303_08609_amd import inputs
from paper_2303_08609_amd.autograd import link_force_l1, wilson_apply, wilson_solve
from paper_2303_08609_amd.ops import Lattice, to_device
from tests._helpers import AP, cached_gauge, rel_err

pytestmark = pytest.mark.gpu
PH = np.array(AP, dtype=np.complex128)


def _expi(x):
    w, v = np.linalg.eigh(x)
    return (v * np.exp(1j * w)) @ np.conj(v.T)


def _rand_th(g):
    a = g.standard_normal((3, 3)) + 1j * g.standard_normal((3, 3))
    x = 0.5 * (a + np.conj(a.T))
    x -= np.trace(x) / 3 * np.eye(3)
    return x / np.sqrt(np.trace(x @ x).real)


def _links(g, dims, n):
    lx, ly, lz, lt = dims
    out = [(3, lt - 1, int(g.integers(lz)), int(g.integers(ly)), int(g.integers(lx)))
           for _ in range(4)]
    while len(out) < n:
        out.append(tuple(int(v) for v in (g.integers(4), g.integers(lt), g.integers(lz),
                                          g.integers(ly), g.integers(lx))))
    return out


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64], ids=["f64", "f32"])
def test_apply_autograd_matches_oracle(dtype):
    print(f"apply autograd {dtype}", flush=True)
    dims, kappa = (4, 6, 2, 8), 0.125
    lat = Lattice(dims, kappa, AP)
    u = inputs.gen_gauge(dims, 0.5, 501)
    psi = inputs.gen_spinor_half(dims, 502)
    eta = inputs.gen_spinor_half(dims, 503)
    ut = to_device(u).to(dtype).requires_grad_(True)
    pt = to_device(psi).to(dtype).requires_grad_(True)
    et = to_device(eta).to(dtype)
    out = wilson_apply(ut, pt, lat)
    loss = (et.conj() * out).real.sum()
    loss.backward()
    tol = 1e-12 if dtype == torch.complex128 else 2e-6
    want_psi = F.grad_psi_l1(u, eta, kappa, PH)
    want_u = F.link_grad_l1(u, psi, eta, kappa, PH)
    assert rel_err(pt.grad.cpu().numpy(), want_psi) <= tol
    assert rel_err(ut.grad.cpu().numpy(), want_u) <= tol
    f = link_force_l1(ut.detach(), pt.detach(), et, lat).cpu().numpy()
    assert rel_err(f, F.link_force_l1(u, psi, eta, kappa, PH)) <= tol


def test_fp32_gradients_16_3x32_vs_fp64_oracle():
    """FP32 autograd at 16^3x32 against the FP64 oracle gradients (no finite
    differences in FP32): spinor gradient and link gradient within 1e-5."""
    print("fp32 gradients 16^3x32", flush=True)
    dims, kappa = (16, 16, 16, 32), 0.125
    lat = Lattice(dims, kappa, AP)
    u = cached_gauge(dims, 0.5, 501)
    psi = inputs.gen_spinor_half(dims, 502)
    eta = inputs.gen_spinor_half(dims, 503)
    ut = to_device(u).to(torch.complex64).requires_grad_(True)
    pt = to_device(psi).to(torch.complex64).requires_grad_(True)
    et = to_device(eta).to(torch.complex64)
    loss = (et.conj() * wilson_apply(ut, pt, lat)).real.sum()
    loss.backward()
    assert rel_err(pt.grad.cpu().numpy(), F.grad_psi_l1(u, eta, kappa, PH)) <= 1e-5
    assert rel_err(ut.grad.cpu().numpy(), F.link_grad_l1(u, psi, eta, kappa, PH)) <= 1e-5


def test_solve_autograd_matches_oracle_small():
    print("solve autograd 4x4x2x4", flush=True)
    dims, kappa = (4, 4, 2, 4), 0.125
    lat = Lattice(dims, kappa, AP)
    u = inputs.gen_gauge(dims, 0.5, 511)
    phi = inputs.gen_spinor_half(dims, 514)
    ut = to_device(u).requires_grad_(True)
    ft = to_device(phi).requires_grad_(True)
    chi = wilson_solve(ut, ft, lat, tol=1e-13)
    loss = (ft.detach().conj() * chi).real.sum()        # L2 = <phi, chi> with phi fixed
    loss.backward()
    # oracle: chi by a dense solve, gradients from the oracle formulas
    from oracle.solvers import cg as ocg
    a = lambda v: W.apply_mdagm(u, v, kappa, PH)
    chi_o, _, _ = ocg(a, phi, 1e-14, 10000)
    assert rel_err(chi.detach().cpu().numpy(), chi_o) < 1e-11
    # L = Re<phi_fixed, chi(U, phi)> equals L2 as a function of U: the link
    # gradient is the oracle's L2 gradient; g_phi = A^-1 phi = chi
    assert rel_err(ft.grad.cpu().numpy(), chi_o) < 1e-11
    want_u = F.link_grad_l2(u, chi_o, kappa, PH)
    assert rel_err(ut.grad.cpu().numpy(), want_u) < 1e-10


def test_fd_links_and_sites_16_3x32_fp64():
    """20 link directions (4 on the antiperiodic t edge) and 20 site
    directions, central differences at step 1e-6, FP64 on the GPU."""
    print("fd 16^3x32", flush=True)
    dims, kappa = (16, 16, 16, 32), 0.125
    lat = Lattice(dims, kappa, AP)
    u = cached_gauge(dims, 0.5, 501)
    psi = inputs.gen_spinor_half(dims, 502)
    eta = inputs.gen_spinor_half(dims, 503)
    ud = to_device(u)
    pt = to_device(psi)
    et = to_device(eta)

    def l1(uu, pp):
        with torch.no_grad():
            return float((et.conj() * wilson_apply(uu, pp, lat)).real.sum())

    f = link_force_l1(ud, pt, et, lat).cpu().numpy()
    # the kernel's force agrees with the oracle formula on the full lattice
    assert rel_err(f, F.link_force_l1(u, psi, eta, kappa, PH)) <= 1e-12
    g = np.random.default_rng(505)
    h = 1e-6
    for link in _links(g, dims, 20):
        x = _rand_th(g)
        up = ud.clone()
        um = ud.clone()
        up[link] = to_device(_expi(h * x) @ u[link])
        um[link] = to_device(_expi(-h * x) @ u[link])
        fd = (l1(up, pt) - l1(um, pt)) / (2 * h)
        an = np.trace(x @ f[link]).real
        assert abs(fd - an) <= 2e-6 * max(1.0, abs(an)), (link, fd, an)
    ptg = pt.clone().requires_grad_(True)
    loss = (et.conj() * wilson_apply(ud, ptg, lat)).real.sum()
    loss.backward()
    gpsi = ptg.grad.cpu().numpy()
    for _ in range(20):
        site = tuple(int(g.integers(n)) for n in psi.shape[:4])
        d = np.zeros_like(psi)
        v = g.standard_normal((4, 3)) + 1j * g.standard_normal((4, 3))
        d[site] = v / np.linalg.norm(v)
        dt = to_device(d)
        fd = (l1(ud, pt + h * dt) - l1(ud, pt - h * dt)) / (2 * h)
        an = np.vdot(gpsi, d).real
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))


def test_fd_l2_links_16_3x32_difference_form():
    """L2 = <phi, (M^dag M)^-1 phi> is ~1e6 at 16^3x32 while one link moves it
    by O(1): the central difference is taken in the difference form
    L(U+) - L(U-) = <chi+, (A- - A+) chi->, A = M^dag M, chi = A^-1 phi,
    on 20 link directions (4 of them t links across the antiperiodic edge)."""
    print("fd L2 16^3x32", flush=True)
    from paper_2303_08609_amd.ops import Format
    from paper_2303_08609_amd.solve import cg
    dims, kappa = (16, 16, 16, 32), 0.125
    lat = Lattice(dims, kappa, AP)
    f64 = Format("f64", "f64", 18)
    u = cached_gauge(dims, 0.5, 501)
    phi = inputs.gen_spinor_half(dims, 504)
    ud = to_device(u).requires_grad_(True)
    ft = to_device(phi)
    chi = wilson_solve(ud, ft, lat, tol=1e-12, mixed=True)
    loss = (ft.conj() * chi).real.sum()
    loss.backward()
    force = torch.zeros_like(ud)
    gu = ud.grad.detach()
    y = 1j * (ud.detach() @ gu.conj().transpose(-1, -2).contiguous())
    hh = 0.5 * (y + y.conj().transpose(-1, -2))
    tr = torch.diagonal(hh, dim1=-2, dim2=-1).sum(-1) / 3
    force = (hh - tr[..., None, None] * torch.eye(3, dtype=hh.dtype, device=hh.device)).cpu().numpy()
    g = np.random.default_rng(506)
    h = 1e-6
    b_p = lat.pack_spinor(ft, f64)
    for link in _links(g, dims, 20):
        x = _rand_th(g)
        up = ud.detach().clone()
        um = ud.detach().clone()
        up[link] = to_device(_expi(h * x) @ u[link])
        um[link] = to_device(_expi(-h * x) @ u[link])
        upp = lat.pack_gauge(up, f64)
        ump = lat.pack_gauge(um, f64)
        inner = Format("f32", "f32", 18)
        chp, _ = cg(lat, f64, upp, b_p, op="MdagM", tol=1e-13, inner=inner,
                    u_inner=lat.pack_gauge(up, inner), inner_tol=1e-5, maxiter=100000)
        chm, _ = cg(lat, f64, ump, b_p, op="MdagM", tol=1e-13, inner=inner,
                    u_inner=lat.pack_gauge(um, inner), inner_tol=1e-5, maxiter=100000)
        am = lat.apply(ump, lat.apply(ump, chm, f64), f64, dagger=True)
        ap = lat.apply(upp, lat.apply(upp, chm, f64), f64, dagger=True)
        cp = lat.unpack_spinor(chp, f64).cpu().numpy()
        diff = (lat.unpack_spinor(am, f64) - lat.unpack_spinor(ap, f64)).cpu().numpy()
        fd = np.vdot(cp, diff).real / (2 * h)
        an = np.trace(x @ force[link]).real
        assert abs(fd - an) <= 1e-5 * max(1.0, abs(an)), (link, fd, an)


def _l2_setup(dims, kappa, dtype):
    lat = Lattice(dims, kappa, AP)
    u = cached_gauge(dims, 0.5, 501)
    phi = inputs.gen_spinor_half(dims, 504)
    return lat, u, phi


def test_fd_l2_sites_16_3x32_difference_form():
    """20 site directions d of phi for L2 = <phi, A^-1 phi>, A = M^dag M, at
    step 1e-6 in FP64.  L(phi + h d) - L(phi - h d) is taken in the
    cancellation-free difference form <2 h d, A^-1 phi+> + <phi-, A^-1 (2 h d)>
    (exact algebra: A^-1 is linear), each A^-1 a GPU solve to 1e-13; the
    gradient is the autograd one, 2 chi."""
    print("fd L2 sites 16^3x32", flush=True)
    from paper_2303_08609_amd.ops import Format
    from paper_2303_08609_amd.solve import cg
    dims, kappa = (16, 16, 16, 32), 0.125
    lat, u, phi = _l2_setup(dims, kappa, torch.complex128)
    f64, f32 = Format("f64", "f64", 18), Format("f32", "f32", 18)
    ud = to_device(u)
    ft = to_device(phi).requires_grad_(True)
    chi = wilson_solve(ud, ft, lat, tol=1e-12, mixed=True)
    loss = (ft.conj() * chi).real.sum()
    loss.backward()
    gphi = ft.grad.cpu().numpy()
    u64, u32 = lat.pack_gauge(ud, f64), lat.pack_gauge(ud, f32)

    def solve(v):
        x, info = cg(lat, f64, u64, lat.pack_spinor(to_device(v), f64), op="MdagM", tol=1e-13, inner=f32,
                     u_inner=u32, inner_tol=1e-5, maxiter=100000)
        assert info["status"] == 0, info
        return lat.unpack_spinor(x, f64).cpu().numpy()

    g = np.random.default_rng(507)
    h = 1e-6
    for _ in range(20):
        site = tuple(int(g.integers(n)) for n in phi.shape[:4])
        d = np.zeros_like(phi)
        v = g.standard_normal((4, 3)) + 1j * g.standard_normal((4, 3))
        d[site] = v / np.linalg.norm(v)
        chi_p = solve(phi + h * d)
        eta = solve(2 * h * d)
        fd = (np.vdot(2 * h * d, chi_p) + np.vdot(phi - h * d, eta)).real / (2 * h)
        an = np.vdot(gphi, d).real
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (site, fd, an)


def test_fp32_l2_gradient_16_3x32_vs_fp64_oracle():
    """FP32 fields (complex64 links and phi) through the autograd solve with
    FP64 defect correction around FP32 inner solves: the link and phi
    gradients of L2 = <phi, (M^dag M)^-1 phi> match the oracle's FP64
    gradients on the same (FP32-rounded) inputs within 1e-5.  The oracle's
    chi is the GPU FP64 solve, accepted after the oracle's own residual check
    (no oracle CG at this size)."""
    print("fp32 L2 gradient 16^3x32", flush=True)
    from tests._helpers import ROUND
    dims, kappa = (16, 16, 16, 32), 0.125
    lat, u, phi = _l2_setup(dims, kappa, torch.complex64)
    u_r, phi_r = ROUND["f32"](u), ROUND["f32"](phi)
    # FP64 reference chi on the rounded inputs, checked by the oracle
    chi64 = wilson_solve(to_device(u_r), to_device(phi_r), lat, tol=1e-13, mixed=True).cpu().numpy()
    res = np.linalg.norm(phi_r - W.apply_mdagm(u_r, chi64, kappa, PH)) / np.linalg.norm(phi_r)
    assert res <= 1e-12, res
    want_u = F.link_grad_l2(u_r, chi64, kappa, PH)
    want_phi = F.grad_phi_l2(chi64)
    ut = to_device(u).to(torch.complex64).requires_grad_(True)
    ft = to_device(phi).to(torch.complex64).requires_grad_(True)
    chi = wilson_solve(ut, ft, lat, tol=1e-10, mixed=True)
    assert chi.dtype == torch.complex64
    loss = (ft.conj() * chi).real.sum()
    loss.backward()
    eu = rel_err(ut.grad.cpu().numpy(), want_u)
    ep = rel_err(ft.grad.cpu().numpy(), want_phi)
    print(f"  link gradient {eu:.2e}, phi gradient {ep:.2e}", flush=True)
    assert eu <= 1e-5 and ep <= 1e-5
