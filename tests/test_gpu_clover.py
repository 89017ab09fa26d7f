"""Clover-type site blocks (site-local D_ee, D_oo of Eqs. (3)-(5)) on the GPU
against the FP64 oracle: packing with and without the FP64 inversion, the
site product, the even-odd operator and its adjoint in every format, the full
system through Eqs. (4)-(5) against a dense solve, and mixed-precision solves.
Bars as for the Wilson operator: FP64 <= 1e-12, FP32 <= 1e-6, FP16 spinors
<= 2e-3, BF16 spinors <= 1e-2 (norm-wise relative)."""
import numpy as np
import pytest
import torch

from oracle import clover as CL
from oracle import solvers as S
from oracle import wilson as W
from oracle.lattice import full_to_half
from paper_2303_08609_amd import inputs
from paper_2303_08609_amd import wilson_eo as WE
from paper_2303_08609_amd.ops import Format, Lattice, to_device
from paper_2303_08609_amd.solve import cg
from tests._helpers import AP, ROUND, cached_gauge, link_as_stored, rel_err

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-6, "f16": 2e-3, "bf16": 1e-2}
FORMATS = [("f64", "f64", 18), ("f64", "f64", 12), ("f32", "f32", 18), ("f32", "f32", 12),
           ("f16", "f16", 18), ("f16", "f16", 12), ("bf16", "f16", 18), ("bf16", "f16", 12)]
PH = np.array(AP, dtype=np.complex128)
KAPPA = 0.126


def _blocks(dims, seed, eps=0.3):
    blocks = inputs.gen_site_blocks(dims, eps, seed)
    a = CL.blocks_to_dirac(blocks)
    return blocks, a, np.linalg.inv(a)


@pytest.mark.parametrize("fmt_t", FORMATS, ids=lambda f: f"{f[0]}-{f[1]}-{f[2]}")
def test_site_product_matches_oracle(fmt_t):
    dims = (4, 6, 2, 4)
    print(f"clover site product fmt={fmt_t}", flush=True)
    fmt = Format(*fmt_t)
    lat = Lattice(dims, KAPPA, AP)
    blocks, a, ainv = _blocks(dims, 900)
    psi = inputs.gen_spinor_half(dims, 901)
    y = inputs.gen_spinor_half(dims, 902)
    x_d, y_d = lat.pack_spinor(to_device(psi), fmt), lat.pack_spinor(to_device(y), fmt)
    psi_r, y_r = ROUND[fmt_t[0]](psi), ROUND[fmt_t[0]](y)
    for invert, mat in ((0, a), (1, ainv)):
        clv = lat.pack_clover(to_device(blocks), fmt, invert=bool(invert))
        for par in (0, 1):
            m = full_to_half(mat, par)
            got = lat.unpack_spinor(lat.clover_site(clv, x_d, fmt, par), fmt).cpu().numpy()
            assert rel_err(got, CL.apply_sites(m, psi_r)) <= TOL[fmt_t[0]], (invert, par)
            got = lat.unpack_spinor(lat.clover_site(clv, x_d, fmt, par, y=y_d, alpha=-0.7), fmt).cpu().numpy()
            assert rel_err(got, y_r - 0.7 * CL.apply_sites(m, psi_r)) <= TOL[fmt_t[0]], (invert, par)


@pytest.mark.parametrize("fmt_t", FORMATS, ids=lambda f: f"{f[0]}-{f[1]}-{f[2]}")
@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (4, 6, 2, 8), (10, 6, 4, 6)],
                         ids=lambda d: "x".join(map(str, d)))
def test_clover_apply_matches_oracle(dims, fmt_t):
    print(f"clover apply dims={dims} fmt={fmt_t}", flush=True)
    sp, lp, reals = fmt_t
    fmt = Format(*fmt_t)
    lat = Lattice(dims, KAPPA, AP)
    u = cached_gauge(dims, 0.5, 910 + sum(dims))
    blocks, a, ainv = _blocks(dims, 911)
    psi = inputs.gen_spinor_half(dims, 912)
    u_d, x_d = lat.pack_gauge(to_device(u), fmt), lat.pack_spinor(to_device(psi), fmt)
    clv = lat.pack_clover(to_device(blocks), fmt)
    u_or, psi_or = link_as_stored(u, lp, reals), ROUND[sp](psi)
    ai_e, ai_o = full_to_half(ainv, 0), full_to_half(ainv, 1)
    for dag in (False, True):
        got = lat.unpack_spinor(lat.clover_apply(u_d, clv, x_d, fmt, dagger=dag), fmt).cpu().numpy()
        want = CL.apply_m_clover(u_or, psi_or, KAPPA, PH, ai_e, ai_o, dagger=dag)
        assert rel_err(got, want) <= TOL[sp], (dag, rel_err(got, want))


def test_scalar_blocks_equal_wilson_and_several_rhs():
    """Blocks a * 1 give the Wilson operator at kappa / a; three right-hand
    sides through one call match one at a time."""
    dims = (4, 4, 2, 6)
    fmt = Format("f64", "f64", 18)
    lat = Lattice(dims, KAPPA, AP)
    u = cached_gauge(dims, 0.5, 920)
    psi = inputs.gen_spinor_half(dims, 921, nrhs=3)
    u_d, x_d = lat.pack_gauge(to_device(u), fmt), lat.pack_spinor(to_device(psi), fmt)
    a = 1.25
    blocks = np.broadcast_to(a * np.eye(6, dtype=np.complex128), (dims[3], dims[2], dims[1], dims[0], 2, 6, 6))
    clv = lat.pack_clover(to_device(np.ascontiguousarray(blocks)), fmt)
    got = lat.clover_apply(u_d, clv, x_d, fmt, nrhs=3)
    lat2 = Lattice(dims, KAPPA / a, AP)
    want = lat2.apply(u_d, x_d, fmt, nrhs=3)
    g = lat.unpack_spinor(got, fmt, nrhs=3).cpu().numpy()
    w = lat.unpack_spinor(want, fmt, nrhs=3).cpu().numpy()
    assert rel_err(g, w) < 1e-13


@pytest.mark.parametrize("method", ["cg", "bicgstab"])
def test_clover_full_system_via_eqs_4_5(method):
    """D xi = eta with D = A - kappa H on 4^4 through Eq. (4) (right-hand side
    A_ee^-1 (eta_e + kappa H_eo A_oo^-1 eta_o)), the even solve and Eq. (5)
    (xi_o = A_oo^-1 (eta_o + kappa H_oe xi_e)), against a dense FP64 solve."""
    print(f"clover full system {method}", flush=True)
    dims = (4, 4, 4, 4)
    fmt = Format("f64", "f64", 18)
    lat = Lattice(dims, KAPPA, AP)
    u = inputs.gen_gauge(dims, 0.3, 101)
    blocks, a, ainv = _blocks(dims, 930)
    eta = inputs.gen_spinor_full(dims, 931)
    u_d = lat.pack_gauge(to_device(u), fmt)
    clv = lat.pack_clover(to_device(blocks), fmt)
    ee = lat.pack_spinor(to_device(full_to_half(eta, 0)), fmt)
    eo = lat.pack_spinor(to_device(full_to_half(eta, 1)), fmt)
    ai_eo = lat.clover_site(clv, eo, fmt, 1)                                  # A_oo^-1 eta_o
    t = lat.hop_axpy(u_d, ai_eo, ee, fmt, out_parity=0, alpha=KAPPA)          # eta_e + kappa H_eo (.)
    b_e = lat.clover_site(clv, t, fmt, 0)                                      # A_ee^-1 (.)
    xe, info = cg(lat, fmt, u_d, b_e, tol=1e-13, maxiter=5000, method=method, clover=clv, check_every=1)
    assert info["status"] == WE.WEO_OK
    xo = lat.clover_hop(u_d, clv, xe, fmt, out_parity=1, y=ai_eo, alpha=KAPPA)  # Eq. (5)
    d = CL.dense_sites(a) - KAPPA * W.dense_hop(u, PH)
    xi = np.linalg.solve(d, eta.reshape(-1)).reshape(eta.shape)
    assert rel_err(lat.unpack_spinor(xe, fmt).cpu().numpy(), full_to_half(xi, 0)) < 1e-11
    assert rel_err(lat.unpack_spinor(xo, fmt).cpu().numpy(), full_to_half(xi, 1)) < 1e-11


@pytest.mark.parametrize("inner", [("f32", "f32", 18), ("f16", "f16", 12)], ids=["f32", "f16-l12"])
def test_clover_mixed_defect_correction(inner):
    print(f"clover mixed dc inner={inner}", flush=True)
    dims, kappa = (8, 8, 8, 16), 0.124
    fmt = Format("f64", "f64", 18)
    fi = Format(*inner)
    lat = Lattice(dims, kappa, AP)
    u = inputs.gen_gauge(dims, 0.7, 301)
    blocks, a, ainv = _blocks(dims, 940, eps=0.2)
    b = inputs.gen_spinor_half(dims, 941)
    u_dev, bl_dev = to_device(u), to_device(blocks)
    x_p, info = cg(lat, fmt, lat.pack_gauge(u_dev, fmt), lat.pack_spinor(to_device(b), fmt), tol=1e-10,
                   inner=fi, u_inner=lat.pack_gauge(u_dev, fi), inner_tol=1e-3 if inner[0] != "f32" else 1e-5,
                   max_outer=60, maxiter=20000, method="bicgstab", clover=lat.pack_clover(bl_dev, fmt),
                   clover_inner=lat.pack_clover(bl_dev, fi))
    assert info["status"] == WE.WEO_OK, info
    x = lat.unpack_spinor(x_p, fmt).cpu().numpy()
    ai_e, ai_o = full_to_half(ainv, 0), full_to_half(ainv, 1)
    r = S.rel_resid(lambda v: CL.apply_m_clover(u, v, kappa, PH, ai_e, ai_o), x, b)
    assert r <= 1e-10
    assert abs(r - info["true_rel_resid"][0]) <= 1e-12


def test_clover_argument_checks():
    dims = (4, 4, 4, 4)
    lat = Lattice(dims, KAPPA, AP)
    fmt = Format("f64", "f64", 18)
    u = lat.new_gauge(fmt)
    b = lat.new_spinor(fmt)
    clv = torch.empty(lat.clover_bytes(fmt), dtype=torch.uint8, device="cuda")
    # D_W with site blocks is not built; mixed needs the inner blocks too
    with pytest.raises(WE.WilsonEOError):
        cg(lat, fmt, u, torch.cat([b, b]), op="DW", clover=clv, maxiter=1)
    with pytest.raises(WE.WilsonEOError):
        cg(lat, fmt, u, b, inner=Format("f32", "f32", 18), u_inner=lat.new_gauge(Format("f32", "f32", 18)),
           clover=clv, maxiter=1)


@pytest.mark.parametrize("fmt_t", [FORMATS[0], FORMATS[3]], ids=["f64-18", "f32-12"])
def test_clover_apply_complex_phases(fmt_t):
    dims = (4, 6, 2, 8)
    bc = tuple(np.exp(1j * np.array([0.4, -1.1, 2.0, 2.9])))
    print(f"clover apply complex phases fmt={fmt_t}", flush=True)
    sp, lp, reals = fmt_t
    fmt = Format(*fmt_t)
    lat = Lattice(dims, KAPPA, bc)
    u = cached_gauge(dims, 0.5, 950)
    blocks, a, ainv = _blocks(dims, 951)
    psi = inputs.gen_spinor_half(dims, 952)
    u_d, x_d = lat.pack_gauge(to_device(u), fmt), lat.pack_spinor(to_device(psi), fmt)
    clv = lat.pack_clover(to_device(blocks), fmt)
    ai_e, ai_o = full_to_half(ainv, 0), full_to_half(ainv, 1)
    for dag in (False, True):
        got = lat.unpack_spinor(lat.clover_apply(u_d, clv, x_d, fmt, dagger=dag), fmt).cpu().numpy()
        want = CL.apply_m_clover(link_as_stored(u, lp, reals), ROUND[sp](psi), KAPPA, np.array(bc), ai_e, ai_o,
                                 dagger=dag)
        assert rel_err(got, want) <= TOL[sp], dag
