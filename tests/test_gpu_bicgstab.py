"""BiCGStab (van der Vorst 1992) on the GPU: solutions against dense FP64
solves and the oracle's residuals, the operator products it saves over CGLS,
mixed-precision defect correction around BiCGStab inner solves, twelve
right-hand sides, and the degenerate cases (zero source, converged start,
singular operator)."""
import numpy as np
import pytest
import torch

from oracle import solvers as S
from oracle import wilson as W
from paper_2303_08609_amd import inputs
from paper_2303_08609_amd import wilson_eo as WE
from paper_2303_08609_amd.ops import Format, Lattice, to_device
from paper_2303_08609_amd.solve import cg
from tests._helpers import AP, ROUND, cached_gauge, rel_err

pytestmark = pytest.mark.gpu

F64 = Format("f64", "f64", 18)
F32 = Format("f32", "f32", 18)
PH = np.array(AP, dtype=np.complex128)


def _resid_m(u, x, b, kappa):
    return S.rel_resid(lambda v: W.apply_m(u, v, kappa, PH), x, b)


def test_bicgstab_fp64_matches_dense_and_oracle_iterates():
    """4^4: the GPU iterate after k iterations equals the oracle's BiCGStab
    after k iterations; to 1e-13 the solution matches a dense solve."""
    print("bicgstab fp64 4^4", flush=True)
    dims, kappa = (4, 4, 4, 4), 0.125
    u = inputs.gen_gauge(dims, 0.3, 101)
    b = inputs.gen_spinor_half(dims, 102)
    lat = Lattice(dims, kappa, AP)
    u_p, b_p = lat.pack_gauge(to_device(u), F64), lat.pack_spinor(to_device(b), F64)
    m = lambda v: W.apply_m(u, v, kappa, PH)
    for k in (1, 2, 5):
        x_p, info = cg(lat, F64, u_p, b_p, tol=1e-30, maxiter=k, check_every=1, method="bicgstab")
        assert info["iters"] == k
        xo, it, _ = S.bicgstab(m, b, 1e-30, k)
        assert rel_err(lat.unpack_spinor(x_p, F64).cpu().numpy(), xo) < 1e-12, k
    x_p, info = cg(lat, F64, u_p, b_p, tol=1e-13, maxiter=1000, check_every=1, method="bicgstab")
    assert info["status"] == WE.WEO_OK
    x = lat.unpack_spinor(x_p, F64).cpu().numpy()
    assert _resid_m(u, x, b, kappa) <= 1.05e-13
    d = W.dense_dirac_wilson(u, kappa, PH)
    from oracle.lattice import full_to_half, half_to_full
    # M x = b  <=>  D_W (x, kappa H_oe x) = (b, 0): compare on the even half
    eta = half_to_full(b, 0, dims)
    xi = np.linalg.solve(d, eta.reshape(-1)).reshape(eta.shape)
    assert rel_err(x, full_to_half(xi, 0)) < 1e-11
    # fewer operator products than CGLS to the same tolerance
    _, info_cgls = cg(lat, F64, u_p, b_p, tol=1e-13, maxiter=1000, check_every=1)
    assert info["applies"] < info_cgls["applies"]


def test_bicgstab_unpreconditioned_dw():
    print("bicgstab D_W 4^4", flush=True)
    from tests.test_gpu_solver import _full_field, _unpack_full
    dims, kappa = (4, 4, 4, 4), 0.125
    lat = Lattice(dims, kappa, AP)
    u = inputs.gen_gauge(dims, 0.3, 101)
    eta = inputs.gen_spinor_full(dims, 102)
    u_p = lat.pack_gauge(to_device(u), F64)
    x, info = cg(lat, F64, u_p, _full_field(lat, F64, eta), op="DW", tol=1e-13, maxiter=2000,
                 method="bicgstab", check_every=1)
    assert info["status"] == WE.WEO_OK
    xi = np.linalg.solve(W.dense_dirac_wilson(u, kappa, PH), eta.reshape(-1)).reshape(eta.shape)
    assert rel_err(_unpack_full(lat, F64, x), xi) < 1e-11


def test_bicgstab_fp32_16_3x32():
    print("bicgstab fp32 16^3x32", flush=True)
    dims, kappa = (16, 16, 16, 32), 0.126
    u = cached_gauge(dims, 0.5, 201)
    b = inputs.gen_spinor_half(dims, 202)
    lat = Lattice(dims, kappa, AP)
    x_p, info = cg(lat, F32, lat.pack_gauge(to_device(u), F32), lat.pack_spinor(to_device(b), F32),
                   tol=1e-6, maxiter=10000, method="bicgstab")
    assert info["status"] == WE.WEO_OK
    x = lat.unpack_spinor(x_p, F32).cpu().numpy()
    assert _resid_m(ROUND["f32"](u), x, ROUND["f32"](b), kappa) <= 3e-6


@pytest.mark.parametrize("inner", [("f32", "f32", 18), ("f16", "f16", 12), ("bf16", "f16", 12)],
                         ids=["f32", "f16-l12", "bf16-l12"])
def test_bicgstab_defect_correction_reaches_1e_10(inner):
    print(f"bicgstab dc inner={inner}", flush=True)
    dims, kappa = (8, 8, 8, 16), 0.1265
    u = inputs.gen_gauge(dims, 0.7, 301)
    b = inputs.gen_spinor_half(dims, 302)
    lat = Lattice(dims, kappa, AP)
    fi = Format(*inner)
    u_dev = to_device(u)
    x_p, info = cg(lat, F64, lat.pack_gauge(u_dev, F64), lat.pack_spinor(to_device(b), F64),
                   tol=1e-10, inner=fi, u_inner=lat.pack_gauge(u_dev, fi),
                   inner_tol=1e-3 if inner[0] != "f32" else 1e-5, max_outer=60, maxiter=20000,
                   method="bicgstab")
    assert info["status"] == WE.WEO_OK, info
    x = lat.unpack_spinor(x_p, F64).cpu().numpy()
    r = _resid_m(u, x, b, kappa)
    assert r <= 1e-10
    assert abs(r - info["true_rel_resid"][0]) <= 1e-12


def test_bicgstab_twelve_rhs_mixed():
    """12 point+noise sources together, FP16 inner BiCGStab, each to 1e-10;
    the batched plain FP64 solve equals one-at-a-time solves."""
    print("bicgstab 12 rhs", flush=True)
    dims, kappa = (8, 8, 8, 8), 0.126
    u = inputs.gen_gauge(dims, 0.5, 401)
    b = inputs.gen_point_noise_sources(dims, 406)
    lat = Lattice(dims, kappa, AP)
    u_dev = to_device(u)
    fi = Format("f16", "f16", 12)
    x_p, info = cg(lat, F64, lat.pack_gauge(u_dev, F64), lat.pack_spinor(to_device(b), F64), nrhs=12,
                   tol=1e-10, inner=fi, u_inner=lat.pack_gauge(u_dev, fi), inner_tol=1e-3,
                   max_outer=60, maxiter=20000, method="bicgstab")
    assert info["status"] == WE.WEO_OK, info
    x = lat.unpack_spinor(x_p, F64, nrhs=12).cpu().numpy()
    for r in range(12):
        assert _resid_m(u, x[r], b[r], kappa) <= 1e-10, r
    u64 = lat.pack_gauge(u_dev, F64)
    xb, _ = cg(lat, F64, u64, lat.pack_spinor(to_device(b[:3]), F64), nrhs=3, tol=1e-11, maxiter=5000,
               method="bicgstab", check_every=1)
    xb = lat.unpack_spinor(xb, F64, nrhs=3).cpu().numpy()
    for r in range(3):
        x1, _ = cg(lat, F64, u64, lat.pack_spinor(to_device(b[r]), F64), tol=1e-11, maxiter=5000,
                   method="bicgstab", check_every=1)
        assert rel_err(xb[r], lat.unpack_spinor(x1, F64).cpu().numpy()) < 1e-9


def test_bicgstab_degenerate_cases():
    print("bicgstab zero source / x0 / singular", flush=True)
    dims, kappa = (4, 4, 4, 4), 0.125
    lat = Lattice(dims, kappa, AP)
    u = inputs.gen_gauge(dims, 0.3, 101)
    u_p = lat.pack_gauge(to_device(u), F64)
    zero = lat.pack_spinor(to_device(np.zeros(lat.half_shape(), dtype=np.complex128)), F64)
    x_p, info = cg(lat, F64, u_p, zero, tol=1e-12, maxiter=100, method="bicgstab")
    assert info["status"] == WE.WEO_OK and info["iters"] == 0
    assert torch.count_nonzero(x_p).item() == 0
    b_p = lat.pack_spinor(to_device(inputs.gen_spinor_half(dims, 102)), F64)
    x_p, info = cg(lat, F64, u_p, b_p, tol=1e-12, maxiter=5000, method="bicgstab")
    _, info2 = cg(lat, F64, u_p, b_p, tol=1e-11, maxiter=5000, x0=x_p, method="bicgstab")
    assert info2["status"] == WE.WEO_OK and info2["iters"] == 0
    # the free field at kappa = 1/8 with periodic phases has a zero mode
    lat0 = Lattice(dims, 0.125, (1, 1, 1, 1))
    u0 = lat0.pack_gauge(to_device(inputs.gen_unit_gauge(dims)), F64)
    b0 = lat0.pack_spinor(to_device(inputs.gen_spinor_half(dims, 7)), F64)
    x_p, info = cg(lat0, F64, u0, b0, tol=1e-10, maxiter=300, method="bicgstab")
    assert info["status"] in (WE.WEO_NOT_CONVERGED, WE.WEO_BREAKDOWN)
    assert info["true_rel_resid"][0] > 1e-3
