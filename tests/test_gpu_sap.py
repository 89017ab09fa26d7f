"""The Schwarz alternating procedure and SAP-preconditioned flexible GCR on
the GPU against the oracle (``oracle/sap.py``):

* K eta (ncy cycles of nmr-step MR block solves on two-coloured Dirichlet
  blocks, FP32) against the oracle's SAP on the same FP32-rounded inputs, on
  several block layouts (blocks of 2^4, 4^4 (256 sites, the largest),
  non-cubic blocks, one block spanning the lattice), complex boundary
  phases, several right-hand sides;
* SAP-GCR solves of D_W: FP64 GCR with the FP32 preconditioner against a
  dense solve (4^4, with and without restarts), plain FP32 GCR at 16^3x32
  against the oracle's residual, and FP64 defect correction around FP32
  SAP-GCR inner solves to 1e-10;
* defect correction around FP32 inner CGLS / BiCGStab / block CG on D_W
  (full fields converted half by half).

Bars: K, relative 1e-5 norm-wise and 1e-4 per site (FP32 storage of the
carried residual and solution between sweeps, and the MR step sizes are
data-dependent); solves as stated per test.
"""
import numpy as np
import pytest
import torch

from oracle import sap as OS
from oracle import wilson as W
from oracle.lattice import full_to_half, half_to_full
from paper_2303_08609_amd import inputs
from paper_2303_08609_amd import wilson_eo as WE
from paper_2303_08609_amd.ops import Format, Lattice, to_device
from paper_2303_08609_amd.solve import cg
from tests._helpers import AP, ROUND, cached_gauge, link_as_stored, rel_err, site_rel_max

pytestmark = pytest.mark.gpu

F64 = Format("f64", "f64", 18)
F32 = Format("f32", "f32", 18)
F32L12 = Format("f32", "f32", 12)


def _full_field(lat, fmt, full, nrhs=None):
    if nrhs is None:
        e = lat.pack_spinor(to_device(full_to_half(full, 0)), fmt)
        o = lat.pack_spinor(to_device(full_to_half(full, 1)), fmt)
        return torch.cat([e, o])
    return torch.cat([_full_field(lat, fmt, full[r]) for r in range(nrhs)])


def _unpack_full(lat, fmt, x, nrhs=None):
    s = lat.spinor_bytes(fmt)
    if nrhs is not None:
        return np.stack([_unpack_full(lat, fmt, x[2 * r * s:2 * (r + 1) * s]) for r in range(nrhs)])
    e = lat.unpack_spinor(x[:s], fmt).cpu().numpy()
    o = lat.unpack_spinor(x[s:2 * s], fmt).cpu().numpy()
    return half_to_full(e, 0, lat.dims) + half_to_full(o, 1, lat.dims)


CASES = [
    # dims, block, ncy, nmr, fmt
    ((4, 4, 4, 4), (2, 2, 2, 2), 2, 4, F32),
    ((8, 4, 4, 8), (4, 2, 2, 4), 3, 3, F32L12),
    ((8, 8, 8, 8), (4, 4, 4, 4), 2, 5, F32),
    ((4, 2, 2, 4), (4, 2, 2, 4), 1, 8, F32),          # one block over the lattice
    ((8, 4, 2, 4), (2, 4, 2, 2), 2, 2, F32L12),       # blocks spanning y and z
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{'x'.join(map(str, c[0]))}-b{''.join(map(str, c[1]))}")
def test_sap_matches_oracle(case):
    dims, block, ncy, nmr, fmt = case
    print(f"SAP dims={dims} block={block} ncy={ncy} nmr={nmr} fmt={fmt}", flush=True)
    ph = np.exp(1j * np.array([0.4, -1.1, 2.0, 2.9]))
    lat = Lattice(dims, 0.124, tuple(ph))
    u = inputs.gen_gauge(dims, 0.5, 1300 + sum(dims))
    eta = inputs.gen_spinor_full(dims, 1301)
    u_d = lat.pack_gauge(to_device(u), fmt)
    got = _unpack_full(lat, fmt, lat.sap(u_d, _full_field(lat, fmt, eta), fmt, block, ncy, nmr))
    want = OS.sap(link_as_stored(u, "f32", fmt.link_reals), ROUND["f32"](eta), 0.124, ph, block, ncy, nmr)
    e, m = rel_err(got, want), site_rel_max(got, want)
    print(f"  norm-wise {e:.2e}, per site {m:.2e}", flush=True)
    assert e <= 1e-5 and m <= 1e-4


def test_sap_several_rhs_match_one_at_a_time():
    dims, block = (8, 4, 4, 8), (4, 2, 2, 2)
    print("SAP 3 rhs", flush=True)
    lat = Lattice(dims, 0.125, AP)
    u_d = lat.pack_gauge(to_device(inputs.gen_gauge(dims, 0.5, 1310)), F32)
    eta = np.stack([inputs.gen_spinor_full(dims, 1311 + r) for r in range(3)])
    together = lat.sap(u_d, _full_field(lat, F32, eta, nrhs=3), F32, block, 2, 4, nrhs=3)
    for r in range(3):
        one = lat.sap(u_d, _full_field(lat, F32, eta[r]), F32, block, 2, 4)
        s = 2 * lat.spinor_bytes(F32)
        assert torch.equal(together[r * s:(r + 1) * s], one), r


@pytest.mark.parametrize("nkv", [2, 8])
def test_sap_gcr_fp64_matches_dense(nkv):
    """FP64 flexible GCR preconditioned by the FP32 SAP (links passed as the
    preconditioner's FP32 copy) on 4^4, against a dense solve of D_W."""
    print(f"SAP-GCR FP64 4^4 nkv={nkv}", flush=True)
    dims, kappa = (4, 4, 4, 4), 0.124
    lat = Lattice(dims, kappa, AP)
    u = inputs.gen_gauge(dims, 0.3, 101)
    eta = inputs.gen_spinor_full(dims, 102)
    ud = to_device(u)
    x, info = cg(lat, F64, lat.pack_gauge(ud, F64), _full_field(lat, F64, eta), op="DW", tol=1e-12,
                 maxiter=500, method="sapgcr", u_inner=lat.pack_gauge(ud, F32), pre=F32, sap_block=(2, 2, 2, 2),
                 sap_ncy=2, sap_nmr=4, gcr_nkv=nkv)
    print(f"  {info}", flush=True)
    assert info["status"] == WE.WEO_OK and info["true_rel_resid"][0] <= 1e-12
    d = W.dense_dirac_wilson(u, kappa, np.array(AP, dtype=np.complex128))
    xi = np.linalg.solve(d, eta.reshape(-1)).reshape(eta.shape)
    assert rel_err(_unpack_full(lat, F64, x), xi) < 1e-10
    # the preconditioner pays: far fewer iterations than CGLS on D_W
    _, info_cg = cg(lat, F64, lat.pack_gauge(ud, F64), _full_field(lat, F64, eta), op="DW", tol=1e-12,
                    maxiter=5000)
    assert info["iters"] < info_cg["iters"] / 3


def test_sap_gcr_fp32_16_3x32():
    """Plain FP32 SAP-GCR (4^4 blocks) at 16^3x32 to 1e-6; the oracle's D_W
    residual of the returned solution on the rounded inputs."""
    print("SAP-GCR FP32 16^3x32", flush=True)
    dims, kappa = (16, 16, 16, 32), 0.125
    lat = Lattice(dims, kappa, AP)
    u = cached_gauge(dims, 0.5, 501)
    eta = inputs.gen_spinor_full(dims, 1320)
    x, info = cg(lat, F32, lat.pack_gauge(to_device(u), F32), _full_field(lat, F32, eta), op="DW", tol=1e-6,
                 maxiter=200, method="sapgcr", sap_block=(4, 4, 4, 4), sap_ncy=4, sap_nmr=4, gcr_nkv=8)
    print(f"  {info}", flush=True)
    assert info["status"] == WE.WEO_OK
    got = _unpack_full(lat, F32, x)
    eta_r = ROUND["f32"](eta)
    r = eta_r - W.dirac_wilson(ROUND["f32"](u), got, kappa, np.array(AP, dtype=np.complex128))
    assert np.linalg.norm(r) / np.linalg.norm(eta_r) <= 3e-6


@pytest.mark.parametrize("method", ["sapgcr", "cg", "bicgstab", "blockcg"])
def test_dw_defect_correction_fp32_inner(method):
    """FP64 defect correction on D_W (full fields, converted half by half)
    around FP32 inner solves, two right-hand sides, to 1e-10: the oracle's
    residual of each solution."""
    print(f"D_W defect correction inner={method}", flush=True)
    dims, kappa = (8, 8, 8, 16), 0.125
    lat = Lattice(dims, kappa, AP)
    u = cached_gauge(dims, 0.5, 850)
    eta = np.stack([inputs.gen_spinor_full(dims, 1330 + r) for r in range(2)])
    ud = to_device(u)
    x, info = cg(lat, F64, lat.pack_gauge(ud, F64), _full_field(lat, F64, eta, nrhs=2), nrhs=2, op="DW",
                 tol=1e-10, inner=F32L12, u_inner=lat.pack_gauge(ud, F32L12), inner_tol=1e-5, max_outer=30,
                 maxiter=20000, method=method, sap_block=(4, 4, 4, 4), sap_ncy=3, sap_nmr=4, gcr_nkv=8)
    print(f"  {info}", flush=True)
    assert info["status"] == WE.WEO_OK
    got = _unpack_full(lat, F64, x, nrhs=2)
    for r in range(2):
        res = eta[r] - W.dirac_wilson(u, got[r], kappa, np.array(AP, dtype=np.complex128))
        assert np.linalg.norm(res) / np.linalg.norm(eta[r]) <= 1e-10, r


def test_dw_defect_correction_fp16_inner_refused():
    dims = (4, 4, 4, 4)
    lat = Lattice(dims, 0.125, AP)
    f16 = Format("f16", "f16", 12)
    u = lat.new_gauge(F64)
    b = torch.cat([lat.new_spinor(F64), lat.new_spinor(F64)])
    with pytest.raises(WE.WilsonEOError):
        cg(lat, F64, u, b, op="DW", inner=f16, u_inner=lat.new_gauge(f16), maxiter=1)
