"""Full-size parity of the timed workloads against the FP64 oracle at sampled
sites (faces, corners and random sites), in the launch configuration the
benchmark uses:

* the FP16- and BF16-spinor operators with FP16 12-real links (the inner
  operator of the mixed-precision solves) at 32^3x64 (kappa = 0.126,
  links exp(0.5 i H)) and at 48^3x96 (kappa = 0.1265, links exp(0.7 i H)),
  apply M, M^dag and the hop;
* the FP64 outer operator at 48^3x96;
* FP64 defect correction to 1e-10 at 48^3x96 with FP16 / BF16 spinor and
  FP16 12-real link inner solves, CGLS and BiCGStab;
* the clover-type operator in full at 16^3x32 and sampled at 32^3x64.

The oracle sees the inputs exactly as the kernels read them: spinors and
links rounded to the storage precision (12-real links with row 2 rebuilt
from the rounded rows), clover inverse blocks rounded after the FP64
inversion.  Bars, norm-wise over the sampled records and per site
(max_s ||a_s - b_s|| / ||b_s||): FP64 1e-12, FP32 1e-6, FP16 spinors 2e-3,
BF16 spinors 1e-2.
"""
import numpy as np
import pytest
import torch

from oracle import clover as CL
from oracle import wilson as W
from oracle.lattice import full_to_half
from paper_2303_08609_amd import inputs
from paper_2303_08609_amd import wilson_eo as WE
from paper_2303_08609_amd.ops import Format, Lattice, to_device
from paper_2303_08609_amd.solve import cg
from tests._helpers import (AP, ROUND, cached_gauge, link_as_stored, rel_err, sample_sites,
                            site_rel_max)

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-6, "f16": 2e-3, "bf16": 1e-2}
PH = np.array(AP, dtype=np.complex128)
LOW = [("f16", "f16", 12), ("bf16", "f16", 12)]


class _StoredLinks:
    """Links as a kernel of the given format reads them, rounded on access
    (the sampled oracle touches only the links around its sites)."""

    def __init__(self, u, prec, reals):
        self.u, self.prec, self.reals = u, prec, reals

    def __getitem__(self, idx):
        return link_as_stored(self.u[idx], self.prec, self.reals)


class _StoredHalf:
    """A one-parity spinor as stored in precision prec, rounded on access."""

    def __init__(self, psi, prec):
        self.psi, self.prec, self.shape = psi, prec, psi.shape

    def __getitem__(self, idx):
        return ROUND[self.prec](self.psi[idx])


def _check(got, want, prec, what):
    e, m = rel_err(got, want), site_rel_max(got, want)
    print(f"  {what}: norm-wise {e:.2e}, per-site max {m:.2e}", flush=True)
    assert e <= TOL[prec], (what, e)
    assert m <= TOL[prec], (what, m)


def _operator_sampled(dims, kappa, eps, seed_u, seed_psi, fmt_t, nsample, seed_sites, u=None):
    sp, lp, reals = fmt_t
    fmt = Format(*fmt_t)
    lat = Lattice(dims, kappa, AP)
    u = cached_gauge(dims, eps, seed_u) if u is None else u
    psi = inputs.gen_spinor_half(dims, seed_psi)
    u_d = lat.pack_gauge(to_device(u), fmt)
    x_d = lat.pack_spinor(to_device(psi), fmt)
    us, ps = _StoredLinks(u, lp, reals), _StoredHalf(psi, sp)
    sites = sample_sites(dims, nsample, seed_sites)
    for dag in (False, True):
        got = lat.unpack_spinor(lat.apply(u_d, x_d, fmt, dagger=dag), fmt).cpu().numpy().reshape(-1, 4, 3)
        want = W.apply_m_at_sites(us, ps, kappa, PH, sites, dagger=dag)
        _check(got[sites], want, sp, f"apply dagger={dag}")
    for dag in (False, True):
        got = lat.unpack_spinor(lat.hop(u_d, x_d, fmt, out_parity=1, dagger=dag), fmt).cpu().numpy()
        want = W.hop_at_sites(us, ps, 0, PH, sites, dagger=dag)
        _check(got.reshape(-1, 4, 3)[sites], want, sp, f"hop to odd dagger={dag}")
    del u_d, x_d
    torch.cuda.empty_cache()


@pytest.mark.parametrize("fmt_t", LOW, ids=["f16-l12", "bf16-l12"])
def test_low_precision_operator_32_3x64_sampled(fmt_t):
    """The single-rhs FP16 / BF16 spinor operator with FP16 12-real links at
    32^3x64 (the benchmark's f16/f16/12 and bf16/f16/12 variants)."""
    print(f"low-precision operator 32^3x64 fmt={fmt_t}", flush=True)
    _operator_sampled((32, 32, 32, 64), 0.126, 0.5, 201, 202, fmt_t, 24, 11)


# ---- 48^3 x 96: one gauge field for every test of the mixed-precision workload ----
DIMS48, KAPPA48, EPS48 = (48, 48, 48, 96), 0.1265, 0.7


@pytest.fixture(scope="module")
def gauge48():
    print("generating the 48^3x96 gauge field", flush=True)
    return cached_gauge(DIMS48, EPS48, 301)


@pytest.mark.parametrize("fmt_t", [("f64", "f64", 18)] + LOW, ids=["f64", "f16-l12", "bf16-l12"])
def test_operator_48_3x96_sampled(gauge48, fmt_t):
    """The outer FP64 operator and the inner FP16 / BF16 ones of the
    mixed-precision workload at 48^3x96."""
    print(f"operator 48^3x96 fmt={fmt_t}", flush=True)
    _operator_sampled(DIMS48, KAPPA48, EPS48, 301, 302, fmt_t, 16, 12, u=gauge48)


@pytest.mark.parametrize("method", ["cg", "bicgstab"])
@pytest.mark.parametrize("inner", LOW, ids=["f16-l12", "bf16-l12"])
def test_mixed_solve_48_3x96_sampled(gauge48, inner, method):
    """FP64 defect correction to 1e-10 around FP16 / BF16 spinor and FP16
    12-real link inner solves (inner tolerance 1e-3) at 48^3x96 with the
    benchmark's source: the library's FP64 true residual meets the
    tolerance, and the oracle's M x at sampled sites matches b there to a
    relative 1e-9 (the global relative residual 1e-10, with room for an
    uneven spread over the sites)."""
    print(f"mixed solve 48^3x96 inner={inner} method={method}", flush=True)
    lat = Lattice(DIMS48, KAPPA48, AP)
    f64, fi = Format("f64", "f64", 18), Format(*inner)
    ud = to_device(gauge48)
    b = inputs.gen_spinor_half(DIMS48, 302)
    x_p, info = cg(lat, f64, lat.pack_gauge(ud, f64), lat.pack_spinor(to_device(b), f64), tol=1e-10, inner=fi,
                   u_inner=lat.pack_gauge(ud, fi), inner_tol=1e-3, max_outer=100, maxiter=50000, method=method)
    del ud
    print(f"  {info}", flush=True)
    assert info["status"] == WE.WEO_OK, info
    assert info["true_rel_resid"][0] <= 1e-10
    x = lat.unpack_spinor(x_p, f64).cpu().numpy()
    del x_p
    torch.cuda.empty_cache()
    sites = sample_sites(DIMS48, 16, 13)
    mx = W.apply_m_at_sites(gauge48, x, KAPPA48, PH, sites)
    bs = b.reshape(-1, 4, 3)[sites]
    r = np.linalg.norm(mx - bs) / np.linalg.norm(bs)
    print(f"  sampled relative residual {r:.2e}", flush=True)
    assert r <= 1e-9
    assert np.linalg.norm(x.reshape(-1, 4, 3)[sites]) > 0.1 * np.linalg.norm(bs)


# ---- clover-type operator -------------------------------------------------------
CLOVER_FMTS = [("f64", "f64", 18), ("f32", "f32", 18), ("f32", "f32", 12), ("f16", "f16", 12),
               ("bf16", "f16", 12)]


def _stored_inverse_blocks(blocks, lp):
    """Inverse site blocks as packed: inverted in FP64, rounded to the link
    precision, as [..., 12, 12] matrices on the Dirac (spin, colour) index."""
    return CL.blocks_to_dirac(ROUND[lp](np.linalg.inv(blocks)))


@pytest.mark.parametrize("fmt_t", CLOVER_FMTS, ids=lambda f: f"{f[0]}-{f[2]}")
def test_clover_apply_16_3x32_full(fmt_t):
    """The clover-type M and M^dag of Eq. (4) on the whole 16^3x32 lattice."""
    print(f"clover apply 16^3x32 fmt={fmt_t}", flush=True)
    sp, lp, reals = fmt_t
    dims, kappa = (16, 16, 16, 32), 0.126
    fmt = Format(*fmt_t)
    lat = Lattice(dims, kappa, AP)
    u = cached_gauge(dims, 0.5, 501)
    blocks = inputs.gen_site_blocks(dims, 0.3, 507)
    psi = inputs.gen_spinor_half(dims, 502)
    u_d, x_d = lat.pack_gauge(to_device(u), fmt), lat.pack_spinor(to_device(psi), fmt)
    clv = lat.pack_clover(to_device(blocks), fmt)
    ainv = _stored_inverse_blocks(blocks, lp)
    ai_e, ai_o = full_to_half(ainv, 0), full_to_half(ainv, 1)
    u_or, psi_or = link_as_stored(u, lp, reals), ROUND[sp](psi)
    for dag in (False, True):
        got = lat.unpack_spinor(lat.clover_apply(u_d, clv, x_d, fmt, dagger=dag), fmt).cpu().numpy()
        want = CL.apply_m_clover(u_or, psi_or, kappa, PH, ai_e, ai_o, dagger=dag)
        _check(got, want, sp, f"clover apply dagger={dag}")


@pytest.mark.parametrize("fmt_t", [("f64", "f64", 18), ("f32", "f32", 18), ("f16", "f16", 12)],
                         ids=["f64-18", "f32-18", "f16-12"])
def test_clover_apply_32_3x64_sampled(fmt_t):
    """The clover-type operator at the benchmark size (32^3x64, blocks
    1 + 0.3 X) in the launch configuration the benchmark times."""
    print(f"clover apply 32^3x64 sampled fmt={fmt_t}", flush=True)
    sp, lp, reals = fmt_t
    dims, kappa = (32, 32, 32, 64), 0.126
    fmt = Format(*fmt_t)
    lat = Lattice(dims, kappa, AP)
    u = cached_gauge(dims, 0.5, 201)
    blocks = inputs.gen_site_blocks(dims, 0.3, 207)
    psi = inputs.gen_spinor_half(dims, 202)
    u_d, x_d = lat.pack_gauge(to_device(u), fmt), lat.pack_spinor(to_device(psi), fmt)
    clv = lat.pack_clover(to_device(blocks), fmt)
    ainv_at = lambda x, y, z, t: _stored_inverse_blocks(blocks[t, z, y, x], lp)
    us, ps = _StoredLinks(u, lp, reals), _StoredHalf(psi, sp)
    sites = sample_sites(dims, 16, 14)
    for dag in (False, True):
        got = lat.unpack_spinor(lat.clover_apply(u_d, clv, x_d, fmt, dagger=dag), fmt).cpu().numpy()
        want = CL.apply_m_clover_at_sites(us, ps, kappa, PH, ainv_at, sites, dagger=dag)
        _check(got.reshape(-1, 4, 3)[sites], want, sp, f"clover apply dagger={dag}")
    del u_d, x_d, clv
    torch.cuda.empty_cache()
