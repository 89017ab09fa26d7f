"""Block CG (O'Leary 1980, Dubrulle's QR form) on the GPU against the oracle:
iterate by iterate on ragged lattices (M X = B through the normal equations,
A X = B for A = M^dag M), converged solutions against the oracle's residuals
and a dense solve, FP32, mixed-precision defect correction around FP32 block
inner solves, clover-type blocks, twelve point sources, and the degenerate
cases (rank-deficient block, zero source, converged start)."""
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


def _ops(u, kappa):
    m = lambda v: W.apply_m(u, v, kappa, PH)
    md = lambda v: W.apply_m(u, v, kappa, PH, dagger=True)
    return m, md


@pytest.mark.parametrize("dims,nrhs", [((10, 6, 2, 6), 3), ((6, 2, 2, 6), 5)], ids=["10x6x2x6-3", "6x2x2x6-5"])
def test_block_cg_iterates_match_oracle_normal_equations(dims, nrhs):
    """FP64, M X = B: after k iterations the GPU block equals the oracle's
    (the chunk counts of these lattices leave ragged tails in every kernel)."""
    print(f"block cg iterates M dims={dims} nrhs={nrhs}", flush=True)
    kappa = 0.125
    u = inputs.gen_gauge(dims, 0.4, 150)
    b = inputs.gen_spinor_half(dims, 151, nrhs=nrhs)
    lat = Lattice(dims, kappa, AP)
    u_p, b_p = lat.pack_gauge(to_device(u), F64), lat.pack_spinor(to_device(b), F64)
    m, md = _ops(u, kappa)
    for k in (1, 2, 5):
        x_p, info = cg(lat, F64, u_p, b_p, nrhs=nrhs, tol=1e-30, maxiter=k, method="blockcg")
        assert info["iters"] == k and info["status"] == WE.WEO_NOT_CONVERGED
        xo, it, hist = S.block_cg(None, list(b), 1e-30, k, apply_m=m, apply_mdag=md)
        x = lat.unpack_spinor(x_p, F64, nrhs=nrhs).cpu().numpy()
        for j in range(nrhs):
            assert rel_err(x[j], xo[j]) < 1e-11, (k, j)
        # the library's recomputed residuals are the oracle's
        res = [S.rel_resid(m, xo[j], b[j]) for j in range(nrhs)]
        assert np.allclose(info["true_rel_resid"], res, rtol=1e-9, atol=0)


def test_block_cg_iterates_match_oracle_mdagm():
    """FP64, (M^dag M) X = B directly: iterates and the converged solution."""
    print("block cg iterates MdagM", flush=True)
    dims, kappa, nrhs = (6, 2, 2, 6), 0.125, 4
    u = inputs.gen_gauge(dims, 0.4, 160)
    b = inputs.gen_spinor_half(dims, 161, nrhs=nrhs)
    lat = Lattice(dims, kappa, AP)
    u_p, b_p = lat.pack_gauge(to_device(u), F64), lat.pack_spinor(to_device(b), F64)
    m, md = _ops(u, kappa)
    a = lambda v: md(m(v))
    for k in (1, 3, 6):
        x_p, info = cg(lat, F64, u_p, b_p, nrhs=nrhs, op="MdagM", tol=1e-30, maxiter=k, method="blockcg")
        xo, _, _ = S.block_cg(a, list(b), 1e-30, k)
        x = lat.unpack_spinor(x_p, F64, nrhs=nrhs).cpu().numpy()
        for j in range(nrhs):
            assert rel_err(x[j], xo[j]) < 1e-11, (k, j)
    x_p, info = cg(lat, F64, u_p, b_p, nrhs=nrhs, op="MdagM", tol=1e-12, maxiter=500, method="blockcg")
    assert info["status"] == WE.WEO_OK
    x = lat.unpack_spinor(x_p, F64, nrhs=nrhs).cpu().numpy()
    for j in range(nrhs):
        assert S.rel_resid(a, x[j], b[j]) <= 1e-12


def test_block_cg_fp64_twelve_point_sources():
    """12 point + noise sources on 8^3x16 to 1e-10: every solution passes the
    oracle's residual check, and the block takes no more iterations than the
    12 separate CGLS recurrences batched together (on these smooth links the
    low end of the spectrum is dense, so the block gains little: 33 and 33)."""
    print("block cg 12 point sources 8^3x16", flush=True)
    dims, kappa = (8, 8, 8, 16), 0.126
    u = inputs.gen_gauge(dims, 0.5, 170)
    b = inputs.gen_point_noise_sources(dims, 171)
    lat = Lattice(dims, kappa, AP)
    u_p, b_p = lat.pack_gauge(to_device(u), F64), lat.pack_spinor(to_device(b), F64)
    m, _ = _ops(u, kappa)
    x_p, info = cg(lat, F64, u_p, b_p, nrhs=12, tol=1e-10, maxiter=2000, method="blockcg")
    assert info["status"] == WE.WEO_OK
    x = lat.unpack_spinor(x_p, F64, nrhs=12).cpu().numpy()
    for j in range(12):
        r = S.rel_resid(m, x[j], b[j])
        assert r <= 1e-10 and abs(r - info["true_rel_resid"][j]) <= 1e-12 * max(1.0, r / 1e-10), j
    _, info_cg = cg(lat, F64, u_p, b_p, nrhs=12, tol=1e-10, maxiter=2000, check_every=1)
    assert info["iters"] <= info_cg["iters"], (info["iters"], info_cg["iters"])


def test_block_cg_fp32_and_dw():
    """FP32 vectors to 1e-6 (16^3x32, 4 rhs), and FP64 on the unpreconditioned
    D_W against a dense solve."""
    print("block cg fp32 16^3x32 and D_W 4^4", flush=True)
    dims, kappa = (16, 16, 16, 32), 0.126
    u = cached_gauge(dims, 0.5, 201)
    b = inputs.gen_spinor_half(dims, 180, nrhs=4)
    lat = Lattice(dims, kappa, AP)
    x_p, info = cg(lat, F32, lat.pack_gauge(to_device(u), F32), lat.pack_spinor(to_device(b), F32), nrhs=4,
                   tol=1e-6, maxiter=2000, method="blockcg")
    assert info["status"] == WE.WEO_OK, info
    x = lat.unpack_spinor(x_p, F32, nrhs=4).cpu().numpy()
    m, _ = _ops(u, kappa)
    for j in range(4):
        assert S.rel_resid(m, x[j], ROUND["f32"](b[j])) <= 1.2e-6, j
    from tests.test_gpu_solver import _full_field, _unpack_full
    dims, kappa = (4, 4, 4, 4), 0.125
    lat = Lattice(dims, kappa, AP)
    u = inputs.gen_gauge(dims, 0.3, 101)
    eta = inputs.gen_spinor_full(dims, 181)
    x, info = cg(lat, F64, lat.pack_gauge(to_device(u), F64), _full_field(lat, F64, eta), op="DW", tol=1e-13,
                 maxiter=2000, method="blockcg")
    assert info["status"] == WE.WEO_OK
    xi = np.linalg.solve(W.dense_dirac_wilson(u, kappa, PH), eta.reshape(-1)).reshape(eta.shape)
    assert rel_err(_unpack_full(lat, F64, x), xi) < 1e-11


def test_block_cg_mixed_defect_correction_12rhs():
    """FP64 defect correction around FP32 block CG inner solves (FP32 12-real
    links), 12 sources on 8^3x16 to 1e-10 against the oracle's residuals."""
    print("block cg mixed 12 rhs", flush=True)
    dims, kappa = (8, 8, 8, 16), 0.126
    u = inputs.gen_gauge(dims, 0.5, 170)
    b = inputs.gen_point_noise_sources(dims, 171)
    lat = Lattice(dims, kappa, AP)
    fi = Format("f32", "f32", 12)
    ud = to_device(u)
    x_p, info = cg(lat, F64, lat.pack_gauge(ud, F64), lat.pack_spinor(to_device(b), F64), nrhs=12, tol=1e-10,
                   inner=fi, u_inner=lat.pack_gauge(ud, fi), inner_tol=1e-4, max_outer=30, maxiter=5000,
                   method="blockcg")
    assert info["status"] == WE.WEO_OK, info
    x = lat.unpack_spinor(x_p, F64, nrhs=12).cpu().numpy()
    m, _ = _ops(u, kappa)
    for j in range(12):
        assert S.rel_resid(m, x[j], b[j]) <= 1e-10, j
    # FP16 inner vectors are not offered for the block method
    with pytest.raises(WE.WilsonEOError):
        f16 = Format("f16", "f16", 12)
        cg(lat, F64, lat.pack_gauge(ud, F64), lat.pack_spinor(to_device(b), F64), nrhs=12, tol=1e-10,
           inner=f16, u_inner=lat.pack_gauge(ud, f16), method="blockcg", maxiter=1)


def test_block_cg_clover():
    print("block cg clover", flush=True)
    from oracle import clover as CL
    from oracle.lattice import full_to_half
    dims, kappa = (4, 4, 4, 8), 0.124
    lat = Lattice(dims, kappa, AP)
    u = inputs.gen_gauge(dims, 0.4, 190)
    blocks = inputs.gen_site_blocks(dims, 0.3, 191)
    ainv = np.linalg.inv(CL.blocks_to_dirac(blocks))
    b = inputs.gen_spinor_half(dims, 192, nrhs=3)
    x_p, info = cg(lat, F64, lat.pack_gauge(to_device(u), F64), lat.pack_spinor(to_device(b), F64), nrhs=3,
                   tol=1e-11, maxiter=1000, method="blockcg", clover=lat.pack_clover(to_device(blocks), F64))
    assert info["status"] == WE.WEO_OK
    x = lat.unpack_spinor(x_p, F64, nrhs=3).cpu().numpy()
    ai_e, ai_o = full_to_half(ainv, 0), full_to_half(ainv, 1)
    for j in range(3):
        r = S.rel_resid(lambda v: CL.apply_m_clover(u, v, kappa, PH, ai_e, ai_o), x[j], b[j])
        assert r <= 1e-11, j


@pytest.mark.parametrize("op", ["M", "MdagM"])
def test_block_cg_deflates_dependent_sources(op):
    """Sources [b0, b1, b0, b0 + 2 b1]: the residual block has rank 2 and the
    dependent columns are deflated.  After 1, 2 and 4 iterations every column
    equals the oracle's (which deflates likewise, FP64 bar 1e-11), the twin
    column equals its twin and the combination the same combination; run to
    1e-11 every column meets the oracle's residual."""
    print(f"block cg deflation op={op}", flush=True)
    dims, kappa = (4, 4, 2, 4), 0.125
    u = inputs.gen_gauge(dims, 0.3, 101)
    lat = Lattice(dims, kappa, AP)
    u_p = lat.pack_gauge(to_device(u), F64)
    b2 = inputs.gen_spinor_half(dims, 200, nrhs=2)
    b = np.stack([b2[0], b2[1], b2[0], b2[0] + 2.0 * b2[1]])
    b_p = lat.pack_spinor(to_device(b), F64)
    m, md = _ops(u, kappa)
    for k in (1, 2, 4):
        x_p, info = cg(lat, F64, u_p, b_p, nrhs=4, op=op, tol=1e-30, maxiter=k, method="blockcg")
        assert info["iters"] == k and info["status"] == WE.WEO_NOT_CONVERGED, info
        x = lat.unpack_spinor(x_p, F64, nrhs=4).cpu().numpy()
        if op == "M":
            xo, _, _ = S.block_cg(None, list(b), 1e-30, k, apply_m=m, apply_mdag=md)
        else:
            xo, _, _ = S.block_cg(lambda v: md(m(v)), list(b), 1e-30, k)
        for j in range(4):
            assert rel_err(x[j], xo[j]) < 1e-11, (k, j)
        assert rel_err(x[2], x[0]) < 1e-12 and rel_err(x[3], x[0] + 2.0 * x[1]) < 1e-12
    x_p, info = cg(lat, F64, u_p, b_p, nrhs=4, op=op, tol=1e-11, maxiter=500, method="blockcg")
    assert info["status"] == WE.WEO_OK, info
    x = lat.unpack_spinor(x_p, F64, nrhs=4).cpu().numpy()
    a = m if op == "M" else (lambda v: md(m(v)))
    for j in range(4):
        assert S.rel_resid(a, x[j], b[j]) <= 1.05e-11, j


def test_block_cg_degenerate_cases():
    """A zero source and a source whose start already solves it stay out of
    the block; the others converge as a block of the rest."""
    print("block cg degenerate", flush=True)
    dims, kappa = (4, 4, 2, 4), 0.125
    u = inputs.gen_gauge(dims, 0.3, 101)
    lat = Lattice(dims, kappa, AP)
    u_p = lat.pack_gauge(to_device(u), F64)
    b = inputs.gen_spinor_half(dims, 201, nrhs=3)
    b[1] = 0
    m, _ = _ops(u, kappa)
    x_p, info = cg(lat, F64, u_p, lat.pack_spinor(to_device(b), F64), nrhs=3, tol=1e-11, maxiter=500,
                   method="blockcg")
    assert info["status"] == WE.WEO_OK
    x = lat.unpack_spinor(x_p, F64, nrhs=3).cpu().numpy()
    assert np.all(x[1] == 0)
    for j in (0, 2):
        assert S.rel_resid(m, x[j], b[j]) <= 1e-11
    # a start that already solves rhs 0 (the previous solution) leaves it as is
    x0 = x_p.clone()
    b[1] = inputs.gen_spinor_half(dims, 202)
    x2_p, info = cg(lat, F64, u_p, lat.pack_spinor(to_device(b), F64), nrhs=3, tol=1e-9, maxiter=500,
                    method="blockcg", x0=x0)
    assert info["status"] == WE.WEO_OK
    x2 = lat.unpack_spinor(x2_p, F64, nrhs=3).cpu().numpy()
    assert np.array_equal(x2[0], x[0]) and np.array_equal(x2[2], x[2])
    assert S.rel_resid(m, x2[1], b[1]) <= 1e-9


@pytest.mark.parametrize("fmt_t,nrhs", [(("f64", "f64", 18), 16), (("f64", "f64", 12), 13), (("f32", "f32", 18), 16),
                                        (("f32", "f32", 12), 7), (("f64", "f64", 18), 1)],
                         ids=["f64-16", "f64l12-13", "f32-16", "f32l12-7", "f64-1"])
def test_block_cg_every_kernel_bucket(fmt_t, nrhs):
    """Block sizes in every compiled bucket of the block kernels (4, 8, 12,
    16; exact and partial), FP64 and FP32 vectors: the iterate after 3 steps
    equals the oracle's (M X = B through the normal equations).  Bars: FP64
    1e-11; FP32 2e-5, since three steps of the recurrence build their s x s
    factors from FP32 vectors (about 20 roundings of 6e-8 each, amplified by
    the conditioning of the Gram matrices)."""
    print(f"block cg bucket fmt={fmt_t} nrhs={nrhs}", flush=True)
    from tests._helpers import link_as_stored
    sp, lp, reals = fmt_t
    fmt = Format(*fmt_t)
    dims, kappa = (6, 4, 2, 6), 0.125
    u = inputs.gen_gauge(dims, 0.4, 210)
    b = inputs.gen_spinor_half(dims, 211, nrhs=nrhs)
    lat = Lattice(dims, kappa, AP)
    x_p, info = cg(lat, fmt, lat.pack_gauge(to_device(u), fmt), lat.pack_spinor(to_device(b), fmt), nrhs=nrhs,
                   tol=1e-30, maxiter=3, method="blockcg")
    assert info["iters"] == 3
    ul = link_as_stored(u, lp, reals)
    m, md = _ops(ul, kappa)
    xo, _, _ = S.block_cg(None, list(ROUND[sp](b)), 1e-30, 3, apply_m=m, apply_mdag=md)
    x = lat.unpack_spinor(x_p, fmt, nrhs=nrhs).cpu().numpy().reshape(nrhs, -1)
    tol = 1e-11 if sp == "f64" else 2e-5
    for j in range(nrhs):
        assert rel_err(x[j], xo[j]) < tol, j


@pytest.mark.parametrize("inner,method", [(("f16", "f16", 12), "bicgstab"), (("f32", "f32", 12), "blockcg")],
                         ids=["f16l12-bicgstab", "f32l12-blockcg"])
def test_twelve_source_solve_32_3x64_sampled(inner, method):
    """The benchmark's 12-source solves at full size (32^3x64, point + noise
    sources, links exp(0.5 i H), FP64 defect correction to 1e-10): the
    library's FP64 true residuals meet the tolerance, and the oracle's M x at
    sampled sites (faces, corners, the source's neighbours, random) differs
    from b there by no more than the residual bound allows."""
    print(f"12-source solve 32^3x64 inner={inner} method={method}", flush=True)
    from tests.test_gpu_apply import _sample_sites
    dims, kappa = (32, 32, 32, 64), 0.126
    lat = Lattice(dims, kappa, AP)
    u = cached_gauge(dims, 0.5, 401)
    b = inputs.gen_point_noise_sources(dims, 406)
    fi = Format(*inner)
    ud = to_device(u)
    x_p, info = cg(lat, F64, lat.pack_gauge(ud, F64), lat.pack_spinor(to_device(b), F64), nrhs=12, tol=1e-10,
                   inner=fi, u_inner=lat.pack_gauge(ud, fi), inner_tol=1e-5 if inner[0] == "f32" else 1e-3,
                   max_outer=100, maxiter=50000, method=method)
    assert info["status"] == WE.WEO_OK, info
    assert max(info["true_rel_resid"][:12]) <= 1e-10
    x = lat.unpack_spinor(x_p, F64, nrhs=12).cpu().numpy().reshape(12, -1, 4, 3)
    del x_p
    sites = _sample_sites(dims, 12, 9)
    for r in range(12):
        xr = x[r].reshape(b[r].shape)
        mx = W.apply_m_at_sites(u, xr, kappa, PH, sites)
        br = b[r].reshape(-1, 4, 3)[sites]
        assert np.linalg.norm(mx - br) <= 1e-10 * np.linalg.norm(b[r]), r
        # relative to b at the sampled sites themselves (the origin, where the
        # point part of b sits, left out): the global relative residual 1e-10
        # with room for an uneven spread over the sites
        rest = [i for i, s in enumerate(sites) if s != 0]
        assert np.linalg.norm((mx - br)[rest]) <= 2e-9 * np.linalg.norm(br[rest]), r
        # and the sampled solution is not trivially small
        assert np.linalg.norm(x[r][sites]) > 0.1 * np.linalg.norm(br)


def test_block_cg_mixed_mdagm_and_dw_fp16_rejected():
    """FP64 defect correction around FP32 block inner solves for M^dag M X = B
    (4 sources) to 1e-10 against the oracle's residuals; on D_W (full fields)
    defect correction with FP16 inner spinors is refused (the FP32 case is
    tested with the other D_W solves)."""
    print("block cg mixed MdagM; D_W mixed FP16 rejected", flush=True)
    from tests.test_gpu_solver import _full_field
    dims, kappa = (6, 4, 4, 8), 0.125
    lat = Lattice(dims, kappa, AP)
    u = inputs.gen_gauge(dims, 0.4, 220)
    ud = to_device(u)
    u64, u32 = lat.pack_gauge(ud, F64), lat.pack_gauge(ud, F32)
    b = inputs.gen_spinor_half(dims, 221, nrhs=4)
    x_p, info = cg(lat, F64, u64, lat.pack_spinor(to_device(b), F64), nrhs=4, op="MdagM", tol=1e-10, inner=F32,
                   u_inner=u32, inner_tol=1e-5, max_outer=30, maxiter=5000, method="blockcg")
    assert info["status"] == WE.WEO_OK, info
    m, md = _ops(u, kappa)
    x = lat.unpack_spinor(x_p, F64, nrhs=4).cpu().numpy()
    for j in range(4):
        assert S.rel_resid(lambda v: md(m(v)), x[j], b[j]) <= 1e-10, j
    bf = _full_field(lat, F64, inputs.gen_spinor_full(dims, 222))
    f16 = Format("f16", "f16", 12)
    u16 = lat.pack_gauge(ud, f16)
    for meth in ("cg", "blockcg"):
        with pytest.raises(WE.WilsonEOError):
            cg(lat, F64, u64, bf, op="DW", tol=1e-10, inner=f16, u_inner=u16, maxiter=10, method=meth)


@pytest.mark.parametrize("fmt,nrhs", [(F64, 3), (F64, 12), (F32, 7), (F32, 16)],
                         ids=["f64-3", "f64-12", "f32-7", "f32-16"])
def test_gram_on_matrix_cores_equals_cell_kernel(monkeypatch, fmt, nrhs):
    """The Gram matrices of block CG computed on the FP64 matrix cores
    (WEO_GRAM=mfma) and by the cell kernel on the vector units (the default)
    give the same block CG iterates to FP64 rounding (one and two 16-column
    tiles, the symmetric and the general product); both agree with the
    oracle's iterate."""
    print(f"gram mfma vs valu fmt={fmt} nrhs={nrhs}", flush=True)
    dims, kappa = (6, 4, 2, 6), 0.125
    u = inputs.gen_gauge(dims, 0.4, 170)
    b = inputs.gen_spinor_half(dims, 171, nrhs=nrhs)
    lat = Lattice(dims, kappa, AP)
    u_p, b_p = lat.pack_gauge(to_device(u), fmt), lat.pack_spinor(to_device(b), fmt)
    xs = {}
    for mode in ("mfma", "valu"):
        if mode == "mfma":
            monkeypatch.setenv("WEO_GRAM", "mfma")
        else:
            monkeypatch.delenv("WEO_GRAM", raising=False)
        x_p, info = cg(lat, fmt, u_p, b_p, nrhs=nrhs, tol=1e-30, maxiter=3, method="blockcg")
        assert info["iters"] == 3, (mode, info)
        xs[mode] = lat.unpack_spinor(x_p, fmt, nrhs=nrhs).cpu().numpy()
    monkeypatch.delenv("WEO_GRAM", raising=False)
    tol = 1e-12 if fmt.spinor == "f64" else 1e-5
    sp = fmt.spinor
    m, md = _ops(u if sp == "f64" else ROUND["f32"](u), kappa)
    xo, _, _ = S.block_cg(None, list(ROUND[sp](b)), 1e-30, 3, apply_m=m, apply_mdag=md)
    for j in range(nrhs):
        assert rel_err(xs["mfma"][j], xs["valu"][j]) < tol, j
        assert rel_err(xs["mfma"][j], xo[j]) < (1e-11 if sp == "f64" else 2e-5), j
