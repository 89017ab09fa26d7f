"""The C ABI library without a GPU: it loads, exports every function the
header declares, passes its host-side index self-test, and rejects bad
arguments before making any HIP call."""
import ctypes as C
import os
import re

import pytest

from paper_2303_08609_amd import wilson_eo as W

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "wilson_eo.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w\s\*]*?\b(\w+)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("defined",)))


def test_header_functions_are_exported_and_bound():
    lib = W.load()
    names = _declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
        assert n in W.exported_names(), f"{n} not bound in wilson_eo.py"


def test_selftest():
    assert W.weo_selftest() == 0


def test_strerror():
    for code in (0, -1, -2, -3, -4, -5, -6, 1, 2):
        assert W.strerror(code) and W.strerror(code) != "unknown status code"
    assert W.strerror(-99) == "unknown status code"


def test_sizes():
    lat = W.make_lattice((32, 32, 32, 64), 0.126)
    f32 = W.make_format(W.WEO_F32, W.WEO_F32, W.WEO_LINK18)
    f32c = W.make_format(W.WEO_F32, W.WEO_F32, W.WEO_LINK12)
    f64 = W.make_format(W.WEO_F64)
    vh = 32 ** 3 * 64 // 2
    assert W.weo_gauge_bytes(lat, f32) == 8 * vh * 72
    assert W.weo_gauge_bytes(lat, f32c) == 8 * vh * 48
    assert W.weo_spinor_bytes(lat, f32, 1) == vh * 96
    assert W.weo_spinor_bytes(lat, f64, 12) == 12 * vh * 192
    hh = W.make_format(W.WEO_BF16, W.WEO_F16, W.WEO_LINK12)
    assert W.weo_format_supported(hh) == 1
    assert W.weo_gauge_bytes(lat, hh) == 8 * vh * 24
    assert W.weo_spinor_bytes(lat, hh, 1) == vh * 48


def test_unsupported_and_bad_formats():
    lat = W.make_lattice((4, 4, 4, 4), 0.1)
    assert W.weo_format_supported(W.make_format(W.WEO_F32, W.WEO_F64)) == 0
    assert W.weo_gauge_bytes(lat, W.make_format(W.WEO_F32, W.WEO_F64)) == 0
    bad = W.make_format(7, 0, 0)
    assert W.weo_spinor_bytes(lat, bad, 1) == 0


@pytest.mark.parametrize("dims", [(3, 4, 4, 4), (4, 4, 4, 0), (4, -2, 4, 4), (1, 1, 1, 1),
                                  (4096, 4096, 4096, 4096)])
def test_bad_dims(dims):
    lat = W.make_lattice(dims, 0.1)
    f = W.make_format(W.WEO_F32)
    assert W.weo_spinor_bytes(lat, f, 1) == 0
    rc = W.wilson_eo_apply(lat, f, 0, 256, 512, 1024, 2048, 1, None)
    assert rc == W.WEO_ERR_DIMS


def test_argument_validation_without_gpu():
    lat = W.make_lattice((4, 4, 4, 4), 0.1)
    f = W.make_format(W.WEO_F32)
    a, b, c, d = 1 << 20, 2 << 20, 3 << 20, 4 << 20     # fake aligned, disjoint
    # null and misaligned pointers
    assert W.wilson_eo_apply(lat, f, 0, None, b, c, d, 1, None) == W.WEO_ERR_ARG
    assert W.wilson_eo_apply(lat, f, 0, a + 8, b, c, d, 1, None) == W.WEO_ERR_ALIGN
    # bad flags and counts
    assert W.wilson_eo_apply(lat, f, 2, a, b, c, d, 1, None) == W.WEO_ERR_ARG
    assert W.wilson_eo_apply(lat, f, 0, a, b, c, d, 0, None) == W.WEO_ERR_ARG
    assert W.wilson_eo_apply(lat, f, 0, a, b, c, d, W.WEO_MAX_RHS + 1, None) == W.WEO_ERR_ARG
    assert W.wilson_eo_hop(lat, f, 2, 0, a, b, c, 1, None) == W.WEO_ERR_ARG
    # overlapping in/out
    assert W.wilson_eo_hop(lat, f, 1, 0, a, b, b + 256, 1, None) == W.WEO_ERR_ARG
    # unsupported combination and unknown enum
    assert W.wilson_eo_hop(lat, W.make_format(W.WEO_F32, W.WEO_F64), 1, 0, a, b, c, 1,
                           None) == W.WEO_ERR_FORMAT
    assert W.wilson_eo_hop(lat, W.make_format(9), 1, 0, a, b, c, 1, None) == W.WEO_ERR_ARG
    # null lattice / format
    assert W.wilson_eo_hop(None, f, 1, 0, a, b, c, 1, None) == W.WEO_ERR_ARG
    assert W.wilson_eo_hop(lat, None, 1, 0, a, b, c, 1, None) == W.WEO_ERR_ARG
    # non-finite kappa or phase
    lat_nan = W.make_lattice((4, 4, 4, 4), float("nan"))
    assert W.wilson_eo_apply(lat_nan, f, 0, a, b, c, d, 1, None) == W.WEO_ERR_ARG
    # pack: bad canonical precision, bad scale
    assert W.weo_pack_spinor(lat, f, 1, a, 5, 1.0, b, None) == W.WEO_ERR_ARG
    assert W.weo_pack_spinor(lat, f, 1, a, 0, float("inf"), b, None) == W.WEO_ERR_ARG
    assert W.weo_pack_gauge(lat, f, a, 0, None, None) == W.WEO_ERR_ARG


def test_python_raises_on_error_codes_and_warns_on_solver_status():
    with pytest.raises(W.WilsonEOError):
        W.check(W.WEO_ERR_ARG, "x")
    for st in (W.WEO_NOT_CONVERGED, W.WEO_BREAKDOWN):
        with pytest.warns(W.SolverWarning):
            assert W.check(st, "x") == st
    import warnings
    with warnings.catch_warnings():
        warnings.simplefilter("error")
        assert W.check(W.WEO_OK, "x") == W.WEO_OK


def test_autograd_solve_raises_on_unconverged_status(monkeypatch):
    """The autograd solve refuses a forward or adjoint solve that did not
    converge (else its gradients would be silently wrong).  The solver
    front end is replaced by one that reports WEO_NOT_CONVERGED, so no GPU is
    needed."""
    from paper_2303_08609_amd import autograd as AG
    from paper_2303_08609_amd.ops import Format

    def fake_cg(*args, **kw):
        return None, {"status": W.WEO_NOT_CONVERGED, "true_rel_resid": [0.5]}
    monkeypatch.setattr(AG, "cg", fake_cg)
    with pytest.raises(W.WilsonEOError) as e:
        AG._solve_normal(None, Format("f32", "f32", 18), None, None, None, 1e-10, False, maxiter=1)
    assert e.value.code == W.WEO_NOT_CONVERGED
    monkeypatch.setattr(AG, "cg", lambda *a, **k: ("x", {"status": W.WEO_OK, "true_rel_resid": [0.0]}))
    assert AG._solve_normal(None, Format("f32", "f32", 18), None, None, None, 1e-10, False)[0] == "x"


def test_face_sizes_and_validation_without_gpu():
    lat = W.make_lattice((16, 8, 12, 8), 0.126)
    lx, ly, lz, lt = 16, 8, 12, 8
    nfs = {0: ly * lz * lt // 2, 1: lx // 2 * lz * lt, 2: lx // 2 * ly * lt, 3: lx // 2 * ly * lz}
    for (sp, lp), cb in (((W.WEO_F64, W.WEO_F64), 16), ((W.WEO_F32, W.WEO_F32), 8),
                         ((W.WEO_F16, W.WEO_F16), 4), ((W.WEO_BF16, W.WEO_F16), 4)):
        f = W.make_format(sp, lp, W.WEO_LINK12)
        for mu, nf in nfs.items():
            assert W.weo_face_bytes(lat, f, mu, 1) == nf * 6 * cb
            assert W.weo_face_bytes(lat, f, mu, 12) == 12 * nf * 6 * cb
            assert W.weo_face_bytes(lat, f, mu, 0) == 0
        assert W.weo_face_bytes(lat, f, 4, 1) == 0 and W.weo_face_bytes(lat, f, -1, 1) == 0
    f = W.make_format(W.WEO_F32)
    a, b, c, d = 1 << 28, 2 << 28, 3 << 28, 4 << 28     # fake aligned, disjoint
    one = (C.c_double * 2)(1.0, 0.0)
    nan = (C.c_double * 2)(float("nan"), 0.0)
    for mu in range(4):
        assert W.wilson_eo_face_pack(lat, f, mu, 1, 0, a, b, c, c, 1, None) == W.WEO_ERR_ARG   # lo == hi
        assert W.wilson_eo_face_pack(lat, f, mu, 1, 0, a, b, b, d, 1, None) == W.WEO_ERR_ARG   # lo over in
        assert W.wilson_eo_face_pack(lat, f, mu, 2, 0, a, b, c, d, 1, None) == W.WEO_ERR_ARG
        assert W.wilson_eo_face_pack(lat, f, mu, 1, 0, a, b + 64, c, d, 1, None) == W.WEO_ERR_ALIGN
        assert W.wilson_eo_face_unpack(lat, f, mu, 1, 0, nan, one, 1.0, a, b, c, d, 1, None) == W.WEO_ERR_ARG
        assert W.wilson_eo_face_unpack(lat, f, mu, 1, 0, None, one, 1.0, a, b, c, d, 1, None) == W.WEO_ERR_ARG
        assert W.wilson_eo_face_unpack(lat, f, mu, 1, 0, one, one, float("inf"), a, b, c, d, 1,
                                       None) == W.WEO_ERR_ARG
        assert W.wilson_eo_face_unpack(lat, f, mu, 1, 0, one, one, 1.0, a, b, c, b, 1, None) == W.WEO_ERR_ARG
    assert W.wilson_eo_face_pack(lat, f, 4, 1, 0, a, b, c, d, 1, None) == W.WEO_ERR_ARG
    assert W.wilson_eo_face_unpack(lat, f, -1, 1, 0, one, one, 1.0, a, b, c, d, 1, None) == W.WEO_ERR_ARG


def test_header_constants_match_the_binding():
    text = open(HEADER).read()
    defs = dict(re.findall(r"^#define\s+(WEO_\w+)\s+(-?\d+)", text, flags=re.M))
    assert len(defs) >= 10
    for name, val in defs.items():
        assert getattr(W, name) == int(val), name


def test_clover_sizes_and_validation_without_gpu():
    lat = W.make_lattice((8, 8, 8, 8), 0.126)
    vh = 8 ** 4 // 2
    for (sp, lp, lf), cb in (((W.WEO_F64, W.WEO_F64, W.WEO_LINK18), 16), ((W.WEO_F32, W.WEO_F32, W.WEO_LINK12), 8),
                             ((W.WEO_BF16, W.WEO_F16, W.WEO_LINK12), 4)):
        # both parities, two blocks of 18 complex (real diagonal in pairs + lower triangle)
        assert W.weo_clover_bytes(lat, W.make_format(sp, lp, lf)) == 2 * 2 * vh * 18 * cb
    f = W.make_format(W.WEO_F32)
    a, b, c, d = 1 << 28, 2 << 28, 3 << 28, 4 << 28
    assert W.weo_pack_clover(lat, f, a, W.WEO_F64, 2, b, None) == W.WEO_ERR_ARG        # invert flag
    assert W.weo_pack_clover(lat, f, a, 7, 1, b, None) == W.WEO_ERR_ARG                # canonical precision
    assert W.weo_pack_clover(lat, f, a, W.WEO_F64, 1, a, None) == W.WEO_ERR_ARG        # overlap
    assert W.wilson_eo_clover_site(lat, f, 2, a, b, None, 1.0, c, 1, None) == W.WEO_ERR_ARG
    assert W.wilson_eo_clover_site(lat, f, 0, a, b, None, 1.0, b, 1, None) == W.WEO_ERR_ARG   # in == out
    assert W.wilson_eo_clover_site(lat, f, 0, a + 16, b, None, 1.0, c, 1, None) == W.WEO_ERR_ALIGN
    assert W.wilson_eo_clover_hop(lat, f, 1, 0, a, b, c, None, float("nan"), d, 1, None) == W.WEO_ERR_ARG
    assert W.wilson_eo_clover_apply(lat, f, 0, a, b, c, c, d, 1, None) == W.WEO_ERR_ARG       # in == out
    assert W.wilson_eo_clover_apply(lat, f, 0, a, None, c, d, b, 1, None) == W.WEO_ERR_ARG


def test_block_cg_parameters_without_gpu():
    """The block method's workspace: every level vector plus its Gram and
    update partials; FP64 or FP32 vectors only (FP32 inner for a mixed solve)."""
    lat = W.make_lattice((8, 8, 8, 16), 0.126)
    f64, f32 = W.make_format(W.WEO_F64), W.make_format(W.WEO_F32)

    def params(method, nrhs=12, mixed=0, inner=None, op=W.WEO_OP_M):
        p = W.weo_solver_params()
        p.op, p.nrhs, p.tol, p.maxiter, p.check_every = op, nrhs, 1e-10, 100, 10
        p.mixed, p.inner_tol, p.max_outer, p.method = mixed, 1e-3, 10, method
        if inner is not None:
            p.inner = inner
        return p
    cg_b = W.wilson_eo_cg_workspace_bytes(lat, f64, params(W.WEO_SOLVER_CG))
    blk = W.wilson_eo_cg_workspace_bytes(lat, f64, params(W.WEO_SOLVER_BLOCK_CG))
    assert cg_b > 0 and blk > cg_b
    for op in (W.WEO_OP_M, W.WEO_OP_MDAGM, W.WEO_OP_DW):
        assert W.wilson_eo_cg_workspace_bytes(lat, f32, params(W.WEO_SOLVER_BLOCK_CG, op=op)) > 0
    assert W.wilson_eo_cg_workspace_bytes(lat, f64, params(W.WEO_SOLVER_BLOCK_CG, mixed=1, inner=f32)) > 0
    f16 = W.make_format(W.WEO_F16, W.WEO_F16, W.WEO_LINK12)
    assert W.wilson_eo_cg_workspace_bytes(lat, f64, params(W.WEO_SOLVER_BLOCK_CG, mixed=1, inner=f16)) == 0
    assert W.wilson_eo_cg_workspace_bytes(lat, f64, params(W.WEO_SOLVER_CG, mixed=1, inner=f16)) > 0
    assert W.wilson_eo_cg_workspace_bytes(lat, f64, params(4)) == 0
    # D_W solves: one precision level, or defect correction around FP32 inner
    # solves (FP16 / BF16 inner spinors are refused for D_W)
    for m in (W.WEO_SOLVER_CG, W.WEO_SOLVER_BICGSTAB, W.WEO_SOLVER_BLOCK_CG):
        assert W.wilson_eo_cg_workspace_bytes(lat, f64, params(m, mixed=1, inner=f32, op=W.WEO_OP_DW)) > 0
        assert W.wilson_eo_cg_workspace_bytes(lat, f64, params(m, mixed=1, inner=f16, op=W.WEO_OP_DW)) == 0
        assert W.wilson_eo_cg_workspace_bytes(lat, f64, params(m, op=W.WEO_OP_DW)) > 0


def test_sap_parameters_without_gpu():
    """SAP and SAP-GCR argument checks before any device work: block extents
    must divide the lattice into 1 or an even number of blocks per direction
    with at most 256 sites each; FP32 spinors and links for the
    preconditioner; D_W only; restart length 1..16."""
    lat = W.make_lattice((8, 8, 8, 16), 0.126)
    f32, f64 = W.make_format(W.WEO_F32), W.make_format(W.WEO_F64)
    f32l12 = W.make_format(W.WEO_F32, W.WEO_F32, W.WEO_LINK12)
    f16 = W.make_format(W.WEO_F16, W.WEO_F16, W.WEO_LINK12)
    full = 8 * 8 * 8 * 16 * 96                       # one FP32 full field
    assert W.wilson_eo_sap_workspace_bytes(lat, f32, 2) == 3 * 2 * full
    assert W.wilson_eo_sap_workspace_bytes(lat, f64, 1) == 0
    assert W.wilson_eo_sap_workspace_bytes(lat, f16, 1) == 0
    a, b, c, d = 1 << 28, 2 << 28, 3 << 28, 4 << 28     # fake aligned, disjoint: rejected first

    def sp(block, ncy=2, nmr=4):
        q = W.weo_sap_params()
        for i in range(4):
            q.block[i] = block[i]
        q.ncy, q.nmr = ncy, nmr
        return q
    ws = 3 * full
    assert W.wilson_eo_sap(lat, f32, sp((3, 4, 4, 4)), a, b, c, d, ws, 1, None) == W.WEO_ERR_ARG
    assert W.wilson_eo_sap(lat, f32, sp((8, 8, 8, 16)), a, b, c, d, ws, 1, None) == W.WEO_ERR_ARG  # 8192 sites
    assert W.wilson_eo_sap(lat, f32, sp((4, 4, 4, 8)), a, b, c, d, ws, 1, None) == W.WEO_ERR_ARG   # 512 sites
    lat6 = W.make_lattice((12, 8, 8, 16), 0.126)
    assert W.wilson_eo_sap(lat6, f32, sp((4, 4, 4, 4)), a, b, c, d, 1 << 30, 1, None) == W.WEO_ERR_ARG  # 3 blocks
    assert W.wilson_eo_sap(lat, f32, sp((4, 4, 4, 4), ncy=0), a, b, c, d, ws, 1, None) == W.WEO_ERR_ARG
    assert W.wilson_eo_sap(lat, f32, sp((4, 4, 4, 4), nmr=65), a, b, c, d, ws, 1, None) == W.WEO_ERR_ARG
    assert W.wilson_eo_sap(lat, f64, sp((4, 4, 4, 4)), a, b, c, d, ws, 1, None) == W.WEO_ERR_FORMAT
    assert W.wilson_eo_sap(lat, f32, sp((4, 4, 4, 4)), a, b, c, d, ws - 256, 1, None) == W.WEO_ERR_WORKSPACE
    assert W.wilson_eo_sap(lat, f32, sp((4, 4, 4, 4)), a, b, b, d, ws, 1, None) == W.WEO_ERR_ARG      # psi = eta

    def params(mixed=0, inner=None, op=W.WEO_OP_DW, nkv=8, block=(4, 4, 4, 4)):
        p = W.weo_solver_params()
        p.op, p.nrhs, p.tol, p.maxiter, p.check_every = op, 2, 1e-10, 100, 10
        p.mixed, p.inner_tol, p.max_outer, p.method = mixed, 1e-3, 10, W.WEO_SOLVER_SAP_GCR
        p.sap = sp(block)
        p.gcr_nkv = nkv
        if inner is not None:
            p.inner = inner
        return p
    assert W.wilson_eo_cg_workspace_bytes(lat, f32, params()) > 0
    assert W.wilson_eo_cg_workspace_bytes(lat, f32l12, params()) > 0
    assert W.wilson_eo_cg_workspace_bytes(lat, f64, params(inner=f32)) > 0          # FP32 preconditioner
    assert W.wilson_eo_cg_workspace_bytes(lat, f64, params(inner=f64)) == 0
    assert W.wilson_eo_cg_workspace_bytes(lat, f64, params(mixed=1, inner=f32l12)) > 0
    assert W.wilson_eo_cg_workspace_bytes(lat, f64, params(mixed=1, inner=f16)) == 0
    assert W.wilson_eo_cg_workspace_bytes(lat, f32, params(op=W.WEO_OP_M)) == 0
    assert W.wilson_eo_cg_workspace_bytes(lat, f32, params(nkv=0)) == 0
    assert W.wilson_eo_cg_workspace_bytes(lat, f32, params(nkv=17)) == 0
    assert W.wilson_eo_cg_workspace_bytes(lat, f32, params(block=(3, 4, 4, 4))) == 0


def test_noalloc_apply_rejects_oversize_before_device_work():
    """The no-allocation apply refuses an intermediate field larger than its
    device array, and bad counts, before any HIP call (fake pointers)."""
    # 32^3x64 FP64: 192 MiB per field, beyond the 128 MiB array
    lat = W.make_lattice((32, 32, 32, 64), 0.126)
    f64 = W.make_format(W.WEO_F64)
    a, b, c = 1 << 28, 2 << 28, 3 << 28           # never touched: rejected first
    assert W.wilson_eo_apply_noalloc(lat, f64, 0, a, b, c, 1, None) == W.WEO_ERR_WORKSPACE
    f32 = W.make_format(W.WEO_F32)
    assert W.wilson_eo_apply_noalloc(lat, f32, 0, a, b, c, 2, None) == W.WEO_ERR_WORKSPACE
    assert W.wilson_eo_apply_noalloc(lat, f32, 0, a, b, c, 0, None) == W.WEO_ERR_ARG
