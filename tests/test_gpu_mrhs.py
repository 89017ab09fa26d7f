"""Multi right-hand-side hops against the oracle, for every launch shape the
autotuner can pick (forced one at a time) and for the tuned choice: 12
sources, several formats, a ragged lattice, both parities and dagger."""
import numpy as np
import pytest

from oracle import wilson as W
from paper_2303_08609_amd import inputs
from paper_2303_08609_amd import wilson_eo as WE
from paper_2303_08609_amd.ops import Format, Lattice, to_device
from tests._helpers import AP, ROUND, link_as_stored, rel_err

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-6, "f16": 2e-3, "bf16": 1e-2}
SHAPES = [(1, 0, 0, 0, 0)] + [(d, s, p, bz, 0) for d in (-1, -2, -3, -4) for s in (64, 128, 256) for p in (0, 1)
                              for bz in (0, 2)] + [(nr, s, p, bz, sp) for nr in (2, 3, 4, 6) for s in (64, 128, 256)
                              for p in (0, 1) for bz in (0, 2) for sp in (0, 1)]


def _setup(dims, fmt_t, nrhs, seed=700):
    sp, lp, reals = fmt_t
    fmt = Format(sp, lp, reals)
    lat = Lattice(dims, 0.126, AP)
    u = inputs.gen_gauge(dims, 0.5, seed)
    psi = inputs.gen_spinor_half(dims, seed + 1, nrhs=nrhs)
    return (lat, fmt, lat.pack_gauge(to_device(u), fmt), lat.pack_spinor(to_device(psi), fmt),
            link_as_stored(u, lp, reals), ROUND[sp](psi))


@pytest.fixture(autouse=True)
def _reset_shape():
    yield
    WE.weo_set_mrhs_shape(0, 0, 0, 0, 0)


@pytest.mark.parametrize("fmt_t", [("f32", "f32", 18), ("f64", "f64", 12), ("bf16", "f16", 12)],
                         ids=["f32-18", "f64-12", "bf16-12"])
@pytest.mark.parametrize("dims", [(6, 4, 4, 10), (16, 8, 4, 6)], ids=["ragged", "strips"])
def test_every_shape_matches_oracle(fmt_t, dims):
    # 6x4x4x10: V/2 = 480, a ragged last workgroup; 16x8x4x6: 64 half sites
    # per (z, t) plane, so the z-strip schedules are taken
    nrhs = 12
    print(f"mrhs shapes fmt={fmt_t} dims={dims}", flush=True)
    lat, fmt, u_d, x_d, u_o, psi_o = _setup(dims, fmt_t, nrhs)
    ph = np.array(AP, dtype=np.complex128)
    want = [W.hop_eo(u_o, psi_o[r], 0, ph) for r in range(nrhs)]
    want_dag = [W.hop_eo(u_o, psi_o[r], 0, ph, dagger=True) for r in range(nrhs)]
    for shape in SHAPES:
        assert WE.weo_set_mrhs_shape(*shape) == WE.WEO_OK
        for dag, ref in ((False, want), (True, want_dag)):
            out = lat.hop(u_d, x_d, fmt, out_parity=1, dagger=dag, nrhs=nrhs)
            got = lat.unpack_spinor(out, fmt, nrhs=nrhs).cpu().numpy()
            for r in range(nrhs):
                assert rel_err(got[r], ref[r]) <= TOL[fmt_t[0]], (shape, dag, r)


COLUMN_SHAPES = [(d, s, p, bz, 0) for d in (-1, -2, -3, -4) for s in (64, 256) for p in (0, 1) for bz in (-1, -2, -4)] + \
    [(-5, w, p, bz, f) for w in (2, 4) for p in (0, 1) for bz in (-2, -4) for f in (0, 3)] + \
    [(nr, 64, 0, -2, sp) for nr in (2, 3) for sp in (0, 1)]


@pytest.mark.parametrize("fmt_t", [("f32", "f32", 18), ("f16", "f16", 12), ("f64", "f64", 12), ("bf16", "f16", 12)],
                         ids=["f32-18", "f16-12", "f64-12", "bf16-12"])
@pytest.mark.parametrize("dims", [(32, 32, 4, 4), (16, 16, 4, 6)], ids=["plane512", "plane128"])
def test_column_schedules_match_oracle(fmt_t, dims):
    """Workgroups that walk columns of half (x, y) planes times 1, 2 or 4
    z-planes along t (negative bz) produce every output site once and
    correctly: 32x32 planes (512 half sites: 256-site workgroups take the
    columns too) and 16x16 planes (128 half sites: only 64-site workgroups
    do, the rest fall back to the lexicographic walk), both parities and
    dagger, 12 sources."""
    nrhs = 12
    print(f"column shapes fmt={fmt_t} dims={dims}", flush=True)
    lat, fmt, u_d, x_d, u_o, psi_o = _setup(dims, fmt_t, nrhs, seed=760)
    ph = np.array(AP, dtype=np.complex128)
    want = {(par, dag): [W.hop_eo(u_o, psi_o[r], 1 - par, ph, dagger=dag) for r in range(nrhs)]
            for par in (0, 1) for dag in (False, True)}
    for shape in COLUMN_SHAPES:
        assert WE.weo_set_mrhs_shape(*shape) == WE.WEO_OK
        for (par, dag), ref in want.items():
            out = lat.hop(u_d, x_d, fmt, out_parity=par, dagger=dag, nrhs=nrhs)
            got = lat.unpack_spinor(out, fmt, nrhs=nrhs).cpu().numpy()
            for r in range(nrhs):
                assert rel_err(got[r], ref[r]) <= TOL[fmt_t[0]], (shape, par, dag, r)


PAIR_SHAPES = [(d, s, p, bz, 0) for d in (-2, -4) for s in (64, 128, 256) for p in (0, 1) for bz in (0, 2)]


@pytest.mark.parametrize("bc", ["ap", "complex"])
@pytest.mark.parametrize("fmt_t", [("f16", "f16", 12), ("f16", "f16", 18)], ids=["f16-12", "f16-18"])
@pytest.mark.parametrize("dims", [(6, 4, 4, 10), (16, 8, 4, 6)], ids=["ragged", "strips"])
def test_fp16_pair_form_matches_oracle(dims, fmt_t, bc):
    """The link-resident hop on packed FP16 pairs (dot2 products, FP32
    accumulation) for FP16 spinors and links: every launch shape, both output
    parities, dagger, real and complex boundary phases, the axpy epilogue;
    against the oracle on the rounded inputs within the FP16 bar."""
    nrhs = 7
    print(f"fp16 pair form fmt={fmt_t} dims={dims} bc={bc}", flush=True)
    phases = AP if bc == "ap" else tuple(np.exp(1j * np.array([0.4, -1.1, 2.0, 2.9])))
    sp, lp, reals = fmt_t
    fmt = Format(sp, lp, reals)
    lat = Lattice(dims, 0.126, phases)
    u = inputs.gen_gauge(dims, 0.5, 720)
    psi = inputs.gen_spinor_half(dims, 721, nrhs=nrhs)
    y = inputs.gen_spinor_half(dims, 722, nrhs=nrhs)
    u_d, x_d, y_d = lat.pack_gauge(to_device(u), fmt), lat.pack_spinor(to_device(psi), fmt), \
        lat.pack_spinor(to_device(y), fmt)
    u_o, psi_o, y_o = link_as_stored(u, lp, reals), ROUND[sp](psi), ROUND[sp](y)
    ph = np.array(phases, dtype=np.complex128)
    for shape in PAIR_SHAPES:
        assert WE.weo_set_mrhs_shape(*shape) == WE.WEO_OK
        for par in (0, 1):
            for dag in (False, True):
                out = lat.hop(u_d, x_d, fmt, out_parity=par, dagger=dag, nrhs=nrhs)
                got = lat.unpack_spinor(out, fmt, nrhs=nrhs).cpu().numpy()
                for r in range(nrhs):
                    want = W.hop_eo(u_o, psi_o[r], 1 - par, ph, dagger=dag)
                    assert rel_err(got[r], want) <= TOL[sp], (shape, par, dag, r, rel_err(got[r], want))
        out = lat.hop_axpy(u_d, x_d, y_d, fmt, out_parity=1, alpha=-0.3, nrhs=nrhs)
        got = lat.unpack_spinor(out, fmt, nrhs=nrhs).cpu().numpy()
        for r in range(nrhs):
            want = y_o[r] - 0.3 * W.hop_eo(u_o, psi_o[r], 0, ph)
            assert rel_err(got[r], want) <= TOL[sp], (shape, "axpy", r)


LDS_SHAPES = [(-5, w, p, bz, f) for w in (2, 3, 4, 6, 8, 12) for p in (0, 1) for bz in (0, 2) for f in (0, 3)] + \
    [(-5, 4, 0, 0, 1), (-5, 2, 1, 2, 4), (-5, 3, 0, 0, 5)]
ALL_FORMATS = [("f64", "f64", 18), ("f64", "f64", 12), ("f32", "f32", 18), ("f32", "f32", 12),
               ("f16", "f16", 18), ("f16", "f16", 12), ("bf16", "f16", 18), ("bf16", "f16", 12)]


@pytest.mark.parametrize("fmt_t", ALL_FORMATS, ids=lambda f: f"{f[0]}-{f[1]}-{f[2]}")
@pytest.mark.parametrize("dims", [(6, 4, 4, 10), (16, 8, 4, 6)], ids=["ragged", "strips"])
def test_lds_form_matches_oracle(dims, fmt_t):
    """The hop with the 64 sites' links staged in LDS and the right-hand
    sides spread over the workgroup's wavefronts: every wavefront count
    (more than the format allows is clamped to its most), persistence,
    z-strip schedule and number of right-hand sides per sweep (all, 1, 3, 4,
    5), 7 right-hand sides (not a multiple of most of these), both output parities, dagger, complex boundary phases and the
    axpy epilogue, against the oracle on the rounded inputs."""
    nrhs = 7
    print(f"lds form fmt={fmt_t} dims={dims}", flush=True)
    phases = tuple(np.exp(1j * np.array([0.4, -1.1, 2.0, 2.9])))
    sp, lp, reals = fmt_t
    fmt = Format(sp, lp, reals)
    lat = Lattice(dims, 0.126, phases)
    u = inputs.gen_gauge(dims, 0.5, 740)
    psi = inputs.gen_spinor_half(dims, 741, nrhs=nrhs)
    y = inputs.gen_spinor_half(dims, 742, nrhs=nrhs)
    u_d, x_d, y_d = lat.pack_gauge(to_device(u), fmt), lat.pack_spinor(to_device(psi), fmt), \
        lat.pack_spinor(to_device(y), fmt)
    u_o, psi_o, y_o = link_as_stored(u, lp, reals), ROUND[sp](psi), ROUND[sp](y)
    ph = np.array(phases, dtype=np.complex128)
    want = {(par, dag): [W.hop_eo(u_o, psi_o[r], 1 - par, ph, dagger=dag) for r in range(nrhs)]
            for par in (0, 1) for dag in (False, True)}
    for shape in LDS_SHAPES:
        assert WE.weo_set_mrhs_shape(*shape) == WE.WEO_OK
        for (par, dag), ref in want.items():
            out = lat.hop(u_d, x_d, fmt, out_parity=par, dagger=dag, nrhs=nrhs)
            got = lat.unpack_spinor(out, fmt, nrhs=nrhs).cpu().numpy()
            for r in range(nrhs):
                assert rel_err(got[r], ref[r]) <= TOL[sp], (shape, par, dag, r, rel_err(got[r], ref[r]))
        out = lat.hop_axpy(u_d, x_d, y_d, fmt, out_parity=1, alpha=-0.3, nrhs=nrhs)
        got = lat.unpack_spinor(out, fmt, nrhs=nrhs).cpu().numpy()
        for r in range(nrhs):
            assert rel_err(got[r], y_o[r] - 0.3 * want[(1, False)][r]) <= TOL[sp], (shape, "axpy", r)


@pytest.mark.parametrize("fmt_t", [("f64", "f64", 12), ("f32", "f32", 18)], ids=["f64-12", "f32-18"])
def test_lds_form_in_solver(fmt_t):
    """Twelve sources solved by CGLS with the LDS form forced for every
    multi-rhs hop (its norm partials drive the solver): every solution's
    oracle residual meets the tolerance."""
    from paper_2303_08609_amd.solve import cg
    print(f"lds form in solver fmt={fmt_t}", flush=True)
    dims, kappa = (8, 8, 8, 8), 0.126
    fmt = Format(*fmt_t)
    lat = Lattice(dims, kappa, AP)
    u = inputs.gen_gauge(dims, 0.5, 401)
    b = inputs.gen_point_noise_sources(dims, 406)
    assert WE.weo_set_mrhs_shape(-5, 4, 0, 0, 0) == WE.WEO_OK
    tol = 1e-10 if fmt_t[0] == "f64" else 1e-5
    x_p, info = cg(lat, fmt, lat.pack_gauge(to_device(u), fmt), lat.pack_spinor(to_device(b), fmt), nrhs=12,
                   tol=tol, maxiter=5000)
    assert info["status"] == WE.WEO_OK, info
    x = lat.unpack_spinor(x_p, fmt, nrhs=12).cpu().numpy()
    u_o, ph = link_as_stored(u, fmt_t[1], fmt_t[2]), np.array(AP, dtype=np.complex128)
    for r in range(12):
        br = ROUND[fmt_t[0]](b[r])
        res = br - W.apply_m(u_o, x[r], kappa, ph)
        assert np.linalg.norm(res) / np.linalg.norm(br) <= 3 * tol, r


@pytest.mark.parametrize("nrhs", [2, 5, 12, 16])
def test_tuned_apply_matches_oracle(nrhs):
    dims = (8, 4, 6, 4)
    print(f"mrhs tuned apply nrhs={nrhs}", flush=True)
    lat, fmt, u_d, x_d, u_o, psi_o = _setup(dims, ("f32", "f32", 12), nrhs, seed=710)
    WE.weo_set_mrhs_shape(0, 0, 0, 0, 0)
    out = lat.apply(u_d, x_d, fmt, nrhs=nrhs)
    got = lat.unpack_spinor(out, fmt, nrhs=nrhs).cpu().numpy()
    ph = np.array(AP, dtype=np.complex128)
    for r in range(nrhs):
        assert rel_err(got[r], W.apply_m(u_o, psi_o[r], lat.kappa, ph)) <= 1e-6
    assert '"nrhs":%d' % nrhs in WE.tuning_report()


def test_bad_shape_rejected():
    assert WE.weo_set_mrhs_shape(5, 64, 0, 0, 0) == WE.WEO_ERR_ARG
    assert WE.weo_set_mrhs_shape(2, 96, 0, 0, 0) == WE.WEO_ERR_ARG
    assert WE.weo_set_mrhs_shape(2, 64, 2, 0, 0) == WE.WEO_ERR_ARG
    assert WE.weo_set_mrhs_shape(2, 64, 0, -65, 0) == WE.WEO_ERR_ARG
    assert WE.weo_set_mrhs_shape(-3, 64, 0, 65, 0) == WE.WEO_ERR_ARG
    assert WE.weo_set_mrhs_shape(-5, 4, 0, -65, 0) == WE.WEO_ERR_ARG
    assert WE.weo_set_mrhs_shape(2, 64, 0, 0, 2) == WE.WEO_ERR_ARG
    assert WE.weo_set_mrhs_shape(-5, 5, 0, 0, 0) == WE.WEO_ERR_ARG
    assert WE.weo_set_mrhs_shape(-5, 64, 0, 0, 0) == WE.WEO_ERR_ARG
    assert WE.weo_set_mrhs_shape(-5, 4, 0, 0, 17) == WE.WEO_ERR_ARG
    assert WE.weo_set_mrhs_shape(-5, 4, 0, 0, -1) == WE.WEO_ERR_ARG
    assert WE.weo_set_mrhs_shape(-6, 64, 0, 0, 0) == WE.WEO_ERR_ARG


def test_in_place_axpy_on_an_untuned_shape():
    """out = out + alpha hop(in) with 12 right-hand sides on a lattice no
    launch has tuned yet: the tuner must not time it by repeated launches
    (each would add to the last), so the result is one application."""
    dims = (6, 4, 4, 8)
    print("in-place axpy, untuned 12 rhs", flush=True)
    lat, fmt, u_d, x_d, u_o, psi_o = _setup(dims, ("f64", "f64", 18), 12, seed=730)
    WE.weo_set_mrhs_shape(0, 0, 0, 0, 0)
    y = inputs.gen_spinor_half(dims, 731, nrhs=12)
    y_d = lat.pack_spinor(to_device(y), fmt)
    lat.hop_axpy(u_d, x_d, y_d, fmt, out_parity=1, alpha=0.3, nrhs=12, out=y_d)
    got = lat.unpack_spinor(y_d, fmt, nrhs=12).cpu().numpy()
    ph = np.array(AP, dtype=np.complex128)
    for r in range(12):
        want = y[r] + 0.3 * W.hop_eo(u_o, psi_o[r], 0, ph)
        assert rel_err(got[r], want) <= 1e-12, r
    # the out-of-place launch of the same shape tunes and agrees
    out = lat.hop_axpy(u_d, x_d, lat.pack_spinor(to_device(y), fmt), fmt, out_parity=1, alpha=0.3, nrhs=12)
    assert rel_err(lat.unpack_spinor(out, fmt, nrhs=12).cpu().numpy(), got) <= 1e-13
    assert '"epilogue":1' in WE.tuning_report()



@pytest.mark.parametrize("fmt_t", [("f32", "f32", 18), ("f16", "f16", 12)], ids=["f32-18", "f16-12"])
def test_twelve_rhs_32_3x64_sampled(fmt_t):
    """The 12-source workload at full size (32^3x64, point + noise sources,
    links exp(0.5 i H)) through the tuned multi-RHS hop and apply, as the
    benchmark and the batched solves launch them; every source checked at
    sampled sites (faces, corners, the point's neighbours, random) against the
    oracle."""
    from tests._helpers import cached_gauge
    from tests.test_gpu_apply import _sample_sites
    dims = (32, 32, 32, 64)
    print(f"12 rhs 32^3x64 sampled fmt={fmt_t}", flush=True)
    sp, lp, reals = fmt_t
    fmt = Format(*fmt_t)
    lat = Lattice(dims, 0.126, AP)
    u = cached_gauge(dims, 0.5, 401)
    b = inputs.gen_point_noise_sources(dims, 406)
    WE.weo_set_mrhs_shape(0, 0, 0, 0, 0)
    ud, bd = lat.pack_gauge(to_device(u), fmt), lat.pack_spinor(to_device(b), fmt)
    hop = lat.unpack_spinor(lat.hop(ud, bd, fmt, out_parity=1, nrhs=12), fmt, nrhs=12).cpu().numpy()
    app = lat.unpack_spinor(lat.apply(ud, bd, fmt, nrhs=12), fmt, nrhs=12).cpu().numpy()
    hop, app = hop.reshape(12, -1, 4, 3), app.reshape(12, -1, 4, 3)
    del ud, bd
    sites = _sample_sites(dims, 12, 9)
    u_or, b_or = link_as_stored(u, lp, reals), ROUND[sp](b)
    ph = np.array(AP, dtype=np.complex128)
    for r in range(12):
        want = W.hop_at_sites(u_or, b_or[r], 0, ph, sites)
        assert rel_err(hop[r][sites], want) <= TOL[sp], ("hop", r)
        want = W.apply_m_at_sites(u_or, b_or[r], 0.126, ph, sites)
        assert rel_err(app[r][sites], want) <= TOL[sp], ("apply", r)


_CACHE_CHILD = r"""
import hashlib, json, sys
import torch
from paper_2303_08609_amd import inputs
from paper_2303_08609_amd import wilson_eo as WE
from paper_2303_08609_amd.ops import Format, Lattice, to_device
dims = (8, 8, 8, 16)
lat = Lattice(dims, 0.125, (1, 1, 1, -1))
fmt = Format("f32", "f32", 18)
u = lat.pack_gauge(to_device(inputs.gen_gauge(dims, 0.5, 760)), fmt)
x = lat.pack_spinor(to_device(inputs.gen_spinor_half(dims, 761, nrhs=12)), fmt)
out = lat.hop(u, x, fmt, 1, nrhs=12)
torch.cuda.synchronize()
rep = [json.loads(l) for l in WE.tuning_report().splitlines() if l.strip()]
print(json.dumps({"report": rep, "sha": hashlib.sha256(out.cpu().numpy().tobytes()).hexdigest()}))
"""


def _cache_child(path):
    import json
    import os
    import subprocess
    import sys
    env = dict(os.environ, WILSON_EO_TUNE_CACHE=str(path))
    env.pop("WEO_TUNE", None)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    p = subprocess.run([sys.executable, "-c", _CACHE_CHILD], env=env, cwd=root, capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 0, p.stderr[-2000:]
    return json.loads(p.stdout.strip().splitlines()[-1])


def test_tuning_cache_across_processes(tmp_path):
    """WILSON_EO_TUNE_CACHE: a first process tunes the 12-rhs hop and writes
    the header and one line; a second reads the shape back (same shape and
    recorded time, nothing appended) and produces the same output bits; a
    file with a foreign header is rewritten by a fresh tuning."""
    path = tmp_path / "tune.txt"
    print("tuning cache: first process", flush=True)
    a = _cache_child(path)
    lines = path.read_text().splitlines()
    assert lines[0].startswith("# wilson_eo tuning cache ") and len(lines) == 2, lines
    print("tuning cache: second process", flush=True)
    b = _cache_child(path)
    assert path.read_text().splitlines() == lines
    assert b["report"] == a["report"] and b["sha"] == a["sha"]
    path.write_text("# some other cache\n8 8 8 16 2 12 0 -1 64 0 0 0 1.00\n")
    print("tuning cache: foreign header", flush=True)
    c = _cache_child(path)
    lines = path.read_text().splitlines()
    assert lines[0].startswith("# wilson_eo tuning cache ") and len(lines) == 2, lines
    assert c["sha"] == a["sha"] or c["report"] != a["report"]
