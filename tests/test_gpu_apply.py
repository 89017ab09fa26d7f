"""Parity of the HIP hop and even-odd operator against the FP64 oracle.

Inputs are the seeded generators' FP64 arrays; the oracle is evaluated on the
same values rounded to the storage format on the CPU.  Bars: FP64 <= 1e-12 and
FP32 <= 1e-6 norm-wise relative; FP16 spinors <= 2e-3, BF16 spinors <= 1e-2.
"""
import numpy as np
import pytest
import torch

from oracle import wilson as W
from paper_2303_08609_amd import inputs
from paper_2303_08609_amd.ops import Format, Lattice, to_device
from tests._helpers import AP, ROUND, cached_gauge, link_as_stored, rel_err, sample_sites, site_rel_max

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-6, "f16": 2e-3, "bf16": 1e-2}
FORMATS = [("f64", "f64", 18), ("f64", "f64", 12), ("f32", "f32", 18), ("f32", "f32", 12),
           ("f16", "f16", 18), ("f16", "f16", 12), ("bf16", "f16", 18), ("bf16", "f16", 12)]
# small lattices: degenerate (2^4), non-cubic axis mixes, ragged last workgroup
DIMS = [(2, 2, 2, 2), (4, 4, 4, 4), (4, 6, 2, 8), (6, 4, 8, 2), (10, 6, 4, 6)]


def _setup(dims, fmt_t, seed, kappa=0.126, bc=AP, nrhs=None, eps=0.5):
    sp, lp, reals = fmt_t
    fmt = Format(sp, lp, reals)
    lat = Lattice(dims, kappa, bc)
    u = cached_gauge(dims, eps, seed)
    psi = inputs.gen_spinor_half(dims, seed + 1, nrhs=nrhs)
    u_dev = lat.pack_gauge(to_device(u), fmt)
    x_dev = lat.pack_spinor(to_device(psi), fmt)
    u_or = link_as_stored(u, lp, reals)
    psi_or = ROUND[sp](psi)
    return lat, fmt, u_dev, x_dev, u_or, psi_or


@pytest.mark.parametrize("fmt_t", FORMATS, ids=lambda f: f"{f[0]}-{f[1]}-{f[2]}")
@pytest.mark.parametrize("dims", DIMS, ids=lambda d: "x".join(map(str, d)))
def test_apply_matches_oracle(dims, fmt_t):
    print(f"apply parity dims={dims} fmt={fmt_t}", flush=True)
    lat, fmt, u_dev, x_dev, u_or, psi_or = _setup(dims, fmt_t, 1000 + sum(dims))
    ph = np.array(lat.bc)
    for dag in (False, True):
        out = lat.apply(u_dev, x_dev, fmt, dagger=dag)
        got = lat.unpack_spinor(out, fmt).cpu().numpy()
        want = W.apply_m(u_or, psi_or, lat.kappa, ph, dagger=dag)
        assert rel_err(got, want) <= TOL[fmt_t[0]], (dag, rel_err(got, want))


@pytest.mark.parametrize("fmt_t", FORMATS[:4], ids=lambda f: f"{f[0]}-{f[2]}")
def test_hop_both_parities_and_complex_phases(fmt_t):
    dims = (4, 6, 2, 8)
    bc = tuple(np.exp(1j * np.array([0.4, -1.1, 2.0, 2.9])))
    print(f"hop parity fmt={fmt_t}", flush=True)
    lat, fmt, u_dev, x_dev, u_or, psi_or = _setup(dims, fmt_t, 77, bc=bc)
    for par in (0, 1):
        for dag in (False, True):
            out = lat.hop(u_dev, x_dev, fmt, out_parity=par, dagger=dag)
            got = lat.unpack_spinor(out, fmt).cpu().numpy()
            want = W.hop_eo(u_or, psi_or, 1 - par, np.array(bc), dagger=dag)
            assert rel_err(got, want) <= TOL[fmt_t[0]], (par, dag)


@pytest.mark.parametrize("fmt_t", [("f64", "f64", 18), ("f32", "f32", 12)], ids=["f64", "f32"])
def test_apply_multi_rhs(fmt_t):
    dims = (4, 4, 2, 6)
    print(f"apply nrhs=3 fmt={fmt_t}", flush=True)
    lat, fmt, u_dev, x_dev, u_or, psi_or = _setup(dims, fmt_t, 91, nrhs=3)
    out = lat.apply(u_dev, x_dev, fmt, nrhs=3)
    got = lat.unpack_spinor(out, fmt, nrhs=3).cpu().numpy()
    for r in range(3):
        want = W.apply_m(u_or, psi_or[r], lat.kappa, np.array(lat.bc))
        assert rel_err(got[r], want) <= TOL[fmt_t[0]]


@pytest.mark.parametrize("fmt_t", [("f64", "f64", 18), ("f32", "f32", 18), ("f32", "f32", 12)],
                         ids=["f64", "f32-18", "f32-12"])
def test_apply_16_3x32_full(fmt_t):
    dims = (16, 16, 16, 32)
    print(f"apply 16^3x32 fmt={fmt_t}", flush=True)
    lat, fmt, u_dev, x_dev, u_or, psi_or = _setup(dims, fmt_t, 501, kappa=0.125)
    out = lat.apply(u_dev, x_dev, fmt)
    got = lat.unpack_spinor(out, fmt).cpu().numpy()
    want = W.apply_m(u_or, psi_or, lat.kappa, np.array(lat.bc))
    assert rel_err(got, want) <= TOL[fmt_t[0]]


_sample_sites = sample_sites


@pytest.mark.parametrize("fmt_t", [("f32", "f32", 18), ("f32", "f32", 12), ("f64", "f64", 18)],
                         ids=["f32-18", "f32-12", "f64-18"])
def test_apply_32_3x64_sampled(fmt_t):
    """Full-size workload (32^3x64, kappa = 0.126, eps = 0.5) in the launch
    configuration the benchmark times; outputs checked at sampled sites."""
    dims = (32, 32, 32, 64)
    print(f"apply 32^3x64 sampled fmt={fmt_t}", flush=True)
    lat, fmt, u_dev, x_dev, u_or, psi_or = _setup(dims, fmt_t, 201, kappa=0.126)
    out = lat.apply(u_dev, x_dev, fmt)
    got = lat.unpack_spinor(out, fmt).cpu().numpy().reshape(-1, 4, 3)
    sites = _sample_sites(dims, 24, 5)
    want = W.apply_m_at_sites(u_or, psi_or, lat.kappa, np.array(lat.bc), sites)
    err = np.linalg.norm(got[sites] - want) / np.linalg.norm(want)
    assert err <= TOL[fmt_t[0]]
    assert site_rel_max(got[sites], want) <= TOL[fmt_t[0]]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_plane_wave_32_3x64(prec):
    """Closed form at full size: unit links, M P_e[e^{ipx} u] = lambda P_e[...]."""
    from oracle.gamma import GAMMA
    from oracle.lattice import full_to_half
    dims = (32, 32, 32, 64)
    kappa = 0.126
    thetas = np.array([0, 0, 0, np.pi])
    n = np.array([3, 30, 7, 11])
    p = (2 * np.pi * n + thetas) / np.array(dims)
    k = sum(GAMMA[mu] * np.sin(p[mu]) for mu in range(4))
    w, v = np.linalg.eigh(k)
    s = np.sqrt((np.sin(p) ** 2).sum())
    c = np.cos(p).sum()
    lam = 1 - kappa ** 2 * (2 * c - 2j * s) ** 2        # eigenvector of +S
    lx, ly, lz, lt = dims
    t, z, y, x = np.meshgrid(range(lt), range(lz), range(ly), range(lx), indexing="ij",
                             sparse=True)
    phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    spinor = np.outer(v[:, 3], np.array([0.6, -0.48j, 0.64]))
    psi_e = full_to_half(phase[..., None, None] * spinor, 0)
    fmt = Format(prec, prec, 18)
    lat = Lattice(dims, kappa, AP)
    u_dev = lat.pack_gauge(to_device(inputs.gen_unit_gauge(dims)), fmt)
    x_dev = lat.pack_spinor(to_device(psi_e), fmt)
    got = lat.unpack_spinor(lat.apply(u_dev, x_dev, fmt), fmt).cpu().numpy()
    ref = lam * ROUND[prec](psi_e)
    assert rel_err(got, ref) <= TOL[prec]


def test_pack_unpack_roundtrip():
    dims = (4, 6, 2, 8)
    lat = Lattice(dims, 0.1)
    psi = inputs.gen_spinor_half(dims, 3, nrhs=2)
    for sp in ("f64", "f32", "f16", "bf16"):
        fmt = Format(sp)
        packed = lat.pack_spinor(to_device(psi), fmt, scale=0.5)
        back = lat.unpack_spinor(packed, fmt, nrhs=2, scale=2.0).cpu().numpy()
        assert np.array_equal(back, 2.0 * ROUND[sp](0.5 * psi)), sp


def test_bitwise_repeatable():
    dims = (8, 8, 8, 8)
    lat, fmt, u_dev, x_dev, _, _ = _setup(dims, ("f32", "f32", 18), 5)
    a = lat.apply(u_dev, x_dev, fmt)
    b = lat.apply(u_dev, x_dev, fmt)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
