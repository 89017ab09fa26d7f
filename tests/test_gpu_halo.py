"""A hop split along t (the one-device share of the domain decomposition of
Sec. 3.6 and 4.1): each slab of consecutive t slices runs the bulk hop with
a zero t phase, packs its two t faces, and adds the faces received from its
neighbours.  Checked against the oracle's hop of the whole lattice for the
whole lattice as one slab exchanging with itself (as the paper's runs on one
node do) and for the lattice cut into 2 and 4 slabs whose faces are passed
between their buffers on the one device.
"""
import numpy as np
import pytest

from oracle import wilson as W
from paper_2303_08609_amd import inputs
from paper_2303_08609_amd.ops import Format, Lattice, to_device
from tests._helpers import ROUND, cached_gauge, link_as_stored, rel_err

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-6, "f16": 2e-3, "bf16": 1e-2}
FORMATS = [("f64", "f64", 18), ("f64", "f64", 12), ("f32", "f32", 18), ("f32", "f32", 12),
           ("f16", "f16", 18), ("f16", "f16", 12), ("bf16", "f16", 18), ("bf16", "f16", 12)]
KAPPA = 0.126


class Slabs:
    """The lattice cut along t into n slabs, each with its own packed links."""

    def __init__(self, dims, fmt, u, bc, n):
        lx, ly, lz, lt = dims
        assert lt % n == 0 and (lt // n) % 2 == 0
        self.n, self.ls, self.fmt, self.bc = n, lt // n, fmt, bc
        self.lat = [Lattice((lx, ly, lz, self.ls), KAPPA, bc) for _ in range(n)]
        self.u = [self.lat[r].pack_gauge(to_device(u[:, r * self.ls:(r + 1) * self.ls]), fmt)
                  for r in range(n)]

    def pack(self, psi_half, nrhs=None):
        """Device fields of each slab from a canonical half-lattice array."""
        sl = (lambda r: psi_half[:, r * self.ls:(r + 1) * self.ls]) if nrhs else \
             (lambda r: psi_half[r * self.ls:(r + 1) * self.ls])
        return [self.lat[r].pack_spinor(to_device(sl(r)), self.fmt) for r in range(self.n)]

    def hop(self, x, out_parity, dagger, nrhs=1, alpha=None, y=None):
        """Bulk hop on every slab, face pack, exchange, face unpack."""
        outs, faces = [], []
        for r in range(self.n):
            bulk = self.lat[r].open_t()
            if y is None:
                o = bulk.hop(self.u[r], x[r], self.fmt, out_parity, dagger, nrhs=nrhs)
            else:
                o = bulk.hop_axpy(self.u[r], x[r], y[r], self.fmt, out_parity, alpha, dagger, nrhs=nrhs)
            outs.append(o)
            faces.append(self.lat[r].face_pack(self.u[r], x[r], self.fmt, out_parity, dagger, nrhs=nrhs))
        phase_t = self.bc[3]
        for r in range(self.n):
            recv_lo = faces[(r - 1) % self.n][1]      # the slab below sends its upper face
            recv_hi = faces[(r + 1) % self.n][0]      # the slab above sends its lower face
            self.lat[r].face_unpack(self.u[r], recv_lo, recv_hi, outs[r], self.fmt, out_parity, dagger,
                                    phase_lo=phase_t if r == 0 else 1.0,
                                    phase_hi=phase_t if r == self.n - 1 else 1.0,
                                    alpha=1.0 if y is None else alpha, nrhs=nrhs)
        return outs

    def gather(self, outs, nrhs=None):
        parts = [self.lat[r].unpack_spinor(outs[r], self.fmt, nrhs=nrhs or 1).cpu().numpy()
                 for r in range(self.n)]
        return np.concatenate(parts, axis=1 if nrhs else 0)


def _inputs(dims, fmt_t, seed, nrhs=None):
    sp, lp, reals = fmt_t
    u = cached_gauge(dims, 0.5, seed)
    psi = inputs.gen_spinor_half(dims, seed + 1, nrhs=nrhs)
    return u, psi, link_as_stored(u, lp, reals), ROUND[sp](psi)


@pytest.mark.parametrize("fmt_t", FORMATS, ids=lambda f: f"{f[0]}-{f[1]}-{f[2]}")
def test_self_exchange_matches_oracle_and_plain_hop(fmt_t):
    """One slab = the whole lattice, its faces sent to itself."""
    dims = (4, 6, 2, 8)
    print(f"self exchange fmt={fmt_t}", flush=True)
    fmt = Format(*fmt_t)
    bc = (1, 1, 1, -1)
    u, psi, u_or, psi_or = _inputs(dims, fmt_t, 810)
    s = Slabs(dims, fmt, u, bc, 1)
    x = s.pack(psi)
    for par in (0, 1):
        for dag in (False, True):
            got = s.gather(s.hop(x, par, dag))
            want = W.hop_eo(u_or, psi_or, 1 - par, np.array(bc, dtype=complex), dagger=dag)
            assert rel_err(got, want) <= TOL[fmt_t[0]], (par, dag, rel_err(got, want))
            plain = s.lat[0].hop(s.u[0], x[0], fmt, par, dag)
            ref = s.lat[0].unpack_spinor(plain, fmt).cpu().numpy()
            assert rel_err(got, ref) <= TOL[fmt_t[0]], (par, dag)


@pytest.mark.parametrize("nslab", [2, 4])
@pytest.mark.parametrize("fmt_t", [FORMATS[0], FORMATS[3], FORMATS[5], FORMATS[6]],
                         ids=lambda f: f"{f[0]}-{f[1]}-{f[2]}")
def test_slabs_exchange_matches_oracle(fmt_t, nslab):
    """2 or 4 slabs (slab length 4 or 2) with a complex t phase at the global
    boundary only."""
    dims = (4, 2, 6, 8)
    bc = tuple(np.exp(1j * np.array([0.3, -0.7, 1.9, 2.6])))
    print(f"{nslab} slabs fmt={fmt_t}", flush=True)
    fmt = Format(*fmt_t)
    u, psi, u_or, psi_or = _inputs(dims, fmt_t, 820 + nslab)
    s = Slabs(dims, fmt, u, bc, nslab)
    x = s.pack(psi)
    for par in (0, 1):
        for dag in (False, True):
            got = s.gather(s.hop(x, par, dag))
            want = W.hop_eo(u_or, psi_or, 1 - par, np.array(bc), dagger=dag)
            assert rel_err(got, want) <= TOL[fmt_t[0]], (par, dag, rel_err(got, want))


@pytest.mark.parametrize("fmt_t", [FORMATS[0], FORMATS[2]], ids=["f64", "f32"])
def test_split_apply_matches_oracle(fmt_t):
    """M = 1 - kappa^2 H_eo H_oe over 2 slabs: the second hop's bulk call
    carries the axpy and the face unpack the same alpha."""
    dims = (6, 4, 4, 8)
    bc = (1, 1, 1, -1)
    print(f"split apply fmt={fmt_t}", flush=True)
    fmt = Format(*fmt_t)
    u, psi, u_or, psi_or = _inputs(dims, fmt_t, 830)
    s = Slabs(dims, fmt, u, bc, 2)
    x = s.pack(psi)
    for dag in (False, True):
        tmp = s.hop(x, 1, dag)
        out = s.hop(tmp, 0, dag, alpha=-KAPPA * KAPPA, y=x)
        got = s.gather(out)
        want = W.apply_m(u_or, psi_or, KAPPA, np.array(bc, dtype=complex), dagger=dag)
        assert rel_err(got, want) <= TOL[fmt_t[0]], (dag, rel_err(got, want))


def test_slabs_multi_rhs():
    """Three right-hand sides through one set of face calls per slab."""
    dims = (4, 4, 4, 8)
    fmt_t = ("f32", "f32", 18)
    bc = (1, 1, 1, -1)
    print("slabs nrhs=3", flush=True)
    fmt = Format(*fmt_t)
    u, psi, u_or, psi_or = _inputs(dims, fmt_t, 840, nrhs=3)
    s = Slabs(dims, fmt, u, bc, 2)
    x = s.pack(psi, nrhs=3)
    got = s.gather(s.hop(x, 1, False, nrhs=3), nrhs=3)
    for r in range(3):
        want = W.hop_eo(u_or, psi_or[r], 0, np.array(bc, dtype=complex))
        assert rel_err(got[r], want) <= TOL["f32"], r
