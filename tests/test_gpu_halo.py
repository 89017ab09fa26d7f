"""A hop split along one or more directions (the one-device share of the domain decomposition of
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


# ---- splits along any set of directions ------------------------------------------

class Grid:
    """The lattice cut into n[mu] blocks along each direction mu (a process
    grid); each block holds its own packed links and fields and runs the bulk
    hop with zero phases in every direction in ``dirs`` (the exchanged ones),
    then packs, exchanges and unpacks the faces of those directions.  A
    direction in ``dirs`` with n[mu] = 1 exchanges with itself (the paper's
    forced communication)."""

    def __init__(self, dims, fmt, u, bc, n, dirs):
        self.dims, self.fmt, self.bc, self.n, self.dirs = dims, fmt, bc, n, tuple(dirs)
        self.ld = tuple(dims[m] // n[m] for m in range(4))
        assert all(dims[m] % n[m] == 0 and self.ld[m] % 2 == 0 for m in range(4))
        self.idx = [(ix, iy, iz, it) for it in range(n[3]) for iz in range(n[2]) for iy in range(n[1])
                    for ix in range(n[0])]
        self.lat = {i: Lattice(self.ld, KAPPA, bc) for i in self.idx}
        self.u = {i: self.lat[i].pack_gauge(to_device(np.ascontiguousarray(u[(slice(None),) + self._sl(i)])), fmt)
                  for i in self.idx}

    def _sl(self, i, half=False):
        """Slices [t][z][y][x] (x halved for one-parity arrays) of block i."""
        lx, ly, lz, lt = self.ld
        ix, iy, iz, it = i
        xs = slice(ix * lx // 2, (ix + 1) * lx // 2) if half else slice(ix * lx, (ix + 1) * lx)
        return (slice(it * lt, (it + 1) * lt), slice(iz * lz, (iz + 1) * lz), slice(iy * ly, (iy + 1) * ly), xs)

    def pack(self, psi_half):
        return {i: self.lat[i].pack_spinor(to_device(np.ascontiguousarray(psi_half[self._sl(i, True)])), self.fmt)
                for i in self.idx}

    def hop(self, x, out_parity, dagger):
        outs, faces = {}, {}
        for i in self.idx:
            outs[i] = self.lat[i].open_dirs(self.dirs).hop(self.u[i], x[i], self.fmt, out_parity, dagger)
            for mu in self.dirs:
                faces[i, mu] = self.lat[i].face_pack(self.u[i], x[i], self.fmt, out_parity, dagger, mu=mu)
        for i in self.idx:
            for mu in self.dirs:
                below = tuple((c - 1) % self.n[m] if m == mu else c for m, c in enumerate(i))
                above = tuple((c + 1) % self.n[m] if m == mu else c for m, c in enumerate(i))
                self.lat[i].face_unpack(self.u[i], faces[below, mu][1], faces[above, mu][0], outs[i], self.fmt,
                                        out_parity, dagger, mu=mu,
                                        phase_lo=self.bc[mu] if i[mu] == 0 else 1.0,
                                        phase_hi=self.bc[mu] if i[mu] == self.n[mu] - 1 else 1.0)
        return outs

    def gather(self, outs):
        lx, ly, lz, lt = self.dims
        full = np.zeros((lt, lz, ly, lx // 2, 4, 3), dtype=np.complex128)
        for i in self.idx:
            full[self._sl(i, True)] = self.lat[i].unpack_spinor(outs[i], self.fmt).cpu().numpy()
        return full


CPH = tuple(np.exp(1j * np.array([0.4, -1.1, 2.0, 2.9])))


@pytest.mark.parametrize("fmt_t", FORMATS, ids=lambda f: f"{f[0]}-{f[1]}-{f[2]}")
def test_forced_exchange_in_all_four_directions(fmt_t):
    """One block = the whole lattice with every direction's faces sent to
    itself (the communication the paper forces in all four directions for
    its single-node runs): bulk hop with all four phases zero plus the x, y,
    z and t faces equals the oracle's hop, both parities, with and without
    dagger, complex boundary phases."""
    dims = (4, 6, 2, 8)
    print(f"forced exchange x,y,z,t fmt={fmt_t}", flush=True)
    u, psi, u_or, psi_or = _inputs(dims, fmt_t, 1401)
    fmt = Format(*fmt_t)
    grid = Grid(dims, fmt, u, CPH, (1, 1, 1, 1), (0, 1, 2, 3))
    x = grid.pack(psi)
    for par in (0, 1):
        for dag in (False, True):
            got = grid.gather(grid.hop(x, par, dag))
            want = W.hop_eo(u_or, psi_or, 1 - par, np.array(CPH), dagger=dag)
            assert rel_err(got, want) <= TOL[fmt_t[0]], (par, dag, rel_err(got, want))


@pytest.mark.parametrize("n", [(1, 1, 2, 2), (2, 1, 1, 2), (2, 2, 1, 1), (4, 1, 1, 1), (2, 2, 2, 2)],
                         ids=lambda n: "x".join(map(str, n)))
@pytest.mark.parametrize("fmt_t", [("f64", "f64", 18), ("f32", "f32", 12)], ids=["f64", "f32-12"])
def test_block_grids_match_oracle(fmt_t, n):
    """The lattice cut into a grid of blocks (the paper's process grid
    [1,1,2,2], x splits across the even-odd compacted direction, all four
    directions at once); each block's faces go to its neighbours, every
    other direction exchanges with itself.  The gathered hop equals the
    oracle's hop of the whole lattice."""
    dims = (8, 4, 4, 8)
    print(f"block grid {n} fmt={fmt_t}", flush=True)
    u, psi, u_or, psi_or = _inputs(dims, fmt_t, 1411)
    fmt = Format(*fmt_t)
    grid = Grid(dims, fmt, u, CPH, n, (0, 1, 2, 3))
    x = grid.pack(psi)
    for par in (0, 1):
        for dag in (False, True):
            got = grid.gather(grid.hop(x, par, dag))
            want = W.hop_eo(u_or, psi_or, 1 - par, np.array(CPH), dagger=dag)
            assert rel_err(got, want) <= TOL[fmt_t[0]], (par, dag, rel_err(got, want))


def test_split_only_some_directions():
    """A 2 x 2 grid in z and t with x and y left to the bulk hop (their phases
    kept): only the split directions exchange faces."""
    dims = (4, 4, 4, 8)
    print("z,t split only", flush=True)
    fmt_t = ("f32", "f32", 18)
    u, psi, u_or, psi_or = _inputs(dims, fmt_t, 1421)
    grid = Grid(dims, Format(*fmt_t), u, CPH, (1, 1, 2, 2), (2, 3))
    x = grid.pack(psi)
    got = grid.gather(grid.hop(x, 1, False))
    want = W.hop_eo(u_or, psi_or, 0, np.array(CPH))
    assert rel_err(got, want) <= 1e-6


@pytest.mark.parametrize("order", ["sequential", "forked"])
def test_split_hop_graph_replays(order):
    """The self-exchanging split hop (all four directions open) captured as
    one HIP graph, the face pack either in line or forked onto a second
    stream and joined before the unpack: every replay, with eager launches
    and synchronisations between replays and the output cleared before
    each, equals the eager sequence bit for bit and the oracle's hop."""
    import torch
    dims = (8, 4, 4, 8)
    print(f"split hop graph {order}", flush=True)
    fmt_t = ("f32", "f32", 18)
    fmt = Format(*fmt_t)
    u, psi, u_or, psi_or = _inputs(dims, fmt_t, 1431)
    lat = Lattice(dims, KAPPA, CPH)
    bulk = lat.open_dirs((0, 1, 2, 3))
    ud = lat.pack_gauge(to_device(u), fmt)
    xd = lat.pack_spinor(to_device(psi), fmt)
    out = lat.new_spinor(fmt)
    bufs = {mu: lat.face_pack(ud, xd, fmt, 1, mu=mu) for mu in range(4)}
    side = torch.cuda.Stream()

    def pack():
        for mu in range(4):
            lat.face_pack(ud, xd, fmt, 1, lo=bufs[mu][0], hi=bufs[mu][1], mu=mu)

    def seq():
        cur = torch.cuda.current_stream()
        if order == "forked":
            side.wait_stream(cur)
            with torch.cuda.stream(side):
                pack()
        else:
            pack()
        bulk.hop(ud, xd, fmt, 1, out=out)
        if order == "forked":
            cur.wait_stream(side)
        for mu in range(4):
            lat.face_unpack(ud, bufs[mu][1], bufs[mu][0], out, fmt, 1, phase_lo=CPH[mu], phase_hi=CPH[mu], mu=mu)

    seq()
    torch.cuda.synchronize()
    eager = out.clone()
    want = W.hop_eo(u_or, psi_or, 0, np.array(CPH))
    assert rel_err(lat.unpack_spinor(eager, fmt).cpu().numpy(), want) <= 1e-6
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        seq()
    other = lat.new_spinor(fmt)
    for k in range(4):
        out.zero_()
        lat.hop(ud, xd, fmt, 0, out=other)            # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), k
