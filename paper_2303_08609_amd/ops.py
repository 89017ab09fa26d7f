"""torch-facing layer over the C ABI: device buffers are torch tensors, launches
go to torch's current HIP stream.  Every operation is one or more calls into
libwilson_eo (``wilson_eo``); nothing is computed in torch or on the CPU.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import wilson_eo as W

PREC = {"f64": W.WEO_F64, "f32": W.WEO_F32, "f16": W.WEO_F16, "bf16": W.WEO_BF16}
LINK = {18: W.WEO_LINK18, 12: W.WEO_LINK12}


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _ptr(t: torch.Tensor | None):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def _canon_prec(t: torch.Tensor) -> int:
    if t.dtype == torch.complex128:
        return W.WEO_F64
    if t.dtype == torch.complex64:
        return W.WEO_F32
    raise ValueError(f"canonical fields are complex128 or complex64, got {t.dtype}")


class Format:
    """Storage format: spinor precision, link precision, link reals (18/12)."""

    def __init__(self, spinor="f32", link=None, link_reals=18):
        self.spinor = spinor
        self.link = link or ("f16" if spinor == "bf16" else spinor)
        self.link_reals = int(link_reals)
        self.c = W.make_format(PREC[self.spinor], PREC[self.link], LINK[self.link_reals])

    def __repr__(self):
        return f"Format({self.spinor}/{self.link}/{self.link_reals})"


class Lattice:
    """Lattice extents (Lx, Ly, Lz, Lt), kappa and boundary phases."""

    def __init__(self, dims, kappa, bc=(1, 1, 1, -1)):
        self.dims = tuple(int(d) for d in dims)
        self.kappa = float(kappa)
        self.bc = tuple(complex(b) for b in bc)
        self.c = W.make_lattice(self.dims, self.kappa, [(b.real, b.imag) for b in self.bc])
        lx, ly, lz, lt = self.dims
        self.volume = lx * ly * lz * lt
        self.vh = self.volume // 2

    def half_shape(self, nrhs=None):
        lx, ly, lz, lt = self.dims
        s = (lt, lz, ly, lx // 2, 4, 3)
        return s if nrhs is None else (nrhs,) + s

    def gauge_shape(self):
        lx, ly, lz, lt = self.dims
        return (4, lt, lz, ly, lx, 3, 3)

    def gauge_bytes(self, fmt: Format) -> int:
        n = W.weo_gauge_bytes(self.c, fmt.c)
        if n == 0:
            raise W.WilsonEOError(W.WEO_ERR_ARG, "weo_gauge_bytes")
        return n

    def spinor_bytes(self, fmt: Format, nrhs=1) -> int:
        n = W.weo_spinor_bytes(self.c, fmt.c, int(nrhs))
        if n == 0:
            raise W.WilsonEOError(W.WEO_ERR_ARG, "weo_spinor_bytes")
        return n

    # ---- buffers ----------------------------------------------------------
    def new_spinor(self, fmt: Format, nrhs=1, device="cuda"):
        return torch.empty(self.spinor_bytes(fmt, nrhs), dtype=torch.uint8, device=device)

    def new_gauge(self, fmt: Format, device="cuda"):
        return torch.empty(self.gauge_bytes(fmt), dtype=torch.uint8, device=device)

    # ---- packing ------------------------------------------------------------
    def pack_gauge(self, u_canon: torch.Tensor, fmt: Format, out=None):
        if tuple(u_canon.shape) != self.gauge_shape():
            raise ValueError(f"gauge shape {tuple(u_canon.shape)} != {self.gauge_shape()}")
        out = self.new_gauge(fmt) if out is None else out
        W.check(W.weo_pack_gauge(self.c, fmt.c, _ptr(u_canon), _canon_prec(u_canon), _ptr(out),
                                 _stream()), "weo_pack_gauge")
        return out

    def pack_spinor(self, s_canon: torch.Tensor, fmt: Format, scale=1.0, out=None):
        nrhs = 1 if s_canon.dim() == 6 else int(s_canon.shape[0])
        want = self.half_shape() if s_canon.dim() == 6 else self.half_shape(nrhs)
        if tuple(s_canon.shape) != want:
            raise ValueError(f"spinor shape {tuple(s_canon.shape)} != {want}")
        out = self.new_spinor(fmt, nrhs) if out is None else out
        W.check(W.weo_pack_spinor(self.c, fmt.c, nrhs, _ptr(s_canon), _canon_prec(s_canon),
                                  float(scale), _ptr(out), _stream()), "weo_pack_spinor")
        return out

    def unpack_spinor(self, packed: torch.Tensor, fmt: Format, nrhs=1, scale=1.0,
                      dtype=torch.complex128):
        shape = self.half_shape() if nrhs == 1 else self.half_shape(nrhs)
        out = torch.empty(shape, dtype=dtype, device=packed.device)
        W.check(W.weo_unpack_spinor(self.c, fmt.c, int(nrhs), _ptr(packed), float(scale),
                                    _ptr(out), _canon_prec(out), _stream()), "weo_unpack_spinor")
        return out

    # ---- operator -----------------------------------------------------------
    def hop(self, u, x, fmt: Format, out_parity, dagger=False, nrhs=1, out=None):
        out = self.new_spinor(fmt, nrhs) if out is None else out
        W.check(W.wilson_eo_hop(self.c, fmt.c, int(out_parity), int(bool(dagger)), _ptr(u),
                                _ptr(x), _ptr(out), int(nrhs), _stream()), "wilson_eo_hop")
        return out

    def hop_axpy(self, u, x, y, fmt: Format, out_parity, alpha, dagger=False, nrhs=1, out=None):
        """out = y + alpha * P_p H P_{1-p} x (out may be y)."""
        out = self.new_spinor(fmt, nrhs) if out is None else out
        W.check(W.wilson_eo_hop_axpy(self.c, fmt.c, int(out_parity), int(bool(dagger)), float(alpha),
                                     _ptr(u), _ptr(x), _ptr(y), _ptr(out), int(nrhs), _stream()),
                "wilson_eo_hop_axpy")
        return out

    # ---- split hop: faces of a block along a direction ------------------------
    def open_t(self):
        """The same slab with a zero t phase: its hop is the bulk part of a
        t-split hop (the terms across the t faces dropped)."""
        return self.open_dirs((3,))

    def open_dirs(self, dirs):
        """The same block with zero phases in the split directions ``dirs``:
        its hop is the bulk part of the split hop."""
        return Lattice(self.dims, self.kappa, tuple(0.0 if m in dirs else b for m, b in enumerate(self.bc)))

    def face_bytes(self, fmt: Format, nrhs=1, mu=3) -> int:
        n = W.weo_face_bytes(self.c, fmt.c, int(mu), int(nrhs))
        if n == 0:
            raise W.WilsonEOError(W.WEO_ERR_ARG, "weo_face_bytes")
        return n

    def face_pack(self, u, x, fmt: Format, out_parity, dagger=False, nrhs=1, lo=None, hi=None, mu=3):
        """(send_lo, send_hi) of direction mu for a hop to out_parity from x."""
        nb = self.face_bytes(fmt, nrhs, mu)
        lo = torch.empty(nb, dtype=torch.uint8, device=x.device) if lo is None else lo
        hi = torch.empty(nb, dtype=torch.uint8, device=x.device) if hi is None else hi
        W.check(W.wilson_eo_face_pack(self.c, fmt.c, int(mu), int(out_parity), int(bool(dagger)), _ptr(u),
                                      _ptr(x), _ptr(lo), _ptr(hi), int(nrhs), _stream()), "wilson_eo_face_pack")
        return lo, hi

    def face_unpack(self, u, recv_lo, recv_hi, out, fmt: Format, out_parity, dagger=False,
                    phase_lo=1.0, phase_hi=1.0, alpha=1.0, nrhs=1, mu=3):
        """Adds the received faces of direction mu to out (in place)."""
        pl = (ctypes.c_double * 2)(complex(phase_lo).real, complex(phase_lo).imag)
        phh = (ctypes.c_double * 2)(complex(phase_hi).real, complex(phase_hi).imag)
        W.check(W.wilson_eo_face_unpack(self.c, fmt.c, int(mu), int(out_parity), int(bool(dagger)), pl, phh,
                                        float(alpha), _ptr(u), _ptr(recv_lo), _ptr(recv_hi), _ptr(out),
                                        int(nrhs), _stream()), "wilson_eo_face_unpack")
        return out

    # ---- clover-type site blocks ---------------------------------------------
    def clover_bytes(self, fmt: Format) -> int:
        n = W.weo_clover_bytes(self.c, fmt.c)
        if n == 0:
            raise W.WilsonEOError(W.WEO_ERR_ARG, "weo_clover_bytes")
        return n

    def pack_clover(self, blocks_canon: torch.Tensor, fmt: Format, invert=True, out=None):
        """Canonical blocks [Lt][Lz][Ly][Lx][2][6][6] -> packed (inverse if invert)."""
        lx, ly, lz, lt = self.dims
        if tuple(blocks_canon.shape) != (lt, lz, ly, lx, 2, 6, 6):
            raise ValueError(f"block shape {tuple(blocks_canon.shape)}")
        out = torch.empty(self.clover_bytes(fmt), dtype=torch.uint8, device=blocks_canon.device) \
            if out is None else out
        W.check(W.weo_pack_clover(self.c, fmt.c, _ptr(blocks_canon), _canon_prec(blocks_canon),
                                  int(bool(invert)), _ptr(out), _stream()), "weo_pack_clover")
        return out

    def clover_site(self, clv, x, fmt: Format, parity, y=None, alpha=1.0, nrhs=1, out=None):
        """out = y + alpha C_parity x (y None: out = C_parity x)."""
        out = self.new_spinor(fmt, nrhs) if out is None else out
        W.check(W.wilson_eo_clover_site(self.c, fmt.c, int(parity), _ptr(clv), _ptr(x), _ptr(y), float(alpha),
                                        _ptr(out), int(nrhs), _stream()), "wilson_eo_clover_site")
        return out

    def clover_hop(self, u, clv, x, fmt: Format, out_parity, dagger=False, y=None, alpha=1.0, nrhs=1,
                   out=None):
        """out = C_p hop(x) (y None) or y + alpha C_p hop(x)."""
        out = self.new_spinor(fmt, nrhs) if out is None else out
        W.check(W.wilson_eo_clover_hop(self.c, fmt.c, int(out_parity), int(bool(dagger)), _ptr(u), _ptr(clv),
                                       _ptr(x), _ptr(y), float(alpha), _ptr(out), int(nrhs), _stream()),
                "wilson_eo_clover_hop")
        return out

    def clover_apply(self, u, clv_inv, x, fmt: Format, dagger=False, nrhs=1, out=None, tmp=None):
        out = self.new_spinor(fmt, nrhs) if out is None else out
        tmp = self.new_spinor(fmt, nrhs) if tmp is None else tmp
        W.check(W.wilson_eo_clover_apply(self.c, fmt.c, int(bool(dagger)), _ptr(u), _ptr(clv_inv), _ptr(x),
                                         _ptr(out), _ptr(tmp), int(nrhs), _stream()), "wilson_eo_clover_apply")
        return out

    # ---- Schwarz alternating procedure (full fields: even half, odd half) -----
    def sap(self, u, eta, fmt: Format, block=(4, 4, 4, 4), ncy=4, nmr=4, nrhs=1, out=None):
        """psi = K eta, ncy SAP cycles with nmr MR steps per block solve, on
        nrhs full fields (FP32 format)."""
        sp = W.weo_sap_params()
        for i in range(4):
            sp.block[i] = int(block[i])
        sp.ncy, sp.nmr = int(ncy), int(nmr)
        nbytes = W.wilson_eo_sap_workspace_bytes(self.c, fmt.c, int(nrhs))
        if nbytes == 0:
            raise W.WilsonEOError(W.WEO_ERR_ARG, "wilson_eo_sap_workspace_bytes")
        ws = torch.empty(nbytes, dtype=torch.uint8, device=eta.device)
        out = self.new_spinor(fmt, 2 * nrhs) if out is None else out
        W.check(W.wilson_eo_sap(self.c, fmt.c, sp, _ptr(u), _ptr(eta), _ptr(out), _ptr(ws), nbytes, int(nrhs),
                                _stream()), "wilson_eo_sap")
        return out

    def apply(self, u, x, fmt: Format, dagger=False, nrhs=1, out=None, tmp=None):
        out = self.new_spinor(fmt, nrhs) if out is None else out
        tmp = self.new_spinor(fmt, nrhs) if tmp is None else tmp
        W.check(W.wilson_eo_apply(self.c, fmt.c, int(bool(dagger)), _ptr(u), _ptr(x), _ptr(out),
                                  _ptr(tmp), int(nrhs), _stream()), "wilson_eo_apply")
        return out


def to_device(a: np.ndarray, device="cuda") -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).to(device)
