"""wilson_eo_apply_noalloc (the operator with its intermediate field in a
library-owned device array) against wilson_eo_apply with a caller buffer,
through the C ABI: two calls in a row, the second on a smaller input, each
bit-identical to the entry point it stands in for (same kernels, same
launches), and the size limit enforced before any device work."""
import ctypes as C

import numpy as np
import pytest
import torch

from oracle import wilson as W
from paper_2303_08609_amd import inputs
from paper_2303_08609_amd import wilson_eo as WE
from paper_2303_08609_amd.ops import Format, Lattice, _ptr, _stream, to_device
from tests._helpers import AP, ROUND, rel_err

pytestmark = pytest.mark.gpu


def _run(dims, fmt_t, nrhs, dagger, seed):
    fmt = Format(*fmt_t)
    lat = Lattice(dims, 0.126, AP)
    u = inputs.gen_gauge(dims, 0.5, seed)
    psi = inputs.gen_spinor_half(dims, seed + 1, nrhs=nrhs if nrhs > 1 else None)
    u_d = lat.pack_gauge(to_device(u), fmt)
    x_d = lat.pack_spinor(to_device(psi), fmt)
    ref = lat.new_spinor(fmt, nrhs)
    tmp = lat.new_spinor(fmt, nrhs)
    rc = WE.wilson_eo_apply(lat.c, fmt.c, int(dagger), _ptr(u_d), _ptr(x_d), _ptr(ref), _ptr(tmp), nrhs,
                            _stream())
    assert rc == WE.WEO_OK
    out = lat.new_spinor(fmt, nrhs)
    out.fill_(0xFF)                       # NaN patterns: every byte must be written
    rc = WE.wilson_eo_apply_noalloc(lat.c, fmt.c, int(dagger), _ptr(u_d), _ptr(x_d), _ptr(out), nrhs,
                                    _stream())
    assert rc == WE.WEO_OK, WE.strerror(rc)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    # and the result is the operator (oracle on the rounded inputs)
    sp, lp, reals = fmt_t
    from tests._helpers import link_as_stored
    got = lat.unpack_spinor(out, fmt, nrhs=nrhs).cpu().numpy()
    got = got if nrhs > 1 else got[None]
    ps = ROUND[sp](psi) if nrhs > 1 else ROUND[sp](psi)[None]
    for r in range(nrhs):
        want = W.apply_m(link_as_stored(u, lp, reals), ps[r], 0.126, np.array(AP), dagger=dagger)
        assert rel_err(got[r], want) <= {"f64": 1e-12, "f32": 1e-6}[sp]


def test_noalloc_apply_two_calls_second_smaller():
    print("noalloc apply: 16^3x32 f32 2 rhs, then 8^4 f64 1 rhs", flush=True)
    _run((16, 16, 16, 32), ("f32", "f32", 18), 2, False, 31)
    _run((8, 8, 8, 8), ("f64", "f64", 12), 1, True, 33)
