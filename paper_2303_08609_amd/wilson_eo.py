"""ctypes binding of libwilson_eo.so (names and arguments as in wilson_eo.h).

Argument marshalling only: every computation runs in the library's HIP
kernels.  The library is loaded from this package directory (or from the
path in WILSON_EO_LIB); if it is missing ``load()`` raises instead of falling
back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os
import warnings

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwilson_eo.so")

WEO_OK = 0
WEO_ERR_ARG = -1
WEO_ERR_DIMS = -2
WEO_ERR_ALIGN = -3
WEO_ERR_FORMAT = -4
WEO_ERR_HIP = -5
WEO_ERR_WORKSPACE = -6
WEO_NOT_CONVERGED = 1
WEO_BREAKDOWN = 2

WEO_F64, WEO_F32, WEO_F16, WEO_BF16 = 0, 1, 2, 3
WEO_LINK18, WEO_LINK12 = 0, 1
WEO_MAX_RHS = 16
WEO_NOALLOC_SCRATCH_BYTES = 134217728
WEO_OP_M, WEO_OP_MDAGM, WEO_OP_DW = 0, 1, 2
WEO_SOLVER_CG, WEO_SOLVER_BICGSTAB, WEO_SOLVER_BLOCK_CG, WEO_SOLVER_SAP_GCR = 0, 1, 2, 3
WEO_FORCE_PROJECT, WEO_FORCE_ACCUMULATE = 1, 2


class weo_lattice(C.Structure):
    _fields_ = [("dims", C.c_int * 4), ("kappa", C.c_double), ("bc", (C.c_double * 2) * 4)]


class weo_format(C.Structure):
    _fields_ = [("spinor_prec", C.c_int), ("link_prec", C.c_int), ("link_fmt", C.c_int)]


class weo_sap_params(C.Structure):
    _fields_ = [("block", C.c_int * 4), ("ncy", C.c_int), ("nmr", C.c_int)]


class weo_solver_params(C.Structure):
    _fields_ = [("op", C.c_int), ("nrhs", C.c_int), ("tol", C.c_double), ("maxiter", C.c_int),
                ("x0_given", C.c_int), ("mixed", C.c_int), ("inner", weo_format),
                ("inner_tol", C.c_double), ("max_outer", C.c_int), ("check_every", C.c_int),
                ("method", C.c_int), ("clover", C.c_void_p), ("clover_inner", C.c_void_p),
                ("sap", weo_sap_params), ("gcr_nkv", C.c_int)]


class weo_solver_info(C.Structure):
    _fields_ = [("status", C.c_int), ("iters", C.c_int), ("outer_iters", C.c_int),
                ("applies", C.c_int), ("true_rel_resid", C.c_double * WEO_MAX_RHS),
                ("seconds", C.c_double)]


_P = C.POINTER
_vp = C.c_void_p
_SIGS = {
    "wilson_eo_strerror": (C.c_char_p, [C.c_int]),
    "weo_selftest": (C.c_int, []),
    "weo_format_supported": (C.c_int, [_P(weo_format)]),
    "weo_set_mrhs_shape": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int]),
    "weo_tuning_report": (C.c_int, [C.c_char_p, C.c_size_t]),
    "weo_gauge_bytes": (C.c_size_t, [_P(weo_lattice), _P(weo_format)]),
    "weo_spinor_bytes": (C.c_size_t, [_P(weo_lattice), _P(weo_format), C.c_int]),
    "weo_pack_gauge": (C.c_int, [_P(weo_lattice), _P(weo_format), _vp, C.c_int, _vp, _vp]),
    "weo_pack_spinor": (C.c_int, [_P(weo_lattice), _P(weo_format), C.c_int, _vp, C.c_int,
                                  C.c_double, _vp, _vp]),
    "weo_unpack_spinor": (C.c_int, [_P(weo_lattice), _P(weo_format), C.c_int, _vp, C.c_double,
                                    _vp, C.c_int, _vp]),
    "wilson_eo_hop": (C.c_int, [_P(weo_lattice), _P(weo_format), C.c_int, C.c_int, _vp, _vp,
                                _vp, C.c_int, _vp]),
    "wilson_eo_hop_axpy": (C.c_int, [_P(weo_lattice), _P(weo_format), C.c_int, C.c_int, C.c_double,
                                     _vp, _vp, _vp, _vp, C.c_int, _vp]),
    "weo_face_bytes": (C.c_size_t, [_P(weo_lattice), _P(weo_format), C.c_int, C.c_int]),
    "wilson_eo_face_pack": (C.c_int, [_P(weo_lattice), _P(weo_format), C.c_int, C.c_int, C.c_int, _vp,
                                      _vp, _vp, _vp, C.c_int, _vp]),
    "wilson_eo_face_unpack": (C.c_int, [_P(weo_lattice), _P(weo_format), C.c_int, C.c_int, C.c_int,
                                        _P(C.c_double), _P(C.c_double), C.c_double, _vp, _vp, _vp,
                                        _vp, C.c_int, _vp]),
    "weo_clover_bytes": (C.c_size_t, [_P(weo_lattice), _P(weo_format)]),
    "weo_pack_clover": (C.c_int, [_P(weo_lattice), _P(weo_format), _vp, C.c_int, C.c_int, _vp, _vp]),
    "wilson_eo_clover_site": (C.c_int, [_P(weo_lattice), _P(weo_format), C.c_int, _vp, _vp, _vp, C.c_double,
                                        _vp, C.c_int, _vp]),
    "wilson_eo_clover_hop": (C.c_int, [_P(weo_lattice), _P(weo_format), C.c_int, C.c_int, _vp, _vp, _vp, _vp,
                                       C.c_double, _vp, C.c_int, _vp]),
    "wilson_eo_clover_apply": (C.c_int, [_P(weo_lattice), _P(weo_format), C.c_int, _vp, _vp, _vp, _vp, _vp,
                                         C.c_int, _vp]),
    "wilson_eo_apply": (C.c_int, [_P(weo_lattice), _P(weo_format), C.c_int, _vp, _vp, _vp,
                                  _vp, C.c_int, _vp]),
    "wilson_eo_apply_noalloc": (C.c_int, [_P(weo_lattice), _P(weo_format), C.c_int, _vp, _vp, _vp,
                                          C.c_int, _vp]),
    "wilson_eo_cg_workspace_bytes": (C.c_size_t, [_P(weo_lattice), _P(weo_format),
                                                  _P(weo_solver_params)]),
    "wilson_eo_cg": (C.c_int, [_P(weo_lattice), _P(weo_format), _P(weo_solver_params), _vp, _vp,
                               _vp, _vp, _vp, C.c_size_t, _P(weo_solver_info), _vp]),
    "wilson_eo_sap_workspace_bytes": (C.c_size_t, [_P(weo_lattice), _P(weo_format), C.c_int]),
    "wilson_eo_sap": (C.c_int, [_P(weo_lattice), _P(weo_format), _P(weo_sap_params), _vp, _vp, _vp, _vp,
                                C.c_size_t, C.c_int, _vp]),
    "wilson_eo_force": (C.c_int, [_P(weo_lattice), _P(weo_format), _vp, _vp, _vp, _vp, _vp,
                                  C.c_double, C.c_int, _vp, C.c_int, _vp]),
}

_lib = None


class WilsonEOError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} (code {code})")


class SolverWarning(RuntimeWarning):
    """A solve ended without meeting its tolerance (WEO_NOT_CONVERGED) or
    broke down (WEO_BREAKDOWN); the returned x is the last iterate."""


def load(path: str | None = None):
    """Load libwilson_eo.so and declare its signatures (idempotent).  The
    environment variable WILSON_EO_LIB names another build of the library
    (e.g. the sanitizer build) to load instead of the in-tree one."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or os.environ.get("WILSON_EO_LIB") or LIB_PATH
    if not os.path.exists(path):
        raise OSError(f"{path} is not built; run `python -m paper_2303_08609_amd.build`")
    lib = C.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_names():
    return list(_SIGS)


def strerror(code: int) -> str:
    return load().wilson_eo_strerror(int(code)).decode()


def check(code: int, where: str) -> int:
    """Raise on a negative (error) code; warn on a positive solver status."""
    if code < 0:
        raise WilsonEOError(code, where)
    if code > 0:
        warnings.warn(f"{where}: {strerror(code)} (status {code})", SolverWarning, stacklevel=2)
    return code


def _call(name):
    def f(*args):
        return getattr(load(), name)(*args)
    f.__name__ = name
    return f


weo_selftest = _call("weo_selftest")
weo_format_supported = _call("weo_format_supported")
weo_set_mrhs_shape = _call("weo_set_mrhs_shape")
weo_tuning_report = _call("weo_tuning_report")


def tuning_report() -> str:
    n = weo_tuning_report(None, 0)
    buf = C.create_string_buffer(n + 1)
    weo_tuning_report(buf, n + 1)
    return buf.value.decode()
weo_gauge_bytes = _call("weo_gauge_bytes")
weo_spinor_bytes = _call("weo_spinor_bytes")
weo_pack_gauge = _call("weo_pack_gauge")
weo_pack_spinor = _call("weo_pack_spinor")
weo_unpack_spinor = _call("weo_unpack_spinor")
wilson_eo_hop = _call("wilson_eo_hop")
wilson_eo_hop_axpy = _call("wilson_eo_hop_axpy")
wilson_eo_apply = _call("wilson_eo_apply")
wilson_eo_apply_noalloc = _call("wilson_eo_apply_noalloc")
weo_clover_bytes = _call("weo_clover_bytes")
weo_pack_clover = _call("weo_pack_clover")
wilson_eo_clover_site = _call("wilson_eo_clover_site")
wilson_eo_clover_hop = _call("wilson_eo_clover_hop")
wilson_eo_clover_apply = _call("wilson_eo_clover_apply")
weo_face_bytes = _call("weo_face_bytes")
wilson_eo_face_pack = _call("wilson_eo_face_pack")
wilson_eo_face_unpack = _call("wilson_eo_face_unpack")
wilson_eo_cg_workspace_bytes = _call("wilson_eo_cg_workspace_bytes")
wilson_eo_cg = _call("wilson_eo_cg")
wilson_eo_force = _call("wilson_eo_force")
wilson_eo_sap_workspace_bytes = _call("wilson_eo_sap_workspace_bytes")
wilson_eo_sap = _call("wilson_eo_sap")
wilson_eo_strerror = _call("wilson_eo_strerror")


def make_lattice(dims, kappa, bc=((1, 0), (1, 0), (1, 0), (-1, 0))) -> weo_lattice:
    lat = weo_lattice()
    for i in range(4):
        lat.dims[i] = int(dims[i])
        b = complex(*bc[i]) if isinstance(bc[i], (tuple, list)) else complex(bc[i])
        lat.bc[i][0] = b.real
        lat.bc[i][1] = b.imag
    lat.kappa = float(kappa)
    return lat


def make_format(spinor_prec=WEO_F32, link_prec=None, link_fmt=WEO_LINK18) -> weo_format:
    f = weo_format()
    f.spinor_prec = int(spinor_prec)
    f.link_prec = int(spinor_prec if link_prec is None else link_prec)
    f.link_fmt = int(link_fmt)
    return f
