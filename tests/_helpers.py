"""Shared test helpers: rounding of canonical inputs to a storage precision on
the CPU (so the oracle sees exactly the values the kernels read), relative
errors, and GPU set-up for the parity tests."""
from __future__ import annotations

import numpy as np

AP = (1, 1, 1, -1)


def round_f32(a):
    return a.astype(np.complex64).astype(np.complex128)


def round_f16(a):
    # the library narrows FP64 input to FP32 first, then to binary16 (RNE)
    r = a.real.astype(np.float32).astype(np.float16).astype(np.float64)
    i = a.imag.astype(np.float32).astype(np.float16).astype(np.float64)
    return r + 1j * i


def _bf16(x):
    f = np.ascontiguousarray(x.astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def round_bf16(a):
    return _bf16(a.real) + 1j * _bf16(a.imag)


ROUND = {"f64": lambda a: a.astype(np.complex128), "f32": round_f32, "f16": round_f16,
         "bf16": round_bf16}


def reconstruct_row2(u):
    r0, r1 = u[..., 0, :], u[..., 1, :]
    r2 = np.conj(np.stack([r0[..., 1] * r1[..., 2] - r0[..., 2] * r1[..., 1],
                           r0[..., 2] * r1[..., 0] - r0[..., 0] * r1[..., 2],
                           r0[..., 0] * r1[..., 1] - r0[..., 1] * r1[..., 0]], axis=-1))
    out = u.copy()
    out[..., 2, :] = r2
    return out


def link_as_stored(u, prec, reals):
    """The links the kernel effectively uses: rounded, and for 12 reals with
    row 2 rebuilt (in FP64 here) from the rounded rows 0 and 1."""
    q = ROUND[prec](u)
    return reconstruct_row2(q) if reals == 12 else q


def rel_err(a, b):
    a = np.asarray(a).reshape(-1)
    b = np.asarray(b).reshape(-1)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def site_rel_max(a, b):
    """Largest per-site relative error max_s ||a_s - b_s|| / ||b_s|| over the
    12-component records of two spinor fields (any leading shape ending in
    (4, 3)): a defect confined to a few sites is not diluted by the rest of
    the field as it is in the norm-wise ``rel_err``."""
    a = np.asarray(a).reshape(-1, 12)
    b = np.asarray(b).reshape(-1, 12)
    return float((np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)).max())


def sample_sites(dims, n, seed):
    """Half indices of sites on every face and corner of the lattice plus n
    random ones (for checks at sampled sites on lattices too large for the
    whole-field oracle)."""
    lx, ly, lz, lt = dims
    vh = lx * ly * lz * lt // 2
    g = np.random.default_rng(seed)
    corners = [0, lx // 2 - 1, vh - 1, vh - lx // 2, (lx // 2) * (ly - 1),
               (lx // 2) * ly * (lz - 1), (lx // 2) * ly * lz * (lt - 1)]
    return sorted(set(corners + [int(v) for v in g.integers(0, vh, n)]))


_GAUGE_CACHE = {}


def cached_gauge(dims, eps, seed):
    """gen_gauge with a small per-process cache (big lattices take seconds)."""
    from paper_2303_08609_amd import inputs
    key = (tuple(dims), float(eps), int(seed))
    if key not in _GAUGE_CACHE:
        if len(_GAUGE_CACHE) > 2:
            _GAUGE_CACHE.clear()
        _GAUGE_CACHE[key] = inputs.gen_gauge(dims, eps, seed)
    return _GAUGE_CACHE[key]
