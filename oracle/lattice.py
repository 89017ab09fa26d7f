"""Lattice coordinates, parity and even/odd compaction (oracle side).

Arrays are ordered [t][z][y][x] with x fastest; dims are given as
(Lx, Ly, Lz, Lt).  A site is even when x + y + z + t is even (paper Sec. 3.3,
Fig. 4).  The sites of one parity are stored compacted along x: the site of
parity p with half index xh in row (y, z, t) has x = 2*xh + ((y+z+t+p) & 1).
All extents must be even so that the checkerboard is consistent across the
periodic wrap.
"""
import numpy as np


def dims_of(psi_full: np.ndarray) -> tuple:
    lt, lz, ly, lx = psi_full.shape[:4]
    return (lx, ly, lz, lt)


def coords(dims):
    """Coordinate arrays x, y, z, t of shape (Lt, Lz, Ly, Lx)."""
    lx, ly, lz, lt = dims
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly),
                             np.arange(lx), indexing="ij")
    return x, y, z, t


def parity_mask(dims, parity: int) -> np.ndarray:
    x, y, z, t = coords(dims)
    return ((x + y + z + t) % 2) == parity


def _x_of_half(dims, parity: int):
    lx, ly, lz, lt = dims
    t, z, y, xh = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly),
                              np.arange(lx // 2), indexing="ij")
    x = 2 * xh + ((y + z + t + parity) % 2)
    return t, z, y, x


def half_to_full(half: np.ndarray, parity: int, dims) -> np.ndarray:
    """Scatter a one-parity array [t][z][y][x/2][...] into a zero full array."""
    lx, ly, lz, lt = dims
    full = np.zeros((lt, lz, ly, lx) + half.shape[4:], dtype=half.dtype)
    t, z, y, x = _x_of_half(dims, parity)
    full[t, z, y, x] = half
    return full


def full_to_half(full: np.ndarray, parity: int) -> np.ndarray:
    """Gather the sites of one parity from a full array."""
    dims = dims_of(full)
    t, z, y, x = _x_of_half(dims, parity)
    return full[t, z, y, x]


def half_index_coords(dims, parity: int, ih: int) -> tuple:
    """(x, y, z, t) of half index ih (x/2 fastest) in the given parity."""
    lx, ly, lz, lt = dims
    xh = ih % (lx // 2)
    r = ih // (lx // 2)
    y = r % ly
    r //= ly
    z = r % lz
    t = r // lz
    return (2 * xh + ((y + z + t + parity) % 2), y, z, t)
