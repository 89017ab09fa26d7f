"""Flop and byte model of the even-odd Wilson operator (oracle).

Paper Sec. 2 quotes 1368 flop per lattice site for D_W with its gamma
convention and a byte-per-flop ratio of 1.12.  The model here counts:

* per hop output site and direction: spin projection 6 complex adds (12 flop),
  SU(3) times two colour vectors 2 x (9 cmul + 6 cadd) (132 flop),
  reconstruction and accumulation 12 complex adds (24 flop): 168 flop; eight
  directions minus the first accumulation (a store): 8 * 168 - 24 = 1320;
* D_W adds the diagonal term psi - kappa * (H psi): a real scale and a complex subtract on
  12 components, 48 flop, giving 1368 = the paper's count;
* one application of M = 1 - kappa^2 H_eo H_oe on the even sublattice is two
  hops over V/2 output sites each: 1320 * V flop (the axpy is not counted).

Bytes are "ideal reuse" algorithmic bytes: each hop reads every link once
(all 4V links), its input spinor once and writes its output once; M also reads
the even input once more for the axpy.  The paper's own ratio counts no reuse:
8 neighbour spinors + 8 links read and one spinor written per site.
"""

FLOP_PER_DIRECTION = 12 + 2 * (9 * 6 + 6 * 2) + 24
FLOP_HOP_SITE = 8 * FLOP_PER_DIRECTION - 24
FLOP_DIAG_SITE = 12 * (2 + 2)   # real kappa times complex, then complex subtract
FLOP_DW_SITE = FLOP_HOP_SITE + FLOP_DIAG_SITE

REAL_BYTES = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}


def spinor_site_bytes(prec: str) -> int:
    return 24 * REAL_BYTES[prec]


def link_bytes(prec: str, reals: int) -> int:
    return reals * REAL_BYTES[prec]


def hop_bytes_per_output_site(spinor_prec: str, link_prec: str, link_reals: int) -> int:
    """8 links + one input spinor read + one output spinor written, per output
    site of one hop (ideal reuse)."""
    return 8 * link_bytes(link_prec, link_reals) + 2 * spinor_site_bytes(spinor_prec)


def apply_bytes_per_site(spinor_prec: str, link_prec: str, link_reals: int) -> float:
    """Per full-lattice site of one M application: two hops over V/2 output
    sites plus the even input read once more for the axpy."""
    return hop_bytes_per_output_site(spinor_prec, link_prec, link_reals) + \
        0.5 * spinor_site_bytes(spinor_prec)


def apply_flop(volume: int) -> int:
    return FLOP_HOP_SITE * volume


def paper_no_reuse_bytes_per_site(real_bytes: int = 4, link_reals: int = 18) -> int:
    """The paper's ratio: 8 neighbour spinors and 8 links read, the site's
    own spinor read for the diagonal term, one spinor written."""
    spinor = 24 * real_bytes
    return 8 * spinor + 8 * link_reals * real_bytes + spinor + spinor


def footprint_bytes(dims, real_bytes: int = 4, link_reals: int = 18):
    """(gauge bytes, full-lattice spinor bytes) of a lattice."""
    lx, ly, lz, lt = dims
    v = lx * ly * lz * lt
    return 4 * v * link_reals * real_bytes, v * 24 * real_bytes
