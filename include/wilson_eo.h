/*
 * wilson_eo.h -- C ABI of libwilson_eo.so, the even-odd preconditioned Wilson
 * fermion operator on AMD MI355X (gfx950).
 *
 * The operator (Kanamori, Nitadori, Matsufuru, HPCAsia 2023 Workshops,
 * arXiv:2303.08609, Sec. 2):
 *
 *   Eq. (1):  D_W = 1 - kappa H,
 *             H(x,y) = sum_mu [ (1 - gamma_mu) U_mu(x) delta_{x+mu,y}
 *                             + (1 + gamma_mu) U_mu(x-mu)^dag delta_{x-mu,y} ]
 *   Eqs. (3)-(4) with D_ee = D_oo = 1 (Wilson):
 *             M = 1 - kappa^2 H_eo H_oe   on the even sublattice,
 *   where H_oe = P_o H P_e maps even sites to odd sites and H_eo = P_e H P_o.
 *
 * Conventions
 *   - Lattice extents Lx, Ly, Lz, Lt; each even and >= 2.  x runs fastest.
 *     A site is even when x+y+z+t is even.  The sites of one parity are
 *     compacted along x (Sec. 3.3, Fig. 4): half index
 *       ih = (x >> 1) + Lx/2 * (y + Ly * (z + Lz * t)).
 *   - gamma matrices: Euclidean Dirac representation,
 *       gamma_k = [[0, -i sigma_k], [i sigma_k, 0]] (k = x, y, z),
 *       gamma_t = diag(1, 1, -1, -1).
 *   - Boundary conditions: a U(1) phase per direction.  A hop that crosses
 *     the lattice edge forward is multiplied by bc[mu], backward by conj(bc[mu]).
 *     Phases are applied inside the kernels, never folded into the links.
 *   - "dagger" selects the Hermitian conjugate operator (H^dag swaps the two
 *     projectors; M^dag = gamma5 M gamma5).
 *   - Canonical host-side layouts (complex, interleaved re/im), accepted by the
 *     pack/unpack calls in complex128 (WEO_F64) or complex64 (WEO_F32):
 *       gauge   [4][Lt][Lz][Ly][Lx][3][3]        U_mu(x)_{ab}, mu = x,y,z,t
 *       spinor  [nrhs][Lt][Lz][Ly][Lx/2][4][3]   one parity, [spin][colour]
 *   - Packed device layouts are private to the library; size them with
 *     weo_gauge_bytes / weo_spinor_bytes and fill them with the pack calls.
 *
 * Memory and streams
 *   - Every buffer pointer is a DEVICE pointer owned by the caller; the library
 *     never allocates, frees or retains caller memory.  Base pointers must be
 *     256-byte aligned (WEO_ERR_ALIGN otherwise).  Input and output buffers
 *     must not overlap (WEO_ERR_ARG where detectable).
 *   - "stream" is a hipStream_t (NULL = the default stream).  pack, unpack,
 *     hop, apply and force are asynchronous on that stream.  wilson_eo_cg
 *     synchronises the stream before it returns.
 *   - Errors are returned, never raised or aborted on; arguments are validated
 *     before any HIP call is made.
 */
#ifndef WILSON_EO_H
#define WILSON_EO_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define WEO_OK              0
#define WEO_ERR_ARG        -1   /* null pointer, bad enum, bad count, aliasing */
#define WEO_ERR_DIMS       -2   /* an extent odd, < 2, or the volume too large */
#define WEO_ERR_ALIGN      -3   /* a base pointer not 256-byte aligned */
#define WEO_ERR_FORMAT     -4   /* precision / link-format combination not built */
#define WEO_ERR_HIP        -5   /* a HIP runtime call failed */
#define WEO_ERR_WORKSPACE  -6   /* workspace missing or smaller than required */
#define WEO_NOT_CONVERGED   1   /* solver hit maxiter / max_outer; x is the best iterate */
#define WEO_BREAKDOWN       2   /* solver met a non-positive or non-finite scalar */

/* ---- precisions and link formats --------------------------------------- */
#define WEO_F64   0
#define WEO_F32   1
#define WEO_F16   2
#define WEO_BF16  3

#define WEO_LINK18 0   /* all 9 complex entries stored */
#define WEO_LINK12 1   /* rows 0 and 1 stored; row 2 = conj(row0 x row1),
                          exact for det U = 1 (SU(3)) */

#define WEO_MAX_RHS 16

typedef struct {
    int    dims[4];    /* Lx, Ly, Lz, Lt: each even and >= 2 */
    double kappa;      /* hopping parameter, kappa = 1/(8 + 2m) (Sec. 2) */
    double bc[4][2];   /* boundary phase (re, im) per direction x, y, z, t */
} weo_lattice;

/* Storage format of the fields an operation reads and writes.  Arithmetic is
 * FP64 for WEO_F64 spinors and FP32 otherwise.  Built combinations
 * (spinor_prec / link_prec / link_fmt):
 *   F64/F64/18|12, F32/F32/18|12, F16/F16/18|12, BF16/F16/18|12.            */
typedef struct {
    int spinor_prec;
    int link_prec;
    int link_fmt;
} weo_format;

/* Human-readable text of a status code (static storage). */
const char* wilson_eo_strerror(int code);

/* Host-only self-test of the library's index arithmetic (fast division,
 * even-odd site decoding, neighbour indices and boundary flags, workgroup
 * remap) against direct coordinate arithmetic.  Needs no GPU.  Returns 0 on
 * success, a positive code naming the failed check otherwise. */
int weo_selftest(void);

/* 1 if the format combination is built into this library, else 0. */
int weo_format_supported(const weo_format* fmt);

/* Launch shape of hops with nrhs > 1 (used by hop, apply and the solvers).
 * The multi-rhs kernels share each loaded link between right-hand sides
 * (the batching the paper's solvers would need for many sources; the paper
 * itself treats one).  nr = 0 (default): an autotuner times every candidate
 * shape on the first call per (lattice, format, nrhs, epilogue) -- on the
 * caller's stream and buffers, with one stream synchronisation -- and caches
 * the fastest for the process.  nr = 1: one lane per (site, rhs).
 * nr in {2, 3, 4, 6} (FP64 uses at most 3): a lane applies each link it
 * loads to nr right-hand sides.  nr = -1 / -3: one lane per site holding its
 * 8 links in registers while it walks all right-hand sides (neighbour ring
 * depth 1 / 3; FP32, FP16 and BF16 spinors, FP64 falls back to nr = 1);
 * nr = -2 / -4: the same with FP16 arithmetic on packed pairs (FP16
 * spinors and links; other formats fall back to -1 / -3).  For these,
 * sites per workgroup is 64, 128 or 256.  nr = -5: the 64 sites' links
 * staged in LDS and shared by `sites` wavefronts (2, 3, 4, 6, 8 or 12;
 * clamped to 4 for FP64 and 8 for FP16/BF16 spinors), each walking every
 * sites-th right-hand side (all formats); here split = 0 sweeps the lattice
 * once for all right-hand sides, split = f in 1..16 once per f of them
 * (the links staged again per sweep).  persist in {0, 1}, bz in -64..64 and
 * split in {0, 1} (for nr > 1) complete the shape.  bz > 0 visits the lattice in strips of bz z-planes, all t per
 * strip; bz < 0 the same in columns of half an (x, y) plane (y below
 * ly / 2, then the rest) times -bz z-planes (both ignored where the lattice
 * or workgroup size does not allow them);
 * split = 1 gives each group of nr rhs its own workgroups and sweep of the
 * lattice.  Returns WEO_ERR_ARG for other values.  The setting is
 * process-wide. */
int weo_set_mrhs_shape(int nr, int sites, int persist, int bz, int split);

/* The autotuner's cached choices as JSON lines in buf (NUL-terminated,
 * truncated to len bytes), one per (lattice, format, nrhs, epilogue: 1 axpy,
 * 2 norm partials); returns the untruncated length.  buf may be NULL to
 * query the length.  A multi-rhs launch is tuned on its first call by
 * timing every candidate shape on the caller's stream and buffers, except
 * an in-place axpy (y is out), which runs untuned.  With the environment
 * variable WILSON_EO_TUNE_CACHE naming a file, tuned shapes are appended to
 * it (a header line with the cache version and GPU architecture, then one
 * text line per key) and read back by later processes, which then skip the
 * timing for those keys; an entry whose shape is not a current candidate
 * for its key is ignored, and a file with another header is rewritten.
 * WEO_TUNE=0 disables tuning (and the cache). */
int weo_tuning_report(char* buf, size_t len);

/* Bytes of the packed gauge field (all 4V links) in format fmt; 0 on error. */
size_t weo_gauge_bytes(const weo_lattice* lat, const weo_format* fmt);

/* Bytes of nrhs packed one-parity spinors (V/2 sites each); 0 on error. */
size_t weo_spinor_bytes(const weo_lattice* lat, const weo_format* fmt, int nrhs);

/* Convert a canonical gauge field (device memory, complex128 if canon_prec is
 * WEO_F64, complex64 if WEO_F32) into the packed format fmt (links rounded to
 * nearest even; WEO_LINK12 drops row 2).  Phases are not applied here. */
int weo_pack_gauge(const weo_lattice* lat, const weo_format* fmt,
                   const void* u_canon, int canon_prec,
                   void* u_packed, void* stream);

/* Convert nrhs canonical one-parity spinors into the packed format, multiplying
 * by scale on the way (scale lets FP16 spinors be kept near unit magnitude). */
int weo_pack_spinor(const weo_lattice* lat, const weo_format* fmt, int nrhs,
                    const void* s_canon, int canon_prec, double scale,
                    void* s_packed, void* stream);

/* Inverse of weo_pack_spinor: canonical = packed * scale. */
int weo_unpack_spinor(const weo_lattice* lat, const weo_format* fmt, int nrhs,
                      const void* s_packed, double scale,
                      void* s_canon, int canon_prec, void* stream);

/* One hopping block (Eq. (1) off-diagonal part, paper Fig. 2, without -kappa):
 *   out = P_{out_parity} H P_{1-out_parity} in      (dagger = 0)
 *   out = P_{out_parity} H^dag P_{1-out_parity} in  (dagger = 1)
 * in and out are nrhs packed spinors of parity 1-out_parity and out_parity. */
int wilson_eo_hop(const weo_lattice* lat, const weo_format* fmt,
                  int out_parity, int dagger,
                  const void* u, const void* in, void* out,
                  int nrhs, void* stream);

/* Hop with an axpy epilogue: out = y + alpha * P_{out_parity} H P_{1-out_parity} in
 * (H^dag with dagger = 1).  With D_ee = D_oo = 1 this gives the steps either
 * side of the even-odd solve of Eqs. (4)-(5):
 *   right-hand side of Eq. (4):  b_e  = eta_e + kappa H_eo eta_o   (out_parity 0)
 *   Eq. (5):                     xi_o = eta_o + kappa H_oe xi_e    (out_parity 1)
 * y (parity out_parity) may be the same buffer as out; in must not overlap out. */
int wilson_eo_hop_axpy(const weo_lattice* lat, const weo_format* fmt,
                       int out_parity, int dagger, double alpha,
                       const void* u, const void* in, const void* y, void* out,
                       int nrhs, void* stream);

/* ---- a hop split along a direction (domain decomposition, Sec. 3.6, 4.1) ---
 * A device holding a block of consecutive mu slices (even length) of the
 * lattice computes its share of a hop in three calls per split direction mu:
 *   1. wilson_eo_hop / wilson_eo_hop_axpy on the block with bc[mu] = {0, 0}
 *      for every split direction: a zero phase drops exactly the terms that
 *      cross the block's mu faces;
 *   2. wilson_eo_face_pack: the two faces its neighbours along mu need, from
 *      the input field (parity 1 - out_parity);
 *   3. after the exchange, wilson_eo_face_unpack adds the two received faces
 *      to the output (slices x_mu = 0 and x_mu = L_mu - 1).
 * Each face holds, per site of one parity, the two-component half spinor of
 * the projected input (6 complex in the spinor precision):
 *   send_lo[f] = (1 - S gamma_mu) psi(f, x_mu = 0)                   -> block below
 *   send_hi[f] = U_mu(f, L_mu-1)^dag (1 + S gamma_mu) psi(f, x_mu = L_mu-1) -> block above
 * with S = +1 (dagger 0) or -1 (dagger 1): the backward face is multiplied
 * by the link on the sender, which owns it.  The receiver rebuilds the full
 * spinor from the half spinor.  Face sites f: for y, z, t the sites of the
 * slice in the library's compacted order (x/2 fastest, then the remaining
 * coordinates in x, y, z, t order); for x, where the slice holds one parity
 * only in every other (y, z, t) row, f = (y + Ly (z + Lz t)) / 2.  With an
 * even block length the sites across a face carry the same f on both sides.
 * The receiver's recv_lo is the block below's send_hi and recv_hi the block
 * above's send_lo; on one device holding the whole lattice recv_lo = send_hi
 * and recv_hi = send_lo (the paper's forced exchange with itself, which its
 * Table 1 runs use in all four directions).  Face buffers hold nrhs faces of
 * weo_face_bytes(lat, fmt, mu, 1) bytes each; layout private to the library.
 * mu outside 0..3: WEO_ERR_ARG (weo_face_bytes: 0). */
size_t weo_face_bytes(const weo_lattice* lat, const weo_format* fmt, int mu, int nrhs);

/* Pack the two mu faces of nrhs input spinors (parity 1 - out_parity) for a
 * hop to out_parity.  send_lo and send_hi must not overlap each other, u or in. */
int wilson_eo_face_pack(const weo_lattice* lat, const weo_format* fmt, int mu,
                        int out_parity, int dagger,
                        const void* u, const void* in,
                        void* send_lo, void* send_hi, int nrhs, void* stream);

/* Add the received mu faces to nrhs output spinors of parity out_parity:
 *   out(f, x_mu = 0)      += alpha conj(phase_lo) [(1 + S gamma_mu) part rebuilt from recv_lo[f]]
 *   out(f, x_mu = L_mu-1) += alpha phase_hi [(1 - S gamma_mu) part rebuilt from U_mu recv_hi[f]]
 * phase_lo / phase_hi (host arrays {re, im}) are the mu boundary phase for a
 * face that is the global lattice edge and {1, 0} otherwise; alpha matches the
 * bulk call (1 for wilson_eo_hop, its alpha for wilson_eo_hop_axpy).
 * Must follow the bulk call on the same stream; only the two face slices of
 * out are touched.  recv_lo / recv_hi must not overlap out. */
int wilson_eo_face_unpack(const weo_lattice* lat, const weo_format* fmt, int mu,
                          int out_parity, int dagger,
                          const double phase_lo[2], const double phase_hi[2], double alpha,
                          const void* u, const void* recv_lo, const void* recv_hi,
                          void* out, int nrhs, void* stream);

/* ---- site-local diagonal blocks (clover-type D_ee, D_oo; Sec. 2) ----------
 * With a clover term the diagonal blocks of Eqs. (3)-(5) act site by site
 * (Sec. 2).  Here D = A - kappa H with A(x) a 12 x 12 Hermitian
 * site matrix commuting with gamma5 (as 1 + c sigma_mu_nu F_mu_nu does), so
 * that D_eo = -kappa H_eo, D_oe = -kappa H_oe and A is given by two 6 x 6
 * Hermitian blocks in the gamma5 eigenbasis (gamma5 = -[[0,1],[1,0]] in 2 x 2
 * spin blocks of the Dirac representation):
 *     psi_A = (psi_{s} + psi_{s+2}) / sqrt2,  s = 0, 1   -> block 0 (gamma5 = -1)
 *     psi_B = (psi_{s} - psi_{s+2}) / sqrt2               -> block 1 (gamma5 = +1)
 * each 6-vector ordered k = 3 s + colour.
 * Canonical layout (complex128 / complex64, full lattice):
 *     blocks [Lt][Lz][Ly][Lx][2][6][6]     B_b(x)_{k,l}
 * Only the lower triangle and the real parts of the diagonal are read (the
 * blocks are Hermitian).  Packed: both parities, in the link precision.
 * With invert = 1 the packed blocks are the inverses (FP64 Gauss-Jordan with
 * partial pivoting on the GPU; a singular block gives non-finite entries). */
size_t weo_clover_bytes(const weo_lattice* lat, const weo_format* fmt);
int weo_pack_clover(const weo_lattice* lat, const weo_format* fmt, const void* canon, int canon_prec,
                    int invert, void* packed, void* stream);

/* out = y + alpha C_p in  (y == NULL: out = C_p in) for nrhs spinors of parity
 * `parity`, C the packed blocks (A or A^-1 as packed).  y may be out; in must
 * not overlap out. */
int wilson_eo_clover_site(const weo_lattice* lat, const weo_format* fmt, int parity,
                          const void* clover, const void* in, const void* y, double alpha,
                          void* out, int nrhs, void* stream);

/* Hop followed by the output parity's blocks:
 *   out = C_p P_p H P_{1-p} in           (y == NULL)
 *   out = y + alpha C_p P_p H P_{1-p} in (H^dag with dagger = 1)
 * With inverse blocks and alpha = kappa this gives Eq. (5),
 * xi_o = A_oo^-1 eta_o + kappa A_oo^-1 H_oe xi_e (y = A_oo^-1 eta_o), and the
 * right-hand side of Eq. (4).  y may be out; in must not overlap out. */
int wilson_eo_clover_hop(const weo_lattice* lat, const weo_format* fmt, int out_parity, int dagger,
                         const void* u, const void* clover, const void* in, const void* y,
                         double alpha, void* out, int nrhs, void* stream);

/* Eq. (4), left-hand side, with site blocks (clover_inv = packed A^-1):
 *   out = M in = in - kappa^2 A_ee^-1 H_eo A_oo^-1 H_oe in   (dagger = 0)
 *   out = M^dag in = in - kappa^2 H_eo^dag A_oo^-1 H_oe^dag A_ee^-1 in  (dagger = 1)
 * tmp: nrhs odd-parity spinors of scratch. */
int wilson_eo_clover_apply(const weo_lattice* lat, const weo_format* fmt, int dagger,
                           const void* u, const void* clover_inv, const void* in, void* out,
                           void* tmp, int nrhs, void* stream);

/* The even-odd operator of Eq. (4), left-hand side, on the even sublattice:
 *   out = M in = in - kappa^2 H_eo H_oe in   (dagger = 0)
 *   out = M^dag in                           (dagger = 1)
 * tmp is caller scratch for nrhs odd-parity spinors (weo_spinor_bytes). */
int wilson_eo_apply(const weo_lattice* lat, const weo_format* fmt, int dagger,
                    const void* u, const void* in, void* out, void* tmp,
                    int nrhs, void* stream);

/* ---- the operator without caller scratch ------------------------------------
 * For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid allocation): wilson_eo_apply
 * with its odd-parity intermediate field (tmp) held in a library-owned device
 * array of WEO_NOALLOC_SCRATCH_BYTES per GPU, kept until the process ends.
 * Allocates nothing.  Same arguments, results and launches as
 * wilson_eo_apply; nrhs * weo_spinor_bytes(lat, fmt, 1) must not exceed
 * WEO_NOALLOC_SCRATCH_BYTES (WEO_ERR_WORKSPACE otherwise; 128 MiB holds one
 * FP32 field of 32^3x64).  The array is the current device's: a non-NULL
 * stream must belong to the current device (WEO_ERR_ARG otherwise).  Every
 * call on one GPU shares that GPU's array, so calls that overlap on one GPU
 * (different streams or host threads) race; serialise them. */
#define WEO_NOALLOC_SCRATCH_BYTES 134217728
int wilson_eo_apply_noalloc(const weo_lattice* lat, const weo_format* fmt, int dagger,
                            const void* u, const void* in, void* out, int nrhs, void* stream);

/* ---- solvers (the paper names none; Sec. 2 says solves dominate) -------- */
#define WEO_OP_M      0   /* solve M x = b by CGLS (CG on the normal equations) */
#define WEO_OP_MDAGM  1   /* solve M^dag M x = b by CG */
#define WEO_OP_DW     2   /* solve D_W x = b of Eq. (2) on the full lattice by CGLS,
                             without even-odd preconditioning (Sec. 2 compares
                             the two systems' condition); b and x hold nrhs
                             full fields, each the packed even half followed by
                             the packed odd half (2 weo_spinor_bytes(.., 1));
                             single-precision-level solves only (mixed = 1 is
                             WEO_ERR_ARG) */

#define WEO_SOLVER_CG        0   /* CGLS for WEO_OP_M / WEO_OP_DW, CG for WEO_OP_MDAGM */
#define WEO_SOLVER_BICGSTAB  1   /* BiCGStab (van der Vorst 1992) on the operator itself:
                                    two operator products per iteration, complex
                                    scalars, FP64 dot products */
#define WEO_SOLVER_BLOCK_CG  2   /* block CG (O'Leary 1980) in Dubrulle's QR form
                                    (2001): the live rhs share one block Krylov
                                    space; CG on M^dag M for WEO_OP_MDAGM, on the
                                    normal equations (carrying b - M x) for
                                    WEO_OP_M / WEO_OP_DW.  FP64 or FP32 vectors
                                    only (a mixed solve needs FP32 inner spinors);
                                    residual columns that become dependent (e.g.
                                    two equal rhs) are deflated: the block
                                    shrinks and the dropped columns follow the
                                    others' coefficients */
#define WEO_SOLVER_SAP_GCR   3   /* flexible GCR (restart gcr_nkv) preconditioned by
                                    the Schwarz alternating procedure (params sap),
                                    WEO_OP_DW only; the right-hand sides are solved
                                    one after the other.  The preconditioner runs in
                                    FP32: with FP32 vectors on the solve's own links,
                                    with FP64 vectors (mixed = 0) on u_inner in the
                                    FP32 format `inner`.  info->iters sums the GCR
                                    iterations over the right-hand sides */

/* ---- Schwarz alternating procedure (QWS's preconditioner, Sec. 1-2) ---------
 * The solver library the paper builds on preconditions its Krylov solver by
 * the Schwarz alternating procedure on a domain-decomposed lattice.  Here:
 * the lattice is cut into blocks of extent block[mu] (each dividing L_mu, with
 * L_mu / block[mu] equal to 1 or even, at most 256 sites per block), coloured
 * by the parity of the block coordinates.  One cycle sweeps the blocks of
 * colour 0, then those of colour 1; a sweep solves every block's own Wilson
 * system D_L e = r_L (D_W of Eq. (1) with the hops that leave the block
 * dropped; where L_mu / block[mu] = 1 the hop across the lattice edge stays
 * inside) by nmr minimal-residual steps started from zero, adds e to the
 * solution and updates the residual.  ncy cycles from zero give psi = K eta,
 * an approximation of D_W^-1 eta.  K is not linear (the MR step sizes depend
 * on the data), so it preconditions flexible GCR. */
typedef struct {
    int block[4];   /* block extents (x, y, z, t) */
    int ncy;        /* cycles, >= 1 */
    int nmr;        /* MR steps per block solve, 1..64 */
} weo_sap_params;

/* Bytes of device workspace wilson_eo_sap needs (three sets of nrhs full
 * fields: carried residual and the two colours' last block solutions). */
size_t wilson_eo_sap_workspace_bytes(const weo_lattice* lat, const weo_format* fmt, int nrhs);

/* psi = K eta for nrhs full fields (each the packed even half followed by the
 * packed odd half, 2 weo_spinor_bytes(lat, fmt, 1) bytes).  fmt: FP32 spinors
 * and FP32 links (18 or 12 reals), else WEO_ERR_FORMAT; invalid block extents,
 * ncy or nmr: WEO_ERR_ARG.  eta, psi and the workspace must not overlap.
 * Asynchronous on stream. */
int wilson_eo_sap(const weo_lattice* lat, const weo_format* fmt, const weo_sap_params* sap,
                  const void* u, const void* eta, void* psi, void* workspace, size_t ws_bytes,
                  int nrhs, void* stream);

typedef struct {
    int        op;          /* WEO_OP_M, WEO_OP_MDAGM or WEO_OP_DW */
    int        nrhs;        /* 1..WEO_MAX_RHS right-hand sides solved together */
    double     tol;         /* target true relative residual ||b - A x|| / ||b|| */
    int        maxiter;     /* cap on inner iterations (per solve) */
    int        x0_given;    /* 1: x holds the initial guess; 0: start from zero */
    int        mixed;       /* 0: iterate in format fmt.
                               1: FP64 defect correction (fmt must be F64) with
                                  inner solves in format `inner` on links u_inner */
    weo_format inner;       /* inner format when mixed = 1 */
    double     inner_tol;   /* relative tolerance of each inner solve; a step
                               whose inner solve can bring every remaining rhs
                               to tol with a tolerance down to inner_tol / 8
                               gets that tighter tolerance.  Right-hand sides
                               that meet tol leave the later steps. */
    int        max_outer;   /* cap on defect-correction steps */
    int        check_every; /* iterations between host convergence checks (>=1) */
    int        method;      /* WEO_SOLVER_CG, WEO_SOLVER_BICGSTAB or
                               WEO_SOLVER_BLOCK_CG (also for the inner solves of
                               defect correction) */
    const void* clover;     /* NULL: Wilson (D_ee = D_oo = 1).  Else packed INVERSE
                               site blocks (weo_pack_clover, invert = 1) in format
                               fmt: the operator is the clover-type M of
                               wilson_eo_clover_apply.  Not with WEO_OP_DW. */
    const void* clover_inner; /* the same blocks packed in format `inner` (mixed
                               only; required with clover) */
    weo_sap_params sap;     /* WEO_SOLVER_SAP_GCR: the preconditioner */
    int        gcr_nkv;     /* WEO_SOLVER_SAP_GCR: restart length, 1..16 */
} weo_solver_params;

typedef struct {
    int    status;                          /* WEO_OK, WEO_NOT_CONVERGED, WEO_BREAKDOWN */
    int    iters;                           /* inner iterations performed */
    int    outer_iters;                     /* defect-correction steps (mixed) */
    int    applies;                         /* operator (M, M^dag, D_W, D_W^dag) applications */
    double true_rel_resid[WEO_MAX_RHS];     /* recomputed at exit, FP64 for mixed */
    double seconds;                         /* wall time inside the call */
} weo_solver_info;

/* Bytes of device workspace wilson_eo_cg needs for these parameters. */
size_t wilson_eo_cg_workspace_bytes(const weo_lattice* lat, const weo_format* fmt,
                                    const weo_solver_params* p);

/* Solve for nrhs right-hand sides b (packed, format fmt, even parity; full
 * fields for WEO_OP_DW) into x.
 * u holds the links in format fmt; u_inner the links in p->inner (mixed only,
 * else ignored).  Synchronises `stream` before returning.
 * With WEO_SOLVER_BLOCK_CG the right-hand sides whose start does not already
 * meet the tolerance form one block (the others are left as they are);
 * info->iters counts block iterations; the block method needs FP64 or FP32
 * spinors (else WEO_ERR_FORMAT); dependent residual columns are deflated.
 * Its Gram matrices run on the vector units; the environment variable
 * WEO_GRAM=mfma (read per call) moves them to the FP64 matrix cores, which
 * gives the same results to FP64 rounding but is slower on MI355X. */
int wilson_eo_cg(const weo_lattice* lat, const weo_format* fmt,
                 const weo_solver_params* p,
                 const void* u, const void* u_inner,
                 const void* b, void* x,
                 void* workspace, size_t ws_bytes,
                 weo_solver_info* info, void* stream);

/* ---- derivatives --------------------------------------------------------- */
#define WEO_FORCE_PROJECT     1   /* write F = TH(i U g^dag) instead of g */
#define WEO_FORCE_ACCUMULATE  2   /* add to g_canon instead of overwriting it */

/* Link gradient of coeff * Re <Lambda, H R> for full-lattice fields given as
 * even and odd packed parts (1 rhs each).  For the link U_mu(x) with boundary
 * phase b (bc[mu] where x_mu = L_mu - 1, else 1):
 *   g = coeff * conj(b) * [ sum_s ((1-gamma_mu) Lambda(x))_s R(x+mu)_s^dag
 *                         + sum_s R(x)_s ((1+gamma_mu) Lambda(x+mu))_s^dag ]
 * which is the gradient in the convention dL = Re tr(g^dag dU).  With
 * WEO_FORCE_PROJECT the su(3) force F = TH(i U g^dag) is written instead
 * (TH = traceless Hermitian part), so that dL/d eps = tr(X F) for
 * U -> exp(i eps X) U.  The derivation follows from Eq. (1) and Eq. (4).
 * For L = Re<eta, M psi>: Lambda = (eta, H_eo^dag eta), R = (psi, H_oe psi),
 * coeff = -kappa^2.  Output: canonical gauge layout in canon_prec; the
 * gradient is accumulated in FP64.  flags: WEO_FORCE_* bits. */
int wilson_eo_force(const weo_lattice* lat, const weo_format* fmt,
                    const void* u,
                    const void* lam_e, const void* lam_o,
                    const void* r_e, const void* r_o,
                    double coeff, int flags,
                    void* g_canon, int canon_prec, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* WILSON_EO_H */
