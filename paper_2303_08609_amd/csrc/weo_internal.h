// Host-side interface between the C ABI / solver code (plain C++) and the HIP
// translation units that own the kernels.  Nothing here is exported.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

#include "weo_geom.h"

namespace weo {

// Per-format facts needed on the host.
struct FmtInfo {
    int spinor_prec, link_prec, link12;
    int spinor_site_bytes;   // 12 complex
    int link_bytes;          // 9 or 6 complex
    int wide;                // 1 if arithmetic is FP64
};
const FmtInfo& fmt_info(int fmt_id);

inline size_t spinor_field_bytes(const Geom& g, int fmt_id) {
    return (size_t)g.vh * (size_t)fmt_info(fmt_id).spinor_site_bytes;
}
inline size_t gauge_block_bytes(const Geom& g, int fmt_id) {   // one (mu, parity) block
    return (size_t)g.vh * (size_t)fmt_info(fmt_id).link_bytes;
}
inline size_t gauge_field_bytes(const Geom& g, int fmt_id) { return 8 * gauge_block_bytes(g, fmt_id); }

// Epilogue of a hop launch: out = hop(in)               (y == nullptr)
//                           out = y + alpha * hop(in)    (y != nullptr)
// with optional per-workgroup partial sums of ||out||^2 (FP64) per rhs.
struct HopLaunch {
    Geom g;
    int fmt;
    int out_par;
    int dagger;
    double phase[4][2];
    const void* u;
    const void* in;
    void* out;
    const void* y;
    double alpha;
    double* partial;      // [nrhs][hop_partials()] or nullptr: one per 64 sites
    int nrhs;
    // epilogue out = alpha hop + cy y + z (z only with y): cy = 1, z = null is
    // the axpy of M; cy = -1 with z = b gives the residual b - M x in one pass
    const void* z = nullptr;
    double cy = 1.0;
    // fused dot with the output, with partial set: dmode 1: <dw, out>,
    // 2: <out, y>; real / imaginary partials laid out like partial
    int dmode = 0;
    const void* dw = nullptr;
    double* pdre = nullptr;
    double* pdim = nullptr;
};

struct TuneCfg {
    int block;    // threads per workgroup (multiple of 64, <= 256)
    int remap;    // XCD-aware workgroup remap on/off
    int bz;       // workgroup schedule: z-strip height (0 = lexicographic)
};
TuneCfg& hop_tune();                       // current single-rhs launch shape
uint32_t hop_partials(const Geom& g);      // norm partials per rhs: one per 64 sites
hipError_t launch_hop(const HopLaunch& h, hipStream_t s);          // picks the kernel
hipError_t launch_hop_single(const HopLaunch& h, hipStream_t s);   // one lane per site
// Multi-rhs kernel: one lane per (site, group of nr rhs); links are loaded
// once per lane and applied to its nr right-hand sides.  s = sites per
// workgroup (64, 128 or 256), up to 256 / s rhs groups per workgroup and the
// rest in grid rows; persist = 1: a grid of min(#blocks, 8 * 256) workgroups
// (a multiple of 8) looping over site blocks.
struct MrhsCfg { int nr, s, persist, bz, split; };
hipError_t launch_hop_mrhs(const HopLaunch& h, const MrhsCfg& c, hipStream_t st);
int set_mrhs_shape(int nr, int sites, int persist, int bz, int split);   // 0 ok, -1 bad
int tuning_report(char* buf, size_t len);             // JSON lines, returns length

// ---- BLAS-1 on packed spinor fields (one parity, nrhs fields) -------------
// Scalars live in device memory (double) so the solver never needs the host
// in the loop.  ``mask`` (may be null) is a per-rhs int array: rhs with
// mask[r] == 0 are left untouched.  Partial sums are [nrhs][blas_blocks()].
uint32_t blas_blocks(const Geom& g);
hipError_t launch_norm2(const Geom& g, int fmt, const void* a, int nrhs,
                        double* partial, hipStream_t s);
// Deterministic final sum: out[r] = sum_b partial[r][b], fixed order.
hipError_t launch_reduce(const double* partial, int nblocks, int nrhs,
                         double* out, hipStream_t s);
// x += alpha_r p; s -= alpha_r q; s_op = s (when the formats differ);
// partial_s = ||s||^2.  x, s in fmt_acc; p, q, s_op in fmt_op.
hipError_t launch_axpy2(const Geom& g, int fmt_acc, int fmt_op, int nrhs,
                        const double* alpha, const int* mask,
                        void* x, const void* p, void* s, const void* q, void* s_op,
                        double* partial_s, hipStream_t st);
// p = r + beta_r p
hipError_t launch_xpay(const Geom& g, int fmt, int nrhs,
                       const double* beta, const int* mask,
                       const void* r, void* p, hipStream_t s);
// out = ca a + cb b (b may be null), optional partial ||out||^2
hipError_t launch_axpby(const Geom& g, int fmt, int nrhs, double ca, const void* a,
                        double cb, const void* b, void* out, double* partial,
                        hipStream_t s);
// out (fmt_out) = in (fmt_in) * scale[r] (scale may be null = 1) [+ out]
hipError_t launch_convert(const Geom& g, int fmt_in, const void* in, int fmt_out,
                          void* out, int nrhs, const double* scale, int accumulate,
                          hipStream_t s);
// clear bytes (a multiple of 16) with a kernel (safe inside graph capture)
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);

// Solver scalar steps, one workgroup per rhs:
//   SCAL_ALPHA: a = sum pa;  alpha = gamma / a (breakdown if a <= 0 or not finite)
//   SCAL_BETA:  a = sum pa, b = sum pb;  beta = a / gamma; gamma = a;
//               ss = (pb ? b : a)
//   SCAL_SCALE: a = sum pa;  nrm = a; sc_in = sqrt(target / a); sc_out = 1/sc_in
enum { SCAL_ALPHA = 0, SCAL_BETA = 1, SCAL_SCALE = 2 };
struct ScalarArgsHost {
    int nrhs, nba, nbb;     // partial counts per rhs of pa and pb
    const double* pa;
    const double* pb;
    double* gamma;
    double* alpha;
    double* beta;
    double* ss;
    int* mask;
    int* flags;
    double target;
    double* sc_in;
    double* sc_out;
    double* nrm;
    const double* bb;   // SCAL_BETA: ||b||^2 per rhs; ss <= tol2 bb masks the rhs off
    double tol2;
};
hipError_t launch_scalars(int kind, const ScalarArgsHost& a, hipStream_t s);

// ---- BiCGStab vector and scalar steps ---------------------------------------
// Complex per-rhs scalars are (re, im) pairs of doubles in device memory.
// x, r, s in fmt_acc; r^, p, v, t, s_op in fmt_op (s_op written only when
// the two formats store spinors differently).  Partials are [nrhs][blas_blocks].
enum { BI_INIT = 0, BI_ALPHA = 1, BI_OMEGA = 2, BI_BETA = 3 };
struct BiScalHost {
    int nrhs;
    double* rho;
    double* alpha;
    double* omega;
    double* beta;
    double* ss;      // ||r||^2 for the host's convergence check
    const double* bb;  // ||b||^2 per rhs: ||r||^2 <= tol2 bb masks the rhs off
    double tol2;
    int* mask;
    int* flags;
};
// partials of <a, b> (a in fmt_a, b in fmt_b)
hipError_t launch_bi_cdot(const Geom& g, int fmt_a, int fmt_b, int nrhs, const int* mask, const void* a,
                          const void* b, double* pre, double* pim, hipStream_t st);
// r^ = p = r (in fmt_op), partials ||r||^2 and <r^, r> (one pass)
hipError_t launch_bi_init(const Geom& g, int fmt_acc, int fmt_op, int nrhs, const int* mask, const void* r,
                          void* rh, void* p, double* prr, double* pre, double* pim, hipStream_t st);
// s = r - alpha v, s_op = s, partial ||s||^2
hipError_t launch_bi_s(const Geom& g, int fmt_acc, int fmt_op, int nrhs, const BiScalHost& h, const void* r,
                       const void* v, void* s, void* s_op, double* partial, hipStream_t st);
// partials of <t, s> and ||t||^2
hipError_t launch_bi_ts(const Geom& g, int fmt_acc, int fmt_op, int nrhs, const int* mask, const void* t,
                        const void* s, double* pre, double* pim, double* ptt, hipStream_t st);
// x += alpha p + omega s, r = s - omega t, partials ||r||^2 and <r^, r>
hipError_t launch_bi_xr(const Geom& g, int fmt_acc, int fmt_op, int nrhs, const BiScalHost& h, void* x,
                        const void* p, const void* s, const void* t, void* r, const void* rh, double* prr,
                        double* pre, double* pim, hipStream_t st);
// p = r + beta (p - omega v)
hipError_t launch_bi_p(const Geom& g, int fmt_acc, int fmt_op, int nrhs, const BiScalHost& h, const void* r,
                       void* p, const void* v, hipStream_t st);
hipError_t launch_bi_scalars(int kind, const BiScalHost& h, int nb, const double* pa, const double* pb,
                             const double* pc, hipStream_t st);

// ---- block CG: Gram matrices and block updates --------------------------------
// A block is s <= kMaxBlock fields of one format; column j is the field at
// base + col[j] * stride.  FP64 and FP32 spinor formats only.
constexpr int kMaxBlock = 16;
constexpr int kGramStride = 2 * kMaxBlock * kMaxBlock;   // doubles of one s x s complex matrix (max)
struct BlockRef {
    uint8_t* base;
    uint64_t stride;
    uint8_t col[kMaxBlock];
};
int block_gram_wg(const Geom& g, int fmt);      // Gram partials: kGramStride doubles each
int block_update_wg(const Geom& g, int fmt);    // norm partials per column of an update
// out[(j s + k) 2 + {re, im}] = <a_j, b_k> for j <= k, 0 below the diagonal
// (FP64 accumulation, deterministic; both matrices of block CG are Hermitian)
hipError_t launch_block_gram(const Geom& g, int fmt, int s, const BlockRef& a, const BlockRef& b, double* part,
                             double* out, hipStream_t st);
// out_j = [in0_j] + a sum_k in1_k T[k][j], T complex s x s row-major (re, im);
// out may be in0 or in1.  nrm (optional, with npart scratch of
// s * block_update_wg doubles): nrm[j] = ||out_j||^2.
hipError_t launch_block_update(const Geom& g, int fmt, int s, const BlockRef& out, const BlockRef* in0,
                               const BlockRef& in1, double a, const double* T, double* npart, double* nrm,
                               hipStream_t st);
// q <- q TA;  p <- q + p TB (with the new q), in place, one pass
hipError_t launch_block_qp(const Geom& g, int fmt, int s, const BlockRef& q, const BlockRef& p, const double* ta,
                           const double* tb, hipStream_t st);

// ---- Schwarz alternating procedure and flexible GCR (sap.hip) -----------------
// Blocks of extent b[mu] (nb[mu] = L_mu / b[mu], each 1 or even; at most 256
// sites), coloured by the parity of the block coordinates.
struct SapGeom {
    int b[4], nb[4];
    int bvol, nblocks;
};
constexpr int kSapMaxSites = 256;
constexpr int kGcrMax = 16;       // vectors one GCR dot / update pass takes
// One sweep over the blocks of one colour (nrhs full fields [even | odd] in
// fmt, FP64 or FP32): nmr MR steps on each block system starting from the
// carried residual rho (plus kappa H dprev from the previous sweep's block
// solutions on the neighbouring blocks, dprev may be null); phi += the block
// solutions, dout = the block solutions, rho = the block residuals.
hipError_t launch_sap_sweep(const Geom& g, int fmt, const SapGeom& sg, int colour, int nmr, double kappa,
                            const double ph[4][2], const void* u, void* rho, void* phi, const void* dprev,
                            void* dout, int nrhs, hipStream_t s);
// Block layout for extents block[mu] on lattice g: 0 with sg filled, or -1
// (an extent not dividing L_mu, L_mu / block[mu] neither 1 nor even, or more
// than kSapMaxSites sites per block).
int make_sap_geom(const Geom& g, const int block[4], SapGeom* sg);
// psi = K eta: ncy SAP cycles (colour 0 then 1) from zero, nmr MR steps per
// block; nrhs full fields in the FP32 format fmt; rho, d0, d1: nrhs full
// fields of scratch each.
hipError_t sap_apply(const Geom& g, int fmt, const SapGeom& sg, int ncy, int nmr, double kappa,
                     const double ph[4][2], const void* u, const void* eta, void* psi, void* rho, void* d0,
                     void* d1, int nrhs, hipStream_t s);
// Partials (gcr_wg of them per value) of <a_l, b>, l < n: value 2 l + {re, im}.
uint32_t gcr_wg(const Geom& gb, int fmt);
hipError_t launch_gcr_dots(const Geom& gb, int fmt, int n, const void* const* a, const void* b, double* part,
                           hipStream_t s);
// b += sum_l (cre_l + i cim_l) a_l; with part: partials of ||b||^2 (value 0)
// and, when r is given, of <b, r> (values 1, 2: re, im).
hipError_t launch_gcr_update(const Geom& gb, int fmt, int n, const void* const* a, const double* cre,
                             const double* cim, void* b, const void* r, double* part, hipStream_t s);

// ---- pack / unpack --------------------------------------------------------
hipError_t launch_pack_gauge(const Geom& g, int fmt, const void* canon, int canon_f64,
                             void* packed, hipStream_t s);
hipError_t launch_pack_spinor(const Geom& g, int fmt, int nrhs, const void* canon,
                              int canon_f64, double scale, void* packed, hipStream_t s);
hipError_t launch_unpack_spinor(const Geom& g, int fmt, int nrhs, const void* packed,
                                double scale, void* canon, int canon_f64, hipStream_t s);

// ---- face exchange of a hop split along a direction ------------------------------
uint32_t face_sites(const Geom& g, int mu);                 // face sites per parity
size_t face_field_bytes(const Geom& g, int fmt, int mu);   // one face of one field
hipError_t launch_face_pack(const Geom& g, int fmt, int mu, int out_par, int dagger, const void* u,
                            const void* in, void* lo, void* hi, int nrhs, hipStream_t s);
hipError_t launch_face_unpack(const Geom& g, int fmt, int mu, int out_par, int dagger, const double ph_lo[2],
                              const double ph_hi[2], double alpha, const void* u, const void* lo,
                              const void* hi, void* out, int nrhs, hipStream_t s);

// ---- clover-type site blocks (layout in clover_core.h) -------------------------
size_t clover_block_bytes(const Geom& g, int fmt);   // one (parity, block) field
size_t clover_field_bytes(const Geom& g, int fmt);   // both parities, both blocks
// canonical blocks [Lt][Lz][Ly][Lx][2][6][6] -> packed (inverted in FP64 if invert)
hipError_t launch_pack_clover(const Geom& g, int fmt, const void* canon, int canon_f64, int invert, void* packed,
                              hipStream_t s);
// out = y + alpha C_parity in  (y == nullptr: out = C_parity in)
hipError_t launch_clover_site(const Geom& g, int fmt, int parity, const void* clv, const void* in, const void* y,
                              double alpha, void* out, int nrhs, hipStream_t s);
// hop whose result is multiplied by the output parity's blocks before the
// axpy / norm epilogue (one lane per site, nrhs grid rows)
hipError_t launch_hop_clover(const HopLaunch& h, const void* clv, hipStream_t s);
// M = 1 - kappa^2 C_e H_eo C_o H_oe or its adjoint (C: packed inverse blocks)
hipError_t launch_apply_clover(const Geom& g, int fmt, const double phase[4][2], double kappa, int dagger,
                               const void* u, const void* clv, const void* in, void* out, void* tmp, int nrhs,
                               double* partial, hipStream_t s);

// ---- force ------------------------------------------------------------------
hipError_t launch_force(const Geom& g, int fmt, const double phase[4][2], const void* u,
                        const void* lam_e, const void* lam_o, const void* r_e,
                        const void* r_o, double coeff, int flags, void* g_canon,
                        int canon_f64, hipStream_t s);

}  // namespace weo
