// Krylov solvers for the even-odd system (host driver; all vector work runs in
// the library's kernels, scalars stay on the device).
//
// The paper (Sec. 2) only states that iterative solvers dominate and that
// their cost is the matrix multiplication; the algorithms are standard:
//
//  CGLS for M x = b (CG on M^dag M x = M^dag b, carrying s = b - M x):
//     s = b - M x;  r = M^dag s;  p = r;  gamma = <r, r>
//     repeat: q = M p;  alpha = gamma / ||q||^2;  x += alpha p;  s -= alpha q;
//             r = M^dag s;  beta = <r, r> / gamma;  gamma = <r, r>;  p = r + beta p
//  The same CGLS on the unpreconditioned D_W = 1 - kappa H of Eq. (1) over
//  both parities (op WEO_OP_DW; a field is its even half followed by its odd
//  half), for comparing iteration counts with the even-odd system.
//  CG for M^dag M x = b:
//     r = b - A x;  p = r;  gamma = <r, r>
//     repeat: t = M p;  q = M^dag t;  alpha = gamma / ||t||^2;  x += alpha p;
//             r -= alpha q;  beta = <r, r> / gamma;  gamma = <r, r>;  p = r + beta p
//  BiCGStab (van der Vorst 1992) for A x = b, any of the operators above
//  (method WEO_SOLVER_BICGSTAB), shadow residual r^ = r_0, two products with
//  A per iteration and complex scalars:
//     v = A p;  alpha = rho / <r^, v>;  s = r - alpha v;  t = A s;
//     omega = <t, s> / ||t||^2;  x += alpha p + omega s;  r = s - omega t;
//     rho' = <r^, r>;  beta = (rho' / rho)(alpha / omega);  p = r + beta (p - omega v)
//  Block CG (method WEO_SOLVER_BLOCK_CG; O'Leary 1980, in the QR form of
//  Dubrulle 2001) for the s live right-hand sides together, on A = M^dag M
//  (for M x = b and D_W through the normal equations, carrying S = B - M X):
//     Q C = R_0 (QR),  P = Q
//     repeat: W = A P;  delta = (P^H W)^-1;  X += P delta C;  S -= (M P) delta C
//             Q' psi = Q - W delta (QR);  C = psi C;  P = Q' + P psi^H;  Q = Q'
//  The QR factorisations are Cholesky QR (Gram matrix on the device in FP64,
//  Cholesky factor on the host); the s x s algebra runs on the host in FP64.
//  With site blocks (clover-type D_ee, D_oo; packed inverse blocks C) the
//  operator is M = 1 - kappa^2 C_e H_eo C_o H_oe of Eq. (4), same solvers.
//  Defect correction (mixed precision): in FP64, r = b - A x; the residual is
//  rescaled to unit RMS component, solved approximately in the inner format
//  (relative tolerance inner_tol) and the correction added back in FP64.
//
// "acc" is the format of the iterate x and residual s (r for CG); "op" the
// format of every vector the operator reads or writes (p, q, r, t).  Norms
// and dot products accumulate in FP64 in every format.  The host looks at the
// residual norms every check_every iterations (one small copy and one stream
// synchronisation); nothing else leaves the device.
#include <hip/hip_runtime_api.h>

#include <chrono>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "../../include/wilson_eo.h"
#include "weo_internal.h"

namespace weo {

int check_lattice(const weo_lattice* lat, Geom* g);
int check_fmt(const weo_format* f, int* id);
int check_ptr(const void* p);
bool overlaps(const void* a, size_t na, const void* b, size_t nb);
void phases_of(const weo_lattice* lat, double ph[4][2]);

namespace {

// WILSON_EO_LOG=1: one line per defect-correction step on stderr.
bool solver_log() {
    const char* e = getenv("WILSON_EO_LOG");
    return e && e[0] == '1';
}

#define HIPCHK(expr)                                  \
    do {                                              \
        if ((expr) != hipSuccess) return WEO_ERR_HIP; \
    } while (0)

struct Carve {
    uint8_t* base;
    size_t size, off;
    void* take(size_t bytes) {
        off = (off + 255) & ~(size_t)255;
        void* p = base ? base + off : nullptr;
        off += bytes;
        return p;
    }
};

// Device scalar block: one entry per rhs for each quantity.
struct Scalars {
    double *gamma, *alpha, *beta, *ss, *bb, *rr, *sc_in, *sc_out, *nrm;
    double *crho, *calpha, *comega, *cbeta;     // BiCGStab complex scalars (re, im)
    int *mask, *flags;
};

struct Workspace {
    // fields (nrhs each)
    void *s_acc, *x_acc, *s_op, *p, *q, *r, *t, *tmp;     // level vectors
    void *rh, *s2;                                        // BiCGStab: shadow residual (op), s (acc)
    void *r64, *t64, *tmp64;                              // outer (mixed) vectors
    double *pa, *pb, *pc;                                 // partial sums
    double *gpart, *upart, *gram, *tm;                    // block CG: partials, Gram, s x s factors
    void *gphi[kGcrMax], *gchi[kGcrMax];                  // SAP-GCR: directions and their images
    void *srho, *sd0, *sd1, *spin, *spout;                // SAP scratch; FP32 copies (FP64 level)
    double *gcpart, *gcsum;                               // GCR partials and sums
    Scalars sc;
    size_t bytes;
};

// The format used for FP32 accumulation vectors (spinor part only matters).
constexpr int kAccF32 = FMT_S_S_18;
constexpr int kBlockFactors = 5;      // s x s factors of block CG held on the device

uint32_t max_partials(const Geom& g) {
    const uint32_t a = (g.vh + 63) / 64;           // smallest legal hop workgroup
    const uint32_t b = blas_blocks(g);
    return a > b ? a : b;
}

Workspace carve_ws(const Geom& g, int fmt, const weo_solver_params* p, int inner_fmt, uint8_t* base,
                   size_t size) {
    Carve c{base, size, 0};
    Workspace w;
    std::memset(&w, 0, sizeof(w));
    const int n = p->nrhs;
    const int op = p->mixed ? inner_fmt : fmt;
    const int acc = p->mixed ? kAccF32 : fmt;
    const size_t fo = (size_t)n * spinor_field_bytes(g, op);
    const size_t fa = (size_t)n * spinor_field_bytes(g, acc);
    w.s_acc = c.take(fa);
    if (p->mixed) w.x_acc = c.take(fa);
    if (fmt_info(acc).spinor_prec != fmt_info(op).spinor_prec) w.s_op = c.take(fo);
    w.p = c.take(fo);
    w.q = c.take(fo);
    w.r = c.take(fo);
    w.t = c.take(fo);
    w.tmp = c.take(fo);
    if (p->method == WEO_SOLVER_BICGSTAB) {
        w.rh = c.take(fo);
        w.s2 = c.take(fa);
    }
    if (p->method == WEO_SOLVER_SAP_GCR) {
        // one right-hand side at a time: single fields of the level format and,
        // for the preconditioner, of its FP32 format
        const int pre = fmt_info(op).spinor_prec == WEO_F32 ? op : inner_fmt;
        const size_t f1 = spinor_field_bytes(g, op), fp = spinor_field_bytes(g, pre);
        for (int k = 0; k < p->gcr_nkv && k < kGcrMax; ++k) {
            w.gphi[k] = c.take(f1);
            w.gchi[k] = c.take(f1);
        }
        w.srho = c.take(fp);
        w.sd0 = c.take(fp);
        w.sd1 = c.take(fp);
        if (pre != op) {
            w.spin = c.take(fp);
            w.spout = c.take(fp);
        }
        w.gcpart = static_cast<double*>(c.take((size_t)2 * kGcrMax * gcr_wg(g, op) * sizeof(double)));
        w.gcsum = static_cast<double*>(c.take((size_t)2 * kGcrMax * sizeof(double)));
    }
    if (p->method == WEO_SOLVER_BLOCK_CG) {
        w.gpart = static_cast<double*>(c.take((size_t)block_gram_wg(g, op) * kGramStride * sizeof(double)));
        w.upart = static_cast<double*>(c.take((size_t)kMaxBlock * block_update_wg(g, op) * sizeof(double)));
        w.gram = static_cast<double*>(c.take(kGramStride * sizeof(double)));
        w.tm = static_cast<double*>(c.take(kBlockFactors * kGramStride * sizeof(double)));
    }
    if (p->mixed) {
        const size_t f64 = (size_t)n * spinor_field_bytes(g, fmt);
        w.r64 = c.take(f64);
        w.t64 = c.take(f64);
        w.tmp64 = c.take(f64);
    }
    const size_t np = (size_t)n * max_partials(g) * sizeof(double);
    w.pa = static_cast<double*>(c.take(np));
    w.pb = static_cast<double*>(c.take(np));
    w.pc = static_cast<double*>(c.take(np));
    double* d = static_cast<double*>(c.take(17 * WEO_MAX_RHS * sizeof(double)));
    int* ip = static_cast<int*>(c.take(2 * WEO_MAX_RHS * sizeof(int)));
    if (d) {
        w.sc.gamma = d; w.sc.alpha = d + 16; w.sc.beta = d + 32; w.sc.ss = d + 48; w.sc.bb = d + 64;
        w.sc.rr = d + 80; w.sc.sc_in = d + 96; w.sc.sc_out = d + 112; w.sc.nrm = d + 128;
        w.sc.crho = d + 144; w.sc.calpha = d + 176; w.sc.comega = d + 208; w.sc.cbeta = d + 240;
        w.sc.mask = ip; w.sc.flags = ip + 16;
    }
    w.bytes = c.off;
    return w;
}

struct Ctx {
    const weo_lattice* lat;
    Geom g;                 // the lattice (hop geometry)
    Geom gb;                // vector geometry: g, or twice the sites for full fields
    bool full;              // operator on full (both-parity) fields
    uint32_t nb_apply;      // norm partials per rhs written by an operator apply
    const void* clv;        // packed inverse site blocks of the current level (clover-type M) or null
    double ph[4][2];
    hipStream_t st;
    int applies;
    // SAP-GCR: preconditioner blocks, cycles, MR steps, restart length, and
    // the FP32 format and links the preconditioner runs on
    SapGeom sap;
    int ncy, nmr, nkv;
    int fmt_pre;
    const void* u_pre;
};

// out = A in with A = M (dagger 0) or M^dag (dagger 1); partial = ||out||^2.
hipError_t apply_m(Ctx& c, int fmt, const void* u, int dagger, const void* in, void* out, void* tmp,
                   int nrhs, double* partial, int dmode = 0, const void* dw = nullptr, double* pdre = nullptr,
                   double* pdim = nullptr) {
    if (c.clv && dmode) return hipErrorInvalidValue;     // the site-block hops fuse no dot
    if (c.clv) {
        ++c.applies;
        return launch_apply_clover(c.g, fmt, c.ph, c.lat->kappa, dagger, u, c.clv, in, out, tmp, nrhs, partial,
                                   c.st);
    }
    HopLaunch h;
    h.g = c.g;
    h.fmt = fmt;
    h.dagger = dagger;
    std::memcpy(h.phase, c.ph, sizeof(h.phase));
    h.u = u;
    h.nrhs = nrhs;
    h.out_par = 1;
    h.in = in;
    h.out = tmp;
    h.y = nullptr;
    h.alpha = 0.0;
    h.partial = nullptr;
    hipError_t e = launch_hop(h, c.st);
    if (e != hipSuccess) return e;
    h.out_par = 0;
    h.in = tmp;
    h.out = out;
    h.y = in;
    h.alpha = -c.lat->kappa * c.lat->kappa;
    h.partial = partial;
    h.dmode = dmode;
    h.dw = dw;
    h.pdre = pdre;
    h.pdim = pdim;
    ++c.applies;
    return launch_hop(h, c.st);
}

// out = D_W in (dagger 0) or D_W^dag in (dagger 1) on full fields [even | odd]:
//   out_e = in_e - kappa H_eo in_o,   out_o = in_o - kappa H_oe in_e
// partial = ||out||^2 over both halves.
hipError_t apply_dw(Ctx& c, int fmt, const void* u, int dagger, const void* in, void* out, int nrhs,
                    double* partial) {
    const size_t half = spinor_field_bytes(c.g, fmt);
    HopLaunch h;
    h.g = c.g;
    h.fmt = fmt;
    h.dagger = dagger;
    std::memcpy(h.phase, c.ph, sizeof(h.phase));
    h.u = u;
    h.nrhs = 1;
    h.alpha = -c.lat->kappa;
    h.partial = nullptr;
    for (int r = 0; r < nrhs; ++r) {
        const uint8_t* ie = static_cast<const uint8_t*>(in) + (size_t)r * 2 * half;
        uint8_t* oe = static_cast<uint8_t*>(out) + (size_t)r * 2 * half;
        for (int par = 0; par < 2; ++par) {
            h.out_par = par;
            h.in = par == 0 ? ie + half : ie;
            h.y = par == 0 ? ie : ie + half;
            h.out = par == 0 ? oe : oe + half;
            hipError_t e = launch_hop(h, c.st);
            if (e != hipSuccess) return e;
        }
    }
    ++c.applies;
    return partial ? launch_norm2(c.gb, fmt, out, nrhs, partial, c.st) : hipSuccess;
}

// The CGLS operator: M (even-odd) or D_W (full fields).
hipError_t apply_a(Ctx& c, int fmt, const void* u, int dagger, const void* in, void* out, void* tmp,
                   int nrhs, double* partial) {
    if (c.full) return apply_dw(c, fmt, u, dagger, in, out, nrhs, partial);
    return apply_m(c, fmt, u, dagger, in, out, tmp, nrhs, partial);
}

// r = b - M x in two hops: tmp = H_oe x, then r = kappa^2 H_eo tmp - x + b
// in the second hop's epilogue (no M x field written and read back);
// partial = ||r||^2 per 64 sites.  Wilson M only (no site blocks).
hipError_t resid_m(Ctx& c, int fmt, const void* u, const void* x, const void* b, void* r, void* tmp, int nrhs,
                   double* partial) {
    HopLaunch h;
    h.g = c.g;
    h.fmt = fmt;
    h.dagger = 0;
    std::memcpy(h.phase, c.ph, sizeof(h.phase));
    h.u = u;
    h.nrhs = nrhs;
    h.out_par = 1;
    h.in = x;
    h.out = tmp;
    h.y = nullptr;
    h.alpha = 0.0;
    h.partial = nullptr;
    hipError_t e = launch_hop(h, c.st);
    if (e != hipSuccess) return e;
    h.out_par = 0;
    h.in = tmp;
    h.out = r;
    h.y = x;
    h.cy = -1.0;
    h.z = b;
    h.alpha = c.lat->kappa * c.lat->kappa;
    h.partial = partial;
    ++c.applies;
    return launch_hop(h, c.st);
}

// out = A x for the solver operator (M, or M^dag M through mid); partial = ||out||^2
// (for M^dag M the partial holds ||M x||^2 only when want_mid_norm).
hipError_t apply_op(Ctx& c, int op, int fmt, const void* u, const void* x, void* out, void* mid, void* tmp,
                    int nrhs, double* partial) {
    if (op != WEO_OP_MDAGM) return apply_a(c, fmt, u, 0, x, out, tmp, nrhs, partial);
    hipError_t e = apply_m(c, fmt, u, 0, x, mid, tmp, nrhs, partial);
    if (e != hipSuccess) return e;
    return apply_m(c, fmt, u, 1, mid, out, tmp, nrhs, nullptr);
}

ScalarArgsHost sargs(const Scalars& s, int nrhs) {
    ScalarArgsHost a;
    std::memset(&a, 0, sizeof(a));
    a.nrhs = nrhs;
    a.gamma = s.gamma; a.alpha = s.alpha; a.beta = s.beta; a.ss = s.ss;
    a.mask = s.mask; a.flags = s.flags; a.sc_in = s.sc_in; a.sc_out = s.sc_out; a.nrm = s.nrm;
    return a;
}

struct LevelResult {
    int iters;
    int breakdown;
};

// Host look at the residual norms: masks off converged rhs, notes breakdowns.
// Returns the number of live rhs (or a negative status); ss and mask are
// left holding what was seen.
int look_at(Ctx& c, const Workspace& w, int nrhs, double tol2, const std::vector<double>& bb,
            std::vector<double>& ss, std::vector<int>& mask, LevelResult* res) {
    std::vector<int> flags(nrhs);
    HIPCHK(hipMemcpyAsync(ss.data(), w.sc.ss, nrhs * sizeof(double), hipMemcpyDeviceToHost, c.st));
    HIPCHK(hipMemcpyAsync(mask.data(), w.sc.mask, nrhs * sizeof(int), hipMemcpyDeviceToHost, c.st));
    HIPCHK(hipMemcpyAsync(flags.data(), w.sc.flags, nrhs * sizeof(int), hipMemcpyDeviceToHost, c.st));
    HIPCHK(hipStreamSynchronize(c.st));
    int live = 0;
    bool changed = false;
    for (int r = 0; r < nrhs; ++r) {
        if (flags[r]) res->breakdown = 1;
        if (mask[r] && ss[r] <= tol2 * bb[r]) { mask[r] = 0; changed = true; }
        live += mask[r] != 0;
    }
    if (changed) {
        HIPCHK(hipMemcpyAsync(w.sc.mask, mask.data(), nrhs * sizeof(int), hipMemcpyHostToDevice, c.st));
        HIPCHK(hipStreamSynchronize(c.st));     // the host vector goes out of scope
    }
    return live;
}

// When the host next looks at the residuals.  The look costs a stream
// synchronisation, so it is not done every iteration: after a look the
// convergence rate of each live rhs since the previous look predicts the
// iteration at which the slowest one reaches its tolerance, and the next look
// is placed there (at most check_every iterations ahead; the first look after
// two iterations).  Converged rhs are masked off on the device as soon as
// their residual passes, so a late look only costs masked-off iterations.
struct LookPlan {
    int every, last_it = 0;
    std::vector<double> last_ss;
    LookPlan(int check_every, const std::vector<double>& ss0) : every(check_every), last_ss(ss0) {}
    int first() const { return every < 2 ? every : 2; }
    int next(int it, const std::vector<double>& ss, const std::vector<int>& mask, const std::vector<double>& bb,
             double tol2) {
        double need = 1.0;
        for (size_t r = 0; r < ss.size(); ++r) {
            if (!mask[r]) continue;
            const double a = last_ss[r], b = ss[r], goal = tol2 * bb[r];
            if (!(a > 0.0) || !(b > 0.0) || !(b < a) || it <= last_it) { need = every; break; }
            const double rate = std::log(b / a) / (double)(it - last_it);   // per iteration, < 0
            const double k = std::log(goal / b) / rate;
            if (k > need) need = k;
        }
        last_ss = ss;
        last_it = it;
        const int k = need >= (double)every ? every : (int)std::ceil(need);
        return it + (k < 1 ? 1 : k);
    }
};

// Iterate one precision level.  On entry: x_acc holds the start (zero or x0),
// s_acc the matching residual (b - M x for CGLS, b - A x for CG), mask the
// live rhs, bb[r] = ||b||^2.  Stops per rhs when ||s||^2 <= tol^2 bb.
int run_level(Ctx& c, const Workspace& w, int op, int fmt_op, int fmt_acc, const void* u, void* x_acc,
              int nrhs, double tol, int maxiter, int check_every, LevelResult* res) {
    const Geom& g = c.gb;
    // the residual doubles as the operator input when both are stored alike
    const bool same = fmt_info(fmt_op).spinor_prec == fmt_info(fmt_acc).spinor_prec;
    void* s_op = same ? w.s_acc : w.s_op;
    const uint32_t nbh = c.nb_apply, nbb = blas_blocks(g);
    ScalarArgsHost sa = sargs(w.sc, nrhs);
    sa.bb = w.sc.bb;
    sa.tol2 = tol * tol;
    res->iters = 0;
    res->breakdown = 0;
    if (!same) HIPCHK(launch_convert(g, fmt_acc, w.s_acc, fmt_op, s_op, nrhs, nullptr, 0, c.st));
    if (op != WEO_OP_MDAGM) {
        // r = M^dag s, gamma = ||r||^2, p = r
        HIPCHK(apply_a(c, fmt_op, u, 1, s_op, w.r, w.tmp, nrhs, w.pa));
    } else {
        HIPCHK(launch_norm2(g, fmt_op, s_op, nrhs, w.pa, c.st));
        HIPCHK(launch_convert(g, fmt_op, s_op, fmt_op, w.r, nrhs, nullptr, 0, c.st));
    }
    HIPCHK(launch_reduce(w.pa, op != WEO_OP_MDAGM ? (int)nbh : (int)nbb, nrhs, w.sc.gamma, c.st));
    HIPCHK(launch_convert(g, fmt_op, w.r, fmt_op, w.p, nrhs, nullptr, 0, c.st));

    std::vector<double> ss(nrhs), bb(nrhs);
    std::vector<int> mask(nrhs);
    const double tol2 = tol * tol;
    // a start that already meets the tolerance costs no iteration
    HIPCHK(launch_norm2(g, fmt_acc, w.s_acc, nrhs, w.pb, c.st));
    HIPCHK(launch_reduce(w.pb, (int)nbb, nrhs, w.sc.ss, c.st));
    HIPCHK(hipMemcpyAsync(ss.data(), w.sc.ss, nrhs * sizeof(double), hipMemcpyDeviceToHost, c.st));
    HIPCHK(hipMemcpyAsync(bb.data(), w.sc.bb, nrhs * sizeof(double), hipMemcpyDeviceToHost, c.st));
    HIPCHK(hipMemcpyAsync(mask.data(), w.sc.mask, nrhs * sizeof(int), hipMemcpyDeviceToHost, c.st));
    HIPCHK(hipStreamSynchronize(c.st));
    {
        int live = 0;
        for (int r = 0; r < nrhs; ++r) {
            if (mask[r] && ss[r] <= tol2 * bb[r]) mask[r] = 0;
            live += mask[r] != 0;
        }
        HIPCHK(hipMemcpyAsync(w.sc.mask, mask.data(), nrhs * sizeof(int), hipMemcpyHostToDevice, c.st));
        HIPCHK(hipStreamSynchronize(c.st));
        if (!live) return WEO_OK;
    }
    LookPlan plan(check_every, ss);
    int look = plan.first();
    for (int it = 1; it <= maxiter; ++it) {
        // q = A p with the alpha denominator in pa
        if (op != WEO_OP_MDAGM) {
            HIPCHK(apply_a(c, fmt_op, u, 0, w.p, w.q, w.tmp, nrhs, w.pa));
        } else {
            HIPCHK(apply_op(c, op, fmt_op, u, w.p, w.q, w.t, w.tmp, nrhs, w.pa));
        }
        sa.pa = w.pa; sa.nba = (int)nbh; sa.pb = nullptr; sa.nbb = 0;
        HIPCHK(launch_scalars(SCAL_ALPHA, sa, c.st));
        // x += alpha p; s -= alpha q (s is the CG residual r for M^dag M)
        HIPCHK(launch_axpy2(g, fmt_acc, fmt_op, nrhs, w.sc.alpha, w.sc.mask, x_acc, w.p, w.s_acc, w.q,
                            same ? nullptr : s_op, w.pb, c.st));
        if (op != WEO_OP_MDAGM) {
            HIPCHK(apply_a(c, fmt_op, u, 1, s_op, w.r, w.tmp, nrhs, w.pc));
            sa.pa = w.pc; sa.nba = (int)nbh; sa.pb = w.pb; sa.nbb = (int)nbb;
            HIPCHK(launch_scalars(SCAL_BETA, sa, c.st));
            HIPCHK(launch_xpay(g, fmt_op, nrhs, w.sc.beta, w.sc.mask, w.r, w.p, c.st));
        } else {
            sa.pa = w.pb; sa.nba = (int)nbb; sa.pb = nullptr; sa.nbb = 0;
            HIPCHK(launch_scalars(SCAL_BETA, sa, c.st));
            HIPCHK(launch_xpay(g, fmt_op, nrhs, w.sc.beta, w.sc.mask, s_op, w.p, c.st));
        }
        res->iters = it;
        if (it == look || it == maxiter) {
            const int live = look_at(c, w, nrhs, tol2, bb, ss, mask, res);
            if (live < 0) return live;
            if (!live) break;
            look = plan.next(it, ss, mask, bb, tol2);
        }
    }
    HIPCHK(hipStreamSynchronize(c.st));
    return WEO_OK;
}

// BiCGStab at one precision level.  Same contract as run_level: x_acc holds
// the start, s_acc the matching residual b - A x, mask the live rhs and
// bb[r] = ||b||^2; stops per rhs when ||r||^2 <= tol^2 bb.  Vectors: r = s_acc,
// s = s2 (fmt_acc); r^ = rh, p, v = q, t, s_op, mid = r (fmt_op).  Any fixed
// r^ serves; keeping it in the operator's format halves its traffic.
int run_level_bicg(Ctx& c, const Workspace& w, int op, int fmt_op, int fmt_acc, const void* u, void* x_acc,
                   int nrhs, double tol, int maxiter, int check_every, LevelResult* res) {
    const Geom& g = c.gb;
    const bool same = fmt_info(fmt_op).spinor_prec == fmt_info(fmt_acc).spinor_prec;
    void* s_op = same ? w.s2 : w.s_op;
    const int nbb = (int)blas_blocks(g);
    const double tol2 = tol * tol;
    BiScalHost B;
    B.nrhs = nrhs;
    B.rho = w.sc.crho; B.alpha = w.sc.calpha; B.omega = w.sc.comega; B.beta = w.sc.cbeta;
    B.ss = w.sc.ss; B.bb = w.sc.bb; B.tol2 = tol2; B.mask = w.sc.mask; B.flags = w.sc.flags;
    res->iters = 0;
    res->breakdown = 0;
    std::vector<double> ss(nrhs);
    std::vector<int> mask(nrhs);
    std::vector<double> bb(nrhs);
    HIPCHK(hipMemcpyAsync(bb.data(), w.sc.bb, nrhs * sizeof(double), hipMemcpyDeviceToHost, c.st));
    // r^ = r (rounded to fmt_op), p = r, rho = <r^, r>, in one pass
    HIPCHK(launch_bi_init(g, fmt_acc, fmt_op, nrhs, w.sc.mask, w.s_acc, w.rh, w.p, w.pa, w.pb, w.pc, c.st));
    HIPCHK(launch_bi_scalars(BI_INIT, B, nbb, w.pa, w.pb, w.pc, c.st));
    int live = look_at(c, w, nrhs, tol2, bb, ss, mask, res);
    if (live < 0) return live;
    if (!live) return WEO_OK;
    LookPlan plan(check_every, ss);
    int look = plan.first();
    // Wilson M with every vector in one format: <r^, v> and (<t, s>, ||t||^2)
    // come from the epilogues of the operator's second hop (the dot partner
    // r^ read there, s being that hop's own axpy input).  With a narrower
    // operator format (FP16 / BF16 inner solves) both stay separate passes:
    // omega from the rounded s cost iterations, and the partner read in the
    // epilogue of the packed FP16 hop cost more than the pass it saves.
    const bool fuse = op == WEO_OP_M && !c.clv && !c.full && same;
    const bool fuse_ts = fuse;
    const int nbh = (int)c.nb_apply;
    for (int it = 1; it <= maxiter; ++it) {
        if (fuse) {
            HIPCHK(apply_m(c, fmt_op, u, 0, w.p, w.q, w.tmp, nrhs, w.pc, 1, w.rh, w.pa, w.pb));
            HIPCHK(launch_bi_scalars(BI_ALPHA, B, nbh, w.pa, w.pb, nullptr, c.st));
        } else {
            HIPCHK(apply_op(c, op, fmt_op, u, w.p, w.q, w.r, w.tmp, nrhs, nullptr));
            HIPCHK(launch_bi_cdot(g, fmt_op, fmt_op, nrhs, w.sc.mask, w.rh, w.q, w.pa, w.pb, c.st));
            HIPCHK(launch_bi_scalars(BI_ALPHA, B, nbb, w.pa, w.pb, nullptr, c.st));
        }
        HIPCHK(launch_bi_s(g, fmt_acc, fmt_op, nrhs, B, w.s_acc, w.q, w.s2, s_op, w.pc, c.st));
        if (fuse_ts) {
            HIPCHK(apply_m(c, fmt_op, u, 0, s_op, w.t, w.tmp, nrhs, w.pc, 2, nullptr, w.pa, w.pb));
            HIPCHK(launch_bi_scalars(BI_OMEGA, B, nbh, w.pa, w.pb, w.pc, c.st));
        } else {
            HIPCHK(apply_op(c, op, fmt_op, u, s_op, w.t, w.r, w.tmp, nrhs, nullptr));
            HIPCHK(launch_bi_ts(g, fmt_acc, fmt_op, nrhs, w.sc.mask, w.t, w.s2, w.pa, w.pb, w.pc, c.st));
            HIPCHK(launch_bi_scalars(BI_OMEGA, B, nbb, w.pa, w.pb, w.pc, c.st));
        }
        HIPCHK(launch_bi_xr(g, fmt_acc, fmt_op, nrhs, B, x_acc, w.p, w.s2, w.t, w.s_acc, w.rh, w.pa, w.pb,
                            w.pc, c.st));
        HIPCHK(launch_bi_scalars(BI_BETA, B, nbb, w.pa, w.pb, w.pc, c.st));
        HIPCHK(launch_bi_p(g, fmt_acc, fmt_op, nrhs, B, w.s_acc, w.p, w.q, c.st));
        res->iters = it;
        if (it == look || it == maxiter) {
            live = look_at(c, w, nrhs, tol2, bb, ss, mask, res);
            if (live < 0) return live;
            if (!live) break;
            look = plan.next(it, ss, mask, bb, tol2);
        }
    }
    HIPCHK(hipStreamSynchronize(c.st));
    return WEO_OK;
}

// ---- block CG ---------------------------------------------------------------
// Small dense complex algebra for the s x s factors, FP64 on the host; row-major.
using cplx = std::complex<double>;
struct Mat {
    int n;
    std::vector<cplx> a;
    explicit Mat(int n_) : n(n_), a((size_t)n_ * n_) {}
    cplx& operator()(int i, int j) { return a[(size_t)i * n + j]; }
    cplx operator()(int i, int j) const { return a[(size_t)i * n + j]; }
    static Mat eye(int n) {
        Mat m(n);
        for (int i = 0; i < n; ++i) m(i, i) = 1.0;
        return m;
    }
};
Mat mul(const Mat& x, const Mat& y) {
    Mat z(x.n);
    for (int i = 0; i < x.n; ++i)
        for (int k = 0; k < x.n; ++k)
            for (int j = 0; j < x.n; ++j) z(i, j) += x(i, k) * y(k, j);
    return z;
}
Mat adj(const Mat& x) {
    Mat z(x.n);
    for (int i = 0; i < x.n; ++i)
        for (int j = 0; j < x.n; ++j) z(i, j) = std::conj(x(j, i));
    return z;
}
// The Hermitian matrix whose upper triangle the device computed (re, im
// interleaved, G[j][k] = <a_j, b_k> for j <= k).
Mat gram_from(const std::vector<double>& g, int n) {
    Mat h(n);
    for (int i = 0; i < n; ++i)
        for (int j = i; j < n; ++j) {
            const cplx v(g[(i * n + j) * 2], i == j ? 0.0 : g[(i * n + j) * 2 + 1]);
            h(i, j) = v;
            h(j, i) = std::conj(v);
        }
    return h;
}
// G = L L^H.  False unless every pivot exceeds rank_eps times its diagonal
// entry (the squared sine of the angle between a column and the span of the
// ones before it): a rank-deficient block, to the vectors' precision.
bool cholesky(const Mat& gm, Mat& l, double rank_eps) {
    const int n = gm.n;
    l = Mat(n);
    for (int j = 0; j < n; ++j) {
        double d = gm(j, j).real();
        for (int k = 0; k < j; ++k) d -= std::norm(l(j, k));
        if (!(d > rank_eps * gm(j, j).real()) || !std::isfinite(d)) return false;
        l(j, j) = std::sqrt(d);
        for (int i = j + 1; i < n; ++i) {
            cplx v = gm(i, j);
            for (int k = 0; k < j; ++k) v -= l(i, k) * std::conj(l(j, k));
            l(i, j) = v / l(j, j).real();
        }
    }
    return true;
}
// inverse of a lower triangular matrix
Mat lower_inv(const Mat& l) {
    const int n = l.n;
    Mat x(n);
    for (int j = 0; j < n; ++j) {
        x(j, j) = 1.0 / l(j, j);
        for (int i = j + 1; i < n; ++i) {
            cplx v = 0.0;
            for (int k = j; k < i; ++k) v -= l(i, k) * x(k, j);
            x(i, j) = v / l(i, i);
        }
    }
    return x;
}
void to_dev_layout(const Mat& m, double* out) {
    for (int i = 0; i < m.n; ++i)
        for (int j = 0; j < m.n; ++j) {
            out[(i * m.n + j) * 2] = m(i, j).real();
            out[(i * m.n + j) * 2 + 1] = m(i, j).imag();
        }
}
// Cholesky factorisation of a Gram matrix G = Z^H Z (n x n) that deflates
// dependent columns: the columns are taken in order, and column i is kept
// when the part of z_i orthogonal to the kept columns before it has squared
// norm d > rank_eps G_ii (the squared sine of its angle to their span), else
// dropped.  On return kept lists the r kept columns and l (n x n, only the
// first r columns used) satisfies G_ij = sum_k l(i, k) conj(l(j, k)) for every
// i, j to that accuracy: with Q = Z_kept L_kk^-H (L_kk the kept rows of l),
// z_j = sum_k Q_k conj(l(j, k)).  False on a non-finite entry.
bool cholesky_deflate(const Mat& gm, Mat& l, std::vector<int>& kept, double rank_eps) {
    const int n = gm.n;
    l = Mat(n);
    kept.clear();
    for (int i = 0; i < n; ++i) {
        for (int k = 0; k < (int)kept.size(); ++k) {
            const int jk = kept[k];
            cplx v = gm(i, jk);
            for (int q = 0; q < k; ++q) v -= l(i, q) * std::conj(l(jk, q));
            l(i, k) = v / l(jk, k).real();
        }
        double d = gm(i, i).real();
        for (int k = 0; k < (int)kept.size(); ++k) d -= std::norm(l(i, k));
        if (!std::isfinite(d)) return false;
        if (d > rank_eps * gm(i, i).real()) {
            l(i, (int)kept.size()) = std::sqrt(d);
            kept.push_back(i);
        }
    }
    return true;
}
// The factors of a deflating QR Z = Q psi (Z with n columns, r kept): T with
// Q = Z T (n x r: row kept[k] holds column k of L_kk^-H, other rows zero)
// and psi^H = l restricted to its first r columns (n x r); both padded to
// n x n with zero columns from r on.
void deflate_factors(const Mat& l, const std::vector<int>& kept, Mat& t, Mat& psih) {
    const int n = l.n, r = (int)kept.size();
    Mat lkk(r);
    for (int a = 0; a < r; ++a)
        for (int b = 0; b < r; ++b) lkk(a, b) = l(kept[a], b);
    const Mat li = lower_inv(lkk);
    t = Mat(n);
    psih = Mat(n);
    for (int a = 0; a < r; ++a)
        for (int m = 0; m < r; ++m) t(kept[a], m) = std::conj(li(m, a));
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < r; ++k) psih(i, k) = l(i, k);
}
// The leading r x r block of an n x n matrix, and back (zero padded).
Mat lead(const Mat& m, int r) {
    Mat z(r);
    for (int i = 0; i < r; ++i)
        for (int j = 0; j < r; ++j) z(i, j) = m(i, j);
    return z;
}
Mat pad(const Mat& m, int n) {
    Mat z(n);
    for (int i = 0; i < m.n && i < n; ++i)
        for (int j = 0; j < m.n && j < n; ++j) z(i, j) = m(i, j);
    return z;
}

// Block CG at one precision level (vectors in one FP64 or FP32 format).  Same
// contract as run_level: x_acc holds the start, s_acc the residual b - M x
// (b - A x for M^dag M), mask the live rhs, bb[r] = ||b||^2.  The live rhs
// form one block; it stops when every one of them meets ||r||^2 <= tol^2 bb
// (r = S, or the recurrence ||C e_j||^2 for M^dag M).  Block vectors: Q = r,
// P = p, W = q, M P = t (fields 0 .. s-1).  Columns of the residual block
// that become dependent are deflated (the block shrinks); breakdown: P^H A P
// not numerically positive definite, or a non-finite Gram matrix.
int run_level_block(Ctx& c, const Workspace& w, int op, int fmt, const void* u, void* x_acc, int nrhs,
                    double tol, int maxiter, LevelResult* res) {
    const Geom& g = c.gb;
    const size_t fb = spinor_field_bytes(g, fmt);
    res->iters = 0;
    res->breakdown = 0;
    std::vector<int> mask(nrhs);
    std::vector<double> bb(nrhs);
    HIPCHK(hipMemcpyAsync(mask.data(), w.sc.mask, nrhs * sizeof(int), hipMemcpyDeviceToHost, c.st));
    HIPCHK(hipMemcpyAsync(bb.data(), w.sc.bb, nrhs * sizeof(double), hipMemcpyDeviceToHost, c.st));
    HIPCHK(hipStreamSynchronize(c.st));
    // rhs whose start already meets the tolerance stay out of the block
    std::vector<double> ss0(nrhs);
    HIPCHK(launch_norm2(g, fmt, w.s_acc, nrhs, w.pb, c.st));
    HIPCHK(launch_reduce(w.pb, (int)blas_blocks(g), nrhs, w.sc.rr, c.st));
    HIPCHK(hipMemcpyAsync(ss0.data(), w.sc.rr, nrhs * sizeof(double), hipMemcpyDeviceToHost, c.st));
    HIPCHK(hipStreamSynchronize(c.st));
    std::vector<int> live;
    for (int r = 0; r < nrhs; ++r)
        if (mask[r] && !(ss0[r] <= tol * tol * bb[r])) live.push_back(r);
    const int s = (int)live.size();
    if (!s) return WEO_OK;
    const bool normal = op != WEO_OP_MDAGM;
    // 64 unit roundoffs of the vector format
    const double rank_eps = 64.0 * (fmt_info(fmt).spinor_prec == WEO_F64 ? 0x1p-53 : 0x1p-24);
    auto ref = [&](void* base, bool mapped) {
        BlockRef b;
        std::memset(&b, 0, sizeof(b));
        b.base = static_cast<uint8_t*>(base);
        b.stride = fb;
        for (int j = 0; j < s; ++j) b.col[j] = (uint8_t)(mapped ? live[j] : j);
        return b;
    };
    const BlockRef X = ref(x_acc, true), S = ref(w.s_acc, true);
    const BlockRef Q = ref(w.r, false), P = ref(w.p, false), W = ref(w.q, false), MP = ref(w.t, false);
    const double tol2 = tol * tol;
    // host copies of the factors: each is rewritten only after a stream
    // synchronisation that follows its last upload
    std::vector<double> h_id(kGramStride), h_dc(kGramStride), h_dl(kGramStride), h_pi(kGramStride),
        h_ph(kGramStride), gh(kGramStride), ssv(s);
    // every exit (early error returns included) waits for the stream before
    // the host buffers above go out of scope (their uploads are asynchronous)
    struct SyncOnExit {
        hipStream_t st;
        ~SyncOnExit() { (void)hipStreamSynchronize(st); }
    } sync_on_exit{c.st};
    double* d_id = w.tm;
    double* d_dc = w.tm + kGramStride;
    double* d_dl = w.tm + 2 * kGramStride;
    double* d_pi = w.tm + 3 * kGramStride;
    double* d_ph = w.tm + 4 * kGramStride;
    // a factor laid out for kernels of width m.n
    auto upload = [&](const Mat& m, std::vector<double>& h, double* d) -> hipError_t {
        to_dev_layout(m, h.data());
        return hipMemcpyAsync(d, h.data(), (size_t)2 * m.n * m.n * sizeof(double), hipMemcpyHostToDevice, c.st);
    };
    // Gram matrix of the first n columns of two blocks (and ||S_j||^2)
    auto gram = [&](const BlockRef& a, const BlockRef& b, Mat& out, int n) -> hipError_t {
        hipError_t e = launch_block_gram(g, fmt, n, a, b, w.gpart, w.gram, c.st);
        if (e != hipSuccess) return e;
        e = hipMemcpyAsync(gh.data(), w.gram, (size_t)2 * n * n * sizeof(double), hipMemcpyDeviceToHost, c.st);
        if (e != hipSuccess) return e;
        if (normal) {
            e = hipMemcpyAsync(ssv.data(), w.sc.ss, s * sizeof(double), hipMemcpyDeviceToHost, c.st);
            if (e != hipSuccess) return e;
        }
        e = hipStreamSynchronize(c.st);
        out = gram_from(gh, n);
        return e;
    };
    // Deflation: the block (Q, P, W, M P) has r <= s columns, the first r of
    // its fields; columns of the residual block that become dependent are
    // dropped by cholesky_deflate, the block shrinks and C (r x s, held as an
    // s x s matrix with zero rows from r on) keeps their coefficients.  X and
    // S keep all s columns: their updates run at width s with zero rows of
    // the coefficient matrix for the dropped directions (the block fields
    // beyond r hold finite values from earlier steps).
    HIPCHK(upload(Mat::eye(s), h_id, d_id));
    // R_0 = S (M^dag M) or A^dag S, gathered into W; ||S_j||^2 into ss
    if (normal) {
        HIPCHK(launch_block_update(g, fmt, s, MP, nullptr, S, 1.0, d_id, w.upart, w.sc.ss, c.st));
        HIPCHK(apply_a(c, fmt, u, 1, w.t, w.q, w.tmp, s, nullptr));
    } else {
        HIPCHK(launch_block_update(g, fmt, s, W, nullptr, S, 1.0, d_id, nullptr, nullptr, c.st));
    }
    Mat gm(s), l(s), t(s), psih(s);
    std::vector<int> kept;
    HIPCHK(gram(W, W, gm, s));
    if (!cholesky_deflate(gm, l, kept, rank_eps)) { res->breakdown = 1; return WEO_OK; }
    int r = (int)kept.size();
    if (!r) return WEO_OK;
    deflate_factors(l, kept, t, psih);
    Mat cm = adj(psih);                                // C = psi_0 (R_0 = Q C)
    HIPCHK(upload(t, h_pi, d_pi));                     // Q = R_0 T
    HIPCHK(launch_block_update(g, fmt, s, Q, nullptr, W, 1.0, d_pi, nullptr, nullptr, c.st));
    HIPCHK(launch_block_update(g, fmt, s, P, nullptr, Q, 1.0, d_id, nullptr, nullptr, c.st));
    auto converged = [&]() {
        for (int j = 0; j < s; ++j) {
            double rr = 0.0;
            if (normal) rr = ssv[j];
            else
                for (int i = 0; i < s; ++i) rr += std::norm(cm(i, j));
            if (!(rr <= tol2 * bb[live[j]])) return false;
        }
        return true;
    };
    if (converged()) return WEO_OK;
    for (int it = 1; it <= maxiter; ++it) {
        // W = A P (M P kept for S)
        if (normal) {
            HIPCHK(apply_a(c, fmt, u, 0, w.p, w.t, w.tmp, r, nullptr));
            HIPCHK(apply_a(c, fmt, u, 1, w.t, w.q, w.tmp, r, nullptr));
        } else {
            HIPCHK(apply_op(c, op, fmt, u, w.p, w.q, w.t, w.tmp, r, nullptr));
        }
        Mat gpw(r), lpw(r);
        HIPCHK(gram(P, W, gpw, r));
        if (!cholesky(gpw, lpw, rank_eps)) { res->breakdown = 1; break; }
        const Mat li = lower_inv(lpw);
        const Mat delta = mul(adj(li), li);            // (P^H W)^-1
        HIPCHK(upload(mul(pad(delta, s), cm), h_dc, d_dc));
        HIPCHK(upload(delta, h_dl, d_dl));
        HIPCHK(launch_block_update(g, fmt, s, X, &X, P, 1.0, d_dc, nullptr, nullptr, c.st));
        if (normal) HIPCHK(launch_block_update(g, fmt, s, S, &S, MP, -1.0, d_dc, w.upart, w.sc.ss, c.st));
        HIPCHK(launch_block_update(g, fmt, r, Q, &Q, W, -1.0, d_dl, nullptr, nullptr, c.st));
        Mat gq(r);
        HIPCHK(gram(Q, Q, gq, r));
        res->iters = it;
        // the carried residuals of the normal equations decide before the
        // new residual block is factorised
        if (normal && converged()) break;
        Mat lq(r), tq(r), pq(r);
        if (!cholesky_deflate(gq, lq, kept, rank_eps)) { res->breakdown = 1; break; }
        const int r2 = (int)kept.size();
        deflate_factors(lq, kept, tq, pq);
        cm = mul(pad(adj(pq), s), cm);                 // C = psi C
        if (converged() || !r2) break;
        HIPCHK(upload(tq, h_pi, d_pi));                // Q' = Q T
        HIPCHK(upload(pq, h_ph, d_ph));                // psi^H
        HIPCHK(launch_block_qp(g, fmt, r, Q, P, d_pi, d_ph, c.st));
        r = r2;
    }
    HIPCHK(hipStreamSynchronize(c.st));
    return WEO_OK;
}

// Format conversion of nrhs solver vectors (scale per rhs, may be null).  A
// full field (D_W) is two packed halves whose record planes depend on the
// format, so it is converted half by half; one-parity fields in one pass.
hipError_t convert_fields(Ctx& c, int fin, const void* in, int fout, void* out, int nrhs, const double* scale,
                          int accumulate) {
    if (!c.full) return launch_convert(c.gb, fin, in, fout, out, nrhs, scale, accumulate, c.st);
    const size_t hi = spinor_field_bytes(c.g, fin), ho = spinor_field_bytes(c.g, fout);
    for (int r = 0; r < nrhs; ++r)
        for (int h = 0; h < 2; ++h) {
            const size_t k = (size_t)2 * r + h;
            const hipError_t e = launch_convert(c.g, fin, static_cast<const uint8_t*>(in) + k * hi, fout,
                                                static_cast<uint8_t*>(out) + k * ho, 1, scale ? scale + r : nullptr,
                                                accumulate, c.st);
            if (e != hipSuccess) return e;
        }
    return hipSuccess;
}

// Flexible GCR preconditioned by SAP, for D_W on full fields (op DW), one
// right-hand side after the other.  Same contract as run_level: x_acc holds
// the start, s_acc the residual b - D x (both in the level format fmt, the
// residual updated in place), mask the live rhs, bb[r] = ||b||^2.  Per
// iteration: phi_k = K r (SAP in FP32, converted when the level is FP64),
// chi_k = D_W phi_k, classical Gram-Schmidt of chi_k against chi_0..k-1 (one
// dot pass and one update pass that also gives ||chi_k||^2 and <chi_k, r>),
// r -= c_k chi_k / ||chi_k||.  The chi_l are kept unnormalised with their
// norms n_l on the host.  At the end of a cycle (nkv directions or
// convergence) x += sum_k alpha_k phi_k from the upper-triangular system.
int run_level_gcr(Ctx& c, const Workspace& w, int fmt, const void* u, void* x_acc, int nrhs, double tol,
                  int maxiter, LevelResult* res) {
    const Geom& gb = c.gb;
    const size_t fb = spinor_field_bytes(gb, fmt);
    const int nkv = c.nkv;
    const uint32_t nwg = gcr_wg(gb, fmt);
    const bool conv = c.fmt_pre != fmt;
    res->iters = 0;
    res->breakdown = 0;
    std::vector<int> mask(nrhs);
    std::vector<double> bb(nrhs);
    HIPCHK(hipMemcpyAsync(mask.data(), w.sc.mask, nrhs * sizeof(int), hipMemcpyDeviceToHost, c.st));
    HIPCHK(hipMemcpyAsync(bb.data(), w.sc.bb, nrhs * sizeof(double), hipMemcpyDeviceToHost, c.st));
    HIPCHK(hipStreamSynchronize(c.st));
    std::vector<double> sums(2 * kGcrMax);
    auto fetch = [&](int nval) -> hipError_t {
        hipError_t e = launch_reduce(w.gcpart, (int)nwg, nval, w.gcsum, c.st);
        if (e != hipSuccess) return e;
        e = hipMemcpyAsync(sums.data(), w.gcsum, nval * sizeof(double), hipMemcpyDeviceToHost, c.st);
        if (e != hipSuccess) return e;
        return hipStreamSynchronize(c.st);
    };
    const double tol2 = tol * tol;
    for (int r = 0; r < nrhs; ++r) {
        if (!mask[r]) continue;
        uint8_t* rv = static_cast<uint8_t*>(w.s_acc) + (size_t)r * fb;
        uint8_t* xv = static_cast<uint8_t*>(x_acc) + (size_t)r * fb;
        // ||r||^2 of the start
        {
            const void* none[1] = {rv};
            const double z = 0.0;
            HIPCHK(launch_gcr_update(gb, fmt, 0, none, &z, &z, rv, nullptr, w.gcpart, c.st));
            HIPCHK(fetch(1));
        }
        double rr = sums[0];
        int it = 0;
        bool breakdown = false;
        while (!(rr <= tol2 * bb[r]) && it < maxiter && !breakdown) {
            std::vector<std::complex<double>> a((size_t)nkv * nkv), cc(nkv);
            std::vector<double> nrm(nkv);
            int k = 0;
            for (; k < nkv && it < maxiter; ++k) {
                void* phi = w.gphi[k];
                void* chi = w.gchi[k];
                // phi_k = K r
                if (conv) {
                    HIPCHK(convert_fields(c, fmt, rv, c.fmt_pre, w.spin, 1, nullptr, 0));
                    HIPCHK(sap_apply(c.g, c.fmt_pre, c.sap, c.ncy, c.nmr, c.lat->kappa, c.ph, c.u_pre, w.spin,
                                     w.spout, w.srho, w.sd0, w.sd1, 1, c.st));
                    HIPCHK(convert_fields(c, c.fmt_pre, w.spout, fmt, phi, 1, nullptr, 0));
                } else {
                    HIPCHK(sap_apply(c.g, fmt, c.sap, c.ncy, c.nmr, c.lat->kappa, c.ph, c.u_pre, rv, phi, w.srho,
                                     w.sd0, w.sd1, 1, c.st));
                }
                // chi_k = D_W phi_k, orthogonalised against chi_0 .. chi_{k-1}
                HIPCHK(apply_dw(c, fmt, u, 0, phi, chi, 1, nullptr));
                std::vector<double> cre(kGcrMax, 0.0), cim(kGcrMax, 0.0);
                if (k > 0) {
                    HIPCHK(launch_gcr_dots(gb, fmt, k, w.gchi, chi, w.gcpart, c.st));
                    HIPCHK(fetch(2 * k));
                    for (int l = 0; l < k; ++l) {
                        const std::complex<double> alk(sums[2 * l] / nrm[l], sums[2 * l + 1] / nrm[l]);
                        a[(size_t)l * nkv + k] = alk;                  // <chi^_l, chi_k>
                        cre[l] = -alk.real() / nrm[l];
                        cim[l] = -alk.imag() / nrm[l];
                    }
                }
                HIPCHK(launch_gcr_update(gb, fmt, k, w.gchi, cre.data(), cim.data(), chi, rv, w.gcpart, c.st));
                HIPCHK(fetch(3));
                nrm[k] = std::sqrt(sums[0]);
                if (!(nrm[k] > 0.0) || !std::isfinite(nrm[k])) { breakdown = true; break; }
                a[(size_t)k * nkv + k] = nrm[k];
                cc[k] = std::complex<double>(sums[1], sums[2]) / nrm[k];     // <chi^_k, r>
                // r -= c_k chi^_k, and ||r||^2
                const double ur = -cc[k].real() / nrm[k], ui = -cc[k].imag() / nrm[k];
                const void* one[1] = {chi};
                HIPCHK(launch_gcr_update(gb, fmt, 1, one, &ur, &ui, rv, nullptr, w.gcpart, c.st));
                HIPCHK(fetch(1));
                rr = sums[0];
                ++it;
                if (rr <= tol2 * bb[r]) { ++k; break; }
            }
            // x += sum alpha_l phi_l with sum_{m >= l} a_lm alpha_m = c_l
            std::vector<std::complex<double>> al(kGcrMax, 0.0);
            for (int l = k - 1; l >= 0; --l) {
                std::complex<double> t = cc[l];
                for (int m = l + 1; m < k; ++m) t -= a[(size_t)l * nkv + m] * al[m];
                al[l] = t / a[(size_t)l * nkv + l];
            }
            if (k > 0) {
                std::vector<double> xr(kGcrMax), xi(kGcrMax);
                for (int l = 0; l < k; ++l) { xr[l] = al[l].real(); xi[l] = al[l].imag(); }
                HIPCHK(launch_gcr_update(gb, fmt, k, w.gphi, xr.data(), xi.data(), xv, nullptr, nullptr, c.st));
            }
        }
        res->iters += it;
        if (breakdown) res->breakdown = 1;
    }
    HIPCHK(hipStreamSynchronize(c.st));
    return WEO_OK;
}

// One precision level with the requested method.
int run_method(Ctx& c, const Workspace& w, int method, int op, int fmt_op, int fmt_acc, const void* u,
               void* x_acc, int nrhs, double tol, int maxiter, int check_every, LevelResult* res) {
    if (method == WEO_SOLVER_BICGSTAB)
        return run_level_bicg(c, w, op, fmt_op, fmt_acc, u, x_acc, nrhs, tol, maxiter, check_every, res);
    if (method == WEO_SOLVER_BLOCK_CG) return run_level_block(c, w, op, fmt_op, u, x_acc, nrhs, tol, maxiter, res);
    if (method == WEO_SOLVER_SAP_GCR) return run_level_gcr(c, w, fmt_op, u, x_acc, nrhs, tol, maxiter, res);
    return run_level(c, w, op, fmt_op, fmt_acc, u, x_acc, nrhs, tol, maxiter, check_every, res);
}

// True relative residuals ||b - A x|| / ||b|| in format fmt (x, b in fmt).
int true_resid(Ctx& c, const Workspace& w, int op, int fmt, const void* u, const void* b, const void* x,
               void* t, void* mid, void* tmp, int nrhs, double* out) {
    const Geom& g = c.gb;
    HIPCHK(apply_op(c, op, fmt, u, x, t, mid, tmp, nrhs, nullptr));
    HIPCHK(launch_axpby(g, fmt, nrhs, 1.0, b, -1.0, t, t, w.pa, c.st));
    HIPCHK(launch_reduce(w.pa, (int)blas_blocks(g), nrhs, w.sc.rr, c.st));
    std::vector<double> rr(nrhs), bb(nrhs);
    HIPCHK(hipMemcpyAsync(rr.data(), w.sc.rr, nrhs * sizeof(double), hipMemcpyDeviceToHost, c.st));
    HIPCHK(hipMemcpyAsync(bb.data(), w.sc.bb, nrhs * sizeof(double), hipMemcpyDeviceToHost, c.st));
    HIPCHK(hipStreamSynchronize(c.st));
    for (int r = 0; r < nrhs; ++r) out[r] = bb[r] > 0 ? std::sqrt(rr[r] / bb[r]) : std::sqrt(rr[r]);
    return WEO_OK;
}

int set_mask(Ctx& c, const Workspace& w, const std::vector<int>& mask) {
    std::vector<int> zero(mask.size(), 0);
    HIPCHK(hipMemcpyAsync(w.sc.mask, mask.data(), mask.size() * sizeof(int), hipMemcpyHostToDevice, c.st));
    HIPCHK(hipMemcpyAsync(w.sc.flags, zero.data(), zero.size() * sizeof(int), hipMemcpyHostToDevice, c.st));
    HIPCHK(hipStreamSynchronize(c.st));   // host vectors go out of scope
    return WEO_OK;
}

// Geometry of the solver's vectors: the lattice's, or (D_W on full fields)
// one with twice the sites per field; vector kernels only use the site count.
Geom vector_geom(const Geom& g, int op) {
    if (op != WEO_OP_DW) return g;
    const int d2[4] = {g.lx, g.ly, g.lz, 2 * g.lt};
    return make_geom(d2);
}

int check_params(const weo_solver_params* p, int fmt, int* inner_fmt) {
    if (!p) return WEO_ERR_ARG;
    if (p->op != WEO_OP_M && p->op != WEO_OP_MDAGM && p->op != WEO_OP_DW) return WEO_ERR_ARG;
    if (p->nrhs < 1 || p->nrhs > WEO_MAX_RHS) return WEO_ERR_ARG;
    if (!(p->tol > 0.0) || !std::isfinite(p->tol) || p->maxiter < 0) return WEO_ERR_ARG;
    if (p->check_every < 1 || (p->x0_given != 0 && p->x0_given != 1)) return WEO_ERR_ARG;
    if (p->mixed != 0 && p->mixed != 1) return WEO_ERR_ARG;
    if (p->method != WEO_SOLVER_CG && p->method != WEO_SOLVER_BICGSTAB && p->method != WEO_SOLVER_BLOCK_CG &&
        p->method != WEO_SOLVER_SAP_GCR)
        return WEO_ERR_ARG;
    if (p->method == WEO_SOLVER_SAP_GCR) {
        if (p->op != WEO_OP_DW || p->gcr_nkv < 1 || p->gcr_nkv > kGcrMax) return WEO_ERR_ARG;
        if (p->sap.ncy < 1 || p->sap.nmr < 1 || p->sap.nmr > 64) return WEO_ERR_ARG;
    }
    // site blocks: the even-odd operator only; the inner level needs its own
    if ((p->clover || p->clover_inner) && p->op == WEO_OP_DW) return WEO_ERR_ARG;
    if (p->mixed && (p->clover != nullptr) != (p->clover_inner != nullptr)) return WEO_ERR_ARG;
    *inner_fmt = fmt;
    if (p->mixed) {
        if (fmt_info(fmt).spinor_prec != WEO_F64) return WEO_ERR_FORMAT;
        const int rc = check_fmt(&p->inner, inner_fmt);
        if (rc != WEO_OK) return rc;
        const int sp = fmt_info(*inner_fmt).spinor_prec;
        if (sp == WEO_F64) return WEO_ERR_FORMAT;
        // block CG keeps every vector in one format: FP32 inner spinors; a
        // D_W level mixes the accumulation format (FP32) with the operator's
        // only where their records coincide (FP32 inner spinors); the SAP
        // preconditioner runs on FP32 spinors and links
        if ((p->method == WEO_SOLVER_BLOCK_CG || p->op == WEO_OP_DW) && sp != WEO_F32) return WEO_ERR_FORMAT;
        if (p->method == WEO_SOLVER_SAP_GCR && fmt_info(*inner_fmt).link_prec != WEO_F32) return WEO_ERR_FORMAT;
        if (!(p->inner_tol > 0.0) || !(p->inner_tol < 1.0) || p->max_outer < 1) return WEO_ERR_ARG;
    } else {
        // a plain solve accumulates in its own format; FP16/BF16 storage is
        // only used as the inner format of a mixed solve
        const int sp = fmt_info(fmt).spinor_prec;
        if (sp != WEO_F64 && sp != WEO_F32) return WEO_ERR_FORMAT;
        if (p->method == WEO_SOLVER_SAP_GCR) {
            if (sp == WEO_F32) {
                if (fmt_info(fmt).link_prec != WEO_F32) return WEO_ERR_FORMAT;
            } else {
                // FP64 vectors: the preconditioner's FP32 format and links
                const int rc = check_fmt(&p->inner, inner_fmt);
                if (rc != WEO_OK) return rc;
                if (fmt_info(*inner_fmt).spinor_prec != WEO_F32 || fmt_info(*inner_fmt).link_prec != WEO_F32)
                    return WEO_ERR_FORMAT;
            }
        }
    }
    return WEO_OK;
}

}  // namespace
}  // namespace weo

using namespace weo;

extern "C" size_t wilson_eo_cg_workspace_bytes(const weo_lattice* lat, const weo_format* fmt,
                                               const weo_solver_params* p) {
    Geom g;
    int id, inner;
    if (check_lattice(lat, &g) != WEO_OK || check_fmt(fmt, &id) != WEO_OK) return 0;
    if (check_params(p, id, &inner) != WEO_OK) return 0;
    if ((uint64_t)vector_geom(g, p->op).vh > (1ull << 26)) return 0;
    SapGeom sg;
    if (p->method == WEO_SOLVER_SAP_GCR && make_sap_geom(g, p->sap.block, &sg) != 0) return 0;
    return carve_ws(vector_geom(g, p->op), id, p, inner, nullptr, 0).bytes;
}

extern "C" int wilson_eo_cg(const weo_lattice* lat, const weo_format* fmt, const weo_solver_params* p,
                            const void* u, const void* u_inner, const void* b, void* x, void* workspace,
                            size_t ws_bytes, weo_solver_info* info, void* stream) {
    const auto t0 = std::chrono::steady_clock::now();
    Geom g;
    int id, inner;
    int rc;
    if ((rc = check_lattice(lat, &g)) != WEO_OK) return rc;
    if ((rc = check_fmt(fmt, &id)) != WEO_OK) return rc;
    if ((rc = check_params(p, id, &inner)) != WEO_OK) return rc;
    if (!info) return WEO_ERR_ARG;
    if ((rc = check_ptr(u)) != WEO_OK || (rc = check_ptr(b)) != WEO_OK || (rc = check_ptr(x)) != WEO_OK)
        return rc;
    const bool pre64 = p->method == WEO_SOLVER_SAP_GCR && !p->mixed && fmt_info(id).spinor_prec == WEO_F64;
    if ((p->mixed || pre64) && (rc = check_ptr(u_inner)) != WEO_OK) return rc;
    SapGeom sg;
    std::memset(&sg, 0, sizeof(sg));
    if (p->method == WEO_SOLVER_SAP_GCR && make_sap_geom(g, p->sap.block, &sg) != 0) return WEO_ERR_ARG;
    if (p->clover && (rc = check_ptr(p->clover)) != WEO_OK) return rc;
    if (p->mixed && p->clover_inner && (rc = check_ptr(p->clover_inner)) != WEO_OK) return rc;
    if ((rc = check_ptr(workspace)) != WEO_OK) return rc == WEO_ERR_ARG ? WEO_ERR_WORKSPACE : rc;
    const Geom gb = vector_geom(g, p->op);
    if ((uint64_t)gb.vh > (1ull << 26)) return WEO_ERR_DIMS;
    const Workspace need = carve_ws(gb, id, p, inner, nullptr, 0);
    if (ws_bytes < need.bytes) return WEO_ERR_WORKSPACE;
    const int n = p->nrhs;
    const size_t fb = (size_t)n * spinor_field_bytes(gb, id);
    if (overlaps(b, fb, x, fb) || overlaps(workspace, ws_bytes, x, fb) || overlaps(workspace, ws_bytes, b, fb))
        return WEO_ERR_ARG;

    std::memset(info, 0, sizeof(*info));
    Workspace w = carve_ws(gb, id, p, inner, static_cast<uint8_t*>(workspace), ws_bytes);
    Ctx c;
    c.lat = lat;
    c.g = g;
    c.gb = gb;
    c.full = p->op == WEO_OP_DW;
    c.nb_apply = c.full ? blas_blocks(gb) : hop_partials(g);
    c.clv = p->clover;
    phases_of(lat, c.ph);
    c.st = static_cast<hipStream_t>(stream);
    c.applies = 0;
    c.sap = sg;
    c.ncy = p->sap.ncy;
    c.nmr = p->sap.nmr;
    c.nkv = p->gcr_nkv;
    // the SAP preconditioner's FP32 format and links: the level's own when
    // its spinors are FP32, else (plain FP64 solve) the inner ones
    c.fmt_pre = pre64 ? inner : (p->mixed ? inner : id);
    c.u_pre = (pre64 || p->mixed) ? u_inner : u;
    const uint32_t nbb = blas_blocks(gb);
    std::vector<int> live(n, 1);
    int status = WEO_OK;

    // bb = ||b||^2
    HIPCHK(launch_norm2(gb, id, b, n, w.pa, c.st));
    HIPCHK(launch_reduce(w.pa, (int)nbb, n, w.sc.bb, c.st));

    if (!p->mixed) {
        // s = b - A x (or b), x = 0 when no start is given
        if (p->x0_given) {
            HIPCHK(apply_op(c, p->op, id, u, x, w.q, w.t, w.tmp, n, nullptr));
            HIPCHK(launch_axpby(gb, id, n, 1.0, b, -1.0, w.q, w.s_acc, nullptr, c.st));
        } else {
            HIPCHK(launch_zero(x, fb, c.st));
            HIPCHK(launch_convert(gb, id, b, id, w.s_acc, n, nullptr, 0, c.st));
        }
        if ((rc = set_mask(c, w, live)) != WEO_OK) return rc;
        LevelResult lr;
        if ((rc = run_method(c, w, p->method, p->op, id, id, u, x, n, p->tol, p->maxiter, p->check_every,
                             &lr)) != WEO_OK)
            return rc;
        info->iters = lr.iters;
        if ((rc = true_resid(c, w, p->op, id, u, b, x, w.q, w.t, w.tmp, n, info->true_rel_resid)) != WEO_OK)
            return rc;
        for (int r = 0; r < n; ++r)
            if (!(info->true_rel_resid[r] <= p->tol)) status = WEO_NOT_CONVERGED;
        // a breakdown matters only where a right-hand side is still unconverged
        if (lr.breakdown && status != WEO_OK) status = WEO_BREAKDOWN;
    } else {
        // FP64 defect correction around inner solves in the inner format.
        // Right-hand sides that meet the tolerance drop out: from then on the
        // FP64 residuals and the inner solves run on the live ones only,
        // compacted to the front of the work fields (live[j] is the rhs in
        // compact slot j), so a last step for a few stragglers costs a few
        // fields, not n.  (M^dag M keeps all n: its residual needs a second
        // FP64 intermediate field.)
        const double target = 12.0 * (double)gb.vh;    // unit RMS per complex component
        if (!p->x0_given) HIPCHK(launch_zero(x, fb, c.st));
        int inner_iters = 0, k = 0;
        bool breakdown = false;
        std::vector<double> rel(n), bb0(n);
        HIPCHK(hipMemcpyAsync(bb0.data(), w.sc.bb, n * sizeof(double), hipMemcpyDeviceToHost, c.st));
        HIPCHK(hipStreamSynchronize(c.st));
        const size_t f1 = spinor_field_bytes(gb, id), fa1 = spinor_field_bytes(gb, kAccF32);
        const bool can_compact = p->op != WEO_OP_MDAGM;
        // the Wilson M residual in one fused pass (site blocks and D_W take
        // the operator, then b - A x)
        const bool fused_resid = p->op == WEO_OP_M && !p->clover;
        auto at = [](const void* base, size_t bytes, int j) {
            return static_cast<uint8_t*>(const_cast<void*>(base)) + (size_t)j * bytes;
        };
        std::vector<int> cur(n);            // rhs of compact slot j (slots of r64, sc_in, sc_out)
        for (int r = 0; r < n; ++r) cur[r] = r;
        for (;;) {
            const int m = (int)cur.size();
            const bool dense = m == n;      // slot j holds rhs j
            // r64 = b - A x, rr = ||r64||^2 for the rhs in cur.  From a zero
            // start the residual is b itself, whose norm partials are still in pa.
            const bool from_zero = k == 0 && !p->x0_given;
            const void* r64 = from_zero ? b : w.r64;
            int nba = (int)nbb;             // partials per rhs in pa
            if (!from_zero && dense && fused_resid) {
                HIPCHK(resid_m(c, id, u, x, b, w.r64, w.tmp64, n, w.pa));
                nba = (int)c.nb_apply;
            } else if (!from_zero && dense) {
                HIPCHK(apply_op(c, p->op, id, u, x, w.t64, w.r64, w.tmp64, n, nullptr));
                HIPCHK(launch_axpby(gb, id, n, 1.0, b, -1.0, w.t64, w.r64, w.pa, c.st));
            } else if (!from_zero) {
                // the live x gathered into r64 (free until the axpby below)
                for (int j = 0; j < m; ++j)
                    HIPCHK(hipMemcpyAsync(at(w.r64, f1, j), at(x, f1, cur[j]), f1, hipMemcpyDeviceToDevice, c.st));
                HIPCHK(apply_op(c, p->op, id, u, w.r64, w.t64, nullptr, w.tmp64, m, nullptr));
                for (int j = 0; j < m; ++j)
                    HIPCHK(launch_axpby(gb, id, 1, 1.0, at(b, f1, cur[j]), -1.0, at(w.t64, f1, j), at(w.r64, f1, j),
                                        w.pa + (size_t)j * nbb, c.st));
            }
            ScalarArgsHost sa = sargs(w.sc, m);
            sa.pa = w.pa; sa.nba = nba; sa.target = target;
            HIPCHK(launch_scalars(SCAL_SCALE, sa, c.st));
            std::vector<double> rr(m);
            HIPCHK(hipMemcpyAsync(rr.data(), w.sc.nrm, m * sizeof(double), hipMemcpyDeviceToHost, c.st));
            HIPCHK(hipStreamSynchronize(c.st));
            std::vector<int> keep;          // compact slots still live
            double worst = 0.0;
            for (int j = 0; j < m; ++j) {
                const int r = cur[j];
                rel[r] = bb0[r] > 0 ? std::sqrt(rr[j] / bb0[r]) : std::sqrt(rr[j]);
                if (!(rel[r] <= p->tol)) keep.push_back(j);
            }
            for (int r = 0; r < n; ++r) worst = std::fmax(worst, rel[r]);
            const int nlive = (int)keep.size();
            if (solver_log())
                fprintf(stderr, "[wilson_eo] outer %d: %d of %d rhs live, worst residual %.3e, inner iterations %d\n",
                        k, nlive, n, worst, inner_iters);
            if (!nlive || k >= p->max_outer || inner_iters >= p->maxiter || breakdown) break;
            // without compaction every rhs stays in its slot (converged ones
            // masked off inside the inner solve)
            std::vector<int> slots = keep;
            if (!can_compact) {
                slots.resize(n);
                for (int j = 0; j < n; ++j) slots[j] = j;
            }
            const int mi = (int)slots.size();
            bool ident = mi == m;
            for (int j = 0; j < mi && ident; ++j) ident = slots[j] == j;
            // inner right-hand sides: the slots' r64 scaled to unit RMS, in
            // FP32, at the front of s_acc; x_acc = 0
            if (ident) {
                HIPCHK(convert_fields(c, id, r64, kAccF32, w.s_acc, mi, w.sc.sc_in, 0));
            } else {
                for (int j = 0; j < mi; ++j)
                    HIPCHK(convert_fields(c, id, at(r64, f1, slots[j]), kAccF32, at(w.s_acc, fa1, j), 1,
                                          w.sc.sc_in + slots[j], 0));
            }
            HIPCHK(launch_zero(w.x_acc, (size_t)mi * fa1, c.st));
            // the inner stopping test compares with ||rhs||^2 = target
            std::vector<double> tg(mi, target);
            HIPCHK(hipMemcpyAsync(w.sc.bb, tg.data(), mi * sizeof(double), hipMemcpyHostToDevice, c.st));
            std::vector<int> mask(mi, 1);
            if (!can_compact)
                for (int j = 0; j < mi; ++j) mask[j] = !(rel[cur[j]] <= p->tol);
            if ((rc = set_mask(c, w, mask)) != WEO_OK) return rc;
            // The inner tolerance: inner_tol, tightened (down to inner_tol / 8)
            // for a step whose solve can then bring every live rhs to tol --
            // one inner solve a little longer instead of one more outer step
            // for the stragglers (an FP64 residual and a Krylov restart).
            double worst_live = 0.0;
            for (int j = 0; j < mi; ++j)
                if (can_compact || !(rel[cur[slots[j]]] <= p->tol)) worst_live = std::fmax(worst_live, rel[cur[slots[j]]]);
            double tin = p->inner_tol;
            const double need = worst_live > 0.0 ? p->tol / worst_live : 1.0;
            if (need < tin && need >= tin / 8.0) tin = std::fmax(0.5 * need, tin / 8.0);
            LevelResult lr;
            c.clv = p->clover_inner;
            rc = run_method(c, w, p->method, p->op, inner, kAccF32, u_inner, w.x_acc, mi, tin,
                            p->maxiter - inner_iters, p->check_every, &lr);
            c.clv = p->clover;
            if (rc != WEO_OK) return rc;
            inner_iters += lr.iters;
            breakdown = breakdown || lr.breakdown;
            // x += x_acc * sc_out (masked rhs have x_acc = 0)
            std::vector<int> next(mi);
            for (int j = 0; j < mi; ++j) next[j] = cur[slots[j]];
            if (ident && dense) {
                HIPCHK(convert_fields(c, kAccF32, w.x_acc, id, x, n, w.sc.sc_out, 1));
            } else {
                for (int j = 0; j < mi; ++j)
                    HIPCHK(convert_fields(c, kAccF32, at(w.x_acc, fa1, j), id, at(x, f1, next[j]), 1,
                                          w.sc.sc_out + slots[j], 1));
            }
            cur.swap(next);
            ++k;
        }
        info->iters = inner_iters;
        info->outer_iters = k;
        for (int r = 0; r < n; ++r) {
            info->true_rel_resid[r] = rel[r];
            if (!(rel[r] <= p->tol)) status = WEO_NOT_CONVERGED;
        }
        if (breakdown && status != WEO_OK) status = WEO_BREAKDOWN;
    }
    info->applies = c.applies;
    info->status = status;
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return status;
}
