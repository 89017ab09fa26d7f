// BLAS-1 kernels on packed one-parity spinor fields and the scalar kernels of
// the Krylov solvers.  Streaming kernels: one lane per (site, rhs), all 12
// complex components of a site per lane, coalesced plane loads.
//
// Reductions are deterministic: every workgroup writes one FP64 partial
// (wavefront shuffle tree, then the workgroup's wavefronts summed in order
// through LDS) and a single-workgroup kernel per right-hand side sums the
// partials in a fixed order.  Dot products and norms always accumulate in
// FP64, whatever the storage precision.
#include <math.h>

#include "weo_device.h"
#include "weo_internal.h"

namespace weo {

static constexpr int kBlk = 256;

template <int P> struct AR { using R = float; };
template <> struct AR<P_F64> { using R = double; };

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum over the workgroup (at most 1024 lanes) in a fixed order; result in
// thread 0.
__device__ __forceinline__ double group_sum(double v) {
    __shared__ double lds[16];
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += lds[w];
    return s;
}

template <class C> __device__ __forceinline__ double norm2_12(const C* v) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 12; ++k) s += (double)v[k].x * (double)v[k].x + (double)v[k].y * (double)v[k].y;
    return s;
}

// Convert a record to another arithmetic type.
template <class CO, class CI> __device__ __forceinline__ void cvt12(const CI* a, CO* b) {
#pragma unroll
    for (int k = 0; k < 12; ++k) { b[k].x = a[k].x; b[k].y = a[k].y; }
}

struct Fields {
    uint32_t vh;
    size_t fb_acc, fb_op;      // bytes of one field in each format
};

// x += alpha_r p ; s -= alpha_r q ; [s_op = s] ; partial = ||s||^2
// x, s in format ACC; p, q (and s_op) in format OP.
template <int ACC, int OP, bool SOP>
__global__ void __launch_bounds__(kBlk) k_axpy2(Fields F, const double* __restrict__ alpha,
                                                const int* __restrict__ mask, uint8_t* x, const uint8_t* p,
                                                uint8_t* s, const uint8_t* q, uint8_t* s_op, double* partial) {
    using RA = typename AR<ACC>::R;
    using RO = typename AR<OP>::R;
    using CA = cx<RA>;
    using CO = cx<RO>;
    const int r = blockIdx.y;
    const uint32_t i = blockIdx.x * kBlk + threadIdx.x;
    double nrm = 0.0;
    const bool live = mask == nullptr || mask[r] != 0;
    if (live && i < F.vh) {
        const RA a = (RA)alpha[r];
        CA xv[12], sv[12];
        CO pv[12], qv[12];
        uint8_t* xr = x + (size_t)r * F.fb_acc;
        uint8_t* sr = s + (size_t)r * F.fb_acc;
        load_rec<ACC, 12>(xr, F.vh, i, xv);
        load_rec<OP, 12>(p + (size_t)r * F.fb_op, F.vh, i, pv);
        load_rec<ACC, 12>(sr, F.vh, i, sv);
        load_rec<OP, 12>(q + (size_t)r * F.fb_op, F.vh, i, qv);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            xv[k].x = fma(a, (RA)pv[k].x, xv[k].x);
            xv[k].y = fma(a, (RA)pv[k].y, xv[k].y);
            sv[k].x = fma(-a, (RA)qv[k].x, sv[k].x);
            sv[k].y = fma(-a, (RA)qv[k].y, sv[k].y);
        }
        store_rec<ACC, 12>(xr, F.vh, i, xv);
        store_rec<ACC, 12>(sr, F.vh, i, sv);
        if constexpr (SOP) {
            CO so[12];
            cvt12(sv, so);
            store_rec<OP, 12>(s_op + (size_t)r * F.fb_op, F.vh, i, so);
        }
        nrm = norm2_12(sv);
    }
    const double t = group_sum(nrm);
    if (threadIdx.x == 0 && partial) partial[(size_t)r * gridDim.x + blockIdx.x] = t;
}

// p = r + beta_r p   (format OP)
template <int OP>
__global__ void __launch_bounds__(kBlk) k_xpay(Fields F, const double* __restrict__ beta,
                                               const int* __restrict__ mask, const uint8_t* rv,
                                               uint8_t* p) {
    using R = typename AR<OP>::R;
    using C = cx<R>;
    const int r = blockIdx.y;
    const uint32_t i = blockIdx.x * kBlk + threadIdx.x;
    if ((mask != nullptr && mask[r] == 0) || i >= F.vh) return;
    const R b = (R)beta[r];
    C a[12], pv[12];
    uint8_t* pr = p + (size_t)r * F.fb_op;
    load_rec<OP, 12>(rv + (size_t)r * F.fb_op, F.vh, i, a);
    load_rec<OP, 12>(pr, F.vh, i, pv);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        pv[k].x = fma(b, pv[k].x, a[k].x);
        pv[k].y = fma(b, pv[k].y, a[k].y);
    }
    store_rec<OP, 12>(pr, F.vh, i, pv);
}

// out = ca a + cb b (b may be null), partial = ||out||^2 (optional)
template <int P>
__global__ void __launch_bounds__(kBlk) k_axpby(Fields F, double ca, const uint8_t* a, double cb,
                                                const uint8_t* b, uint8_t* out, double* partial) {
    using R = typename AR<P>::R;
    using C = cx<R>;
    const int r = blockIdx.y;
    const uint32_t i = blockIdx.x * kBlk + threadIdx.x;
    double nrm = 0.0;
    if (i < F.vh) {
        C av[12], bv[12];
        load_rec<P, 12>(a + (size_t)r * F.fb_op, F.vh, i, av);
        if (b) load_rec<P, 12>(b + (size_t)r * F.fb_op, F.vh, i, bv);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            R x = (R)ca * av[k].x, y = (R)ca * av[k].y;
            if (b) { x = fma((R)cb, bv[k].x, x); y = fma((R)cb, bv[k].y, y); }
            av[k].x = x; av[k].y = y;
        }
        store_rec<P, 12>(out + (size_t)r * F.fb_op, F.vh, i, av);
        if (partial) {
            C st[12];
            if constexpr (P == P_F64 || P == P_F32) {
#pragma unroll
                for (int k = 0; k < 12; ++k) st[k] = av[k];
            } else {
                round_rec<P, 12>(av, st);
            }
            nrm = norm2_12(st);
        }
    }
    if (partial) {
        const double t = group_sum(nrm);
        if (threadIdx.x == 0) partial[(size_t)r * gridDim.x + blockIdx.x] = t;
    }
}

// partial = ||a||^2
template <int P>
__global__ void __launch_bounds__(kBlk) k_norm2(Fields F, const uint8_t* a, double* partial) {
    using C = cx<typename AR<P>::R>;
    const int r = blockIdx.y;
    const uint32_t i = blockIdx.x * kBlk + threadIdx.x;
    double nrm = 0.0;
    if (i < F.vh) {
        C av[12];
        load_rec<P, 12>(a + (size_t)r * F.fb_op, F.vh, i, av);
        nrm = norm2_12(av);
    }
    const double t = group_sum(nrm);
    if (threadIdx.x == 0) partial[(size_t)r * gridDim.x + blockIdx.x] = t;
}

// out (format PO) = in (format PI) * scale_r  [+ out]
template <int PI, int PO, bool ACCUM>
__global__ void __launch_bounds__(kBlk) k_convert(uint32_t vh, size_t fb_in, size_t fb_out, const uint8_t* in,
                                                  uint8_t* out, const double* __restrict__ scale) {
    using RI = typename AR<PI>::R;
    using RO = typename AR<PO>::R;
    using RW = typename AR<(PI == P_F64 || PO == P_F64) ? P_F64 : P_F32>::R;
    const int r = blockIdx.y;
    const uint32_t i = blockIdx.x * kBlk + threadIdx.x;
    if (i >= vh) return;
    cx<RI> a[12];
    load_rec<PI, 12>(in + (size_t)r * fb_in, vh, i, a);
    const RW sc = scale ? (RW)scale[r] : RW(1);
    cx<RO> o[12];
    if constexpr (ACCUM) load_rec<PO, 12>(out + (size_t)r * fb_out, vh, i, o);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        RW x = sc * (RW)a[k].x, y = sc * (RW)a[k].y;
        if constexpr (ACCUM) { x += (RW)o[k].x; y += (RW)o[k].y; }
        o[k].x = (RO)x;
        o[k].y = (RO)y;
    }
    store_rec<PO, 12>(out + (size_t)r * fb_out, vh, i, o);
}

__global__ void k_zero(uint4* p, size_t n16) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n16) p[i] = make_uint4(0u, 0u, 0u, 0u);
}

// out[r] = sum_b partial[r][b] in a fixed order (one workgroup per rhs).
// The final sums run in one workgroup per rhs; 1024 lanes keep the strided
// first pass short when there are tens of thousands of partials.
static constexpr int kRed = 1024;

__device__ __forceinline__ double reduce_row(const double* row, int nb) {
    double v = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) v += row[b];
    __syncthreads();       // the LDS slots may be reused by a second reduction
    return group_sum(v);
}

__global__ void __launch_bounds__(kRed) k_reduce(const double* partial, int nb, double* out) {
    const int r = blockIdx.x;
    const double s = reduce_row(partial + (size_t)r * nb, nb);
    if (threadIdx.x == 0) out[r] = s;
}

// Solver scalar steps (one workgroup per rhs).  Scalar block layout per rhs r:
//   sc[SC_GAMMA*n + r] ... see solver.cpp (kind selects the formula).
struct ScalarArgs {
    int nrhs, nba, nbb;
    const double* pa;    // partials for the first reduction
    const double* pb;    // partials for the second reduction (or null)
    double* gamma;       // <r, r> of the previous step
    double* alpha;
    double* beta;
    double* ss;          // ||s||^2 (or ||r||^2) reported to the host
    int* mask;
    int* flags;          // flags[r] |= 1 on breakdown
    double target;       // SCAL_SCALE: squared norm the scaled vector should have
    double* sc_in;       // SCAL_SCALE: scale into the inner format
    double* sc_out;      // SCAL_SCALE: scale back
    double* nrm;         // SCAL_SCALE: the reduced norm^2
    const double* bb;    // SCAL_BETA: ||b||^2 (or null: no device-side stop)
    double tol2;
};

__global__ void __launch_bounds__(kRed) k_scalars(int kind, ScalarArgs A) {
    const int r = blockIdx.x;
    const double a = reduce_row(A.pa + (size_t)r * A.nba, A.nba);
    double b = 0.0;
    if (A.pb) b = reduce_row(A.pb + (size_t)r * A.nbb, A.nbb);
    if (threadIdx.x != 0) return;
    const bool live = A.mask == nullptr || A.mask[r] != 0;
    if (kind == SCAL_ALPHA) {
        // a = ||M p||^2 (CGLS) or <p, A p> (CG); alpha = gamma / a
        double al = 0.0;
        if (live) {
            if (A.gamma[r] == 0.0) {
                // exact zero residual (e.g. b = 0): converged, nothing to do
                A.mask[r] = 0;
            } else if (!(a > 0.0) || !isfinite(a) || !isfinite(A.gamma[r])) {
                A.flags[r] |= 1;
                A.mask[r] = 0;
            } else {
                al = A.gamma[r] / a;
            }
        }
        A.alpha[r] = al;
    } else if (kind == SCAL_BETA) {
        // a = new <r, r>, b = ||s||^2 (CGLS) or unused (CG, then ss = a)
        double be = 0.0;
        if (live) {
            if (!isfinite(a)) {
                A.flags[r] |= 1;
                A.mask[r] = 0;
            } else {
                be = A.gamma[r] > 0.0 ? a / A.gamma[r] : 0.0;
                A.gamma[r] = a;
            }
            A.ss[r] = A.pb ? b : a;
            // converged: stop updating this rhs at once (the host sees it at
            // its next look); iterating on would only push the low-precision
            // vectors into underflow
            if (A.bb && A.ss[r] <= A.tol2 * A.bb[r]) A.mask[r] = 0;
        }
        A.beta[r] = be;
    } else {
        // SCAL_SCALE: nrm = a; sc_in = sqrt(target / a); sc_out = 1 / sc_in
        A.nrm[r] = a;
        const double si = a > 0.0 ? sqrt(A.target / a) : 1.0;
        A.sc_in[r] = si;
        A.sc_out[r] = 1.0 / si;
    }
}

// ---- BiCGStab (van der Vorst 1992) ----------------------------------------------
// Complex scalars per rhs are (re, im) pairs in FP64 device memory.  Vectors:
// x, r, r^ (shadow), s in format ACC; p, v, t (and s_op, the operator's copy of
// s) in format OP.  Masked rhs are left untouched and contribute zero partials.

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
    const double d = b.x * b.x + b.y * b.y;
    return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
__device__ __forceinline__ double2 cget(const double* p, int r) { return make_double2(p[2 * r], p[2 * r + 1]); }
__device__ __forceinline__ void cset(double* p, int r, double2 v) { p[2 * r] = v.x; p[2 * r + 1] = v.y; }

// Sums three values over the workgroup in a fixed order; results in thread 0.
__device__ __forceinline__ void group_sum3(double a, double b, double c, double* out) {
    __shared__ double lds[3][16];
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_sum(c);
    if ((threadIdx.x & 63) == 0) {
        lds[0][threadIdx.x >> 6] = a;
        lds[1][threadIdx.x >> 6] = b;
        lds[2][threadIdx.x >> 6] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        out[0] = out[1] = out[2] = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
            out[0] += lds[0][w];
            out[1] += lds[1][w];
            out[2] += lds[2][w];
        }
    }
}

struct BiArgs {
    double* rho;
    double* alpha;
    double* omega;
    double* beta;
    double* ss;
    const double* bb;
    double tol2;
    int* mask;
    int* flags;
};

__device__ __forceinline__ bool bi_live(const int* mask, int r) { return mask == nullptr || mask[r] != 0; }

// partial <a, b> = sum conj(a) b, a in PA (field size F.fb_acc), b in PB (F.fb_op)
template <int PA, int PB>
__global__ void __launch_bounds__(kBlk) k_bi_cdot(Fields F, const int* __restrict__ mask, const uint8_t* a,
                                                  const uint8_t* b, double* pre, double* pim) {
    using CA = cx<typename AR<PA>::R>;
    using CO = cx<typename AR<PB>::R>;
    const int r = blockIdx.y;
    const uint32_t i = blockIdx.x * kBlk + threadIdx.x;
    double re = 0.0, im = 0.0;
    if (bi_live(mask, r) && i < F.vh) {
        CA av[12];
        CO bv[12];
        load_rec<PA, 12>(a + (size_t)r * F.fb_acc, F.vh, i, av);
        load_rec<PB, 12>(b + (size_t)r * F.fb_op, F.vh, i, bv);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            re += (double)av[k].x * (double)bv[k].x + (double)av[k].y * (double)bv[k].y;
            im += (double)av[k].x * (double)bv[k].y - (double)av[k].y * (double)bv[k].x;
        }
    }
    double out[3];
    group_sum3(re, im, 0.0, out);
    if (threadIdx.x == 0) {
        pre[(size_t)r * gridDim.x + blockIdx.x] = out[0];
        pim[(size_t)r * gridDim.x + blockIdx.x] = out[1];
    }
}

// BiCGStab start in one pass: r^ = p = r rounded to OP; partials ||r||^2
// (every rhs) and <r^, r> (live rhs; r^ as stored, r in ACC)
template <int ACC, int OP>
__global__ void __launch_bounds__(kBlk) k_bi_init(Fields F, const int* __restrict__ mask, const uint8_t* r,
                                                  uint8_t* rh, uint8_t* p, double* prr, double* pre, double* pim) {
    using CA = cx<typename AR<ACC>::R>;
    using CO = cx<typename AR<OP>::R>;
    const int q = blockIdx.y;
    const uint32_t i = blockIdx.x * kBlk + threadIdx.x;
    double rr = 0.0, re = 0.0, im = 0.0;
    if (i < F.vh) {
        CA rv[12];
        load_rec<ACC, 12>(r + (size_t)q * F.fb_acc, F.vh, i, rv);
        CO ro[12];
        cvt12(rv, ro);
        store_rec<OP, 12>(rh + (size_t)q * F.fb_op, F.vh, i, ro);
        store_rec<OP, 12>(p + (size_t)q * F.fb_op, F.vh, i, ro);
        rr = norm2_12(rv);
        if (bi_live(mask, q)) {
            CO hv[12];
            round_rec<OP, 12>(ro, hv);
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                re += (double)hv[k].x * (double)rv[k].x + (double)hv[k].y * (double)rv[k].y;
                im += (double)hv[k].x * (double)rv[k].y - (double)hv[k].y * (double)rv[k].x;
            }
        }
    }
    double out[3];
    group_sum3(rr, re, im, out);
    if (threadIdx.x == 0) {
        prr[(size_t)q * gridDim.x + blockIdx.x] = out[0];
        pre[(size_t)q * gridDim.x + blockIdx.x] = out[1];
        pim[(size_t)q * gridDim.x + blockIdx.x] = out[2];
    }
}

// s = r - alpha v  [s_op = s];  partial = ||s||^2
template <int ACC, int OP, bool SOP>
__global__ void __launch_bounds__(kBlk) k_bi_s(Fields F, BiArgs B, const uint8_t* rv, const uint8_t* v,
                                               uint8_t* s, uint8_t* s_op, double* partial) {
    using RA = typename AR<ACC>::R;
    using CA = cx<RA>;
    using CO = cx<typename AR<OP>::R>;
    const int r = blockIdx.y;
    const uint32_t i = blockIdx.x * kBlk + threadIdx.x;
    double nrm = 0.0;
    if (bi_live(B.mask, r) && i < F.vh) {
        const double2 al = cget(B.alpha, r);
        const RA ar = (RA)al.x, ai = (RA)al.y;
        CA rr[12];
        CO vv[12];
        load_rec<ACC, 12>(rv + (size_t)r * F.fb_acc, F.vh, i, rr);
        load_rec<OP, 12>(v + (size_t)r * F.fb_op, F.vh, i, vv);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            const RA vx = (RA)vv[k].x, vy = (RA)vv[k].y;
            rr[k].x = rr[k].x - (ar * vx - ai * vy);
            rr[k].y = rr[k].y - (ar * vy + ai * vx);
        }
        store_rec<ACC, 12>(s + (size_t)r * F.fb_acc, F.vh, i, rr);
        if constexpr (SOP) {
            CO so[12];
            cvt12(rr, so);
            store_rec<OP, 12>(s_op + (size_t)r * F.fb_op, F.vh, i, so);
        }
        nrm = norm2_12(rr);
    }
    const double t = group_sum(nrm);
    if (threadIdx.x == 0) partial[(size_t)r * gridDim.x + blockIdx.x] = t;
}

// partials <t, s> (re, im) and ||t||^2; t in OP, s in ACC
template <int ACC, int OP>
__global__ void __launch_bounds__(kBlk) k_bi_ts(Fields F, const int* __restrict__ mask, const uint8_t* t,
                                                const uint8_t* s, double* pre, double* pim, double* ptt) {
    using CA = cx<typename AR<ACC>::R>;
    using CO = cx<typename AR<OP>::R>;
    const int r = blockIdx.y;
    const uint32_t i = blockIdx.x * kBlk + threadIdx.x;
    double re = 0.0, im = 0.0, tt = 0.0;
    if (bi_live(mask, r) && i < F.vh) {
        CO tv[12];
        CA sv[12];
        load_rec<OP, 12>(t + (size_t)r * F.fb_op, F.vh, i, tv);
        load_rec<ACC, 12>(s + (size_t)r * F.fb_acc, F.vh, i, sv);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            const double tx = tv[k].x, ty = tv[k].y, sx = sv[k].x, sy = sv[k].y;
            re += tx * sx + ty * sy;
            im += tx * sy - ty * sx;
            tt += tx * tx + ty * ty;
        }
    }
    double out[3];
    group_sum3(re, im, tt, out);
    if (threadIdx.x == 0) {
        const size_t o = (size_t)r * gridDim.x + blockIdx.x;
        pre[o] = out[0];
        pim[o] = out[1];
        ptt[o] = out[2];
    }
}

// x += alpha p + omega s;  r = s - omega t;  partials ||r||^2 and <r^, r>
// (r^ in OP)
template <int ACC, int OP>
__global__ void __launch_bounds__(kBlk) k_bi_xr(Fields F, BiArgs B, uint8_t* x, const uint8_t* p,
                                                const uint8_t* s, const uint8_t* t, uint8_t* rv,
                                                const uint8_t* rh, double* prr, double* pre, double* pim) {
    using RA = typename AR<ACC>::R;
    using CA = cx<RA>;
    using CO = cx<typename AR<OP>::R>;
    const int r = blockIdx.y;
    const uint32_t i = blockIdx.x * kBlk + threadIdx.x;
    double nrm = 0.0, re = 0.0, im = 0.0;
    if (bi_live(B.mask, r) && i < F.vh) {
        const double2 al = cget(B.alpha, r), om = cget(B.omega, r);
        const RA ar = (RA)al.x, ai = (RA)al.y, wr = (RA)om.x, wi = (RA)om.y;
        CA xv[12], sv[12];
        CO pv[12], tv[12];
        uint8_t* xrow = x + (size_t)r * F.fb_acc;
        load_rec<ACC, 12>(xrow, F.vh, i, xv);
        load_rec<OP, 12>(p + (size_t)r * F.fb_op, F.vh, i, pv);
        load_rec<ACC, 12>(s + (size_t)r * F.fb_acc, F.vh, i, sv);
        load_rec<OP, 12>(t + (size_t)r * F.fb_op, F.vh, i, tv);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            const RA px = (RA)pv[k].x, py = (RA)pv[k].y, tx = (RA)tv[k].x, ty = (RA)tv[k].y;
            xv[k].x += (ar * px - ai * py) + (wr * sv[k].x - wi * sv[k].y);
            xv[k].y += (ar * py + ai * px) + (wr * sv[k].y + wi * sv[k].x);
            sv[k].x -= wr * tx - wi * ty;          // sv becomes the new r
            sv[k].y -= wr * ty + wi * tx;
        }
        store_rec<ACC, 12>(xrow, F.vh, i, xv);
        store_rec<ACC, 12>(rv + (size_t)r * F.fb_acc, F.vh, i, sv);
        CO hv[12];
        load_rec<OP, 12>(rh + (size_t)r * F.fb_op, F.vh, i, hv);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            const double hx = hv[k].x, hy = hv[k].y, rx = sv[k].x, ry = sv[k].y;
            nrm += rx * rx + ry * ry;
            re += hx * rx + hy * ry;
            im += hx * ry - hy * rx;
        }
    }
    double out[3];
    group_sum3(nrm, re, im, out);
    if (threadIdx.x == 0) {
        const size_t o = (size_t)r * gridDim.x + blockIdx.x;
        prr[o] = out[0];
        pre[o] = out[1];
        pim[o] = out[2];
    }
}

// p = r + beta (p - omega v);  r in ACC, p and v in OP
template <int ACC, int OP>
__global__ void __launch_bounds__(kBlk) k_bi_p(Fields F, BiArgs B, const uint8_t* rv, uint8_t* p,
                                               const uint8_t* v) {
    using RA = typename AR<ACC>::R;
    using CA = cx<RA>;
    using CO = cx<typename AR<OP>::R>;
    const int r = blockIdx.y;
    const uint32_t i = blockIdx.x * kBlk + threadIdx.x;
    if (!bi_live(B.mask, r) || i >= F.vh) return;
    const double2 be = cget(B.beta, r), om = cget(B.omega, r);
    const RA br = (RA)be.x, bi = (RA)be.y, wr = (RA)om.x, wi = (RA)om.y;
    CA rr[12];
    CO pv[12], vv[12];
    uint8_t* prow = p + (size_t)r * F.fb_op;
    load_rec<ACC, 12>(rv + (size_t)r * F.fb_acc, F.vh, i, rr);
    load_rec<OP, 12>(prow, F.vh, i, pv);
    load_rec<OP, 12>(v + (size_t)r * F.fb_op, F.vh, i, vv);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        const RA vx = (RA)vv[k].x, vy = (RA)vv[k].y;
        const RA dx = (RA)pv[k].x - (wr * vx - wi * vy);
        const RA dy = (RA)pv[k].y - (wr * vy + wi * vx);
        rr[k].x += br * dx - bi * dy;
        rr[k].y += br * dy + bi * dx;
    }
    CO po[12];
    cvt12(rr, po);
    store_rec<OP, 12>(prow, F.vh, i, po);
}

// Scalar steps, one workgroup per rhs; pa, pb, pc are [nrhs][nb] partials.
//   BI_INIT:  pa = ||r||^2, pb, pc = <r^, r> -> ss, rho = <r^, r>, alpha = omega = 1
//   BI_ALPHA: pa, pb = <r^, v>     -> alpha = rho / <r^, v>
//   BI_OMEGA: pa, pb = <t, s>, pc = ||t||^2 -> omega = <t, s> / ||t||^2 (0 if t = 0)
//   BI_BETA:  pa = ||r||^2, pb, pc = <r^, r> -> ss, beta = (rho'/rho)(alpha/omega), rho = rho'
// ||r||^2 <= tol2 ||b||^2 masks the rhs off (converged, also for b = 0); a
// vanishing or non-finite denominator is a breakdown (flag, masked off).
__global__ void __launch_bounds__(kRed) k_bi_scalars(int kind, BiArgs B, int nb, const double* pa,
                                                     const double* pb, const double* pc) {
    const int r = blockIdx.x;
    const double a = reduce_row(pa + (size_t)r * nb, nb);
    const double b = pb ? reduce_row(pb + (size_t)r * nb, nb) : 0.0;
    const double c = pc ? reduce_row(pc + (size_t)r * nb, nb) : 0.0;
    if (threadIdx.x != 0) return;
    if (!bi_live(B.mask, r)) return;
    auto fail = [&]() { B.flags[r] |= 1; B.mask[r] = 0; };
    if (kind == BI_INIT) {
        cset(B.rho, r, make_double2(b, c));
        cset(B.alpha, r, make_double2(1.0, 0.0));
        cset(B.omega, r, make_double2(1.0, 0.0));
        cset(B.beta, r, make_double2(0.0, 0.0));
        B.ss[r] = a;
        if (!isfinite(a)) fail();
        else if (a <= B.tol2 * B.bb[r]) B.mask[r] = 0;      // includes b = 0
    } else if (kind == BI_ALPHA) {
        const double2 d = make_double2(a, b);
        if (!(d.x * d.x + d.y * d.y > 0.0) || !isfinite(d.x) || !isfinite(d.y)) { fail(); return; }
        cset(B.alpha, r, cdiv(cget(B.rho, r), d));
    } else if (kind == BI_OMEGA) {
        if (!isfinite(a) || !isfinite(b) || !isfinite(c)) { fail(); return; }
        cset(B.omega, r, c > 0.0 ? make_double2(a / c, b / c) : make_double2(0.0, 0.0));
    } else {
        B.ss[r] = a;
        if (isfinite(a) && a <= B.tol2 * B.bb[r]) {      // converged (or exact)
            cset(B.beta, r, make_double2(0.0, 0.0));
            B.mask[r] = 0;
            return;
        }
        const double2 rn = make_double2(b, c), rho = cget(B.rho, r), om = cget(B.omega, r);
        if (!isfinite(a) || !isfinite(b) || !isfinite(c) || !(om.x * om.x + om.y * om.y > 0.0) ||
            !(rho.x * rho.x + rho.y * rho.y > 0.0)) {
            fail();
            return;
        }
        cset(B.beta, r, cmul(cdiv(rn, rho), cdiv(cget(B.alpha, r), om)));
        cset(B.rho, r, rn);
    }
}

// ------------------------------------------------------------------ host ----
static inline Fields fields(const Geom& g, int fmt_acc, int fmt_op) {
    Fields F;
    F.vh = g.vh;
    F.fb_acc = spinor_field_bytes(g, fmt_acc);
    F.fb_op = spinor_field_bytes(g, fmt_op);
    return F;
}

uint32_t blas_blocks(const Geom& g) { return (g.vh + kBlk - 1) / kBlk; }

static inline int sp_of(int fmt) { return fmt_info(fmt).spinor_prec; }

#define WEO_SP_SWITCH(P, CALL)                                   \
    switch (P) {                                                 \
        case P_F64: { constexpr int SPV = P_F64; CALL; break; }  \
        case P_F32: { constexpr int SPV = P_F32; CALL; break; }  \
        case P_F16: { constexpr int SPV = P_F16; CALL; break; }  \
        case P_BF16: { constexpr int SPV = P_BF16; CALL; break; } \
        default: return hipErrorInvalidValue;                    \
    }

hipError_t launch_axpy2(const Geom& g, int fmt_acc, int fmt_op, int nrhs, const double* alpha,
                        const int* mask, void* x, const void* p, void* s, const void* q, void* s_op,
                        double* partial_s, hipStream_t st) {
    const Fields F = fields(g, fmt_acc, fmt_op);
    const dim3 grid(blas_blocks(g), nrhs), block(kBlk);
    auto* X = static_cast<uint8_t*>(x);
    auto* Pp = static_cast<const uint8_t*>(p);
    auto* S = static_cast<uint8_t*>(s);
    auto* Q = static_cast<const uint8_t*>(q);
    auto* SO = static_cast<uint8_t*>(s_op);
    const int pa = sp_of(fmt_acc), po = sp_of(fmt_op);
    if (pa == P_F64 && po == P_F64)
        hipLaunchKernelGGL((k_axpy2<P_F64, P_F64, false>), grid, block, 0, st, F, alpha, mask, X, Pp, S, Q, SO, partial_s);
    else if (pa == P_F32 && po == P_F32)
        hipLaunchKernelGGL((k_axpy2<P_F32, P_F32, false>), grid, block, 0, st, F, alpha, mask, X, Pp, S, Q, SO, partial_s);
    else if (pa == P_F32 && po == P_F16)
        hipLaunchKernelGGL((k_axpy2<P_F32, P_F16, true>), grid, block, 0, st, F, alpha, mask, X, Pp, S, Q, SO, partial_s);
    else if (pa == P_F32 && po == P_BF16)
        hipLaunchKernelGGL((k_axpy2<P_F32, P_BF16, true>), grid, block, 0, st, F, alpha, mask, X, Pp, S, Q, SO, partial_s);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_xpay(const Geom& g, int fmt, int nrhs, const double* beta, const int* mask,
                       const void* r, void* p, hipStream_t st) {
    const Fields F = fields(g, fmt, fmt);
    const dim3 grid(blas_blocks(g), nrhs), block(kBlk);
    auto* R = static_cast<const uint8_t*>(r);
    auto* Pp = static_cast<uint8_t*>(p);
    WEO_SP_SWITCH(sp_of(fmt), hipLaunchKernelGGL((k_xpay<SPV>), grid, block, 0, st, F, beta, mask, R, Pp))
    return hipGetLastError();
}

hipError_t launch_axpby(const Geom& g, int fmt, int nrhs, double ca, const void* a, double cb,
                        const void* b, void* out, double* partial, hipStream_t st) {
    const Fields F = fields(g, fmt, fmt);
    const dim3 grid(blas_blocks(g), nrhs), block(kBlk);
    auto* A = static_cast<const uint8_t*>(a);
    auto* B = static_cast<const uint8_t*>(b);
    auto* O = static_cast<uint8_t*>(out);
    WEO_SP_SWITCH(sp_of(fmt), hipLaunchKernelGGL((k_axpby<SPV>), grid, block, 0, st, F, ca, A, cb, B, O, partial))
    return hipGetLastError();
}

hipError_t launch_norm2(const Geom& g, int fmt, const void* a, int nrhs, double* partial, hipStream_t st) {
    const Fields F = fields(g, fmt, fmt);
    const dim3 grid(blas_blocks(g), nrhs), block(kBlk);
    auto* A = static_cast<const uint8_t*>(a);
    WEO_SP_SWITCH(sp_of(fmt), hipLaunchKernelGGL((k_norm2<SPV>), grid, block, 0, st, F, A, partial))
    return hipGetLastError();
}

template <int PI>
static hipError_t convert_to(const Geom& g, int po, size_t fbi, size_t fbo, const uint8_t* in, uint8_t* out,
                             int nrhs, const double* scale, int accumulate, hipStream_t st) {
    const dim3 grid(blas_blocks(g), nrhs), block(kBlk);
#define WEO_CVT(PO)                                                                                  \
    if (accumulate)                                                                                   \
        hipLaunchKernelGGL((k_convert<PI, PO, true>), grid, block, 0, st, g.vh, fbi, fbo, in, out, scale); \
    else                                                                                              \
        hipLaunchKernelGGL((k_convert<PI, PO, false>), grid, block, 0, st, g.vh, fbi, fbo, in, out, scale);
    switch (po) {
        case P_F64: WEO_CVT(P_F64) break;
        case P_F32: WEO_CVT(P_F32) break;
        case P_F16: WEO_CVT(P_F16) break;
        case P_BF16: WEO_CVT(P_BF16) break;
        default: return hipErrorInvalidValue;
    }
#undef WEO_CVT
    return hipGetLastError();
}

hipError_t launch_convert(const Geom& g, int fmt_in, const void* in, int fmt_out, void* out, int nrhs,
                          const double* scale, int accumulate, hipStream_t st) {
    const size_t fbi = spinor_field_bytes(g, fmt_in), fbo = spinor_field_bytes(g, fmt_out);
    auto* I = static_cast<const uint8_t*>(in);
    auto* O = static_cast<uint8_t*>(out);
    const int po = sp_of(fmt_out);
    switch (sp_of(fmt_in)) {
        case P_F64: return convert_to<P_F64>(g, po, fbi, fbo, I, O, nrhs, scale, accumulate, st);
        case P_F32: return convert_to<P_F32>(g, po, fbi, fbo, I, O, nrhs, scale, accumulate, st);
        case P_F16: return convert_to<P_F16>(g, po, fbi, fbo, I, O, nrhs, scale, accumulate, st);
        case P_BF16: return convert_to<P_BF16>(g, po, fbi, fbo, I, O, nrhs, scale, accumulate, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t st) {
    // bytes is a multiple of 16 for every buffer the library clears
    const size_t n16 = bytes / 16;
    if (n16 == 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)((n16 + 255) / 256)), dim3(256), 0, st,
                       static_cast<uint4*>(p), n16);
    return hipGetLastError();
}

hipError_t launch_reduce(const double* partial, int nblocks, int nrhs, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce, dim3(nrhs), dim3(kRed), 0, st, partial, nblocks, out);
    return hipGetLastError();
}

hipError_t launch_scalars(int kind, const ScalarArgsHost& h, hipStream_t st) {
    ScalarArgs A;
    A.nrhs = h.nrhs; A.nba = h.nba; A.nbb = h.nbb; A.pa = h.pa; A.pb = h.pb;
    A.gamma = h.gamma; A.alpha = h.alpha; A.beta = h.beta; A.ss = h.ss;
    A.mask = h.mask; A.flags = h.flags; A.target = h.target;
    A.sc_in = h.sc_in; A.sc_out = h.sc_out; A.nrm = h.nrm;
    A.bb = h.bb; A.tol2 = h.tol2;
    hipLaunchKernelGGL(k_scalars, dim3(h.nrhs), dim3(kRed), 0, st, kind, A);
    return hipGetLastError();
}

}  // namespace weo

namespace weo {

static BiArgs bi_args(const BiScalHost& h) {
    BiArgs B;
    B.rho = h.rho; B.alpha = h.alpha; B.omega = h.omega; B.beta = h.beta;
    B.ss = h.ss; B.bb = h.bb; B.tol2 = h.tol2; B.mask = h.mask; B.flags = h.flags;
    return B;
}

// Dispatch over the (acc, op) storage pairs the solvers use.
#define WEO_BI_PAIRS(ACCP, OPP, CALL)                                                         \
    if (ACCP == P_F64 && OPP == P_F64) { constexpr int A_ = P_F64, O_ = P_F64; CALL; }        \
    else if (ACCP == P_F32 && OPP == P_F32) { constexpr int A_ = P_F32, O_ = P_F32; CALL; }   \
    else if (ACCP == P_F32 && OPP == P_F16) { constexpr int A_ = P_F32, O_ = P_F16; CALL; }   \
    else if (ACCP == P_F32 && OPP == P_BF16) { constexpr int A_ = P_F32, O_ = P_BF16; CALL; } \
    else return hipErrorInvalidValue;

template <int PA>
static hipError_t bi_cdot_b(int pb, const Fields& F, dim3 grid, const int* mask, const uint8_t* A,
                            const uint8_t* Bv, double* pre, double* pim, hipStream_t st) {
    const dim3 block(kBlk);
    WEO_SP_SWITCH(pb, hipLaunchKernelGGL((k_bi_cdot<PA, SPV>), grid, block, 0, st, F, mask, A, Bv, pre, pim))
    return hipGetLastError();
}

hipError_t launch_bi_cdot(const Geom& g, int fmt_a, int fmt_b, int nrhs, const int* mask, const void* a,
                          const void* b, double* pre, double* pim, hipStream_t st) {
    const Fields F = fields(g, fmt_a, fmt_b);
    const dim3 grid(blas_blocks(g), nrhs);
    auto* A = static_cast<const uint8_t*>(a);
    auto* Bv = static_cast<const uint8_t*>(b);
    const int pb = sp_of(fmt_b);
    WEO_SP_SWITCH(sp_of(fmt_a), return bi_cdot_b<SPV>(pb, F, grid, mask, A, Bv, pre, pim, st))
    return hipSuccess;
}

hipError_t launch_bi_s(const Geom& g, int fmt_acc, int fmt_op, int nrhs, const BiScalHost& h, const void* r,
                       const void* v, void* s, void* s_op, double* partial, hipStream_t st) {
    const Fields F = fields(g, fmt_acc, fmt_op);
    const dim3 grid(blas_blocks(g), nrhs), block(kBlk);
    const BiArgs B = bi_args(h);
    auto* R = static_cast<const uint8_t*>(r);
    auto* V = static_cast<const uint8_t*>(v);
    auto* S = static_cast<uint8_t*>(s);
    auto* SO = static_cast<uint8_t*>(s_op);
    const bool sop = sp_of(fmt_acc) != sp_of(fmt_op);
    WEO_BI_PAIRS(sp_of(fmt_acc), sp_of(fmt_op),
                 if (sop) hipLaunchKernelGGL((k_bi_s<A_, O_, true>), grid, block, 0, st, F, B, R, V, S, SO, partial);
                 else hipLaunchKernelGGL((k_bi_s<A_, O_, false>), grid, block, 0, st, F, B, R, V, S, SO, partial))
    return hipGetLastError();
}

hipError_t launch_bi_init(const Geom& g, int fmt_acc, int fmt_op, int nrhs, const int* mask, const void* r,
                          void* rh, void* p, double* prr, double* pre, double* pim, hipStream_t st) {
    const Fields F = fields(g, fmt_acc, fmt_op);
    const dim3 grid(blas_blocks(g), nrhs), block(kBlk);
    auto* R = static_cast<const uint8_t*>(r);
    auto* RH = static_cast<uint8_t*>(rh);
    auto* Pp = static_cast<uint8_t*>(p);
    WEO_BI_PAIRS(sp_of(fmt_acc), sp_of(fmt_op),
                 hipLaunchKernelGGL((k_bi_init<A_, O_>), grid, block, 0, st, F, mask, R, RH, Pp, prr, pre, pim))
    return hipGetLastError();
}

hipError_t launch_bi_ts(const Geom& g, int fmt_acc, int fmt_op, int nrhs, const int* mask, const void* t,
                        const void* s, double* pre, double* pim, double* ptt, hipStream_t st) {
    const Fields F = fields(g, fmt_acc, fmt_op);
    const dim3 grid(blas_blocks(g), nrhs), block(kBlk);
    auto* T = static_cast<const uint8_t*>(t);
    auto* S = static_cast<const uint8_t*>(s);
    WEO_BI_PAIRS(sp_of(fmt_acc), sp_of(fmt_op),
                 hipLaunchKernelGGL((k_bi_ts<A_, O_>), grid, block, 0, st, F, mask, T, S, pre, pim, ptt))
    return hipGetLastError();
}

hipError_t launch_bi_xr(const Geom& g, int fmt_acc, int fmt_op, int nrhs, const BiScalHost& h, void* x,
                        const void* p, const void* s, const void* t, void* r, const void* rh, double* prr,
                        double* pre, double* pim, hipStream_t st) {
    const Fields F = fields(g, fmt_acc, fmt_op);
    const dim3 grid(blas_blocks(g), nrhs), block(kBlk);
    const BiArgs B = bi_args(h);
    auto* X = static_cast<uint8_t*>(x);
    auto* Pp = static_cast<const uint8_t*>(p);
    auto* S = static_cast<const uint8_t*>(s);
    auto* T = static_cast<const uint8_t*>(t);
    auto* R = static_cast<uint8_t*>(r);
    auto* RH = static_cast<const uint8_t*>(rh);
    WEO_BI_PAIRS(sp_of(fmt_acc), sp_of(fmt_op),
                 hipLaunchKernelGGL((k_bi_xr<A_, O_>), grid, block, 0, st, F, B, X, Pp, S, T, R, RH, prr, pre, pim))
    return hipGetLastError();
}

hipError_t launch_bi_p(const Geom& g, int fmt_acc, int fmt_op, int nrhs, const BiScalHost& h, const void* r,
                       void* p, const void* v, hipStream_t st) {
    const Fields F = fields(g, fmt_acc, fmt_op);
    const dim3 grid(blas_blocks(g), nrhs), block(kBlk);
    const BiArgs B = bi_args(h);
    auto* R = static_cast<const uint8_t*>(r);
    auto* Pp = static_cast<uint8_t*>(p);
    auto* V = static_cast<const uint8_t*>(v);
    WEO_BI_PAIRS(sp_of(fmt_acc), sp_of(fmt_op),
                 hipLaunchKernelGGL((k_bi_p<A_, O_>), grid, block, 0, st, F, B, R, Pp, V))
    return hipGetLastError();
}
#undef WEO_BI_PAIRS

hipError_t launch_bi_scalars(int kind, const BiScalHost& h, int nb, const double* pa, const double* pb,
                             const double* pc, hipStream_t st) {
    hipLaunchKernelGGL(k_bi_scalars, dim3(h.nrhs), dim3(kRed), 0, st, kind, bi_args(h), nb, pa, pb, pc);
    return hipGetLastError();
}

}  // namespace weo
