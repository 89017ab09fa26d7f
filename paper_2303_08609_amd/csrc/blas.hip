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
    hipLaunchKernelGGL(k_scalars, dim3(h.nrhs), dim3(kRed), 0, st, kind, A);
    return hipGetLastError();
}

}  // namespace weo
