// Clover-type site blocks: packing (optionally inverting, in FP64) and the
// site-local product out = y + alpha A in on one parity (paper Sec. 2,
// Eqs. (3)-(5) with site-local D_ee, D_oo).  The block layout and the chiral
// basis are described in clover_core.h.
#include "clover_core.h"
#include "hop_core.h"

namespace weo {

// Canonical blocks (complex, [Lt][Lz][Ly][Lx][2][6][6]) -> packed records.
// One lane per (site, block).  The block is read as Hermitian: its lower
// triangle and the real parts of its diagonal.  With INV the packed record
// holds its inverse, by Gauss-Jordan elimination with partial pivoting in
// FP64 (a singular block gives non-finite entries).
template <int CP, bool CANON_F64, bool INV>
__global__ void __launch_bounds__(64) k_pack_clover(Geom g, const void* canon, uint8_t* packed,
                                                    size_t block_bytes) {
    const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t v = 2ull * g.vh;
    if (gid >= 2 * v) return;
    const uint64_t site = gid >> 1;
    const int blk = (int)(gid & 1);
    // lexicographic site -> coordinates, parity, half index
    const uint32_t x = (uint32_t)(site % (uint64_t)g.lx);
    const uint64_t r1 = site / (uint64_t)g.lx;
    const uint32_t y = (uint32_t)(r1 % (uint64_t)g.ly);
    const uint64_t r2 = r1 / (uint64_t)g.ly;
    const uint32_t z = (uint32_t)(r2 % (uint64_t)g.lz);
    const uint32_t t = (uint32_t)(r2 / (uint64_t)g.lz);
    const int par = (int)((x + y + z + t) & 1u);
    const uint32_t ih = (x >> 1) + (uint32_t)g.sy * y + (uint32_t)g.sz * z + (uint32_t)g.st * t;

    double m[6][6][2];
    const uint64_t off = (site * 2 + (uint64_t)blk) * 36;
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            double re, im;
            if constexpr (CANON_F64) {
                const double* c = static_cast<const double*>(canon) + 2 * (off + 6 * i + j);
                re = c[0]; im = c[1];
            } else {
                const float* c = static_cast<const float*>(canon) + 2 * (off + 6 * i + j);
                re = c[0]; im = c[1];
            }
            if (i == j) im = 0.0;
            m[i][j][0] = re; m[i][j][1] = im;
            m[j][i][0] = re; m[j][i][1] = -im;
        }
    if constexpr (INV) {
        double a[6][12][2];
        for (int i = 0; i < 6; ++i)
            for (int j = 0; j < 12; ++j) {
                a[i][j][0] = j < 6 ? m[i][j][0] : (j - 6 == i ? 1.0 : 0.0);
                a[i][j][1] = j < 6 ? m[i][j][1] : 0.0;
            }
        for (int c = 0; c < 6; ++c) {
            int pr = c;
            double best = a[c][c][0] * a[c][c][0] + a[c][c][1] * a[c][c][1];
            for (int r = c + 1; r < 6; ++r) {
                const double w = a[r][c][0] * a[r][c][0] + a[r][c][1] * a[r][c][1];
                if (w > best) { best = w; pr = r; }
            }
            if (pr != c)
                for (int j = 0; j < 12; ++j) {
                    const double t0 = a[c][j][0], t1 = a[c][j][1];
                    a[c][j][0] = a[pr][j][0]; a[c][j][1] = a[pr][j][1];
                    a[pr][j][0] = t0; a[pr][j][1] = t1;
                }
            // row c /= pivot
            const double pr0 = a[c][c][0], pi0 = a[c][c][1];
            const double den = pr0 * pr0 + pi0 * pi0;
            const double ir = pr0 / den, ii = -pi0 / den;
            for (int j = 0; j < 12; ++j) {
                const double xr = a[c][j][0], xi = a[c][j][1];
                a[c][j][0] = xr * ir - xi * ii;
                a[c][j][1] = xr * ii + xi * ir;
            }
            for (int r = 0; r < 6; ++r) {
                if (r == c) continue;
                const double fr = a[r][c][0], fi = a[r][c][1];
                for (int j = 0; j < 12; ++j) {
                    a[r][j][0] -= fr * a[c][j][0] - fi * a[c][j][1];
                    a[r][j][1] -= fr * a[c][j][1] + fi * a[c][j][0];
                }
            }
        }
        for (int i = 0; i < 6; ++i)
            for (int j = 0; j < 6; ++j) { m[i][j][0] = a[i][6 + j][0]; m[i][j][1] = a[i][6 + j][1]; }
    }
    // pack: diagonal pairs, then the lower triangle row by row
    using CR = typename St<CP>::real;
    cx<CR> rec[kCloverSlots];
#pragma unroll
    for (int k = 0; k < 3; ++k) { rec[k].x = (CR)m[2 * k][2 * k][0]; rec[k].y = (CR)m[2 * k + 1][2 * k + 1][0]; }
    int k = 3;
#pragma unroll
    for (int i = 1; i < 6; ++i)
#pragma unroll
        for (int j = 0; j < i; ++j, ++k) { rec[k].x = (CR)m[i][j][0]; rec[k].y = (CR)m[i][j][1]; }
    store_rec<CP, kCloverSlots>(packed + (size_t)(2 * par + blk) * block_bytes, g.vh, ih, rec);
}

// out = y + alpha A_p in   (y == nullptr: out = A_p in), one parity, nrhs fields
template <int SP, int CP, bool AXPY>
__global__ void __launch_bounds__(256) k_clover_site(uint32_t vh, size_t spinor_bytes, const uint8_t* clv,
                                                     size_t block_bytes, const uint8_t* in, const uint8_t* y,
                                                     double alpha, uint8_t* out) {
    using R = typename Arith<SP>::R;
    using C = cx<R>;
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= vh) return;
    const size_t off = (size_t)blockIdx.y * spinor_bytes;
    C v[12];
    load_rec<SP, 12>(in + off, vh, i, v);
    clover_apply_site<CP>(clv, block_bytes, vh, i, v);
    if constexpr (AXPY) {
        C yv[12];
        load_rec<SP, 12>(y + off, vh, i, yv);
        const R a = (R)alpha;
#pragma unroll
        for (int k = 0; k < 12; ++k) { v[k].x = fma(a, v[k].x, yv[k].x); v[k].y = fma(a, v[k].y, yv[k].y); }
    }
    store_rec<SP, 12>(out + off, vh, i, v);
}

// ------------------------------------------------------------------ host ----
size_t clover_block_bytes(const Geom& g, int fmt) {
    const int cb = fmt_info(fmt).link_bytes / (fmt_info(fmt).link12 ? 6 : 9);   // bytes per complex
    return (size_t)g.vh * (size_t)(kCloverSlots * cb);
}
size_t clover_field_bytes(const Geom& g, int fmt) { return 4 * clover_block_bytes(g, fmt); }

template <int CP>
static hipError_t pack_clover_cp(const Geom& g, int fmt, const void* canon, int canon_f64, int invert,
                                 void* packed, hipStream_t s) {
    const uint64_t n = 4ull * g.vh;                 // sites x blocks
    const dim3 block(64), grid((unsigned)((n + 63) / 64));
    auto* P = static_cast<uint8_t*>(packed);
    const size_t bb = clover_block_bytes(g, fmt);
    if (canon_f64) {
        if (invert) hipLaunchKernelGGL((k_pack_clover<CP, true, true>), grid, block, 0, s, g, canon, P, bb);
        else hipLaunchKernelGGL((k_pack_clover<CP, true, false>), grid, block, 0, s, g, canon, P, bb);
    } else {
        if (invert) hipLaunchKernelGGL((k_pack_clover<CP, false, true>), grid, block, 0, s, g, canon, P, bb);
        else hipLaunchKernelGGL((k_pack_clover<CP, false, false>), grid, block, 0, s, g, canon, P, bb);
    }
    return hipGetLastError();
}

hipError_t launch_pack_clover(const Geom& g, int fmt, const void* canon, int canon_f64, int invert, void* packed,
                              hipStream_t s) {
    switch (fmt_info(fmt).link_prec) {
        case P_F64: return pack_clover_cp<P_F64>(g, fmt, canon, canon_f64, invert, packed, s);
        case P_F32: return pack_clover_cp<P_F32>(g, fmt, canon, canon_f64, invert, packed, s);
        case P_F16: return pack_clover_cp<P_F16>(g, fmt, canon, canon_f64, invert, packed, s);
        default: return hipErrorInvalidValue;
    }
}

template <int SP, int CP>
static hipError_t site_fmt(const Geom& g, int fmt, int parity, const void* clv, const void* in, const void* y,
                           double alpha, void* out, int nrhs, hipStream_t s) {
    const dim3 block(256), grid((g.vh + 255) / 256, nrhs);
    const size_t bb = clover_block_bytes(g, fmt);
    const uint8_t* C = static_cast<const uint8_t*>(clv) + (size_t)(2 * parity) * bb;
    const size_t sb = spinor_field_bytes(g, fmt);
    auto* I = static_cast<const uint8_t*>(in);
    auto* Y = static_cast<const uint8_t*>(y);
    auto* O = static_cast<uint8_t*>(out);
    if (y) hipLaunchKernelGGL((k_clover_site<SP, CP, true>), grid, block, 0, s, g.vh, sb, C, bb, I, Y, alpha, O);
    else hipLaunchKernelGGL((k_clover_site<SP, CP, false>), grid, block, 0, s, g.vh, sb, C, bb, I, Y, alpha, O);
    return hipGetLastError();
}

hipError_t launch_clover_site(const Geom& g, int fmt, int parity, const void* clv, const void* in, const void* y,
                              double alpha, void* out, int nrhs, hipStream_t s) {
    switch (fmt) {
        case FMT_D_D_18: case FMT_D_D_12: return site_fmt<P_F64, P_F64>(g, fmt, parity, clv, in, y, alpha, out, nrhs, s);
        case FMT_S_S_18: case FMT_S_S_12: return site_fmt<P_F32, P_F32>(g, fmt, parity, clv, in, y, alpha, out, nrhs, s);
        case FMT_H_H_18: case FMT_H_H_12: return site_fmt<P_F16, P_F16>(g, fmt, parity, clv, in, y, alpha, out, nrhs, s);
        case FMT_B_H_18: case FMT_B_H_12: return site_fmt<P_BF16, P_F16>(g, fmt, parity, clv, in, y, alpha, out, nrhs, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace weo
