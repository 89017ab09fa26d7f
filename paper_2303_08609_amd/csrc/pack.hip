// Conversion between the canonical (interleaved complex, lexicographic) field
// layouts of the C ABI and the packed structure-of-arrays layouts the kernels
// read.  Runs once per gauge configuration / source, not in the solver loop.
//
// Canonical gauge  [4][Lt][Lz][Ly][Lx][3][3]       -> packed [mu][parity][planes][V/2]
// Canonical spinor [nrhs][Lt][Lz][Ly][Lx/2][4][3]  <-> packed [rhs][planes][V/2]
// The canonical one-parity order (x/2 fastest) is the packed half index, so
// spinor conversion is a per-site transpose.  Conversions round to nearest
// even; FP64 input bound for FP16/BF16 storage is rounded to FP32 first.
#include "weo_device.h"
#include "weo_internal.h"

namespace weo {

template <class CR> struct CanonC;
template <> struct CanonC<double> { using type = double2; };
template <> struct CanonC<float> { using type = float2; };

template <int P, class CR>
__device__ __forceinline__ cx<typename St<P>::real> narrow(const typename CanonC<CR>::type& v, double scale) {
    using R = typename St<P>::real;
    cx<R> r;
    r.x = (R)((double)v.x * scale);
    r.y = (R)((double)v.y * scale);
    return r;
}

// One thread per link: idx in [0, 4V).
template <int LP, bool L12, class CR>
__global__ void __launch_bounds__(256) k_pack_gauge(Geom g, const typename CanonC<CR>::type* __restrict__ canon,
                                                    uint8_t* __restrict__ packed, size_t block_bytes) {
    const uint64_t v = (uint64_t)g.vh * 2;
    const uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= 4 * v) return;
    const int mu = (int)(idx / v);
    const uint64_t site = idx - (uint64_t)mu * v;
    const int x = (int)(site % (uint64_t)g.lx);
    uint64_t r = site / (uint64_t)g.lx;
    const int y = (int)(r % (uint64_t)g.ly); r /= (uint64_t)g.ly;
    const int z = (int)(r % (uint64_t)g.lz);
    const int t = (int)(r / (uint64_t)g.lz);
    const int par = (x + y + z + t) & 1;
    const uint32_t ih = (uint32_t)(x >> 1) + (uint32_t)g.lxh * ((uint32_t)y + (uint32_t)g.ly * ((uint32_t)z + (uint32_t)g.lz * (uint32_t)t));
    constexpr int NC = L12 ? 6 : 9;
    cx<typename St<LP>::real> w[9];
#pragma unroll
    for (int k = 0; k < NC; ++k) w[k] = narrow<LP, CR>(canon[idx * 9 + k], 1.0);
    store_rec<LP, NC>(packed + (size_t)(2 * mu + par) * block_bytes, g.vh, ih, w);
}

// One thread per (rhs, site).
template <int SP, class CR>
__global__ void __launch_bounds__(256) k_pack_spinor(Geom g, int nrhs, const typename CanonC<CR>::type* __restrict__ canon,
                                                     double scale, uint8_t* __restrict__ packed, size_t field_bytes) {
    const uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (uint64_t)nrhs * g.vh) return;
    const uint32_t r = (uint32_t)(idx / g.vh), ih = (uint32_t)(idx - (uint64_t)r * g.vh);
    cx<typename St<SP>::real> w[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) w[k] = narrow<SP, CR>(canon[idx * 12 + k], scale);
    store_rec<SP, 12>(packed + (size_t)r * field_bytes, g.vh, ih, w);
}

template <int SP, class CR>
__global__ void __launch_bounds__(256) k_unpack_spinor(Geom g, int nrhs, const uint8_t* __restrict__ packed,
                                                       size_t field_bytes, double scale,
                                                       typename CanonC<CR>::type* __restrict__ canon) {
    const uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (uint64_t)nrhs * g.vh) return;
    const uint32_t r = (uint32_t)(idx / g.vh), ih = (uint32_t)(idx - (uint64_t)r * g.vh);
    cx<typename St<SP>::real> w[12];
    load_rec<SP, 12>(packed + (size_t)r * field_bytes, g.vh, ih, w);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        typename CanonC<CR>::type o;
        o.x = (CR)((double)w[k].x * scale);
        o.y = (CR)((double)w[k].y * scale);
        canon[idx * 12 + k] = o;
    }
}

static inline dim3 grid_for(uint64_t n) { return dim3((unsigned)((n + 255) / 256)); }

template <class CR>
static hipError_t pack_gauge_t(const Geom& g, int fmt, const void* canon, void* packed, hipStream_t s) {
    const auto* c = static_cast<const typename CanonC<CR>::type*>(canon);
    auto* p = static_cast<uint8_t*>(packed);
    const size_t bb = gauge_block_bytes(g, fmt);
    const dim3 grid = grid_for((uint64_t)g.vh * 8), block(256);
    switch (fmt) {
        case FMT_D_D_18: hipLaunchKernelGGL((k_pack_gauge<P_F64, false, CR>), grid, block, 0, s, g, c, p, bb); break;
        case FMT_D_D_12: hipLaunchKernelGGL((k_pack_gauge<P_F64, true, CR>), grid, block, 0, s, g, c, p, bb); break;
        case FMT_S_S_18: hipLaunchKernelGGL((k_pack_gauge<P_F32, false, CR>), grid, block, 0, s, g, c, p, bb); break;
        case FMT_S_S_12: hipLaunchKernelGGL((k_pack_gauge<P_F32, true, CR>), grid, block, 0, s, g, c, p, bb); break;
        case FMT_H_H_18: case FMT_B_H_18:
            hipLaunchKernelGGL((k_pack_gauge<P_F16, false, CR>), grid, block, 0, s, g, c, p, bb); break;
        case FMT_H_H_12: case FMT_B_H_12:
            hipLaunchKernelGGL((k_pack_gauge<P_F16, true, CR>), grid, block, 0, s, g, c, p, bb); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_pack_gauge(const Geom& g, int fmt, const void* canon, int canon_f64, void* packed,
                             hipStream_t s) {
    return canon_f64 ? pack_gauge_t<double>(g, fmt, canon, packed, s)
                     : pack_gauge_t<float>(g, fmt, canon, packed, s);
}

template <class CR>
static hipError_t pack_spinor_t(const Geom& g, int fmt, int nrhs, const void* canon, double scale,
                                void* packed, hipStream_t s) {
    const auto* c = static_cast<const typename CanonC<CR>::type*>(canon);
    auto* p = static_cast<uint8_t*>(packed);
    const size_t fb = spinor_field_bytes(g, fmt);
    const dim3 grid = grid_for((uint64_t)g.vh * nrhs), block(256);
    switch (fmt_info(fmt).spinor_prec) {
        case P_F64: hipLaunchKernelGGL((k_pack_spinor<P_F64, CR>), grid, block, 0, s, g, nrhs, c, scale, p, fb); break;
        case P_F32: hipLaunchKernelGGL((k_pack_spinor<P_F32, CR>), grid, block, 0, s, g, nrhs, c, scale, p, fb); break;
        case P_F16: hipLaunchKernelGGL((k_pack_spinor<P_F16, CR>), grid, block, 0, s, g, nrhs, c, scale, p, fb); break;
        case P_BF16: hipLaunchKernelGGL((k_pack_spinor<P_BF16, CR>), grid, block, 0, s, g, nrhs, c, scale, p, fb); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_pack_spinor(const Geom& g, int fmt, int nrhs, const void* canon, int canon_f64,
                              double scale, void* packed, hipStream_t s) {
    return canon_f64 ? pack_spinor_t<double>(g, fmt, nrhs, canon, scale, packed, s)
                     : pack_spinor_t<float>(g, fmt, nrhs, canon, scale, packed, s);
}

template <class CR>
static hipError_t unpack_spinor_t(const Geom& g, int fmt, int nrhs, const void* packed, double scale,
                                  void* canon, hipStream_t s) {
    auto* c = static_cast<typename CanonC<CR>::type*>(canon);
    const auto* p = static_cast<const uint8_t*>(packed);
    const size_t fb = spinor_field_bytes(g, fmt);
    const dim3 grid = grid_for((uint64_t)g.vh * nrhs), block(256);
    switch (fmt_info(fmt).spinor_prec) {
        case P_F64: hipLaunchKernelGGL((k_unpack_spinor<P_F64, CR>), grid, block, 0, s, g, nrhs, p, fb, scale, c); break;
        case P_F32: hipLaunchKernelGGL((k_unpack_spinor<P_F32, CR>), grid, block, 0, s, g, nrhs, p, fb, scale, c); break;
        case P_F16: hipLaunchKernelGGL((k_unpack_spinor<P_F16, CR>), grid, block, 0, s, g, nrhs, p, fb, scale, c); break;
        case P_BF16: hipLaunchKernelGGL((k_unpack_spinor<P_BF16, CR>), grid, block, 0, s, g, nrhs, p, fb, scale, c); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_unpack_spinor(const Geom& g, int fmt, int nrhs, const void* packed, double scale,
                                void* canon, int canon_f64, hipStream_t s) {
    return canon_f64 ? unpack_spinor_t<double>(g, fmt, nrhs, packed, scale, canon, s)
                     : unpack_spinor_t<float>(g, fmt, nrhs, packed, scale, canon, s);
}

}  // namespace weo
