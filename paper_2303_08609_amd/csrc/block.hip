// Block kernels of block CG (several right-hand sides sharing one Krylov
// space): the Gram matrix G = A^H B of two blocks of s fields, and the block
// update out = in0 + a (in1 T) with an s x s complex matrix T.
//
// A packed spinor field of one parity is a flat array of 16-byte chunks
// (its records are whole 16-byte planes): two FP32 complex numbers or one
// FP64 complex per chunk.  Inner products and linear combinations of fields
// act chunk by chunk, so these kernels never look at sites.
//
// Gram: one wavefront per workgroup.  Each pass stages 64 consecutive chunks
// of every column of A and B in LDS; the lanes then split the s x s result
// into 4 x 4 cells and the 64 chunks among groups of lanes, accumulating in
// FP64.  Each workgroup writes one partial matrix; a second kernel sums the
// partials in a fixed order (deterministic).
#include <algorithm>

#include "weo_device.h"
#include "weo_internal.h"

namespace weo {

static constexpr int kGramWG = 1024;      // workgroups of the Gram kernel (max)
static constexpr int kUpdBlk = 256;       // lanes per workgroup of the update
static constexpr int kUpdWG = 2048;       // workgroups of the update (max)
static constexpr int kLdsPad = 65;        // row stride in chunks (bank spread)

template <int SP> struct Chunk;
template <> struct Chunk<P_F32> {
    using R = float;
    static constexpr int N = 2;           // complex numbers per chunk
    __device__ static void unpack(const uint4& w, cx<R>* v) {
        v[0].x = __uint_as_float(w.x); v[0].y = __uint_as_float(w.y);
        v[1].x = __uint_as_float(w.z); v[1].y = __uint_as_float(w.w);
    }
    __device__ static uint4 pack(const cx<R>* v) {
        return make_uint4(__float_as_uint(v[0].x), __float_as_uint(v[0].y), __float_as_uint(v[1].x),
                          __float_as_uint(v[1].y));
    }
};
template <> struct Chunk<P_F64> {
    using R = double;
    static constexpr int N = 1;
    __device__ static void unpack(const uint4& w, cx<R>* v) {
        v[0].x = __hiloint2double((int)w.y, (int)w.x);
        v[0].y = __hiloint2double((int)w.w, (int)w.z);
    }
    __device__ static uint4 pack(const cx<R>* v) {
        const unsigned long long a = (unsigned long long)__double_as_longlong(v[0].x);
        const unsigned long long b = (unsigned long long)__double_as_longlong(v[0].y);
        return make_uint4((unsigned)a, (unsigned)(a >> 32), (unsigned)b, (unsigned)(b >> 32));
    }
};

__device__ __forceinline__ const uint4* col_ptr(const BlockRef& r, int j) {
    return reinterpret_cast<const uint4*>(r.base + (uint64_t)r.col[j] * r.stride);
}

// part[blockIdx.x][(j s + k) 2 + {re, im}] = sum over this workgroup's chunks
// of conj(a_j) b_k.  SAME: b is a (loaded once).
template <int SP, bool SAME>
__global__ void __launch_bounds__(64) k_bgram(uint64_t nch, int s, BlockRef A, BlockRef B, double* part) {
    using K = Chunk<SP>;
    using R = typename K::R;
    __shared__ uint4 la[kMaxBlock * kLdsPad];
    __shared__ uint4 lb[SAME ? 1 : kMaxBlock * kLdsPad];
    const uint4* lbp = SAME ? la : lb;
    const int lane = threadIdx.x;
    const int nb = (s + 3) >> 2, cells = nb * nb, ng = 64 / cells;
    const int grp = lane / cells, cell = lane - grp * cells;
    const int j0 = (cell / nb) * 4, k0 = (cell % nb) * 4;
    double acc[4][4][2];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b][0] = acc[a][b][1] = 0.0;

    for (uint64_t c0 = (uint64_t)blockIdx.x * 64; c0 < nch; c0 += (uint64_t)gridDim.x * 64) {
        const uint64_t ch = c0 + (uint64_t)lane;
        const bool in = ch < nch;
#pragma unroll
        for (int j = 0; j < kMaxBlock; ++j) {
            if (j < s) {
                la[j * kLdsPad + lane] = in ? col_ptr(A, j)[ch] : make_uint4(0, 0, 0, 0);
                if constexpr (!SAME) lb[j * kLdsPad + lane] = in ? col_ptr(B, j)[ch] : make_uint4(0, 0, 0, 0);
            }
        }
        __syncthreads();
        if (grp < ng) {
            for (int m = grp; m < 64; m += ng) {
                cx<R> a[4][K::N], b[4][K::N];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    K::unpack(la[(j0 + q) * kLdsPad + m], a[q]);
                    K::unpack(lbp[(k0 + q) * kLdsPad + m], b[q]);
                }
#pragma unroll
                for (int e = 0; e < K::N; ++e)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const double ax = a[q][e].x, ay = a[q][e].y;
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const double bx = b[r][e].x, by = b[r][e].y;
                            acc[q][r][0] = fma(ax, bx, fma(ay, by, acc[q][r][0]));
                            acc[q][r][1] = fma(ax, by, fma(-ay, bx, acc[q][r][1]));
                        }
                    }
            }
        }
        __syncthreads();
    }
    // sum the lane groups in order (LDS reused as doubles: 64 lanes x 32)
    double* red = reinterpret_cast<double*>(la);
    static_assert(sizeof(la) >= 64 * 32 * sizeof(double), "LDS too small for the reduction");
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            red[lane * 32 + (q * 4 + r) * 2] = acc[q][r][0];
            red[lane * 32 + (q * 4 + r) * 2 + 1] = acc[q][r][1];
        }
    __syncthreads();
    if (lane < cells) {
        double* out = part + (size_t)blockIdx.x * kGramStride;
        for (int e = 0; e < 32; ++e) {
            double v = 0.0;
            for (int gi = 0; gi < ng; ++gi) v += red[(gi * cells + lane) * 32 + e];
            const int q = (e >> 1) >> 2, r = (e >> 1) & 3;
            const int j = j0 + q, k = k0 + r;
            if (j < s && k < s) out[(j * s + k) * 2 + (e & 1)] = v;
        }
    }
}

// out[t] = sum_w part[w][t] in order, t < 2 s^2
__global__ void __launch_bounds__(512) k_bgram_reduce(const double* part, int nwg, int n, double* out) {
    const int t = threadIdx.x;
    if (t >= n) return;
    double v = 0.0;
    for (int w = 0; w < nwg; ++w) v += part[(size_t)w * kGramStride + t];
    out[t] = v;
}

// out_j = [in0_j] + a sum_k in1_k T[k][j]   (j < s), chunk by chunk.
// out may be in0 or in1 (each lane reads all its chunks before it writes).
// npart (optional): per-workgroup partials of ||out_j||^2, [j][gridDim.x].
template <int SP, bool IN0, bool NORM>
__global__ void __launch_bounds__(kUpdBlk) k_bupdate(uint64_t nch, int s, BlockRef out, BlockRef in0,
                                                       BlockRef in1, double a, const double* T, double* npart) {
    using K = Chunk<SP>;
    using R = typename K::R;
    __shared__ cx<R> t[kMaxBlock * kMaxBlock];
    for (int i = threadIdx.x; i < s * s; i += blockDim.x) {
        t[i].x = (R)(a * T[2 * i]);
        t[i].y = (R)(a * T[2 * i + 1]);
    }
    __syncthreads();
    double nrm[kMaxBlock];
#pragma unroll
    for (int j = 0; j < kMaxBlock; ++j) nrm[j] = 0.0;
    for (uint64_t ch = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; ch < nch;
         ch += (uint64_t)gridDim.x * blockDim.x) {
        cx<R> v[kMaxBlock][K::N];
#pragma unroll
        for (int k = 0; k < kMaxBlock; ++k)
            if (k < s) K::unpack(col_ptr(in1, k)[ch], v[k]);
#pragma unroll
        for (int j = 0; j < kMaxBlock; ++j) {
            if (j < s) {
                cx<R> o[K::N];
                if constexpr (IN0) {
                    K::unpack(col_ptr(in0, j)[ch], o);
                } else {
#pragma unroll
                    for (int e = 0; e < K::N; ++e) o[e].x = o[e].y = R(0);
                }
#pragma unroll
                for (int k = 0; k < kMaxBlock; ++k) {
                    if (k < s) {
                        const cx<R> tk = t[k * s + j];
#pragma unroll
                        for (int e = 0; e < K::N; ++e) o[e] = fma_(v[k][e], tk, o[e]);
                    }
                }
                *reinterpret_cast<uint4*>(out.base + (uint64_t)out.col[j] * out.stride + ch * 16) = K::pack(o);
                if constexpr (NORM) {
#pragma unroll
                    for (int e = 0; e < K::N; ++e)
                        nrm[j] += (double)o[e].x * o[e].x + (double)o[e].y * o[e].y;
                }
            }
        }
    }
    if constexpr (NORM) {
        __shared__ double wsum[kUpdBlk / 64];
#pragma unroll
        for (int j = 0; j < kMaxBlock; ++j) {
            if (j < s) {
                double v = nrm[j];
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
                if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = v;
                __syncthreads();
                if (threadIdx.x == 0) {
                    double tot = 0.0;
                    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tot += wsum[w];
                    npart[(size_t)j * gridDim.x + blockIdx.x] = tot;
                }
                __syncthreads();
            }
        }
    }
}

// ------------------------------------------------------------------ host ----
static uint64_t chunks(const Geom& g, int fmt) { return spinor_field_bytes(g, fmt) / 16; }

int block_gram_wg(const Geom& g, int fmt) {
    const uint64_t n = (chunks(g, fmt) + 63) / 64;
    return (int)(n < (uint64_t)kGramWG ? n : (uint64_t)kGramWG);
}
int block_update_wg(const Geom& g, int fmt) {
    const uint64_t n = (chunks(g, fmt) + kUpdBlk - 1) / kUpdBlk;
    return (int)(n < (uint64_t)kUpdWG ? n : (uint64_t)kUpdWG);
}

hipError_t launch_block_gram(const Geom& g, int fmt, int s, const BlockRef& a, const BlockRef& b, double* part,
                             double* out, hipStream_t st) {
    if (s < 1 || s > kMaxBlock) return hipErrorInvalidValue;
    const uint64_t n = chunks(g, fmt);
    const int wg = block_gram_wg(g, fmt);
    const bool same = a.base == b.base && a.stride == b.stride &&
                      std::equal(a.col, a.col + s, b.col);
    switch (fmt_info(fmt).spinor_prec) {
        case P_F64:
            if (same) hipLaunchKernelGGL((k_bgram<P_F64, true>), dim3(wg), dim3(64), 0, st, n, s, a, b, part);
            else hipLaunchKernelGGL((k_bgram<P_F64, false>), dim3(wg), dim3(64), 0, st, n, s, a, b, part);
            break;
        case P_F32:
            if (same) hipLaunchKernelGGL((k_bgram<P_F32, true>), dim3(wg), dim3(64), 0, st, n, s, a, b, part);
            else hipLaunchKernelGGL((k_bgram<P_F32, false>), dim3(wg), dim3(64), 0, st, n, s, a, b, part);
            break;
        default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bgram_reduce, dim3(1), dim3(512), 0, st, part, wg, 2 * s * s, out);
    return hipGetLastError();
}

template <int SP>
static void bupdate_sp(uint64_t n, int wg, int s, const BlockRef& out, const BlockRef* in0, const BlockRef& in1,
                       double a, const double* T, double* npart, hipStream_t st) {
    const BlockRef z = in0 ? *in0 : in1;
    if (in0 && npart) hipLaunchKernelGGL((k_bupdate<SP, true, true>), dim3(wg), dim3(kUpdBlk), 0, st, n, s, out, z, in1, a, T, npart);
    else if (in0) hipLaunchKernelGGL((k_bupdate<SP, true, false>), dim3(wg), dim3(kUpdBlk), 0, st, n, s, out, z, in1, a, T, npart);
    else if (npart) hipLaunchKernelGGL((k_bupdate<SP, false, true>), dim3(wg), dim3(kUpdBlk), 0, st, n, s, out, z, in1, a, T, npart);
    else hipLaunchKernelGGL((k_bupdate<SP, false, false>), dim3(wg), dim3(kUpdBlk), 0, st, n, s, out, z, in1, a, T, npart);
}

hipError_t launch_block_update(const Geom& g, int fmt, int s, const BlockRef& out, const BlockRef* in0,
                               const BlockRef& in1, double a, const double* T, double* npart, double* nrm,
                               hipStream_t st) {
    if (s < 1 || s > kMaxBlock || (nrm && !npart)) return hipErrorInvalidValue;
    const uint64_t n = chunks(g, fmt);
    const int wg = block_update_wg(g, fmt);
    double* np = nrm ? npart : nullptr;
    switch (fmt_info(fmt).spinor_prec) {
        case P_F64: bupdate_sp<P_F64>(n, wg, s, out, in0, in1, a, T, np, st); break;
        case P_F32: bupdate_sp<P_F32>(n, wg, s, out, in0, in1, a, T, np, st); break;
        default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !nrm) return e;
    return launch_reduce(npart, wg, s, nrm, st);
}

}  // namespace weo
