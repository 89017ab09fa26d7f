// Block kernels of block CG (several right-hand sides sharing one Krylov
// space): the Gram matrix G = A^H B of two blocks of s fields, and the block
// update out = in0 + a (in1 T) with an s x s complex matrix T.
//
// A packed spinor field of one parity is a flat array of 16-byte chunks
// (its records are whole 16-byte planes): two FP32 complex numbers or one
// FP64 complex per chunk.  Inner products and linear combinations of fields
// act chunk by chunk, so these kernels never look at sites.
//
// Gram matrices accumulate in FP64 (products of FP32 inputs are exact in
// FP64); every workgroup writes one partial matrix and a second kernel sums
// the partials in a fixed order (deterministic).
#include <algorithm>
#include <cstdlib>
#include <cstring>

#include "weo_device.h"
#include "weo_internal.h"

namespace weo {

static constexpr int kGramWG = 1024;      // workgroups of the Gram kernel (max; measured faster than 2048)
static constexpr int kMaxCells = 10;      // 4 x 4 cells of the upper triangle of a 16 x 16 matrix
static constexpr int kUpdBlk = 256;       // lanes per workgroup of the update kernels
static constexpr int kUpdWG = 2048;       // workgroups of the update kernels (max)

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

// Column pointers of a block with constant indices (a runtime index into the
// argument's col[] would place the argument in scratch memory).
__device__ __forceinline__ const uint4* col_sel(const BlockRef& r, int j) {
    int c = 0;
#pragma unroll
    for (int t = 0; t < kMaxBlock; ++t)
        if (t == j) c = r.col[t];
    return reinterpret_cast<const uint4*>(r.base + (uint64_t)c * r.stride);
}

// Partial Gram sums, one column of part per workgroup:
//   part[((j s + k) 2 + {re, im}) nwg + blockIdx.x] = sum of conj(a_j) b_k
// over this workgroup's chunks, for j <= k; zero below the diagonal (both
// Gram matrices of block CG are Hermitian).  The upper triangle is cut into
// 4 x 4 cells, one wavefront per cell: per step a wave streams 64 consecutive
// chunks of its 4 a columns and 4 b columns (each column is read by the
// waves of its row or column of cells; the repeats come from the L1 cache).
// SAME: b is a.
template <int SP, bool SAME>
__global__ void __launch_bounds__(64 * kMaxCells) k_bgram(uint64_t nch, int s, BlockRef A, BlockRef B,
                                                            double* part) {
    using K = Chunk<SP>;
    using R = typename K::R;
    const int nb = (s + 3) >> 2;
    const int c = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int jb = 0, rem = c;
    while (rem >= nb - jb) { rem -= nb - jb; ++jb; }
    const int j0 = 4 * jb, k0 = 4 * (jb + rem);
    // columns past s read column s - 1 (always valid memory); the entries
    // they produce are never stored
    const uint4* pa[4];
    const uint4* pb[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        pa[r] = col_sel(A, j0 + r < s ? j0 + r : s - 1);
        pb[r] = col_sel(SAME ? A : B, k0 + r < s ? k0 + r : s - 1);
    }
    double acc[4][4][2];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b][0] = acc[a][b][1] = 0.0;
    for (uint64_t ch = (uint64_t)blockIdx.x * 64 + lane; ch < nch; ch += (uint64_t)gridDim.x * 64) {
        cx<R> a[4][K::N], b[4][K::N];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            K::unpack(pa[r][ch], a[r]);
            K::unpack(pb[r][ch], b[r]);
        }
#pragma unroll
        for (int e = 0; e < K::N; ++e)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const double ax = a[r][e].x, ay = a[r][e].y;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const double bx = b[t][e].x, by = b[t][e].y;
                    acc[r][t][0] = fma(ax, bx, fma(ay, by, acc[r][t][0]));
                    acc[r][t][1] = fma(ax, by, fma(-ay, bx, acc[r][t][1]));
                }
            }
    }
    const size_t nwg = gridDim.x;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                double v = acc[r][t][q];
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
                const int j = j0 + r, k = k0 + t;
                if (lane == 0 && j < s && k < s) part[((size_t)(j * s + k) * 2 + q) * nwg + blockIdx.x] = j <= k ? v : 0.0;
            }
    // entries below the diagonal in cells off it belong to no wave
    for (int t = threadIdx.x; t < 2 * s * s; t += blockDim.x) {
        const int j = (t >> 1) / s, k = (t >> 1) % s;
        if ((j >> 2) > (k >> 2)) part[(size_t)t * nwg + blockIdx.x] = 0.0;
    }
}

// The same partial Gram sums on the FP64 matrix cores.  A block of s
// complex fields is read as a tall real matrix X with 2s <= 32 columns
// (column c < s: the real parts of field c, s <= c < 2s: the imaginary parts
// of field c - s, the rest zero) and one row per complex component; then
// R = X_A^T X_B is accumulated by v_mfma_f64_16x16x4f64 in 16 x 16 tiles, four
// rows per instruction, and
//     Re <a_j, b_k> = R[j][k] + R[s+j][s+k],  Im <a_j, b_k> = R[j][s+k] - R[s+j][k].
// Each wavefront walks every (gridDim.x x 8)-th group of four rows, the
// loads of four groups issued before their products; lane l supplies row
// l / 16 of column l % 16 (tile 0) and 16 + l % 16 (tile 1) of both
// operands, and holds rows l / 16 + 4 i (i = 0..3), column l % 16 of each
// accumulator tile.  FP32 values are exact in FP64.  SAME: b is a
// (R symmetric: three tiles).
typedef double gd4 __attribute__((ext_vector_type(4)));

template <int SP>
__device__ __forceinline__ const uint8_t* gram_col(const BlockRef& X, int s, int c, bool* live) {
    constexpr int RB = SP == P_F64 ? 8 : 4;          // bytes of one real
    *live = c < 2 * s;
    const int f = c < s ? c : (c < 2 * s ? c - s : 0);
    return reinterpret_cast<const uint8_t*>(col_sel(X, f)) + (c >= s && c < 2 * s ? RB : 0);
}

template <int SP>
__device__ __forceinline__ double gram_val(const uint8_t* p, bool live, uint64_t k, uint64_t nrows) {
    constexpr int CB = SP == P_F64 ? 16 : 8;         // bytes of one complex
    if (!live || k >= nrows) return 0.0;
    if constexpr (SP == P_F64) return *reinterpret_cast<const double*>(p + k * CB);
    else return (double)*reinterpret_cast<const float*>(p + k * CB);
}

static constexpr int kGramMfmaWaves = 8;    // wavefronts per workgroup of k_bgram_mfma
static constexpr int kGramMfmaUnroll = 4;   // row groups whose loads are issued together

template <int SP, bool SAME>
__global__ void __launch_bounds__(64 * kGramMfmaWaves) k_bgram_mfma(uint64_t nch, int s, BlockRef A, BlockRef B,
                                                                     double* part) {
    __shared__ double R[32][33];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint64_t nrows = nch * (SP == P_F64 ? 1 : 2);
    const uint64_t nsteps = (nrows + 3) / 4;
    bool la0, la1, lb0 = false, lb1 = false;
    const uint8_t* a0 = gram_col<SP>(A, s, lane & 15, &la0);
    const uint8_t* a1 = gram_col<SP>(A, s, 16 + (lane & 15), &la1);
    const uint8_t* b0 = a0;
    const uint8_t* b1 = a1;
    if constexpr (!SAME) {
        b0 = gram_col<SP>(B, s, lane & 15, &lb0);
        b1 = gram_col<SP>(B, s, 16 + (lane & 15), &lb1);
    }
    const bool two = 2 * s > 16;                     // the second column tile is needed
    gd4 d00 = {0, 0, 0, 0}, d01 = d00, d10 = d00, d11 = d00;
    const uint64_t stride = (uint64_t)gridDim.x * kGramMfmaWaves;
    for (uint64_t st = (uint64_t)blockIdx.x * kGramMfmaWaves + wv; st < nsteps; st += kGramMfmaUnroll * stride) {
        // the loads of several row groups first (each lane's value of its
        // row and columns), then their products
        double x0[kGramMfmaUnroll], y0[kGramMfmaUnroll], x1[kGramMfmaUnroll], y1[kGramMfmaUnroll];
#pragma unroll
        for (int u = 0; u < kGramMfmaUnroll; ++u) {
            const uint64_t k = 4 * (st + u * stride) + (uint64_t)(lane >> 4);
            x0[u] = gram_val<SP>(a0, la0, k, nrows);
            y0[u] = SAME ? x0[u] : gram_val<SP>(b0, lb0, k, nrows);
            x1[u] = two ? gram_val<SP>(a1, la1, k, nrows) : 0.0;
            y1[u] = SAME ? x1[u] : (two ? gram_val<SP>(b1, lb1, k, nrows) : 0.0);
        }
#pragma unroll
        for (int u = 0; u < kGramMfmaUnroll; ++u) {
            d00 = __builtin_amdgcn_mfma_f64_16x16x4f64(x0[u], y0[u], d00, 0, 0, 0);
            if (two) {
                d01 = __builtin_amdgcn_mfma_f64_16x16x4f64(x0[u], y1[u], d01, 0, 0, 0);
                if constexpr (!SAME) d10 = __builtin_amdgcn_mfma_f64_16x16x4f64(x1[u], y0[u], d10, 0, 0, 0);
                d11 = __builtin_amdgcn_mfma_f64_16x16x4f64(x1[u], y1[u], d11, 0, 0, 0);
            }
        }
    }
    // the wavefronts' tiles summed into R in wavefront order (deterministic);
    // element i of lane l is row l / 16 + 4 i, column l % 16 of its tile
    // (measured on gfx950)
    for (int t = threadIdx.x; t < 32 * 33; t += blockDim.x) (&R[0][0])[t] = 0.0;
    __syncthreads();
    const int rg = lane >> 4, cn = lane & 15;
    for (int w = 0; w < kGramMfmaWaves; ++w) {
        if (w == wv) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                R[rg + 4 * i][cn] += d00[i];
                R[rg + 4 * i][16 + cn] += d01[i];
                R[16 + rg + 4 * i][16 + cn] += d11[i];
                if constexpr (!SAME) R[16 + rg + 4 * i][cn] += d10[i];
            }
        }
        __syncthreads();
    }
    if constexpr (SAME) {
        if (wv == 0) {
#pragma unroll
            for (int i = 0; i < 4; ++i) R[16 + rg + 4 * i][cn] = R[cn][16 + rg + 4 * i];
        }
        __syncthreads();
    }
    const size_t nwg = gridDim.x;
    for (int t = threadIdx.x; t < s * s; t += blockDim.x) {
        const int j = t / s, kk = t % s;
        double re = 0.0, im = 0.0;
        if (j <= kk) {
            re = R[j][kk] + R[s + j][s + kk];
            im = R[j][s + kk] - R[s + j][kk];
        }
        part[((size_t)t * 2 + 0) * nwg + blockIdx.x] = re;
        part[((size_t)t * 2 + 1) * nwg + blockIdx.x] = im;
    }
}

// out_j = [in0_j] + a sum_k in1_k T[k][j]   (j < s), chunk by chunk: one
// lane per chunk holds the chunk of every column in registers (NB >= s, a
// multiple of 4, sizes the arrays) and reads all of them before it writes,
// so out may be in0 or in1.  npart (optional): per-workgroup partials of
// ||out_j||^2, [j][gridDim.x].
template <int SP, int NB, bool EXACT, bool IN0, bool NORM>
__global__ void __launch_bounds__(kUpdBlk) k_bupdate(uint64_t nch, int s_arg, BlockRef out, BlockRef in0,
                                                       BlockRef in1, double a, const double* T, double* npart) {
    using K = Chunk<SP>;
    using R = typename K::R;
    const int s = EXACT ? NB : s_arg;        // EXACT: the block size is NB
    __shared__ cx<R> t[NB * NB];
    for (int i = threadIdx.x; i < s * s; i += blockDim.x) {
        t[(i / s) * NB + i % s].x = (R)(a * T[2 * i]);
        t[(i / s) * NB + i % s].y = (R)(a * T[2 * i + 1]);
    }
    __syncthreads();
    double nrm[NORM ? NB : 1];
#pragma unroll
    for (int j = 0; j < (NORM ? NB : 1); ++j) nrm[j] = 0.0;
    for (uint64_t ch = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; ch < nch;
         ch += (uint64_t)gridDim.x * blockDim.x) {
        // keep the factor in LDS where hoisting it out of the loop spills or
        // measured slower (FP64, the 16-wide bucket, the norm variant)
        if constexpr (SP == P_F64 || NB > 12 || NORM) __asm__ volatile("" ::: "memory");
        cx<R> v[NB][K::N], y[IN0 ? NB : 1][K::N];
#pragma unroll
        for (int k = 0; k < NB; ++k)
            if (k < s) K::unpack(col_ptr(in1, k)[ch], v[k]);
        if constexpr (IN0) {
#pragma unroll
            for (int j = 0; j < NB; ++j)
                if (j < s) K::unpack(col_ptr(in0, j)[ch], y[j]);
        }
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            if (j < s) {
                cx<R> o[K::N];
#pragma unroll
                for (int e = 0; e < K::N; ++e) {
                    if constexpr (IN0) o[e] = y[j][e];
                    else o[e].x = o[e].y = R(0);
                }
#pragma unroll
                for (int k = 0; k < NB; ++k) {
                    if (k < s) {
                        const cx<R> tk = t[k * NB + j];
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
        for (int j = 0; j < NB; ++j) {
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

// The last step of a block CG iteration, in one pass (one lane per chunk,
// NB as for k_bupdate):
//   Q <- Q TA;   P <- Q + P TB   (the new Q)
template <int SP, int NB, bool EXACT>
__global__ void __launch_bounds__(kUpdBlk) k_bqp(uint64_t nch, int s_arg, BlockRef Q, BlockRef P, const double* TA,
                                                   const double* TB) {
    using K = Chunk<SP>;
    using R = typename K::R;
    const int s = EXACT ? NB : s_arg;
    __shared__ cx<R> ta[NB * NB], tb[NB * NB];
    for (int i = threadIdx.x; i < s * s; i += blockDim.x) {
        const int d = (i / s) * NB + i % s;
        ta[d].x = (R)TA[2 * i]; ta[d].y = (R)TA[2 * i + 1];
        tb[d].x = (R)TB[2 * i]; tb[d].y = (R)TB[2 * i + 1];
    }
    __syncthreads();
    for (uint64_t ch = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; ch < nch;
         ch += (uint64_t)gridDim.x * blockDim.x) {
        __asm__ volatile("" ::: "memory");      // the factors stay in LDS (measured faster)
        cx<R> vq[NB][K::N], vp[NB][K::N];
#pragma unroll
        for (int k = 0; k < NB; ++k)
            if (k < s) {
                K::unpack(col_ptr(Q, k)[ch], vq[k]);
                K::unpack(col_ptr(P, k)[ch], vp[k]);
            }
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            if (j < s) {
                cx<R> oq[K::N], op[K::N];
#pragma unroll
                for (int e = 0; e < K::N; ++e) oq[e].x = oq[e].y = R(0);
#pragma unroll
                for (int k = 0; k < NB; ++k)
                    if (k < s) {
                        const cx<R> t = ta[k * NB + j];
#pragma unroll
                        for (int e = 0; e < K::N; ++e) oq[e] = fma_(vq[k][e], t, oq[e]);
                    }
#pragma unroll
                for (int e = 0; e < K::N; ++e) op[e] = oq[e];
#pragma unroll
                for (int k = 0; k < NB; ++k)
                    if (k < s) {
                        const cx<R> t = tb[k * NB + j];
#pragma unroll
                        for (int e = 0; e < K::N; ++e) op[e] = fma_(vp[k][e], t, op[e]);
                    }
                *reinterpret_cast<uint4*>(Q.base + (uint64_t)Q.col[j] * Q.stride + ch * 16) = K::pack(oq);
                *reinterpret_cast<uint4*>(P.base + (uint64_t)P.col[j] * P.stride + ch * 16) = K::pack(op);
            }
        }
    }
}

// ------------------------------------------------------------------ host ----
static uint64_t chunks(const Geom& g, int fmt) { return spinor_field_bytes(g, fmt) / 16; }

// Gram matrices by the cell kernel on the vector units (k_bgram), or with
// WEO_GRAM=mfma on the FP64 matrix cores (k_bgram_mfma); read per call.  The
// cell kernel is the default: at 32^3x64 with 12 FP32 fields it takes 409 us
// (Q^H Q) and 472 us (P^H W) against 878 us and 1743 us on the matrix cores,
// whose operands arrive as scattered 4-byte loads.
static bool gram_on_matrix_cores() {
    const char* e = getenv("WEO_GRAM");
    return e && strcmp(e, "mfma") == 0;
}

int block_gram_wg(const Geom& g, int fmt) {          // 64 chunks per workgroup and step
    const uint64_t n = (chunks(g, fmt) + 63) / 64;
    return (int)(n < (uint64_t)kGramWG ? n : (uint64_t)kGramWG);
}
int block_update_wg(const Geom& g, int fmt) {        // one chunk per lane and step
    const uint64_t n = (chunks(g, fmt) + kUpdBlk - 1) / kUpdBlk;
    return (int)(n < (uint64_t)kUpdWG ? n : (uint64_t)kUpdWG);
}

hipError_t launch_block_gram(const Geom& g, int fmt, int s, const BlockRef& a, const BlockRef& b, double* part,
                             double* out, hipStream_t st) {
    if (s < 1 || s > kMaxBlock) return hipErrorInvalidValue;
    const uint64_t n = chunks(g, fmt);
    const int wg = block_gram_wg(g, fmt);
    const bool same = a.base == b.base && a.stride == b.stride && std::equal(a.col, a.col + s, b.col);
    if (gram_on_matrix_cores()) {
        const dim3 grid(wg), block(64 * kGramMfmaWaves);
        switch (fmt_info(fmt).spinor_prec) {
            case P_F64:
                if (same) hipLaunchKernelGGL((k_bgram_mfma<P_F64, true>), grid, block, 0, st, n, s, a, b, part);
                else hipLaunchKernelGGL((k_bgram_mfma<P_F64, false>), grid, block, 0, st, n, s, a, b, part);
                break;
            case P_F32:
                if (same) hipLaunchKernelGGL((k_bgram_mfma<P_F32, true>), grid, block, 0, st, n, s, a, b, part);
                else hipLaunchKernelGGL((k_bgram_mfma<P_F32, false>), grid, block, 0, st, n, s, a, b, part);
                break;
            default: return hipErrorInvalidValue;
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        return launch_reduce(part, wg, 2 * s * s, out, st);
    }
    const int nb = (s + 3) / 4;
    const dim3 grid(wg), block(64 * nb * (nb + 1) / 2);
    switch (fmt_info(fmt).spinor_prec) {
        case P_F64:
            if (same) hipLaunchKernelGGL((k_bgram<P_F64, true>), grid, block, 0, st, n, s, a, b, part);
            else hipLaunchKernelGGL((k_bgram<P_F64, false>), grid, block, 0, st, n, s, a, b, part);
            break;
        case P_F32:
            if (same) hipLaunchKernelGGL((k_bgram<P_F32, true>), grid, block, 0, st, n, s, a, b, part);
            else hipLaunchKernelGGL((k_bgram<P_F32, false>), grid, block, 0, st, n, s, a, b, part);
            break;
        default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_reduce(part, wg, 2 * s * s, out, st);
}

template <int SP, int NB, bool EX>
static void bupdate_ex(uint64_t n, int wg, int s, const BlockRef& out, const BlockRef* in0, const BlockRef& in1,
                       double a, const double* T, double* npart, hipStream_t st) {
    const BlockRef z = in0 ? *in0 : in1;
    const dim3 grid(wg), block(kUpdBlk);
    if (in0 && npart) hipLaunchKernelGGL((k_bupdate<SP, NB, EX, true, true>), grid, block, 0, st, n, s, out, z, in1, a, T, npart);
    else if (in0) hipLaunchKernelGGL((k_bupdate<SP, NB, EX, true, false>), grid, block, 0, st, n, s, out, z, in1, a, T, npart);
    else if (npart) hipLaunchKernelGGL((k_bupdate<SP, NB, EX, false, true>), grid, block, 0, st, n, s, out, z, in1, a, T, npart);
    else hipLaunchKernelGGL((k_bupdate<SP, NB, EX, false, false>), grid, block, 0, st, n, s, out, z, in1, a, T, npart);
}

template <int SP, int NB>
static void bupdate_nb(uint64_t n, int wg, int s, const BlockRef& out, const BlockRef* in0, const BlockRef& in1,
                       double a, const double* T, double* npart, hipStream_t st) {
    if (s == NB) bupdate_ex<SP, NB, true>(n, wg, s, out, in0, in1, a, T, npart, st);
    else bupdate_ex<SP, NB, false>(n, wg, s, out, in0, in1, a, T, npart, st);
}

template <int SP>
static void bupdate_sp(uint64_t n, int wg, int s, const BlockRef& out, const BlockRef* in0, const BlockRef& in1,
                       double a, const double* T, double* npart, hipStream_t st) {
    if (s <= 4) bupdate_nb<SP, 4>(n, wg, s, out, in0, in1, a, T, npart, st);
    else if (s <= 8) bupdate_nb<SP, 8>(n, wg, s, out, in0, in1, a, T, npart, st);
    else if (s <= 12) bupdate_nb<SP, 12>(n, wg, s, out, in0, in1, a, T, npart, st);
    else bupdate_nb<SP, 16>(n, wg, s, out, in0, in1, a, T, npart, st);
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

namespace weo {

template <int SP, int NB>
static void bqp_nb(uint64_t n, int wg, int s, const BlockRef& q, const BlockRef& p, const double* ta,
                   const double* tb, hipStream_t st) {
    const dim3 grid(wg), block(kUpdBlk);
    if (s == NB) hipLaunchKernelGGL((k_bqp<SP, NB, true>), grid, block, 0, st, n, s, q, p, ta, tb);
    else hipLaunchKernelGGL((k_bqp<SP, NB, false>), grid, block, 0, st, n, s, q, p, ta, tb);
}

template <int SP>
static void bqp_sp(uint64_t n, int wg, int s, const BlockRef& q, const BlockRef& p, const double* ta,
                   const double* tb, hipStream_t st) {
    if (s <= 4) bqp_nb<SP, 4>(n, wg, s, q, p, ta, tb, st);
    else if (s <= 8) bqp_nb<SP, 8>(n, wg, s, q, p, ta, tb, st);
    else if (s <= 12) bqp_nb<SP, 12>(n, wg, s, q, p, ta, tb, st);
    else bqp_nb<SP, 16>(n, wg, s, q, p, ta, tb, st);
}

hipError_t launch_block_qp(const Geom& g, int fmt, int s, const BlockRef& q, const BlockRef& p, const double* ta,
                           const double* tb, hipStream_t st) {
    if (s < 1 || s > kMaxBlock) return hipErrorInvalidValue;
    const uint64_t n = chunks(g, fmt);
    const int wg = block_update_wg(g, fmt);
    switch (fmt_info(fmt).spinor_prec) {
        case P_F64: bqp_sp<P_F64>(n, wg, s, q, p, ta, tb, st); break;
        case P_F32: bqp_sp<P_F32>(n, wg, s, q, p, ta, tb, st); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace weo
