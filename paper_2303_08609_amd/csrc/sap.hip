// Schwarz alternating procedure (SAP) on two-coloured Dirichlet blocks of
// the Wilson matrix D_W = 1 - kappa H (Eq. (1)), and the vector kernels of
// the flexible GCR solver it preconditions.
//
// The lattice is cut into blocks of extent b = (bx, by, bz, bt) (n_mu =
// L_mu / b_mu blocks along mu, each 1 or even), coloured by the parity of the
// block coordinates.  One sweep over the blocks of one colour runs nmr steps
// of the minimal residual iteration on each block's own system D_L e = rho_L
// (every hop leaving the block dropped; where n_mu = 1 the hop across the
// lattice edge stays inside) and adds e to the solution.  The residual is
// carried, not recomputed: inside a swept block it is the MR residual; on the
// blocks of the other colour it changes only by the hops out of the swept
// blocks, +kappa H e, which the next sweep of that colour adds when it loads
// its blocks (from the increment e of the previous sweep, kept in dprev).
//
// The block solves run in FP32 (FP32 spinors and links, FP64 block sums):
// SAP is a preconditioner of a flexible Krylov method, so its accuracy only
// affects the iteration count, and FP32 keeps a block's residual, solution
// and links in one CU's LDS and registers (FP64 would spill).
//
// One workgroup per block (lane = site, at most 256 sites), so a block's
// whole solve runs out of LDS and registers: the block residual is shared
// through LDS for the in-block hops, the block sums of MR reduce through
// wavefront shuffles and LDS, and the fields are read and written once per
// sweep.  The workgroups of the other colour exit at once.
#include "hop_core.h"
#include "weo_internal.h"

namespace weo {

struct SapParams {
    Geom g;
    int b[4], nb[4];        // block extents; blocks per direction
    int bvol;               // sites per block
    int colour;
    int nmr;
    double kappa;
    double ph[4][2];
    const uint8_t* u;
    size_t link_block;
    size_t half_bytes;      // one parity of one field
    uint8_t* rho;           // nrhs full fields [rhs][even | odd]: residual (read, written)
    uint8_t* phi;           // solution, += the block solutions
    const uint8_t* dprev;   // block solutions of the previous sweep (other colour) or null
    uint8_t* dout;          // block solutions of this sweep
};

template <int SP> struct SapLds {
    using R = typename Arith<SP>::R;
    cx<R> res[12][kSapMaxSites];      // the block residual, shared for the in-block hops
    cx<R> e[12][kSapMaxSites];        // the block solution (each lane its own slot)
    double red[4][3];
};

// One hop term K = 2 mu (+mu) or 2 mu + 1 (-mu) of site x (parity p, half
// index ih) on the neighbour record psi, weighted by w (0 drops the term).
template <int SP, int LP, bool L12, int K, class C>
__device__ __forceinline__ void sap_term(const SapParams& P, const uint8_t* ubase, const Nbr& nb, uint32_t ih,
                                         int p, const C* psi, bool on, C* acc) {
    constexpr int MU = K / 2;
    constexpr bool FWD = (K & 1) == 0;
    using R = decltype(C().x);
    C u[9];
    load_link_as<LP, L12, false>(ubase + (size_t)(2 * MU + (FWD ? p : 1 - p)) * P.link_block, P.g.vh,
                                 FWD ? ih : nb.i[K], u);
    const R pr = (R)P.ph[MU][0], pi = (R)(FWD ? P.ph[MU][1] : -P.ph[MU][1]);
    C w = nb.edge[K] ? mk<C>(pr, pi) : mk<C>(R(1), R(0));
    w = on ? w : mk<C>(R(0), R(0));
    hop_dir<MU, FWD ? 1 : -1, FWD, true>(psi, u, true, w, acc);
}

template <int SP, int LP, bool L12>
__global__ void __launch_bounds__(kSapMaxSites) k_sap_sweep(const SapParams P) {
    using R = typename Arith<SP>::R;
    using C = cx<R>;
    __shared__ SapLds<SP> L;
    uint32_t bi = blockIdx.x;
    int bc[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) { bc[m] = (int)(bi % (uint32_t)P.nb[m]); bi /= (uint32_t)P.nb[m]; }
    if (((bc[0] + bc[1] + bc[2] + bc[3]) & 1) != P.colour) return;      // the whole workgroup
    const int l = threadIdx.x;
    const bool act = l < P.bvol;
    const int ls = act ? l : 0;
    int lc[4], stride[4];
    {
        int r = ls, s = 1;
#pragma unroll
        for (int m = 0; m < 4; ++m) { lc[m] = r % P.b[m]; r /= P.b[m]; stride[m] = s; s *= P.b[m]; }
    }
    Site st;
    st.x = bc[0] * P.b[0] + lc[0];
    st.y = bc[1] * P.b[1] + lc[1];
    st.z = bc[2] * P.b[2] + lc[2];
    st.t = bc[3] * P.b[3] + lc[3];
    st.xh = st.x >> 1;
    st.ih = (uint32_t)st.xh + (uint32_t)P.g.lxh * ((uint32_t)st.y + (uint32_t)P.g.ly *
                                                   ((uint32_t)st.z + (uint32_t)P.g.lz * (uint32_t)st.t));
    const int p = (st.x + st.y + st.z + st.t) & 1;
    const Nbr nb = neighbours(P.g, st);
    // in-block neighbours (local index, and whether the hop stays inside)
    int nl[8];
    bool in[8];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const bool whole = P.nb[m] == 1;
        const bool f = lc[m] + 1 < P.b[m], b = lc[m] > 0;
        in[2 * m] = act && (f || whole);
        in[2 * m + 1] = act && (b || whole);
        nl[2 * m] = f ? ls + stride[m] : ls - (P.b[m] - 1) * stride[m];
        nl[2 * m + 1] = b ? ls - stride[m] : ls + (P.b[m] - 1) * stride[m];
    }
    const size_t fb = 2 * P.half_bytes;
    const size_t off = (size_t)blockIdx.y * fb;
    const uint32_t n = P.g.vh;
    C res[12];
    if (act) load_rec<SP, 12>(P.rho + off + (size_t)p * P.half_bytes, n, st.ih, res);
    else
#pragma unroll
        for (int k = 0; k < 12; ++k) res[k] = czero<C>();
    // hops into the block from the previous sweep's solutions on the
    // neighbouring blocks: rho += kappa H dprev on the block's faces
    if (P.dprev) {
        C acc[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[k] = czero<C>();
        const uint8_t* dp = P.dprev + off + (size_t)(1 - p) * P.half_bytes;
        bool any = false;
#pragma unroll
        for (int k = 0; k < 8; ++k) any = any || (act && !in[k]);
        if (any) {
#define WEO_SAP_EXT(K)                                                        \
            if (act && !in[K]) {                                              \
                C q[12];                                                      \
                load_rec<SP, 12>(dp, n, nb.i[K], q);                          \
                sap_term<SP, LP, L12, K>(P, P.u, nb, st.ih, p, q, true, acc);      \
            }
            WEO_SAP_EXT(0) WEO_SAP_EXT(1) WEO_SAP_EXT(2) WEO_SAP_EXT(3)
            WEO_SAP_EXT(4) WEO_SAP_EXT(5) WEO_SAP_EXT(6) WEO_SAP_EXT(7)
#undef WEO_SAP_EXT
            const R kap = (R)P.kappa;
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                res[k].x = fma(kap, acc[k].x, res[k].x);
                res[k].y = fma(kap, acc[k].y, res[k].y);
            }
        }
    }
#pragma unroll
    for (int k = 0; k < 12; ++k) L.e[k][l] = czero<C>();
    const int nw = (blockDim.x + 63) >> 6;
#pragma unroll 1
    for (int it = 0; it < P.nmr; ++it) {
        __syncthreads();                       // readers of the previous residual are done
#pragma unroll
        for (int k = 0; k < 12; ++k) L.res[k][l] = res[k];
        __syncthreads();
        C q[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) q[k] = czero<C>();
        // the links stay in registers across the MR steps (the compiler
        // hoists their loads out of the loop)
#define WEO_SAP_IN(K)                                                         \
        {                                                                     \
            const uint8_t* ub = P.u;                                          \
            C v[12];                                                          \
            const int j = in[K] ? nl[K] : l;                                  \
            _Pragma("unroll") for (int k = 0; k < 12; ++k) v[k] = L.res[k][j]; \
            sap_term<SP, LP, L12, K>(P, ub, nb, st.ih, p, v, in[K], q);           \
            __builtin_amdgcn_sched_barrier(0);                                \
        }
        WEO_SAP_IN(0) WEO_SAP_IN(1) WEO_SAP_IN(2) WEO_SAP_IN(3)
        WEO_SAP_IN(4) WEO_SAP_IN(5) WEO_SAP_IN(6) WEO_SAP_IN(7)
#undef WEO_SAP_IN
        // q = D_L res = res - kappa H_L res
        const R kap = (R)P.kappa;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            q[k].x = act ? fma(-kap, q[k].x, res[k].x) : R(0);
            q[k].y = act ? fma(-kap, q[k].y, res[k].y) : R(0);
            const double qx = q[k].x, qy = q[k].y, rx = res[k].x, ry = res[k].y;
            s0 += qx * rx + qy * ry;           // <q, res>
            s1 += qx * ry - qy * rx;
            s2 += qx * qx + qy * qy;           // <q, q>
        }
        s0 = wave_sum64(s0);
        s1 = wave_sum64(s1);
        s2 = wave_sum64(s2);
        if ((l & 63) == 0) { L.red[l >> 6][0] = s0; L.red[l >> 6][1] = s1; L.red[l >> 6][2] = s2; }
        __syncthreads();
        double t0 = 0.0, t1 = 0.0, t2 = 0.0;
        for (int w = 0; w < nw; ++w) { t0 += L.red[w][0]; t1 += L.red[w][1]; t2 += L.red[w][2]; }
        const double a0 = t2 > 0.0 ? t0 / t2 : 0.0, a1 = t2 > 0.0 ? t1 / t2 : 0.0;
        const C al = mk<C>((R)a0, (R)a1);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            L.e[k][l] = fma_(al, res[k], L.e[k][l]);
            res[k] = sub(res[k], mul(al, q[k]));
        }
    }
    if (!act) return;
    C e[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) e[k] = L.e[k][l];
    const size_t po = off + (size_t)p * P.half_bytes;
    store_rec<SP, 12>(P.rho + po, n, st.ih, res);
    store_rec<SP, 12>(P.dout + po, n, st.ih, e);
    C ph[12];
    load_rec<SP, 12>(P.phi + po, n, st.ih, ph);
#pragma unroll
    for (int k = 0; k < 12; ++k) ph[k] = add(ph[k], e[k]);
    store_rec<SP, 12>(P.phi + po, n, st.ih, ph);
}

}  // namespace weo

// ---- flexible GCR vectors ------------------------------------------------------
// Fields as flat arrays of 16-byte chunks (two FP32 or one FP64 complex).
namespace weo {

template <int SP> struct GChunk;
template <> struct GChunk<P_F32> {
    static constexpr int N = 2;
    __device__ static void unpack(const uint4& w, double2* v) {
        v[0] = make_double2(__uint_as_float(w.x), __uint_as_float(w.y));
        v[1] = make_double2(__uint_as_float(w.z), __uint_as_float(w.w));
    }
    __device__ static uint4 pack(const double2* v) {
        return make_uint4(__float_as_uint((float)v[0].x), __float_as_uint((float)v[0].y),
                          __float_as_uint((float)v[1].x), __float_as_uint((float)v[1].y));
    }
};
template <> struct GChunk<P_F64> {
    static constexpr int N = 1;
    __device__ static void unpack(const uint4& w, double2* v) {
        v[0].x = __hiloint2double((int)w.y, (int)w.x);
        v[0].y = __hiloint2double((int)w.w, (int)w.z);
    }
    __device__ static uint4 pack(const double2* v) {
        const unsigned long long a = (unsigned long long)__double_as_longlong(v[0].x);
        const unsigned long long b = (unsigned long long)__double_as_longlong(v[0].y);
        return make_uint4((unsigned)a, (unsigned)(a >> 32), (unsigned)b, (unsigned)(b >> 32));
    }
};

constexpr int kGcrWG = 1024;
struct GcrVecs {
    const uint4* v[kGcrMax];
    int n;
};
struct GcrCoef {
    double re[kGcrMax], im[kGcrMax];
};

// part[(l 2 + {re, im}) nwg + wg] = sum over the workgroup's chunks of conj(a_l) b
template <int SP>
__global__ void __launch_bounds__(256) k_gcr_dots(uint64_t nch, GcrVecs A, const uint4* b, double* part) {
    using K = GChunk<SP>;
    double sr[kGcrMax], si[kGcrMax];
#pragma unroll
    for (int l = 0; l < kGcrMax; ++l) sr[l] = si[l] = 0.0;
    for (uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nch; c += (uint64_t)gridDim.x * blockDim.x) {
        double2 bv[K::N];
        K::unpack(b[c], bv);
#pragma unroll
        for (int l = 0; l < kGcrMax; ++l) {
            if (l < A.n) {
                double2 av[K::N];
                K::unpack(A.v[l][c], av);
#pragma unroll
                for (int e = 0; e < K::N; ++e) {
                    sr[l] = fma(av[e].x, bv[e].x, fma(av[e].y, bv[e].y, sr[l]));
                    si[l] = fma(av[e].x, bv[e].y, fma(-av[e].y, bv[e].x, si[l]));
                }
            }
        }
    }
    __shared__ double red[4][2 * kGcrMax];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int l = 0; l < kGcrMax; ++l) {
        if (l < A.n) {
            const double a = wave_sum64(sr[l]), c = wave_sum64(si[l]);
            if (lane == 0) { red[w][2 * l] = a; red[w][2 * l + 1] = c; }
        }
    }
    __syncthreads();
    if (threadIdx.x < 2 * A.n) {
        double t = 0.0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t += red[q][threadIdx.x];
        part[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = t;
    }
}

// b += sum_l c_l a_l; partials ||b||^2 at part[0 .. nwg) and, with r, <b, r>
// at part[nwg .. 3 nwg) (re then im)
template <int SP>
__global__ void __launch_bounds__(256) k_gcr_update(uint64_t nch, GcrVecs A, GcrCoef cf, uint4* b, const uint4* r,
                                                    double* part) {
    using K = GChunk<SP>;
    double nn = 0.0, dr = 0.0, di = 0.0;
    for (uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nch; c += (uint64_t)gridDim.x * blockDim.x) {
        double2 bv[K::N];
        K::unpack(b[c], bv);
#pragma unroll
        for (int l = 0; l < kGcrMax; ++l) {
            if (l < A.n) {              // constant indices keep the arguments in registers
                double2 av[K::N];
                K::unpack(A.v[l][c], av);
#pragma unroll
                for (int e = 0; e < K::N; ++e) {
                    bv[e].x = fma(cf.re[l], av[e].x, fma(-cf.im[l], av[e].y, bv[e].x));
                    bv[e].y = fma(cf.re[l], av[e].y, fma(cf.im[l], av[e].x, bv[e].y));
                }
            }
        }
        const uint4 wv = K::pack(bv);
        b[c] = wv;
        if (part) {
            double2 st[K::N];
            K::unpack(wv, st);                 // the stored values
            double2 rv[K::N];
            if (r) K::unpack(r[c], rv);
#pragma unroll
            for (int e = 0; e < K::N; ++e) {
                nn = fma(st[e].x, st[e].x, fma(st[e].y, st[e].y, nn));
                if (r) {
                    dr = fma(st[e].x, rv[e].x, fma(st[e].y, rv[e].y, dr));
                    di = fma(st[e].x, rv[e].y, fma(-st[e].y, rv[e].x, di));
                }
            }
        }
    }
    if (!part) return;
    __shared__ double red[4][3];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    nn = wave_sum64(nn);
    dr = wave_sum64(dr);
    di = wave_sum64(di);
    if (lane == 0) { red[w][0] = nn; red[w][1] = dr; red[w][2] = di; }
    __syncthreads();
    if (threadIdx.x < 3) {
        double t = 0.0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t += red[q][threadIdx.x];
        part[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = t;
    }
}

}  // namespace weo

// ------------------------------------------------------------------ host ----
namespace weo {

template <int SP, int LP, bool L12>
static hipError_t sap_launch(const SapParams& P, dim3 grid, dim3 block, hipStream_t s) {
    hipLaunchKernelGGL((k_sap_sweep<SP, LP, L12>), grid, block, 0, s, P);
    return hipGetLastError();
}

hipError_t launch_sap_sweep(const Geom& g, int fmt, const SapGeom& sg, int colour, int nmr, double kappa,
                            const double ph[4][2], const void* u, void* rho, void* phi, const void* dprev,
                            void* dout, int nrhs, hipStream_t s) {
    SapParams P;
    P.g = g;
    for (int m = 0; m < 4; ++m) { P.b[m] = sg.b[m]; P.nb[m] = sg.nb[m]; P.ph[m][0] = ph[m][0]; P.ph[m][1] = ph[m][1]; }
    P.bvol = sg.bvol;
    P.colour = colour;
    P.nmr = nmr;
    P.kappa = kappa;
    P.u = static_cast<const uint8_t*>(u);
    P.link_block = gauge_block_bytes(g, fmt);
    P.half_bytes = spinor_field_bytes(g, fmt);
    P.rho = static_cast<uint8_t*>(rho);
    P.phi = static_cast<uint8_t*>(phi);
    P.dprev = static_cast<const uint8_t*>(dprev);
    P.dout = static_cast<uint8_t*>(dout);
    const dim3 grid((unsigned)sg.nblocks, (unsigned)nrhs);
    const dim3 block((unsigned)((sg.bvol + 63) / 64 * 64));
    switch (fmt) {
        case FMT_S_S_18: return sap_launch<P_F32, P_F32, false>(P, grid, block, s);
        case FMT_S_S_12: return sap_launch<P_F32, P_F32, true>(P, grid, block, s);
        default: return hipErrorInvalidValue;
    }
}

int make_sap_geom(const Geom& g, const int block[4], SapGeom* sg) {
    const int L[4] = {g.lx, g.ly, g.lz, g.lt};
    int vol = 1, nbt = 1;
    for (int m = 0; m < 4; ++m) {
        const int b = block[m];
        if (b < 1 || b > L[m] || L[m] % b) return -1;
        const int n = L[m] / b;
        if (n != 1 && (n & 1)) return -1;
        sg->b[m] = b;
        sg->nb[m] = n;
        vol *= b;
        nbt *= n;
        if (vol > kSapMaxSites) return -1;
    }
    sg->bvol = vol;
    sg->nblocks = nbt;
    return 0;
}

hipError_t sap_apply(const Geom& g, int fmt, const SapGeom& sg, int ncy, int nmr, double kappa,
                     const double ph[4][2], const void* u, const void* eta, void* psi, void* rho, void* d0,
                     void* d1, int nrhs, hipStream_t s) {
    const size_t bytes = (size_t)nrhs * 2 * spinor_field_bytes(g, fmt);
    hipError_t e = hipMemcpyAsync(rho, eta, bytes, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    if ((e = launch_zero(psi, bytes, s)) != hipSuccess) return e;
    // with one block along every direction there is one colour and no hop
    // between blocks
    const bool two = sg.nblocks > 1;
    const void* prev = nullptr;
    for (int cy = 0; cy < ncy; ++cy)
        for (int c = 0; c < (two ? 2 : 1); ++c) {
            void* out = c ? d1 : d0;
            e = launch_sap_sweep(g, fmt, sg, c, nmr, kappa, ph, u, rho, psi, prev, out, nrhs, s);
            if (e != hipSuccess) return e;
            prev = two ? out : nullptr;
        }
    return hipSuccess;
}

uint32_t gcr_wg(const Geom& gb, int fmt) {
    const uint64_t nch = spinor_field_bytes(gb, fmt) / 16;
    const uint64_t w = (nch + 255) / 256;
    return (uint32_t)(w < (uint64_t)kGcrWG ? w : (uint64_t)kGcrWG);
}

static GcrVecs gcr_vecs(int n, const void* const* v) {
    GcrVecs a;
    a.n = n;
    for (int l = 0; l < kGcrMax; ++l) a.v[l] = static_cast<const uint4*>(l < n ? v[l] : v[0]);
    return a;
}

hipError_t launch_gcr_dots(const Geom& gb, int fmt, int n, const void* const* a, const void* b, double* part,
                           hipStream_t s) {
    if (n < 1 || n > kGcrMax) return hipErrorInvalidValue;
    const uint64_t nch = spinor_field_bytes(gb, fmt) / 16;
    const GcrVecs A = gcr_vecs(n, a);
    const dim3 grid(gcr_wg(gb, fmt)), block(256);
    const uint4* bp = static_cast<const uint4*>(b);
    if (fmt_info(fmt).spinor_prec == P_F64)
        hipLaunchKernelGGL((k_gcr_dots<P_F64>), grid, block, 0, s, nch, A, bp, part);
    else if (fmt_info(fmt).spinor_prec == P_F32)
        hipLaunchKernelGGL((k_gcr_dots<P_F32>), grid, block, 0, s, nch, A, bp, part);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_gcr_update(const Geom& gb, int fmt, int n, const void* const* a, const double* cre,
                             const double* cim, void* b, const void* r, double* part, hipStream_t s) {
    if (n < 0 || n > kGcrMax) return hipErrorInvalidValue;
    const uint64_t nch = spinor_field_bytes(gb, fmt) / 16;
    const void* dummy[1] = {b};
    const GcrVecs A = gcr_vecs(n, n ? a : dummy);
    GcrCoef cf;
    for (int l = 0; l < kGcrMax; ++l) { cf.re[l] = l < n ? cre[l] : 0.0; cf.im[l] = l < n ? cim[l] : 0.0; }
    const dim3 grid(gcr_wg(gb, fmt)), block(256);
    uint4* bp = static_cast<uint4*>(b);
    const uint4* rp = static_cast<const uint4*>(r);
    if (fmt_info(fmt).spinor_prec == P_F64)
        hipLaunchKernelGGL((k_gcr_update<P_F64>), grid, block, 0, s, nch, A, cf, bp, rp, part);
    else if (fmt_info(fmt).spinor_prec == P_F32)
        hipLaunchKernelGGL((k_gcr_update<P_F32>), grid, block, 0, s, nch, A, cf, bp, rp, part);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace weo
