// Hopping-term kernels of the even-odd Wilson operator (paper Sec. 2, Eq. (1)
// and the serial algorithm of Fig. 2): for every output site x of one parity
//
//   out(x) = sum_mu [ (1 - gamma_mu) b+ U_mu(x) in(x+mu)
//                   + (1 + gamma_mu) b- U_mu(x-mu)^dag in(x-mu) ]
//
// computed per direction as: spin projection to a two-component half spinor,
// an SU(3) product on its two colour vectors, reconstruction of the lower
// components and accumulation.  "dagger" swaps the projectors.
//
// gamma matrices are the Dirac representation; with psi = (p0, p1, p2, p3)
// (spin components, each a colour 3-vector) and S = +1 for (1 - gamma_mu),
// S = -1 for (1 + gamma_mu), the projections used below are
//   x: h0 = p0 + S i p3, h1 = p1 + S i p2;  lower = (-S i h1, -S i h0)
//   y: h0 = p0 + S p3,   h1 = p1 - S p2;    lower = (-S h1,    S h0)
//   z: h0 = p0 + S i p2, h1 = p1 - S i p3;  lower = (-S i h0,  S i h1)
//   t: S = +1: 2 (p2, p3) in the lower pair only; S = -1: 2 (p0, p1) upper only.
//
// One lane per output site; the lanes of a wavefront are consecutive sites, so
// every plane load is one coalesced 1 KiB request.  No atomics: each output
// record has exactly one writer.
#include <stdlib.h>

#include "weo_device.h"
#include "weo_internal.h"

namespace weo {

template <int SP> struct Arith { using R = float; };
template <> struct Arith<P_F64> { using R = double; };

struct HopParams {
    Geom g;
    int out_par;
    int remap;
    double ph[4][2];
    const uint8_t* u;       // packed gauge field
    const uint8_t* in;      // nrhs fields of parity 1 - out_par
    uint8_t* out;           // nrhs fields of parity out_par
    const uint8_t* y;       // axpy addend (parity out_par) or null
    double alpha;
    double* partial;
    size_t spinor_bytes;    // bytes of one packed spinor field
    size_t link_block;      // bytes of one (mu, parity) link block
};

// Link U as 9 complex numbers (row-major); a 12-real record is completed with
// row 2 = conj(row0 x row1), exact for det U = 1.
template <int LP, bool L12, class C>
__device__ __forceinline__ void load_link(const uint8_t* base, uint32_t n, uint32_t i, C* u) {
    if constexpr (L12) {
        load_rec<LP, 6>(base, n, i, u);
        u[6] = conj_(sub(mul(u[1], u[5]), mul(u[2], u[4])));
        u[7] = conj_(sub(mul(u[2], u[3]), mul(u[0], u[5])));
        u[8] = conj_(sub(mul(u[0], u[4]), mul(u[1], u[3])));
    } else {
        load_rec<LP, 9>(base, n, i, u);
    }
}

// Link record of a precision possibly narrower than the arithmetic type.
template <int LP, bool L12, class C>
__device__ __forceinline__ void load_link_as(const uint8_t* base, uint32_t n, uint32_t i, C* u) {
    using LR = typename St<LP>::real;
    if constexpr (sizeof(LR) == sizeof(decltype(C().x))) {
        load_link<LP, L12>(base, n, i, u);
    } else {
        cx<LR> w[9];
        load_link<LP, L12>(base, n, i, w);
#pragma unroll
        for (int k = 0; k < 9; ++k) { u[k].x = w[k].x; u[k].y = w[k].y; }
    }
}

// One direction: project with (1 - S gamma_mu), optional boundary phase,
// multiply by U (FWD) or U^dag (!FWD), reconstruct and accumulate.
template <int MU, int S, bool FWD, class C>
__device__ __forceinline__ void hop_dir(const C* p, const C* u, bool edge, C phase, C* acc) {
    C h0[3], h1[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const C p0 = p[c], p1 = p[3 + c], p2 = p[6 + c], p3 = p[9 + c];
        if constexpr (MU == 0) {
            h0[c] = S > 0 ? add(p0, imul(p3)) : sub(p0, imul(p3));
            h1[c] = S > 0 ? add(p1, imul(p2)) : sub(p1, imul(p2));
        } else if constexpr (MU == 1) {
            h0[c] = S > 0 ? add(p0, p3) : sub(p0, p3);
            h1[c] = S > 0 ? sub(p1, p2) : add(p1, p2);
        } else if constexpr (MU == 2) {
            h0[c] = S > 0 ? add(p0, imul(p2)) : sub(p0, imul(p2));
            h1[c] = S > 0 ? sub(p1, imul(p3)) : add(p1, imul(p3));
        } else {
            h0[c] = S > 0 ? p2 : p0;
            h1[c] = S > 0 ? p3 : p1;
        }
    }
    if (edge) {
#pragma unroll
        for (int c = 0; c < 3; ++c) { h0[c] = mul(phase, h0[c]); h1[c] = mul(phase, h1[c]); }
    }
    C g0[3], g1[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if constexpr (FWD) {
            g0[a] = mul(u[3 * a], h0[0]);
            g1[a] = mul(u[3 * a], h1[0]);
            g0[a] = fma_(u[3 * a + 1], h0[1], g0[a]);
            g1[a] = fma_(u[3 * a + 1], h1[1], g1[a]);
            g0[a] = fma_(u[3 * a + 2], h0[2], g0[a]);
            g1[a] = fma_(u[3 * a + 2], h1[2], g1[a]);
        } else {
            g0[a] = mulc(u[a], h0[0]);
            g1[a] = mulc(u[a], h1[0]);
            g0[a] = fmac_(u[3 + a], h0[1], g0[a]);
            g1[a] = fmac_(u[3 + a], h1[1], g1[a]);
            g0[a] = fmac_(u[6 + a], h0[2], g0[a]);
            g1[a] = fmac_(u[6 + a], h1[2], g1[a]);
        }
    }
    using R = decltype(C().x);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if constexpr (MU == 3) {
            if constexpr (S > 0) {
                acc[6 + a].x = fma(R(2), g0[a].x, acc[6 + a].x); acc[6 + a].y = fma(R(2), g0[a].y, acc[6 + a].y);
                acc[9 + a].x = fma(R(2), g1[a].x, acc[9 + a].x); acc[9 + a].y = fma(R(2), g1[a].y, acc[9 + a].y);
            } else {
                acc[a].x = fma(R(2), g0[a].x, acc[a].x); acc[a].y = fma(R(2), g0[a].y, acc[a].y);
                acc[3 + a].x = fma(R(2), g1[a].x, acc[3 + a].x); acc[3 + a].y = fma(R(2), g1[a].y, acc[3 + a].y);
            }
        } else {
            acc[a] = add(acc[a], g0[a]);
            acc[3 + a] = add(acc[3 + a], g1[a]);
            if constexpr (MU == 0) {          // lower = (-S i g1, -S i g0)
                acc[6 + a] = S > 0 ? sub(acc[6 + a], imul(g1[a])) : add(acc[6 + a], imul(g1[a]));
                acc[9 + a] = S > 0 ? sub(acc[9 + a], imul(g0[a])) : add(acc[9 + a], imul(g0[a]));
            } else if constexpr (MU == 1) {   // lower = (-S g1, S g0)
                acc[6 + a] = S > 0 ? sub(acc[6 + a], g1[a]) : add(acc[6 + a], g1[a]);
                acc[9 + a] = S > 0 ? add(acc[9 + a], g0[a]) : sub(acc[9 + a], g0[a]);
            } else {                          // lower = (-S i g0, S i g1)
                acc[6 + a] = S > 0 ? sub(acc[6 + a], imul(g0[a])) : add(acc[6 + a], imul(g0[a]));
                acc[9 + a] = S > 0 ? add(acc[9 + a], imul(g1[a])) : sub(acc[9 + a], imul(g1[a]));
            }
        }
    }
}

// Both neighbours of direction MU for one rhs.
template <int SP, int LP, bool L12, bool DAG, int MU, class C>
__device__ __forceinline__ void hop_mu(const HopParams& P, const uint8_t* in, const Nbr& nb,
                                       uint32_t ih, C* acc) {
    constexpr int SF = DAG ? -1 : 1;      // forward term: (1 - SF gamma)
    const uint32_t n = P.g.vh;
    C phase;
    phase.x = (decltype(C().x))P.ph[MU][0];
    phase.y = (decltype(C().x))P.ph[MU][1];
    {
        C u[9], p[12];
        load_link_as<LP, L12>(P.u + (size_t)(2 * MU + P.out_par) * P.link_block, n, ih, u);
        load_rec<SP, 12>(in, n, nb.i[2 * MU], p);
        hop_dir<MU, SF, true>(p, u, nb.edge[2 * MU], phase, acc);
    }
    {
        C u[9], p[12];
        const uint32_t j = nb.i[2 * MU + 1];
        load_link_as<LP, L12>(P.u + (size_t)(2 * MU + 1 - P.out_par) * P.link_block, n, j, u);
        load_rec<SP, 12>(in, n, j, p);
        hop_dir<MU, -SF, false>(p, u, nb.edge[2 * MU + 1], conj_(phase), acc);
    }
}

// Wavefront + workgroup sum of a double; result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* lds) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) lds[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int w = 0; w < nw; ++w) s += lds[w];
    }
    return s;
}

template <int SP, int LP, bool L12, bool DAG, bool AXPY, bool NORM>
__global__ void __launch_bounds__(256) k_hop(const HopParams P) {
    using R = typename Arith<SP>::R;
    using C = cx<R>;
    const uint32_t blk = xcd_block(blockIdx.x, gridDim.x, P.remap);
    const uint32_t ih = blk * blockDim.x + threadIdx.x;
    const int rhs = blockIdx.y;
    const uint8_t* in = P.in + (size_t)rhs * P.spinor_bytes;
    uint8_t* out = P.out + (size_t)rhs * P.spinor_bytes;
    double nrm = 0.0;
    if (ih < P.g.vh) {
        const Site s = decode(P.g, ih, P.out_par);
        const Nbr nb = neighbours(P.g, s);
        C acc[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[k] = czero<C>();
        hop_mu<SP, LP, L12, DAG, 0>(P, in, nb, ih, acc);
        hop_mu<SP, LP, L12, DAG, 1>(P, in, nb, ih, acc);
        hop_mu<SP, LP, L12, DAG, 2>(P, in, nb, ih, acc);
        hop_mu<SP, LP, L12, DAG, 3>(P, in, nb, ih, acc);
        if constexpr (AXPY) {
            C yv[12];
            load_rec<SP, 12>(P.y + (size_t)rhs * P.spinor_bytes, P.g.vh, ih, yv);
            const R a = (R)P.alpha;
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                acc[k].x = fma(a, acc[k].x, yv[k].x);
                acc[k].y = fma(a, acc[k].y, yv[k].y);
            }
        }
        store_rec<SP, 12>(out, P.g.vh, ih, acc);
        if constexpr (NORM) {
            // norm of the value as stored (rounded to the storage precision)
            C st[12];
            if constexpr (SP == P_F64 || SP == P_F32) {
#pragma unroll
                for (int k = 0; k < 12; ++k) st[k] = acc[k];
            } else {
                load_rec<SP, 12>(out, P.g.vh, ih, st);
            }
#pragma unroll
            for (int k = 0; k < 12; ++k)
                nrm += (double)st[k].x * (double)st[k].x + (double)st[k].y * (double)st[k].y;
        }
    }
    if constexpr (NORM) {
        __shared__ double lds[16];
        const double s = block_sum(nrm, lds);
        if (threadIdx.x == 0) P.partial[(size_t)rhs * gridDim.x + blockIdx.x] = s;
    }
}

// ------------------------------------------------------------------ host ----
static TuneCfg g_hop_tune = {256, 1, 1};
TuneCfg& hop_tune() { return g_hop_tune; }

// Launch-shape overrides from the environment (WEO_HOP_BLOCK, WEO_HOP_REMAP),
// read once; values outside the legal range are ignored.
static void read_env_tuning() {
    static bool done = false;
    if (done) return;
    done = true;
    if (const char* b = getenv("WEO_HOP_BLOCK")) {
        const int v = atoi(b);
        if (v >= 64 && v <= 256 && v % 64 == 0) g_hop_tune.block = v;
    }
    if (const char* r = getenv("WEO_HOP_REMAP")) g_hop_tune.remap = atoi(r) ? 1 : 0;
}

uint32_t hop_blocks(const Geom& g, int /*nrhs*/) {
    return (g.vh + (uint32_t)g_hop_tune.block - 1) / (uint32_t)g_hop_tune.block;
}

template <int SP, int LP, bool L12>
static hipError_t launch_fmt(const HopLaunch& h, const HopParams& P, dim3 grid, dim3 block,
                             hipStream_t s) {
    const bool axpy = h.y != nullptr, norm = h.partial != nullptr;
#define WEO_HOP_CASE(D, A, N)                                                         \
    if (h.dagger == D && axpy == A && norm == N) {                                    \
        hipLaunchKernelGGL((k_hop<SP, LP, L12, D, A, N>), grid, block, 0, s, P);      \
        return hipGetLastError();                                                     \
    }
    WEO_HOP_CASE(0, false, false) WEO_HOP_CASE(1, false, false)
    WEO_HOP_CASE(0, true, false)  WEO_HOP_CASE(1, true, false)
    WEO_HOP_CASE(0, false, true)  WEO_HOP_CASE(1, false, true)
    WEO_HOP_CASE(0, true, true)   WEO_HOP_CASE(1, true, true)
#undef WEO_HOP_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_hop(const HopLaunch& h, hipStream_t s) {
    read_env_tuning();
    HopParams P;
    P.g = h.g;
    P.out_par = h.out_par;
    P.remap = g_hop_tune.remap;
    for (int m = 0; m < 4; ++m) { P.ph[m][0] = h.phase[m][0]; P.ph[m][1] = h.phase[m][1]; }
    P.u = static_cast<const uint8_t*>(h.u);
    P.in = static_cast<const uint8_t*>(h.in);
    P.out = static_cast<uint8_t*>(h.out);
    P.y = static_cast<const uint8_t*>(h.y);
    P.alpha = h.alpha;
    P.partial = h.partial;
    P.spinor_bytes = spinor_field_bytes(h.g, h.fmt);
    P.link_block = gauge_block_bytes(h.g, h.fmt);
    const dim3 block(g_hop_tune.block);
    const dim3 grid(hop_blocks(h.g, h.nrhs), h.nrhs);
    switch (h.fmt) {
        case FMT_D_D_18: return launch_fmt<P_F64, P_F64, false>(h, P, grid, block, s);
        case FMT_D_D_12: return launch_fmt<P_F64, P_F64, true>(h, P, grid, block, s);
        case FMT_S_S_18: return launch_fmt<P_F32, P_F32, false>(h, P, grid, block, s);
        case FMT_S_S_12: return launch_fmt<P_F32, P_F32, true>(h, P, grid, block, s);
        case FMT_H_H_18: return launch_fmt<P_F16, P_F16, false>(h, P, grid, block, s);
        case FMT_H_H_12: return launch_fmt<P_F16, P_F16, true>(h, P, grid, block, s);
        case FMT_B_H_18: return launch_fmt<P_BF16, P_F16, false>(h, P, grid, block, s);
        case FMT_B_H_12: return launch_fmt<P_BF16, P_F16, true>(h, P, grid, block, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace weo
