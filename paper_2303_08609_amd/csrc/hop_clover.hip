// Hop with a clover-type site block applied to its result (paper Sec. 2,
// Eqs. (3)-(5) with site-local D_ee, D_oo):
//     out = C_p P_p H P_{1-p} in            (y == nullptr)
//     out = y + alpha C_p P_p H P_{1-p} in  (y != nullptr)
// with C_p the packed site blocks of the output parity (normally the inverse
// blocks A_pp^-1).  Same lane-per-site structure and neighbour pipeline as the
// plain hop; the block product runs after the 8 directions, when the
// neighbour ring is no longer live.
#include "clover_core.h"
#include "hop_core.h"

// WEO_CLV_PREFETCH = 0 loads the blocks after the 8 directions instead.
#ifndef WEO_CLV_PREFETCH
#define WEO_CLV_PREFETCH 1
#endif

namespace weo {

struct CloverHopParams {
    HopParams h;
    const uint8_t* clv;     // the output parity's two block fields
    size_t block_bytes;
};

// The neighbour pipeline of the plain hop, with the two block records of the
// site loaded in the steps whose ring slot is no longer needed (the last D
// directions), so their latency hides behind the last directions' arithmetic.
template <int SP, int LP, bool L12, bool DAG, bool CPH, int D, int K, class C>
__device__ __forceinline__ void clv_step(const CloverHopParams& Q, const uint8_t* in, const Nbr& nb, uint32_t ih,
                                         NbrRaw<SP, LP, L12> (&ring)[D + 1], RawRec<LP, kCloverSlots> (&cb)[2],
                                         C* acc) {
    const HopParams& P = Q.h;
    if constexpr (K + D < 8) {
        issue<SP, LP, L12, K + D>(P, in, nb, ih, ring[(K + D) % (D + 1)]);
    } else if constexpr (K + D == 8) {
        cb[0].load(Q.clv, P.g.vh, ih);
        if constexpr (D == 1) cb[1].load(Q.clv + Q.block_bytes, P.g.vh, ih);
    } else if constexpr (K + D == 9) {
        cb[1].load(Q.clv + Q.block_bytes, P.g.vh, ih);
    }
    __builtin_amdgcn_sched_barrier(0);
    consume<SP, LP, L12, DAG, CPH, K>(P, nb, ring[K % (D + 1)], acc);
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (K + 1 < 8) clv_step<SP, LP, L12, DAG, CPH, D, K + 1>(Q, in, nb, ih, ring, cb, acc);
}

template <int SP, int LP, bool L12, bool DAG, bool AXPY, bool NORM, bool CPH>
__global__ void __launch_bounds__(256) k_hop_clv(const CloverHopParams Q) {
    using R = typename Arith<SP>::R;
    using C = cx<R>;
    const HopParams& P = Q.h;
    const uint32_t blk = xcd_block(blockIdx.x, gridDim.x, P.remap);
    const uint32_t ih = block_first_site(P.sched, P.g, blk, blockDim.x) + threadIdx.x;
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
        constexpr int D = hop_pipe<SP>();
        static_assert(D <= 2, "block prefetch placed for ring depths up to 2");
        NbrRaw<SP, LP, L12> ring[D + 1];
        if constexpr (D > 0) pipe_prologue<SP, LP, L12, DAG, CPH, D>(P, in, nb, ih, ring);
        if constexpr (D == 0) {
            hop_mu<SP, LP, L12, DAG, CPH, 0>(P, in, nb, ih, acc);
            hop_mu<SP, LP, L12, DAG, CPH, 1>(P, in, nb, ih, acc);
            hop_mu<SP, LP, L12, DAG, CPH, 2>(P, in, nb, ih, acc);
            hop_mu<SP, LP, L12, DAG, CPH, 3>(P, in, nb, ih, acc);
            clover_apply_site<LP>(Q.clv, Q.block_bytes, P.g.vh, ih, acc);
        } else if constexpr (WEO_CLV_PREFETCH != 0) {
            RawRec<LP, kCloverSlots> cb[2];
            clv_step<SP, LP, L12, DAG, CPH, D, 0>(Q, in, nb, ih, ring, cb, acc);
            clover_apply_raw<LP>(cb[0], cb[1], acc);
        } else {
            pipe_step<SP, LP, L12, DAG, CPH, D, 0>(P, in, nb, ih, ring, acc);
            clover_apply_site<LP>(Q.clv, Q.block_bytes, P.g.vh, ih, acc);
        }
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
        store_rec<SP, 12, C, hop_nt_store<SP>()>(out, P.g.vh, ih, acc);
        if constexpr (NORM) {
            C st[12];
            if constexpr (SP == P_F64 || SP == P_F32) {
#pragma unroll
                for (int k = 0; k < 12; ++k) st[k] = acc[k];
            } else {
                round_rec<SP, 12>(acc, st);
            }
#pragma unroll
            for (int k = 0; k < 12; ++k)
                nrm += (double)st[k].x * (double)st[k].x + (double)st[k].y * (double)st[k].y;
        }
    }
    if constexpr (NORM) {
        const double t = wave_sum64(nrm);
        const uint32_t chunk = (block_first_site(P.sched, P.g, blk, blockDim.x) + (threadIdx.x & ~63u)) >> 6;
        const uint32_t nchunk = (P.g.vh + 63) >> 6;
        if ((threadIdx.x & 63) == 0 && chunk < nchunk) P.partial[(size_t)rhs * nchunk + chunk] = t;
    }
}

// ------------------------------------------------------------------ host ----
template <int SP, int LP, bool L12>
static hipError_t clv_fmt(const HopLaunch& h, const CloverHopParams& Q, dim3 grid, dim3 block, hipStream_t s) {
    const bool axpy = h.y != nullptr, norm = h.partial != nullptr;
    bool cph = false;
    for (int m = 0; m < 4; ++m) cph = cph || h.phase[m][1] != 0.0;
#define WEO_CLV(D, A, N)                                                                       \
    if (h.dagger == D && axpy == A && norm == N) {                                             \
        if (cph) hipLaunchKernelGGL((k_hop_clv<SP, LP, L12, D, A, N, true>), grid, block, 0, s, Q);  \
        else hipLaunchKernelGGL((k_hop_clv<SP, LP, L12, D, A, N, false>), grid, block, 0, s, Q);     \
        return hipGetLastError();                                                              \
    }
    WEO_CLV(0, false, false) WEO_CLV(1, false, false)
    WEO_CLV(0, true, false)  WEO_CLV(1, true, false)
    WEO_CLV(0, false, true)  WEO_CLV(1, false, true)
    WEO_CLV(0, true, true)   WEO_CLV(1, true, true)
#undef WEO_CLV
    return hipErrorInvalidValue;
}

hipError_t launch_hop_clover(const HopLaunch& h, const void* clv, hipStream_t s) {
    const TuneCfg& tc = hop_tune();
    CloverHopParams Q;
    HopParams& P = Q.h;
    P.g = h.g;
    P.out_par = h.out_par;
    P.remap = tc.remap;
    for (int m = 0; m < 4; ++m) { P.ph[m][0] = h.phase[m][0]; P.ph[m][1] = h.phase[m][1]; }
    P.u = static_cast<const uint8_t*>(h.u);
    P.in = static_cast<const uint8_t*>(h.in);
    P.out = static_cast<uint8_t*>(h.out);
    P.y = static_cast<const uint8_t*>(h.y);
    P.z = nullptr;            // the clover epilogue takes y only, no fused dot
    P.cy = 1.0;
    P.dmode = 0;
    P.dw = nullptr;
    P.pdre = P.pdim = nullptr;
    P.alpha = h.alpha;
    P.partial = h.partial;
    P.spinor_bytes = spinor_field_bytes(h.g, h.fmt);
    P.link_block = gauge_block_bytes(h.g, h.fmt);
    P.sched = make_sched(h.g, tc.bz, (uint32_t)tc.block);
    Q.block_bytes = clover_block_bytes(h.g, h.fmt);
    Q.clv = static_cast<const uint8_t*>(clv) + (size_t)(2 * h.out_par) * Q.block_bytes;
    const dim3 block(tc.block), grid((h.g.vh + (uint32_t)tc.block - 1) / (uint32_t)tc.block, h.nrhs);
    switch (h.fmt) {
        case FMT_D_D_18: return clv_fmt<P_F64, P_F64, false>(h, Q, grid, block, s);
        case FMT_D_D_12: return clv_fmt<P_F64, P_F64, true>(h, Q, grid, block, s);
        case FMT_S_S_18: return clv_fmt<P_F32, P_F32, false>(h, Q, grid, block, s);
        case FMT_S_S_12: return clv_fmt<P_F32, P_F32, true>(h, Q, grid, block, s);
        case FMT_H_H_18: return clv_fmt<P_F16, P_F16, false>(h, Q, grid, block, s);
        case FMT_H_H_12: return clv_fmt<P_F16, P_F16, true>(h, Q, grid, block, s);
        case FMT_B_H_18: return clv_fmt<P_BF16, P_F16, false>(h, Q, grid, block, s);
        case FMT_B_H_12: return clv_fmt<P_BF16, P_F16, true>(h, Q, grid, block, s);
        default: return hipErrorInvalidValue;
    }
}

// M = 1 - kappa^2 C_e H_eo C_o H_oe (dagger 0) or its adjoint
// 1 - kappa^2 H_eo^dag C_o H_oe^dag C_e (dagger 1; C Hermitian) on the even
// parity, C the packed inverse blocks; partial = ||out||^2 per 64 sites.
hipError_t launch_apply_clover(const Geom& g, int fmt, const double phase[4][2], double kappa, int dagger,
                               const void* u, const void* clv, const void* in, void* out, void* tmp, int nrhs,
                               double* partial, hipStream_t s) {
    HopLaunch h;
    h.g = g;
    h.fmt = fmt;
    h.dagger = dagger;
    for (int m = 0; m < 4; ++m) { h.phase[m][0] = phase[m][0]; h.phase[m][1] = phase[m][1]; }
    h.u = u;
    h.nrhs = nrhs;
    hipError_t e;
    if (!dagger) {
        // tmp_o = C_o H_oe in;  out = in - kappa^2 C_e H_eo tmp_o
        h.out_par = 1; h.in = in; h.out = tmp; h.y = nullptr; h.alpha = 0.0; h.partial = nullptr;
        if ((e = launch_hop_clover(h, clv, s)) != hipSuccess) return e;
        h.out_par = 0; h.in = tmp; h.out = out; h.y = in; h.alpha = -kappa * kappa; h.partial = partial;
        return launch_hop_clover(h, clv, s);
    }
    // out = C_e in;  tmp_o = C_o H_oe^dag out;  out = in - kappa^2 H_eo^dag tmp_o
    if ((e = launch_clover_site(g, fmt, 0, clv, in, nullptr, 0.0, out, nrhs, s)) != hipSuccess) return e;
    h.out_par = 1; h.in = out; h.out = tmp; h.y = nullptr; h.alpha = 0.0; h.partial = nullptr;
    if ((e = launch_hop_clover(h, clv, s)) != hipSuccess) return e;
    h.out_par = 0; h.in = tmp; h.out = out; h.y = in; h.alpha = -kappa * kappa; h.partial = partial;
    return launch_hop_single(h, s);
}

}  // namespace weo
