// Single right-hand-side hopping kernel of the even-odd Wilson operator
// (paper Sec. 2, Eq. (1), serial algorithm of Fig. 2); the per-direction
// arithmetic lives in hop_core.h.  One lane per output site; several
// right-hand sides run as independent grid rows.
#include <stdlib.h>

#include "hop_core.h"

namespace weo {

template <int SP> struct Waves { static constexpr int n = WEO_WAVES_F32; };
template <> struct Waves<P_F64> { static constexpr int n = WEO_WAVES_F64; };

template <int SP, int LP, bool L12, bool DAG, bool AXPY, bool NORM, bool CPH, bool DOT = false>
__global__ void __launch_bounds__(256, Waves<SP>::n > 0 ? Waves<SP>::n : 1) k_hop(const HopParams P) {
    using R = typename Arith<SP>::R;
    using C = cx<R>;
    const uint32_t blk = xcd_block(blockIdx.x, gridDim.x, P.remap);
    const uint32_t ih = block_first_site(P.sched, P.g, blk, blockDim.x) + threadIdx.x;
    const int rhs = blockIdx.y;
    const uint8_t* in = P.in + (size_t)rhs * P.spinor_bytes;
    uint8_t* out = P.out + (size_t)rhs * P.spinor_bytes;
    double nrm = 0.0, dre = 0.0, dim = 0.0;
    if (ih < P.g.vh) {
        const Site s = decode(P.g, ih, P.out_par);
        const Nbr nb = neighbours(P.g, s);
        C acc[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[k] = czero<C>();
        constexpr int D = hop_pipe<SP>();
        if constexpr (D > 0) {
            NbrRaw<SP, LP, L12> ring[D + 1];
            pipe_prologue<SP, LP, L12, DAG, CPH, D>(P, in, nb, ih, ring);
            pipe_step<SP, LP, L12, DAG, CPH, D, 0>(P, in, nb, ih, ring, acc);
        } else {
            hop_mu<SP, LP, L12, DAG, CPH, 0>(P, in, nb, ih, acc);
            hop_mu<SP, LP, L12, DAG, CPH, 1>(P, in, nb, ih, acc);
            hop_mu<SP, LP, L12, DAG, CPH, 2>(P, in, nb, ih, acc);
            hop_mu<SP, LP, L12, DAG, CPH, 3>(P, in, nb, ih, acc);
        }
        if constexpr (AXPY) hop_addends<SP>(P, (size_t)rhs, ih, acc);
        store_rec<SP, 12, C, hop_nt_store<SP>()>(out, P.g.vh, ih, acc);
        if constexpr (NORM) hop_reduce<SP, DOT>(P, (size_t)rhs, ih, acc, nrm, dre, dim);
    }
    if constexpr (NORM) {
        // one partial per 64-site chunk (one wavefront)
        const uint32_t chunk = (block_first_site(P.sched, P.g, blk, blockDim.x) + (threadIdx.x & ~63u)) >> 6;
        hop_partials_out<DOT>(P, (size_t)rhs, chunk, (P.g.vh + 63) >> 6, (threadIdx.x & 63) == 0, nrm, dre, dim);
    }
}

// ------------------------------------------------------------------ host ----
static TuneCfg g_hop_tune = {256, 1, 0};
TuneCfg& hop_tune() { return g_hop_tune; }

// Launch-shape overrides from the environment (WEO_HOP_BLOCK, WEO_HOP_REMAP,
// WEO_HOP_BZ),
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
    if (const char* z = getenv("WEO_HOP_BZ")) {
        const int v = atoi(z);
        if (v >= 0 && v <= 64) g_hop_tune.bz = v;
    }
}

uint32_t hop_partials(const Geom& g) { return (g.vh + 63) / 64; }

static uint32_t hop_blocks(const Geom& g) {
    return (g.vh + (uint32_t)g_hop_tune.block - 1) / (uint32_t)g_hop_tune.block;
}

template <int SP, int LP, bool L12>
static hipError_t launch_fmt(const HopLaunch& h, const HopParams& P, dim3 grid, dim3 block,
                             hipStream_t s) {
    const bool axpy = h.y != nullptr, norm = h.partial != nullptr;
    bool cph = false;
    for (int m = 0; m < 4; ++m) cph = cph || h.phase[m][1] != 0.0;
    if (h.dmode) {
        // the fused dot: an M epilogue (axpy and norm) only
        if (!axpy || !norm) return hipErrorInvalidValue;
#define WEO_HOP_DOT(D)                                                                                   \
        if (h.dagger == D) {                                                                             \
            if (cph) hipLaunchKernelGGL((k_hop<SP, LP, L12, D, true, true, true, true>), grid, block, 0, s, P);   \
            else hipLaunchKernelGGL((k_hop<SP, LP, L12, D, true, true, false, true>), grid, block, 0, s, P);  \
            return hipGetLastError();                                                                    \
        }
        WEO_HOP_DOT(0) WEO_HOP_DOT(1)
#undef WEO_HOP_DOT
        return hipErrorInvalidValue;
    }
#define WEO_HOP_CASE(D, A, N)                                                            \
    if (h.dagger == D && axpy == A && norm == N) {                                       \
        if (cph)                                                                          \
            hipLaunchKernelGGL((k_hop<SP, LP, L12, D, A, N, true>), grid, block, 0, s, P);  \
        else                                                                              \
            hipLaunchKernelGGL((k_hop<SP, LP, L12, D, A, N, false>), grid, block, 0, s, P); \
        return hipGetLastError();                                                         \
    }
    WEO_HOP_CASE(0, false, false) WEO_HOP_CASE(1, false, false)
    WEO_HOP_CASE(0, true, false)  WEO_HOP_CASE(1, true, false)
    WEO_HOP_CASE(0, false, true)  WEO_HOP_CASE(1, false, true)
    WEO_HOP_CASE(0, true, true)   WEO_HOP_CASE(1, true, true)
#undef WEO_HOP_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_hop_single(const HopLaunch& h, hipStream_t s) {
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
    P.z = static_cast<const uint8_t*>(h.z);
    P.cy = h.cy;
    P.dmode = h.dmode;
    P.dw = static_cast<const uint8_t*>(h.dw);
    P.pdre = h.pdre;
    P.pdim = h.pdim;
    P.alpha = h.alpha;
    P.partial = h.partial;
    P.spinor_bytes = spinor_field_bytes(h.g, h.fmt);
    P.link_block = gauge_block_bytes(h.g, h.fmt);
    P.sched = make_sched(h.g, g_hop_tune.bz, (uint32_t)g_hop_tune.block);
    const dim3 block(g_hop_tune.block);
    const dim3 grid(hop_blocks(h.g), h.nrhs);
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
