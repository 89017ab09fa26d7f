// Face exchange for a hop whose lattice is split along t (one slab of
// consecutive time slices per device, the domain decomposition of the
// paper's Sec. 3.6 and 4.1, restated for a t split).
//
// A slab's hop is the bulk hop with the t boundary phase set to zero (which
// drops exactly the two terms that cross the slab's t faces) plus the two
// face terms added here:
//   * pack (sender side, input parity q = 1 - out_parity):
//       lo[f] = (1 - S gamma_t) psi(f, t = 0)            for the slab below
//       hi[f] = U_t(f, Lt-1)^dag (1 + S gamma_t) psi(f, t = Lt-1)
//                                                          for the slab above
//     with S = +1 (-1 for the dagger), stored as the two non-zero spin rows
//     (6 complex), the factor 2 of the t projector applied on the receiver;
//   * unpack (receiver side, output parity p):
//       out(f, 0)    += alpha 2 conj(phase_lo) recv_lo[f]          (upper or lower rows)
//       out(f, Lt-1) += alpha 2 phase_hi U_t(f, Lt-1) recv_hi[f]
// where f = (x>>1) + Lx/2 (y + Ly z) indexes the sites of one parity in a
// t slice: with an even slab length the site across either face has the
// same f.  The backward face is multiplied by U^dag on the sender, which
// owns that link, so the receiver never needs a neighbour's links.
#include "hop_core.h"

namespace weo {

struct FaceParams {
    Geom g;
    int out_par;
    uint32_t nf;             // face sites per parity (Lx Ly Lz / 2)
    const uint8_t* u;
    const uint8_t* in;       // pack: input field; unpack: unused
    uint8_t* out;            // unpack: output field (read-modify-write)
    uint8_t* lo;             // pack: written; unpack: read
    uint8_t* hi;
    size_t spinor_bytes;     // one field
    size_t face_bytes;       // one face of one field
    size_t link_block;       // one (mu, parity) block of links
    double ph_lo[2], ph_hi[2];
    double alpha;
};

// Spin rows kept by (1 - s gamma_t) in the Dirac representation:
// s > 0 keeps rows 2, 3; s < 0 keeps rows 0, 1.
template <int S> __device__ __forceinline__ constexpr int t_rows() { return S > 0 ? 6 : 0; }

template <int SP, int LP, bool L12, bool DAG>
__global__ void __launch_bounds__(64) k_face_pack(const FaceParams P) {
    using R = typename Arith<SP>::R;
    using C = cx<R>;
    constexpr int SF = DAG ? -1 : 1;
    const uint32_t f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= P.nf) return;
    const int rhs = blockIdx.y;
    const uint8_t* in = P.in + (size_t)rhs * P.spinor_bytes;
    C p[12], h[6];
    if (blockIdx.z == 0) {
        // t = 0 slice: the forward term (projector 1 - SF gamma_t) of the slab below
        load_rec<SP, 12>(in, P.g.vh, f, p);
        constexpr int o = t_rows<SF>();
#pragma unroll
        for (int k = 0; k < 6; ++k) h[k] = p[o + k];
        store_rec<SP, 6>(P.lo + (size_t)rhs * P.face_bytes, P.nf, f, h);
    } else {
        // t = Lt-1 slice: the backward term (projector 1 + SF gamma_t, U^dag)
        // of the slab above
        const uint32_t ih = f + (uint32_t)(P.g.lt - 1) * (uint32_t)P.g.st;
        load_rec<SP, 12>(in, P.g.vh, ih, p);
        C u[9];
        load_link_as<LP, L12, false>(P.u + (size_t)(2 * 3 + 1 - P.out_par) * P.link_block, P.g.vh, ih, u);
        constexpr int o = t_rows<-SF>();
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                C g = mulc(u[a], p[o + 3 * s]);
                g = fmac_(u[3 + a], p[o + 3 * s + 1], g);
                g = fmac_(u[6 + a], p[o + 3 * s + 2], g);
                h[3 * s + a] = g;
            }
        store_rec<SP, 6>(P.hi + (size_t)rhs * P.face_bytes, P.nf, f, h);
    }
}

template <int SP, int LP, bool L12, bool DAG>
__global__ void __launch_bounds__(64) k_face_unpack(const FaceParams P) {
    using R = typename Arith<SP>::R;
    using C = cx<R>;
    constexpr int SF = DAG ? -1 : 1;
    const uint32_t f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= P.nf) return;
    const int rhs = blockIdx.y;
    uint8_t* out = P.out + (size_t)rhs * P.spinor_bytes;
    const R two_a = (R)(2.0 * P.alpha);
    C acc[12], h[6], g[6];
    if (blockIdx.z == 0) {
        // output slice t = 0: backward term from the slab below (already U^dag h)
        const uint32_t ih = f;
        load_rec<SP, 12>(out, P.g.vh, ih, acc);
        load_rec<SP, 6>(P.lo + (size_t)rhs * P.face_bytes, P.nf, f, h);
        const C ph = mk<C>((R)P.ph_lo[0], -(R)P.ph_lo[1]);
#pragma unroll
        for (int k = 0; k < 6; ++k) g[k] = mul(ph, h[k]);
        constexpr int o = t_rows<-SF>();
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            acc[o + k].x = fma(two_a, g[k].x, acc[o + k].x);
            acc[o + k].y = fma(two_a, g[k].y, acc[o + k].y);
        }
        store_rec<SP, 12>(out, P.g.vh, ih, acc);
    } else {
        // output slice t = Lt-1: forward term from the slab above, times U_t(x)
        const uint32_t ih = f + (uint32_t)(P.g.lt - 1) * (uint32_t)P.g.st;
        load_rec<SP, 12>(out, P.g.vh, ih, acc);
        load_rec<SP, 6>(P.hi + (size_t)rhs * P.face_bytes, P.nf, f, h);
        C u[9];
        load_link_as<LP, L12, false>(P.u + (size_t)(2 * 3 + P.out_par) * P.link_block, P.g.vh, ih, u);
        const C ph = mk<C>((R)P.ph_hi[0], (R)P.ph_hi[1]);
#pragma unroll
        for (int k = 0; k < 6; ++k) h[k] = mul(ph, h[k]);
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                C t = mul(u[3 * a], h[3 * s]);
                t = fma_(u[3 * a + 1], h[3 * s + 1], t);
                t = fma_(u[3 * a + 2], h[3 * s + 2], t);
                g[3 * s + a] = t;
            }
        constexpr int o = t_rows<SF>();
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            acc[o + k].x = fma(two_a, g[k].x, acc[o + k].x);
            acc[o + k].y = fma(two_a, g[k].y, acc[o + k].y);
        }
        store_rec<SP, 12>(out, P.g.vh, ih, acc);
    }
}

// ------------------------------------------------------------------ host ----
size_t face_field_bytes(const Geom& g, int fmt) {
    return (size_t)g.st * 6 * (size_t)(fmt_info(fmt).spinor_site_bytes / 12);
}

static FaceParams face_params(const Geom& g, int fmt, int out_par) {
    FaceParams P;
    P.g = g;
    P.out_par = out_par;
    P.nf = (uint32_t)g.st;
    P.u = nullptr;
    P.in = nullptr;
    P.out = nullptr;
    P.lo = nullptr;
    P.hi = nullptr;
    P.spinor_bytes = spinor_field_bytes(g, fmt);
    P.face_bytes = face_field_bytes(g, fmt);
    P.link_block = gauge_block_bytes(g, fmt);
    P.ph_lo[0] = P.ph_hi[0] = 1.0;
    P.ph_lo[1] = P.ph_hi[1] = 0.0;
    P.alpha = 1.0;
    return P;
}

template <int SP, int LP, bool L12>
static hipError_t face_fmt(bool unpack, int dagger, const FaceParams& P, int nrhs, hipStream_t s) {
    // small grids: 64-lane workgroups spread a face over more compute units
    const dim3 block(64), grid((P.nf + 63) / 64, nrhs, 2);
    if (unpack) {
        if (dagger) hipLaunchKernelGGL((k_face_unpack<SP, LP, L12, true>), grid, block, 0, s, P);
        else hipLaunchKernelGGL((k_face_unpack<SP, LP, L12, false>), grid, block, 0, s, P);
    } else {
        if (dagger) hipLaunchKernelGGL((k_face_pack<SP, LP, L12, true>), grid, block, 0, s, P);
        else hipLaunchKernelGGL((k_face_pack<SP, LP, L12, false>), grid, block, 0, s, P);
    }
    return hipGetLastError();
}

static hipError_t face_dispatch(int fmt, bool unpack, int dagger, const FaceParams& P, int nrhs,
                                hipStream_t s) {
    switch (fmt) {
        case FMT_D_D_18: return face_fmt<P_F64, P_F64, false>(unpack, dagger, P, nrhs, s);
        case FMT_D_D_12: return face_fmt<P_F64, P_F64, true>(unpack, dagger, P, nrhs, s);
        case FMT_S_S_18: return face_fmt<P_F32, P_F32, false>(unpack, dagger, P, nrhs, s);
        case FMT_S_S_12: return face_fmt<P_F32, P_F32, true>(unpack, dagger, P, nrhs, s);
        case FMT_H_H_18: return face_fmt<P_F16, P_F16, false>(unpack, dagger, P, nrhs, s);
        case FMT_H_H_12: return face_fmt<P_F16, P_F16, true>(unpack, dagger, P, nrhs, s);
        case FMT_B_H_18: return face_fmt<P_BF16, P_F16, false>(unpack, dagger, P, nrhs, s);
        case FMT_B_H_12: return face_fmt<P_BF16, P_F16, true>(unpack, dagger, P, nrhs, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_face_pack(const Geom& g, int fmt, int out_par, int dagger, const void* u,
                            const void* in, void* lo, void* hi, int nrhs, hipStream_t s) {
    FaceParams P = face_params(g, fmt, out_par);
    P.u = static_cast<const uint8_t*>(u);
    P.in = static_cast<const uint8_t*>(in);
    P.lo = static_cast<uint8_t*>(lo);
    P.hi = static_cast<uint8_t*>(hi);
    return face_dispatch(fmt, false, dagger, P, nrhs, s);
}

hipError_t launch_face_unpack(const Geom& g, int fmt, int out_par, int dagger, const double ph_lo[2],
                              const double ph_hi[2], double alpha, const void* u, const void* lo,
                              const void* hi, void* out, int nrhs, hipStream_t s) {
    FaceParams P = face_params(g, fmt, out_par);
    P.u = static_cast<const uint8_t*>(u);
    P.lo = const_cast<uint8_t*>(static_cast<const uint8_t*>(lo));
    P.hi = const_cast<uint8_t*>(static_cast<const uint8_t*>(hi));
    P.out = static_cast<uint8_t*>(out);
    for (int k = 0; k < 2; ++k) { P.ph_lo[k] = ph_lo[k]; P.ph_hi[k] = ph_hi[k]; }
    P.alpha = alpha;
    return face_dispatch(fmt, true, dagger, P, nrhs, s);
}

}  // namespace weo
