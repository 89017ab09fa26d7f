// Face exchange for a hop whose lattice is split along a direction mu (one
// block of consecutive mu slices per device: the domain decomposition of the
// paper's Sec. 3.6 and 4.1, restated for a GPU).
//
// A block's hop is the bulk hop with the mu boundary phase set to zero (which
// drops exactly the terms that cross the block's two mu faces) plus the two
// face terms added here, for every split direction:
//   * pack (sender side, input parity q = 1 - out_parity):
//       lo[f] = (1 - S gamma_mu) psi(f, x_mu = 0)               for the block below
//       hi[f] = U_mu(f, L-1)^dag (1 + S gamma_mu) psi(f, x_mu = L-1)
//                                                                 for the block above
//     with S = +1 (-1 for the dagger), each stored as its two-component
//     half spinor (6 complex: the projector has rank 2; for t the two
//     surviving spin rows, the factor 2 applied on the receiver);
//   * unpack (receiver side, output parity p):
//       out(f, x_mu = 0)   += alpha conj(phase_lo) [rebuilt (1 + S gamma_mu) part of recv_lo[f]]
//       out(f, x_mu = L-1) += alpha phase_hi [rebuilt (1 - S gamma_mu) part of U_mu(f, L-1) recv_hi[f]]
// The backward face is multiplied by U^dag on the sender, which owns that
// link, so the receiver never needs a neighbour's links.
//
// Face sites f of one parity.  For y, z and t the face is the slice x_mu = 0
// (or L-1) with its sites in the library's compacted order (x/2 fastest,
// then the other coordinates in x, y, z, t order); with an even block length
// the site across either face has the same f.  For x the even-odd
// compaction itself runs along x: the slice x = 0 holds the sites of one
// parity in only every other (y, z, t) row, so f = (y + Ly (z + Lz t)) / 2
// (the rows are compacted along y), which again pairs the two sides' sites.
#include "hop_core.h"

namespace weo {

struct FaceParams {
    Geom g;
    int out_par;
    uint32_t nf;             // face sites per parity
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

// Half index of face site f on side `side` (0: x_mu = 0, 1: x_mu = L_mu - 1)
// for a site of parity par.
template <int MU>
__device__ __forceinline__ uint32_t face_site(const Geom& g, uint32_t f, int side, int par) {
    const uint32_t lxh = (uint32_t)g.lxh, ly = (uint32_t)g.ly, lz = (uint32_t)g.lz;
    if constexpr (MU == 3) {
        return f + (side ? (uint32_t)(g.lt - 1) * (uint32_t)g.st : 0u);
    } else if constexpr (MU == 2) {
        const uint32_t xh = f % lxh, r = f / lxh, y = r % ly, t = r / ly;
        const uint32_t z = side ? lz - 1 : 0u;
        return xh + lxh * (y + ly * (z + lz * t));
    } else if constexpr (MU == 1) {
        const uint32_t xh = f % lxh, r = f / lxh, z = r % lz, t = r / lz;
        const uint32_t y = side ? ly - 1 : 0u;
        return xh + lxh * (y + ly * (z + lz * t));
    } else {
        const uint32_t x = side ? (uint32_t)g.lx - 1 : 0u;
        const uint32_t r0 = 2 * f, y0 = r0 % ly, rest = r0 / ly, z = rest % lz, t = rest / lz;
        const uint32_t y = y0 + ((y0 + z + t + x + (uint32_t)par) & 1u);    // the row holding parity par at x
        return (x >> 1) + lxh * (y + ly * (z + lz * t));
    }
}

// Spin projection with (1 - S gamma_mu) to a half spinor (the rules of hop_dir).
template <int MU, int S, class C>
__device__ __forceinline__ void face_project(const C* p, C* h) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const C p0 = p[c], p1 = p[3 + c], p2 = p[6 + c], p3 = p[9 + c];
        C h0, h1;
        if constexpr (MU == 0) {
            h0 = S > 0 ? add(p0, imul(p3)) : sub(p0, imul(p3));
            h1 = S > 0 ? add(p1, imul(p2)) : sub(p1, imul(p2));
        } else if constexpr (MU == 1) {
            h0 = S > 0 ? add(p0, p3) : sub(p0, p3);
            h1 = S > 0 ? sub(p1, p2) : add(p1, p2);
        } else if constexpr (MU == 2) {
            h0 = S > 0 ? add(p0, imul(p2)) : sub(p0, imul(p2));
            h1 = S > 0 ? sub(p1, imul(p3)) : add(p1, imul(p3));
        } else {
            h0 = S > 0 ? p2 : p0;
            h1 = S > 0 ? p3 : p1;
        }
        h[c] = h0;
        h[3 + c] = h1;
    }
}

// acc += a * (the full spinor of (1 - S gamma_mu) rebuilt from half spinor g)
template <int MU, int S, class C, class R>
__device__ __forceinline__ void face_rebuild(const C* g, R a, C* acc) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const C g0 = g[c], g1 = g[3 + c];
        C u0 = g0, u1 = g1, l0, l1;         // upper rows; lower rows
        if constexpr (MU == 0) {
            l0 = S > 0 ? scal(R(-1), imul(g1)) : imul(g1);
            l1 = S > 0 ? scal(R(-1), imul(g0)) : imul(g0);
        } else if constexpr (MU == 1) {
            l0 = S > 0 ? scal(R(-1), g1) : g1;
            l1 = S > 0 ? g0 : scal(R(-1), g0);
        } else if constexpr (MU == 2) {
            l0 = S > 0 ? scal(R(-1), imul(g0)) : imul(g0);
            l1 = S > 0 ? imul(g1) : scal(R(-1), imul(g1));
        }
        if constexpr (MU == 3) {
            // (1 - S gamma_t) = 2 x the projector on rows 2, 3 (S > 0) or 0, 1
            const int o = S > 0 ? 6 : 0;
            acc[o + c].x = fma(R(2) * a, g0.x, acc[o + c].x);
            acc[o + c].y = fma(R(2) * a, g0.y, acc[o + c].y);
            acc[o + 3 + c].x = fma(R(2) * a, g1.x, acc[o + 3 + c].x);
            acc[o + 3 + c].y = fma(R(2) * a, g1.y, acc[o + 3 + c].y);
        } else {
            acc[c].x = fma(a, u0.x, acc[c].x);         acc[c].y = fma(a, u0.y, acc[c].y);
            acc[3 + c].x = fma(a, u1.x, acc[3 + c].x); acc[3 + c].y = fma(a, u1.y, acc[3 + c].y);
            acc[6 + c].x = fma(a, l0.x, acc[6 + c].x); acc[6 + c].y = fma(a, l0.y, acc[6 + c].y);
            acc[9 + c].x = fma(a, l1.x, acc[9 + c].x); acc[9 + c].y = fma(a, l1.y, acc[9 + c].y);
        }
    }
}

template <int SP, int LP, bool L12, bool DAG, int MU>
__global__ void __launch_bounds__(64) k_face_pack(const FaceParams P) {
    using R = typename Arith<SP>::R;
    using C = cx<R>;
    constexpr int SF = DAG ? -1 : 1;
    const uint32_t f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= P.nf) return;
    const int rhs = blockIdx.y;
    const int q = 1 - P.out_par;
    const uint8_t* in = P.in + (size_t)rhs * P.spinor_bytes;
    C p[12], h[6];
    if (blockIdx.z == 0) {
        // slice x_mu = 0: the forward term (projector 1 - SF gamma_mu) of the block below
        load_rec<SP, 12>(in, P.g.vh, face_site<MU>(P.g, f, 0, q), p);
        face_project<MU, SF>(p, h);
        store_rec<SP, 6>(P.lo + (size_t)rhs * P.face_bytes, P.nf, f, h);
    } else {
        // slice x_mu = L-1: the backward term (projector 1 + SF gamma_mu, U^dag)
        // of the block above
        const uint32_t ih = face_site<MU>(P.g, f, 1, q);
        load_rec<SP, 12>(in, P.g.vh, ih, p);
        C u[9], w[6];
        load_link_as<LP, L12, false>(P.u + (size_t)(2 * MU + q) * P.link_block, P.g.vh, ih, u);
        face_project<MU, -SF>(p, w);
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                C g = mulc(u[a], w[3 * s]);
                g = fmac_(u[3 + a], w[3 * s + 1], g);
                g = fmac_(u[6 + a], w[3 * s + 2], g);
                h[3 * s + a] = g;
            }
        store_rec<SP, 6>(P.hi + (size_t)rhs * P.face_bytes, P.nf, f, h);
    }
}

template <int SP, int LP, bool L12, bool DAG, int MU>
__global__ void __launch_bounds__(64) k_face_unpack(const FaceParams P) {
    using R = typename Arith<SP>::R;
    using C = cx<R>;
    constexpr int SF = DAG ? -1 : 1;
    const uint32_t f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= P.nf) return;
    const int rhs = blockIdx.y;
    uint8_t* out = P.out + (size_t)rhs * P.spinor_bytes;
    const R a = (R)P.alpha;
    C acc[12], h[6], g[6];
    if (blockIdx.z == 0) {
        // output slice x_mu = 0: backward term from the block below (already U^dag h)
        const uint32_t ih = face_site<MU>(P.g, f, 0, P.out_par);
        load_rec<SP, 12>(out, P.g.vh, ih, acc);
        load_rec<SP, 6>(P.lo + (size_t)rhs * P.face_bytes, P.nf, f, h);
        const C ph = mk<C>((R)P.ph_lo[0], -(R)P.ph_lo[1]);
#pragma unroll
        for (int k = 0; k < 6; ++k) g[k] = mul(ph, h[k]);
        face_rebuild<MU, -SF>(g, a, acc);
        store_rec<SP, 12>(out, P.g.vh, ih, acc);
    } else {
        // output slice x_mu = L-1: forward term from the block above, times U_mu(x)
        const uint32_t ih = face_site<MU>(P.g, f, 1, P.out_par);
        load_rec<SP, 12>(out, P.g.vh, ih, acc);
        load_rec<SP, 6>(P.hi + (size_t)rhs * P.face_bytes, P.nf, f, h);
        C u[9];
        load_link_as<LP, L12, false>(P.u + (size_t)(2 * MU + P.out_par) * P.link_block, P.g.vh, ih, u);
        const C ph = mk<C>((R)P.ph_hi[0], (R)P.ph_hi[1]);
#pragma unroll
        for (int k = 0; k < 6; ++k) h[k] = mul(ph, h[k]);
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                C t = mul(u[3 * b], h[3 * s]);
                t = fma_(u[3 * b + 1], h[3 * s + 1], t);
                t = fma_(u[3 * b + 2], h[3 * s + 2], t);
                g[3 * s + b] = t;
            }
        face_rebuild<MU, SF>(g, a, acc);
        store_rec<SP, 12>(out, P.g.vh, ih, acc);
    }
}

// ------------------------------------------------------------------ host ----
uint32_t face_sites(const Geom& g, int mu) {
    switch (mu) {
        case 0: return (uint32_t)(g.ly * g.lz * g.lt / 2);
        case 1: return (uint32_t)(g.lxh * g.lz * g.lt);
        case 2: return (uint32_t)(g.lxh * g.ly * g.lt);
        default: return (uint32_t)g.st;
    }
}

size_t face_field_bytes(const Geom& g, int fmt, int mu) {
    return (size_t)face_sites(g, mu) * 6 * (size_t)(fmt_info(fmt).spinor_site_bytes / 12);
}

static FaceParams face_params(const Geom& g, int fmt, int mu, int out_par) {
    FaceParams P;
    P.g = g;
    P.out_par = out_par;
    P.nf = face_sites(g, mu);
    P.u = nullptr;
    P.in = nullptr;
    P.out = nullptr;
    P.lo = nullptr;
    P.hi = nullptr;
    P.spinor_bytes = spinor_field_bytes(g, fmt);
    P.face_bytes = face_field_bytes(g, fmt, mu);
    P.link_block = gauge_block_bytes(g, fmt);
    P.ph_lo[0] = P.ph_hi[0] = 1.0;
    P.ph_lo[1] = P.ph_hi[1] = 0.0;
    P.alpha = 1.0;
    return P;
}

template <int SP, int LP, bool L12, int MU>
static hipError_t face_mu(bool unpack, int dagger, const FaceParams& P, int nrhs, hipStream_t s) {
    // small grids: 64-lane workgroups spread a face over more compute units
    const dim3 block(64), grid((P.nf + 63) / 64, nrhs, 2);
    if (unpack) {
        if (dagger) hipLaunchKernelGGL((k_face_unpack<SP, LP, L12, true, MU>), grid, block, 0, s, P);
        else hipLaunchKernelGGL((k_face_unpack<SP, LP, L12, false, MU>), grid, block, 0, s, P);
    } else {
        if (dagger) hipLaunchKernelGGL((k_face_pack<SP, LP, L12, true, MU>), grid, block, 0, s, P);
        else hipLaunchKernelGGL((k_face_pack<SP, LP, L12, false, MU>), grid, block, 0, s, P);
    }
    return hipGetLastError();
}

template <int SP, int LP, bool L12>
static hipError_t face_fmt(int mu, bool unpack, int dagger, const FaceParams& P, int nrhs, hipStream_t s) {
    switch (mu) {
        case 0: return face_mu<SP, LP, L12, 0>(unpack, dagger, P, nrhs, s);
        case 1: return face_mu<SP, LP, L12, 1>(unpack, dagger, P, nrhs, s);
        case 2: return face_mu<SP, LP, L12, 2>(unpack, dagger, P, nrhs, s);
        case 3: return face_mu<SP, LP, L12, 3>(unpack, dagger, P, nrhs, s);
        default: return hipErrorInvalidValue;
    }
}

static hipError_t face_dispatch(int fmt, int mu, bool unpack, int dagger, const FaceParams& P, int nrhs,
                                hipStream_t s) {
    switch (fmt) {
        case FMT_D_D_18: return face_fmt<P_F64, P_F64, false>(mu, unpack, dagger, P, nrhs, s);
        case FMT_D_D_12: return face_fmt<P_F64, P_F64, true>(mu, unpack, dagger, P, nrhs, s);
        case FMT_S_S_18: return face_fmt<P_F32, P_F32, false>(mu, unpack, dagger, P, nrhs, s);
        case FMT_S_S_12: return face_fmt<P_F32, P_F32, true>(mu, unpack, dagger, P, nrhs, s);
        case FMT_H_H_18: return face_fmt<P_F16, P_F16, false>(mu, unpack, dagger, P, nrhs, s);
        case FMT_H_H_12: return face_fmt<P_F16, P_F16, true>(mu, unpack, dagger, P, nrhs, s);
        case FMT_B_H_18: return face_fmt<P_BF16, P_F16, false>(mu, unpack, dagger, P, nrhs, s);
        case FMT_B_H_12: return face_fmt<P_BF16, P_F16, true>(mu, unpack, dagger, P, nrhs, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_face_pack(const Geom& g, int fmt, int mu, int out_par, int dagger, const void* u,
                            const void* in, void* lo, void* hi, int nrhs, hipStream_t s) {
    FaceParams P = face_params(g, fmt, mu, out_par);
    P.u = static_cast<const uint8_t*>(u);
    P.in = static_cast<const uint8_t*>(in);
    P.lo = static_cast<uint8_t*>(lo);
    P.hi = static_cast<uint8_t*>(hi);
    return face_dispatch(fmt, mu, false, dagger, P, nrhs, s);
}

hipError_t launch_face_unpack(const Geom& g, int fmt, int mu, int out_par, int dagger, const double ph_lo[2],
                              const double ph_hi[2], double alpha, const void* u, const void* lo,
                              const void* hi, void* out, int nrhs, hipStream_t s) {
    FaceParams P = face_params(g, fmt, mu, out_par);
    P.u = static_cast<const uint8_t*>(u);
    P.lo = const_cast<uint8_t*>(static_cast<const uint8_t*>(lo));
    P.hi = const_cast<uint8_t*>(static_cast<const uint8_t*>(hi));
    P.out = static_cast<uint8_t*>(out);
    for (int k = 0; k < 2; ++k) { P.ph_lo[k] = ph_lo[k]; P.ph_hi[k] = ph_hi[k]; }
    P.alpha = alpha;
    return face_dispatch(fmt, mu, true, dagger, P, nrhs, s);
}

}  // namespace weo
