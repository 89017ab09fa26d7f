// Link derivative of the bilinear form coeff * Re <Lambda, H R> (the hopping
// term of paper Eq. (1)) for full-lattice fields given as packed even and odd
// parts.  The link U_mu(x) enters H in the forward term at x (projector
// 1 - gamma_mu, boundary phase b) and in the backward term at x + mu
// (projector 1 + gamma_mu, phase conj(b)); collecting the coefficients of dU
// gives, with dL = Re tr(g^dag dU),
//
//   g = coeff conj(b) [ sum_s w_s v_s^dag + sum_s v'_s w'_s^dag ],
//   w = (1 - gamma_mu) Lambda(x),  v = R(x + mu),
//   v' = R(x),  w' = (1 + gamma_mu) Lambda(x + mu).
//
// With project, F = TH(i U g^dag) is written (TH: traceless Hermitian part),
// the su(3) force for U -> exp(i eps X) U.  One lane per link; output in the
// canonical gauge layout [4][Lt][Lz][Ly][Lx][3][3].
#include "weo_device.h"
#include "weo_internal.h"

namespace weo {

// (1 - S gamma_mu) psi as a full 4-spinor (Dirac representation; see hop.hip
// for the projection formulas).
template <int MU, int S, class C>
__device__ __forceinline__ void proj_full(const C* p, C* o) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const C p0 = p[c], p1 = p[3 + c], p2 = p[6 + c], p3 = p[9 + c];
        C h0, h1, l0, l1;
        if constexpr (MU == 0) {
            h0 = S > 0 ? add(p0, imul(p3)) : sub(p0, imul(p3));
            h1 = S > 0 ? add(p1, imul(p2)) : sub(p1, imul(p2));
            l0 = S > 0 ? sub(czero<C>(), imul(h1)) : imul(h1);
            l1 = S > 0 ? sub(czero<C>(), imul(h0)) : imul(h0);
        } else if constexpr (MU == 1) {
            h0 = S > 0 ? add(p0, p3) : sub(p0, p3);
            h1 = S > 0 ? sub(p1, p2) : add(p1, p2);
            l0 = S > 0 ? sub(czero<C>(), h1) : h1;
            l1 = S > 0 ? h0 : sub(czero<C>(), h0);
        } else if constexpr (MU == 2) {
            h0 = S > 0 ? add(p0, imul(p2)) : sub(p0, imul(p2));
            h1 = S > 0 ? sub(p1, imul(p3)) : add(p1, imul(p3));
            l0 = S > 0 ? sub(czero<C>(), imul(h0)) : imul(h0);
            l1 = S > 0 ? imul(h1) : sub(czero<C>(), imul(h1));
        } else {
            const C z = czero<C>();
            h0 = S > 0 ? z : add(p0, p0);
            h1 = S > 0 ? z : add(p1, p1);
            l0 = S > 0 ? add(p2, p2) : z;
            l1 = S > 0 ? add(p3, p3) : z;
        }
        o[c] = h0; o[3 + c] = h1; o[6 + c] = l0; o[9 + c] = l1;
    }
}

template <int MU, class C>
__device__ __forceinline__ void proj_pair(const C* lam_x, const C* lam_xp, C* w, C* wp) {
    proj_full<MU, 1>(lam_x, w);     // (1 - gamma_mu) Lambda(x)
    proj_full<MU, -1>(lam_xp, wp);  // (1 + gamma_mu) Lambda(x + mu)
}

template <int SP, int LP, bool L12, class CR>
__global__ void __launch_bounds__(256) k_force(Geom g, double4 ph01, double4 ph23, const uint8_t* u, size_t link_block,
                                               const uint8_t* lam_e, const uint8_t* lam_o,
                                               const uint8_t* r_e, const uint8_t* r_o, double coeff,
                                               int flags, typename cx_t<CR>::type* out) {
    const bool project = flags & 1, accumulate = flags & 2;
    using R = double;            // the force is accumulated in FP64
    using C = cx<R>;
    const uint64_t v = (uint64_t)g.vh * 2;
    const uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= 4 * v) return;
    const int mu = (int)(idx / v);
    const uint64_t site = idx - (uint64_t)mu * v;
    int c[4];
    c[0] = (int)(site % (uint64_t)g.lx);
    uint64_t rr = site / (uint64_t)g.lx;
    c[1] = (int)(rr % (uint64_t)g.ly); rr /= (uint64_t)g.ly;
    c[2] = (int)(rr % (uint64_t)g.lz);
    c[3] = (int)(rr / (uint64_t)g.lz);
    const int L[4] = {g.lx, g.ly, g.lz, g.lt};
    const int par = (c[0] + c[1] + c[2] + c[3]) & 1;
    auto hidx = [&](const int* q) {
        return (uint32_t)(q[0] >> 1) + (uint32_t)g.lxh * ((uint32_t)q[1] + (uint32_t)g.ly * ((uint32_t)q[2] + (uint32_t)g.lz * (uint32_t)q[3]));
    };
    const uint32_t ih = hidx(c);
    int f[4] = {c[0], c[1], c[2], c[3]};
    bool edge = false;
    if (++f[mu] == L[mu]) { f[mu] = 0; edge = true; }
    const uint32_t jh = hidx(f);
    const uint8_t* lam_x = par ? lam_o : lam_e;
    const uint8_t* lam_f = par ? lam_e : lam_o;
    const uint8_t* r_x = par ? r_o : r_e;
    const uint8_t* r_f = par ? r_e : r_o;
    using RS = typename St<SP>::real;
    cx<RS> a0[12], a1[12], b0[12], b1[12];
    load_rec<SP, 12>(lam_x, g.vh, ih, a0);
    load_rec<SP, 12>(lam_f, g.vh, jh, a1);
    load_rec<SP, 12>(r_x, g.vh, ih, b0);
    load_rec<SP, 12>(r_f, g.vh, jh, b1);
    C lx[12], lf[12], vp[12], vv[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        lx[k] = mk<C>(a0[k].x, a0[k].y); lf[k] = mk<C>(a1[k].x, a1[k].y);
        vp[k] = mk<C>(b0[k].x, b0[k].y); vv[k] = mk<C>(b1[k].x, b1[k].y);
    }
    C w[12], wp[12];
    switch (mu) {
        case 0: proj_pair<0>(lx, lf, w, wp); break;
        case 1: proj_pair<1>(lx, lf, w, wp); break;
        case 2: proj_pair<2>(lx, lf, w, wp); break;
        default: proj_pair<3>(lx, lf, w, wp); break;
    }
    // G_ab = sum_s w_s[a] conj(v_s[b]) + v'_s[a] conj(w'_s[b])
    C G[9];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            C acc = czero<C>();
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                acc = fma_(w[3 * s + a], conj_(vv[3 * s + b]), acc);
                acc = fma_(vp[3 * s + a], conj_(wp[3 * s + b]), acc);
            }
            G[3 * a + b] = acc;
        }
    // coeff * conj(b)
    C phase = mk<C>(1.0, 0.0);
    if (edge) {
        const double pr = mu == 0 ? ph01.x : mu == 1 ? ph01.z : mu == 2 ? ph23.x : ph23.z;
        const double pi = mu == 0 ? ph01.y : mu == 1 ? ph01.w : mu == 2 ? ph23.y : ph23.w;
        phase = mk<C>(pr, -pi);
    }
    phase = scal(coeff, phase);
#pragma unroll
    for (int k = 0; k < 9; ++k) G[k] = mul(phase, G[k]);
    C res[9];
    if (!project) {
#pragma unroll
        for (int k = 0; k < 9; ++k) res[k] = G[k];
    } else {
        // F = TH(i U G^dag)
        C U[9];
        cx<typename St<LP>::real> uw[9];
        const int lpar = par;
        if constexpr (L12) {
            load_rec<LP, 6>(u + (size_t)(2 * mu + lpar) * link_block, g.vh, ih, uw);
        } else {
            load_rec<LP, 9>(u + (size_t)(2 * mu + lpar) * link_block, g.vh, ih, uw);
        }
#pragma unroll
        for (int k = 0; k < (L12 ? 6 : 9); ++k) U[k] = mk<C>(uw[k].x, uw[k].y);
        if constexpr (L12) {
            U[6] = conj_(sub(mul(U[1], U[5]), mul(U[2], U[4])));
            U[7] = conj_(sub(mul(U[2], U[3]), mul(U[0], U[5])));
            U[8] = conj_(sub(mul(U[0], U[4]), mul(U[1], U[3])));
        }
        C Y[9];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                // (U G^dag)_ab = sum_k U_ak conj(G_bk)
                C acc = czero<C>();
#pragma unroll
                for (int k = 0; k < 3; ++k) acc = fma_(U[3 * a + k], conj_(G[3 * b + k]), acc);
                Y[3 * a + b] = imul(acc);
            }
        // H = (Y + Y^dag)/2 minus trace/3
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const C y = Y[3 * a + b], yt = conj_(Y[3 * b + a]);
                res[3 * a + b] = scal(0.5, add(y, yt));
            }
        const double tr = (res[0].x + res[4].x + res[8].x) / 3.0;
        res[0].x -= tr; res[4].x -= tr; res[8].x -= tr;
        res[0].y = 0.0; res[4].y = 0.0; res[8].y = 0.0;
    }
    typename cx_t<CR>::type* o = out + idx * 9;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        double x = res[k].x, y = res[k].y;
        if (accumulate) { x += (double)o[k].x; y += (double)o[k].y; }
        o[k].x = (CR)x;
        o[k].y = (CR)y;
    }
}

template <class CR>
static hipError_t force_t(const Geom& g, int fmt, const double ph[4][2], const void* u, const void* le,
                          const void* lo, const void* re, const void* ro, double coeff, int flags, void* out,
                          hipStream_t s) {
    const double4 p01 = make_double4(ph[0][0], ph[0][1], ph[1][0], ph[1][1]);
    const double4 p23 = make_double4(ph[2][0], ph[2][1], ph[3][0], ph[3][1]);
    const size_t lb = gauge_block_bytes(g, fmt);
    auto* U = static_cast<const uint8_t*>(u);
    auto* LE = static_cast<const uint8_t*>(le);
    auto* LO = static_cast<const uint8_t*>(lo);
    auto* RE = static_cast<const uint8_t*>(re);
    auto* RO = static_cast<const uint8_t*>(ro);
    auto* O = static_cast<typename cx_t<CR>::type*>(out);
    const dim3 grid((unsigned)(((uint64_t)g.vh * 8 + 255) / 256)), block(256);
#define WEO_F(SP, LP, L12) \
    hipLaunchKernelGGL((k_force<SP, LP, L12, CR>), grid, block, 0, s, g, p01, p23, U, lb, LE, LO, RE, RO, coeff, flags, O)
    switch (fmt) {
        case FMT_D_D_18: WEO_F(P_F64, P_F64, false); break;
        case FMT_D_D_12: WEO_F(P_F64, P_F64, true); break;
        case FMT_S_S_18: WEO_F(P_F32, P_F32, false); break;
        case FMT_S_S_12: WEO_F(P_F32, P_F32, true); break;
        case FMT_H_H_18: WEO_F(P_F16, P_F16, false); break;
        case FMT_H_H_12: WEO_F(P_F16, P_F16, true); break;
        case FMT_B_H_18: WEO_F(P_BF16, P_F16, false); break;
        case FMT_B_H_12: WEO_F(P_BF16, P_F16, true); break;
        default: return hipErrorInvalidValue;
    }
#undef WEO_F
    return hipGetLastError();
}

hipError_t launch_force(const Geom& g, int fmt, const double phase[4][2], const void* u, const void* lam_e,
                        const void* lam_o, const void* r_e, const void* r_o, double coeff, int flags,
                        void* g_canon, int canon_f64, hipStream_t s) {
    return canon_f64 ? force_t<double>(g, fmt, phase, u, lam_e, lam_o, r_e, r_o, coeff, flags, g_canon, s)
                     : force_t<float>(g, fmt, phase, u, lam_e, lam_o, r_e, r_o, coeff, flags, g_canon, s);
}

}  // namespace weo
