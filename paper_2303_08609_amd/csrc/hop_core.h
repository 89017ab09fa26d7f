// Device building blocks of the hopping-term kernels of the even-odd Wilson operator (paper Sec. 2, Eq. (1)
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
#pragma once

#include "weo_device.h"
#include "weo_internal.h"

namespace weo {

// Per-precision kernel shape, chosen by measurement on MI355X at 32^3x64:
//   pipe  d >= 1: the raw words of neighbour k + d are loaded while neighbour
//         k is computed (a register ring of d + 1 records, kept in order by
//         scheduling barriers); 0: one direction at a time as written.
//   nt    links are read with streaming (non-temporal) loads: every link is
//         used once per hop, so it should not evict the spinors that the
//         neighbouring sites re-read through L2.
//   nt_store  the output records are written with streaming stores.
// FP64 keeps regular link loads (its streaming variant measured slower) and
// a one-deep ring (a two-deep ring spills), and streams its output (hop
// 349 -> 336 us at 32^3x64; neutral to slightly slower for the narrower
// formats); FP16/BF16 records are small enough for a two-deep ring.
// WEO_HOP_PIPE / WEO_NT_LINKS / WEO_NT_STORE (-D) override all precisions at
// once for experiments.
template <int SP> struct HopShape;
template <> struct HopShape<P_F64> {
    static constexpr int pipe = 1; static constexpr bool nt = false; static constexpr bool nt_store = true;
};
template <> struct HopShape<P_F32> {
    static constexpr int pipe = 1; static constexpr bool nt = true; static constexpr bool nt_store = false;
};
template <> struct HopShape<P_F16> {
    static constexpr int pipe = 2; static constexpr bool nt = true; static constexpr bool nt_store = false;
};
template <> struct HopShape<P_BF16> {
    static constexpr int pipe = 2; static constexpr bool nt = true; static constexpr bool nt_store = false;
};
#ifdef WEO_HOP_PIPE
template <int SP> constexpr int hop_pipe() { return WEO_HOP_PIPE; }
#else
template <int SP> constexpr int hop_pipe() { return HopShape<SP>::pipe; }
#endif
#ifdef WEO_NT_LINKS
template <int SP> constexpr bool hop_nt() { return WEO_NT_LINKS != 0; }
#else
template <int SP> constexpr bool hop_nt() { return HopShape<SP>::nt; }
#endif
#ifdef WEO_NT_STORE
template <int SP> constexpr bool hop_nt_store() { return WEO_NT_STORE != 0; }
#else
template <int SP> constexpr bool hop_nt_store() { return HopShape<SP>::nt_store; }
#endif
//   WEO_WAVES_F32 / WEO_WAVES_F64: minimum waves per SIMD requested (0 = the
//   compiler's choice).
#ifndef WEO_WAVES_F32
#define WEO_WAVES_F32 0
#endif
#ifndef WEO_WAVES_F64
#define WEO_WAVES_F64 0
#endif

// FP16 values of the 12-real formats are converted to FP32 where they are
// unpacked (an empty asm pins the converted values).  Left alone, the
// compiler folds the conversions into mixed-precision FMAs and keeps the raw
// words live longer: FP16/FP16/12 then needs 150 VGPRs instead of 114
// (3 instead of 4 waves per SIMD) and its hop runs 8 % slower.  The 18-real
// formats measured no gain from it.
template <int SP, int LP, bool L12> constexpr bool hop_pin_f16() { return L12; }

template <class V> __device__ __forceinline__ void pin_values(V* v, int n) {
#pragma unroll
    for (int k = 0; k < n; ++k) asm volatile("" : "+v"(v[k].x), "+v"(v[k].y));
}

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
    const uint8_t* z;       // second addend (with y only) or null
    double cy;              // coefficient of y
    // fused dot with the output (needs partial; kernels built with DOT only):
    // dmode 1: <dw, out>, 2: <out, y>; real and imaginary partials per 64
    // sites into pdre, pdim
    int dmode;
    const uint8_t* dw;
    double* pdre;
    double* pdim;
    double alpha;
    double* partial;
    size_t spinor_bytes;    // bytes of one packed spinor field
    size_t link_block;      // bytes of one (mu, parity) link block
    Sched sched;            // workgroup -> sites order
};

// Epilogue of a hop with addends: acc = alpha acc + cy y (+ z) for rhs r at
// site ih (cy = 1 rounds exactly as a plain axpy).
template <int SP, class C>
__device__ __forceinline__ void hop_addends(const HopParams& P, size_t r, uint32_t ih, C* acc) {
    using R = decltype(C().x);
    C yv[12];
    load_rec<SP, 12>(P.y + r * P.spinor_bytes, P.g.vh, ih, yv);
    const R a = (R)P.alpha, c = (R)P.cy;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        acc[k].x = fma(a, acc[k].x, c * yv[k].x);
        acc[k].y = fma(a, acc[k].y, c * yv[k].y);
    }
    if (P.z) {
        C zv[12];
        load_rec<SP, 12>(P.z + r * P.spinor_bytes, P.g.vh, ih, zv);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            acc[k].x += zv[k].x;
            acc[k].y += zv[k].y;
        }
    }
}

// Per-lane contributions of the output record acc (rhs r, site ih) to the
// fused reductions, taken on the value as stored (rounded to SP): ||out||^2
// and, with P.dmode, the complex dot <dw, out> = sum conj(dw) out (1) or
// <out, y> = sum conj(out) y (2).
// DOT is a compile-time switch: the dot code costs registers even when not
// taken, which pushed the link-resident kernels to a lower occupancy.
template <int SP, bool DOT = false, class C>
__device__ __forceinline__ void hop_reduce(const HopParams& P, size_t r, uint32_t ih, const C* acc, double& nrm,
                                           double& dre, double& dim) {
    C st[12];
    if constexpr (SP == P_F64 || SP == P_F32) {
#pragma unroll
        for (int k = 0; k < 12; ++k) st[k] = acc[k];
    } else {
        round_rec<SP, 12>(acc, st);
    }
#pragma unroll
    for (int k = 0; k < 12; ++k) nrm += (double)st[k].x * (double)st[k].x + (double)st[k].y * (double)st[k].y;
    if constexpr (DOT) {
        C w[12];
        load_rec<SP, 12>((P.dmode == 1 ? P.dw : P.y) + r * P.spinor_bytes, P.g.vh, ih, w);
        const double sg = P.dmode == 1 ? 1.0 : -1.0;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            const double ox = st[k].x, oy = st[k].y, wx = w[k].x, wy = w[k].y;
            dre += ox * wx + oy * wy;
            dim += sg * (wx * oy - wy * ox);
        }
    }
}

// The wavefront's sums of hop_reduce for rhs r into the partial arrays (one
// entry per 64 sites); every lane of the wavefront calls it.
template <bool DOT = false>
__device__ __forceinline__ void hop_partials_out(const HopParams& P, size_t r, uint32_t chunk, uint32_t nchunk,
                                                 bool lead, double nrm, double dre, double dim) {
    const double t = wave_sum64(nrm);
    if (lead && chunk < nchunk) P.partial[r * nchunk + chunk] = t;
    if constexpr (DOT) {
        const double a = wave_sum64(dre), b = wave_sum64(dim);
        if (lead && chunk < nchunk) {
            P.pdre[r * nchunk + chunk] = a;
            P.pdim[r * nchunk + chunk] = b;
        }
    }
}

// Link U as 9 complex numbers (row-major); a 12-real record is completed with
// row 2 = conj(row0 x row1), exact for det U = 1.
template <int LP, bool L12, bool NT = false, class C>
__device__ __forceinline__ void load_link(const uint8_t* base, uint32_t n, uint32_t i, C* u) {
    if constexpr (L12) {
        load_rec<LP, 6, NT>(base, n, i, u);
        u[6] = conj_(sub(mul(u[1], u[5]), mul(u[2], u[4])));
        u[7] = conj_(sub(mul(u[2], u[3]), mul(u[0], u[5])));
        u[8] = conj_(sub(mul(u[0], u[4]), mul(u[1], u[3])));
    } else {
        load_rec<LP, 9, NT>(base, n, i, u);
    }
}

// Link record of a precision possibly narrower than the arithmetic type.
template <int LP, bool L12, bool NT, class C>
__device__ __forceinline__ void load_link_as(const uint8_t* base, uint32_t n, uint32_t i, C* u) {
    using LR = typename St<LP>::real;
    if constexpr (sizeof(LR) == sizeof(decltype(C().x))) {
        load_link<LP, L12, NT>(base, n, i, u);
    } else {
        cx<LR> w[9];
        load_link<LP, L12, NT>(base, n, i, w);
#pragma unroll
        for (int k = 0; k < 9; ++k) { u[k].x = w[k].x; u[k].y = w[k].y; }
    }
}

// One direction: project with (1 - S gamma_mu), boundary phase (complex when
// CPH, else real), multiply by U (FWD) or U^dag (!FWD), reconstruct and
// accumulate.
template <int MU, int S, bool FWD, bool CPH, class C, bool APPLY_PHASE = true>
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
    // Boundary phase: applied without a branch, so that the loads of the
    // next neighbours can be scheduled ahead of this arithmetic.  (Callers
    // that fold the phase into the link pass APPLY_PHASE = false.)
    if constexpr (!APPLY_PHASE) {
    } else if constexpr (CPH) {
        const C ph = edge ? phase : mk<C>(1, 0);
#pragma unroll
        for (int c = 0; c < 3; ++c) { h0[c] = mul(ph, h0[c]); h1[c] = mul(ph, h1[c]); }
    } else {
        const auto sg = edge ? phase.x : decltype(phase.x)(1);
#pragma unroll
        for (int c = 0; c < 3; ++c) { h0[c] = scal(sg, h0[c]); h1[c] = scal(sg, h1[c]); }
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
template <int SP, int LP, bool L12, bool DAG, bool CPH, int MU, class C>
__device__ __forceinline__ void hop_mu(const HopParams& P, const uint8_t* in, const Nbr& nb,
                                       uint32_t ih, C* acc) {
    constexpr int SF = DAG ? -1 : 1;      // forward term: (1 - SF gamma)
    const uint32_t n = P.g.vh;
    C phase;
    phase.x = (decltype(C().x))P.ph[MU][0];
    phase.y = (decltype(C().x))P.ph[MU][1];
    {
        C u[9], p[12];
        load_link_as<LP, L12, hop_nt<SP>()>(P.u + (size_t)(2 * MU + P.out_par) * P.link_block, n, ih, u);
        load_rec<SP, 12>(in, n, nb.i[2 * MU], p);
        hop_dir<MU, SF, true, CPH>(p, u, nb.edge[2 * MU], phase, acc);
    }
    {
        C u[9], p[12];
        const uint32_t j = nb.i[2 * MU + 1];
        load_link_as<LP, L12, hop_nt<SP>()>(P.u + (size_t)(2 * MU + 1 - P.out_par) * P.link_block, n, j, u);
        load_rec<SP, 12>(in, n, j, p);
        hop_dir<MU, -SF, false, CPH>(p, u, nb.edge[2 * MU + 1], conj_(phase), acc);
    }
}

// ---- pipelined form ---------------------------------------------------------
// Neighbour k = 2 mu + (0: forward x + mu, 1: backward x - mu).
template <int SP, int LP, bool L12>
struct NbrRaw {
    RawRec<SP, 12> sp;
    RawRec<LP, L12 ? 6 : 9, hop_nt<SP>()> ln;
};

template <int SP, int LP, bool L12, int K>
__device__ __forceinline__ void issue(const HopParams& P, const uint8_t* in, const Nbr& nb, uint32_t ih,
                                      NbrRaw<SP, LP, L12>& r) {
    constexpr int MU = K / 2;
    const uint32_t n = P.g.vh;
    if constexpr ((K & 1) == 0) {
        r.ln.load(P.u + (size_t)(2 * MU + P.out_par) * P.link_block, n, ih);
    } else {
        r.ln.load(P.u + (size_t)(2 * MU + 1 - P.out_par) * P.link_block, n, nb.i[K]);
    }
    r.sp.load(in, n, nb.i[K]);
}

template <int SP, int LP, bool L12, bool DAG, bool CPH, int K, class C>
__device__ __forceinline__ void consume(const HopParams& P, const Nbr& nb, const NbrRaw<SP, LP, L12>& r,
                                        C* acc) {
    constexpr int MU = K / 2;
    constexpr int SF = DAG ? -1 : 1;
    using R = decltype(C().x);
    C p[12], u[9];
    r.sp.unpack(p);
    if constexpr (hop_pin_f16<SP, LP, L12>() && SP == P_F16) pin_values(p, 12);
    {
        using LR = typename St<LP>::real;
        cx<LR> w[9];
        r.ln.unpack(w);
        if constexpr (hop_pin_f16<SP, LP, L12>() && LP == P_F16) pin_values(w, L12 ? 6 : 9);
#pragma unroll
        for (int k = 0; k < (L12 ? 6 : 9); ++k) { u[k].x = (R)w[k].x; u[k].y = (R)w[k].y; }
        if constexpr (L12) {
            u[6] = conj_(sub(mul(u[1], u[5]), mul(u[2], u[4])));
            u[7] = conj_(sub(mul(u[2], u[3]), mul(u[0], u[5])));
            u[8] = conj_(sub(mul(u[0], u[4]), mul(u[1], u[3])));
        }
    }
    C phase;
    phase.x = (R)P.ph[MU][0];
    phase.y = (R)P.ph[MU][1];
    if constexpr ((K & 1) == 0) hop_dir<MU, SF, true, CPH>(p, u, nb.edge[K], phase, acc);
    else hop_dir<MU, -SF, false, CPH>(p, u, nb.edge[K], conj_(phase), acc);
}

template <int SP, int LP, bool L12, bool DAG, bool CPH, int D, int K, class C>
__device__ __forceinline__ void pipe_step(const HopParams& P, const uint8_t* in, const Nbr& nb, uint32_t ih,
                                          NbrRaw<SP, LP, L12> (&ring)[D + 1], C* acc) {
    if constexpr (K + D < 8) issue<SP, LP, L12, K + D>(P, in, nb, ih, ring[(K + D) % (D + 1)]);
    __builtin_amdgcn_sched_barrier(0);
    consume<SP, LP, L12, DAG, CPH, K>(P, nb, ring[K % (D + 1)], acc);
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (K + 1 < 8) pipe_step<SP, LP, L12, DAG, CPH, D, K + 1>(P, in, nb, ih, ring, acc);
}

template <int SP, int LP, bool L12, bool DAG, bool CPH, int D, int K = 0>
__device__ __forceinline__ void pipe_prologue(const HopParams& P, const uint8_t* in, const Nbr& nb, uint32_t ih,
                                              NbrRaw<SP, LP, L12> (&ring)[D + 1]) {
    if constexpr (K < D) {
        issue<SP, LP, L12, K>(P, in, nb, ih, ring[K]);
        pipe_prologue<SP, LP, L12, DAG, CPH, D, K + 1>(P, in, nb, ih, ring);
    }
}

}  // namespace weo
