// Multi right-hand-side hopping kernel and its autotuner.
//
// A lane owns one output site and a group of NR right-hand sides: each link
// is loaded once and applied to NR spinors, so for 12 right-hand sides the
// link traffic falls by NR compared with 12 single-rhs launches; the NR
// spinor loads per neighbour also give each lane more independent memory
// requests in flight.  The boundary phase is folded into the link once per
// neighbour ((ph U) h forward, (ph U)^dag h = conj(ph) U^dag h backward)
// instead of into NR half spinors.
//
// Workgroups are blockDim.x sites (a multiple of 64) by blockDim.y groups of
// NR rhs (at most 256 lanes), further groups in grid rows; each wavefront
// therefore has one rhs group, and the groups of one workgroup share their
// links through the caches.  Optionally the grid is
// persistent (a multiple of 8 workgroups looping over site blocks), with the
// same XCD-contiguous block order as the single-rhs kernel.
//
// The launch shape (NR, sites per workgroup, persistence) is picked per
// (lattice, format, nrhs) by timing every candidate on the first call with
// that key on the caller's stream and buffers (one stream synchronisation),
// then cached for the life of the process.  The candidates also cover the
// workgroup schedule (z-strips of 2, 4 or 8 planes, make_sched), which keeps
// the +-t neighbours of 12 fields inside L2.  WEO_TUNE=0 in the environment
// disables the search and uses NR = 3, 64 sites, no persistence;
// WILSON_EO_TUNE_CACHE=<file> keeps the tuned shapes across processes.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "hop_core.h"

namespace weo {

// The LDS-staged form (k_hop_lw) in MrhsCfg::nr (MrhsCfg::s then holds the
// wavefronts per workgroup).
constexpr int kNrLw = -5;
// Output records of the multi-RHS kernels are written with streaming stores
// in every precision: with many fields per site the output lines would
// otherwise take L2 from the input records that the +-z and +-t neighbours
// read again (FP32/18 and FP16/12 at 12 rhs: 4 % faster).  -D
// WEO_MRHS_NT_STORE=0 restores regular stores for comparison.
#ifdef WEO_MRHS_NT_STORE
template <int SP> constexpr bool mrhs_nt_store() { return WEO_MRHS_NT_STORE != 0; }
#else
template <int SP> constexpr bool mrhs_nt_store() { return true; }
#endif
#ifndef LW_CROSS
#define LW_CROSS (SP != P_F64)
#endif

struct MrhsParams {
    HopParams h;
    int nrhs;
    uint32_t nblk;      // site blocks of blockDim.x sites
    int rhs_per_row;    // LDS-staged form: right-hand sides per grid row
};

// Raw words of one neighbour: its link and the NR spinor records.
template <int SP, int LP, bool L12, int NR>
struct MrhsRaw {
    RawRec<LP, L12 ? 6 : 9, hop_nt<SP>()> ln;
    RawRec<SP, 12> sp[NR];
};

template <int SP, int LP, bool L12, int NR, int K>
__device__ __forceinline__ void mrhs_issue(const MrhsParams& M, const Nbr& nb, uint32_t ih, int r0,
                                           MrhsRaw<SP, LP, L12, NR>& r) {
    constexpr int MU = K / 2;
    constexpr bool FWD = (K & 1) == 0;
    const HopParams& P = M.h;
    const uint32_t n = P.g.vh;
    r.ln.load(P.u + (size_t)(2 * MU + (FWD ? P.out_par : 1 - P.out_par)) * P.link_block, n,
              FWD ? ih : nb.i[K]);
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        // rhs beyond nrhs (last group) recompute the last one; never stored
        const int rr = r0 + q < M.nrhs ? r0 + q : M.nrhs - 1;
        r.sp[q].load(P.in + (size_t)rr * P.spinor_bytes, n, nb.i[K]);
    }
}

template <int SP, int LP, bool L12, bool DAG, int NR, int K, class C>
__device__ __forceinline__ void mrhs_consume(const MrhsParams& M, const Nbr& nb,
                                             const MrhsRaw<SP, LP, L12, NR>& r, C (&acc)[NR][12]) {
    constexpr int MU = K / 2;
    constexpr bool FWD = (K & 1) == 0;
    constexpr int SF = DAG ? -1 : 1;
    using R = decltype(C().x);
    const HopParams& P = M.h;
    C u[9];
    {
        cx<typename St<LP>::real> w[9];
        r.ln.unpack(w);
        if constexpr (hop_pin_f16<SP, LP, L12>() && LP == P_F16) pin_values(w, L12 ? 6 : 9);
#pragma unroll
        for (int k = 0; k < (L12 ? 6 : 9); ++k) { u[k].x = (R)w[k].x; u[k].y = (R)w[k].y; }
        if constexpr (L12) {
            u[6] = conj_(sub(mul(u[1], u[5]), mul(u[2], u[4])));
            u[7] = conj_(sub(mul(u[2], u[3]), mul(u[0], u[5])));
            u[8] = conj_(sub(mul(u[0], u[4]), mul(u[1], u[3])));
        }
        const C ph = nb.edge[K] ? mk<C>((R)P.ph[MU][0], (R)P.ph[MU][1]) : mk<C>(R(1), R(0));
#pragma unroll
        for (int k = 0; k < 9; ++k) u[k] = mul(ph, u[k]);
    }
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        C p[12];
        r.sp[q].unpack(p);
        if constexpr (hop_pin_f16<SP, LP, L12>() && SP == P_F16) pin_values(p, 12);
        hop_dir<MU, FWD ? SF : -SF, FWD, false, C, false>(p, u, false, C{}, acc[q]);
    }
}

// Prefetch depth: with D = 1 the next neighbour's words are loaded while this
// one is computed; for larger NR the doubled raw storage costs more
// occupancy than the overlap gains, so D = 0 (the NR + 1 records of one
// neighbour are still in flight together).
template <int SP, int NR> constexpr int mrhs_depth() {
    if constexpr (SP == P_F64) return 0;
    else if constexpr (SP == P_F32) return NR <= 2 ? 1 : 0;
    else return NR <= 3 ? 1 : 0;
}

template <int SP, int LP, bool L12, bool DAG, int NR, int D, int K, class C>
__device__ __forceinline__ void mrhs_step(const MrhsParams& M, const Nbr& nb, uint32_t ih, int r0,
                                          MrhsRaw<SP, LP, L12, NR> (&ring)[D + 1], C (&acc)[NR][12]) {
    if constexpr (D == 0) mrhs_issue<SP, LP, L12, NR, K>(M, nb, ih, r0, ring[0]);
    else if constexpr (K + 1 < 8) mrhs_issue<SP, LP, L12, NR, K + 1>(M, nb, ih, r0, ring[(K + 1) & 1]);
    __builtin_amdgcn_sched_barrier(0);
    mrhs_consume<SP, LP, L12, DAG, NR, K>(M, nb, ring[D == 0 ? 0 : (K & 1)], acc);
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (K + 1 < 8) mrhs_step<SP, LP, L12, DAG, NR, D, K + 1>(M, nb, ih, r0, ring, acc);
}

template <int SP, int LP, bool L12, bool DAG, int NR>
__global__ void __launch_bounds__(256) k_hop_mrhs(const MrhsParams M) {
    using R = typename Arith<SP>::R;
    using C = cx<R>;
    const HopParams& P = M.h;
    // the rhs group is uniform across a wavefront (blockDim.x is a multiple
    // of 64): keep it in a scalar register so that every spinor address is a
    // scalar base plus the lane's 32-bit offset
    const int r0 = __builtin_amdgcn_readfirstlane((int)(blockIdx.y * blockDim.y + threadIdx.y) * NR);
    const uint32_t S = blockDim.x;
    const uint32_t nchunk = (P.g.vh + 63) >> 6;
    for (uint32_t b = blockIdx.x; b < M.nblk; b += gridDim.x) {
        const uint32_t blk = xcd_block(b, M.nblk, P.remap);
        const uint32_t base = block_first_site(P.sched, P.g, blk, S);
        const uint32_t ih = base + threadIdx.x;
        double nrm[NR], dre[NR], dim[NR];
#pragma unroll
        for (int q = 0; q < NR; ++q) nrm[q] = dre[q] = dim[q] = 0.0;
        if (ih < P.g.vh && r0 < M.nrhs) {
            const Site s = decode(P.g, ih, P.out_par);
            const Nbr nb = neighbours(P.g, s);
            C acc[NR][12];
#pragma unroll
            for (int q = 0; q < NR; ++q)
#pragma unroll
                for (int k = 0; k < 12; ++k) acc[q][k] = czero<C>();
            constexpr int D = mrhs_depth<SP, NR>();
            MrhsRaw<SP, LP, L12, NR> ring[D + 1];
            if constexpr (D > 0) mrhs_issue<SP, LP, L12, NR, 0>(M, nb, ih, r0, ring[0]);
            mrhs_step<SP, LP, L12, DAG, NR, D, 0>(M, nb, ih, r0, ring, acc);
            // Pin the accumulators here: the epilogue below is conditional per
            // rhs, and without this the compiler sinks the whole accumulation
            // of the later rhs into those branches, keeping every partial
            // product live until the end.
#pragma unroll
            for (int q = 0; q < NR; ++q)
#pragma unroll
                for (int k = 0; k < 12; ++k) asm volatile("" : "+v"(acc[q][k].x), "+v"(acc[q][k].y));
#pragma unroll
            for (int q = 0; q < NR; ++q) {
                const int r = r0 + q;
                if (r < M.nrhs) {
                    if (P.y) hop_addends<SP>(P, (size_t)r, ih, acc[q]);
                    uint8_t* out = P.out + (size_t)r * P.spinor_bytes;
                    store_rec<SP, 12, C, mrhs_nt_store<SP>()>(out, P.g.vh, ih, acc[q]);
                    if (P.partial) hop_reduce<SP>(P, (size_t)r, ih, acc[q], nrm[q], dre[q], dim[q]);
                }
            }
        }
        if (P.partial) {
            const uint32_t chunk = (base + (threadIdx.x & ~63u)) >> 6;
#pragma unroll
            for (int q = 0; q < NR; ++q)
                if (r0 + q < M.nrhs)          // wave-uniform
                    hop_partials_out(P, (size_t)(r0 + q), chunk, nchunk, (threadIdx.x & 63) == 0, nrm[q], dre[q],
                                     dim[q]);
        }
    }
}

// ---- link-resident form -------------------------------------------------------
// One lane per site keeps the raw words of its 8 links in registers and
// walks the right-hand sides one after the other, so every link is read once
// per launch while each wavefront touches one spinor field at a time (the
// neighbour records stay in L2 as for a single right-hand side).  Built for
// FP32, FP16 and BF16 spinors (FP64 links would not fit the register file).
template <class RR> __device__ __forceinline__ void lr_pin(RR& r) {
    constexpr int NW = sizeof(r.w) / sizeof(uint4);
#pragma unroll
    for (int p = 0; p < NW; ++p) asm volatile("" : "+v"(r.w[p].x), "+v"(r.w[p].y), "+v"(r.w[p].z), "+v"(r.w[p].w));
    asm volatile("" : "+v"(r.t8.x), "+v"(r.t8.y), "+v"(r.t4));
}

template <int SP, int LP, bool L12, bool DAG, bool CPH, int K, class C>
__device__ __forceinline__ void lr_consume(const HopParams& P, const Nbr& nb,
                                           const RawRec<LP, L12 ? 6 : 9, hop_nt<SP>()>& ln,
                                           const RawRec<SP, 12>& sp, C* acc) {
    constexpr int MU = K / 2;
    constexpr int SF = DAG ? -1 : 1;
    using R = decltype(C().x);
    C p[12], u[9];
    sp.unpack(p);
    if constexpr (hop_pin_f16<SP, LP, L12>() && SP == P_F16) pin_values(p, 12);
    {
        cx<typename St<LP>::real> w[9];
        ln.unpack(w);
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

// Neighbour records flow through a ring of D+1 slots (D+1 divides 8, so a
// direction always lands in the same slot); the last D directions of one
// right-hand side prefetch the first D records of the next.
template <int SP, int LP, bool L12, bool DAG, bool CPH, int D, int K, class C>
__device__ __forceinline__ void lr_step(const HopParams& P, const uint8_t* in, const uint8_t* in_next,
                                        const Nbr& nb,
                                        const RawRec<LP, L12 ? 6 : 9, hop_nt<SP>()> (&lk)[8],
                                        RawRec<SP, 12> (&ring)[D + 1], C* acc) {
    if constexpr (K + D < 8) ring[(K + D) % (D + 1)].load(in, P.g.vh, nb.i[K + D]);
    else ring[(K + D) % (D + 1)].load(in_next, P.g.vh, nb.i[K + D - 8]);
    __builtin_amdgcn_sched_barrier(0);
    lr_consume<SP, LP, L12, DAG, CPH, K>(P, nb, lk[K], ring[K % (D + 1)], acc);
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (K + 1 < 8) lr_step<SP, LP, L12, DAG, CPH, D, K + 1>(P, in, in_next, nb, lk, ring, acc);
}

template <int SP, int LP, bool L12, bool DAG, bool CPH, int D>
__global__ void __launch_bounds__(256) k_hop_lr(const MrhsParams M) {
    static_assert(8 % (D + 1) == 0, "ring size must divide the 8 directions");
    using R = typename Arith<SP>::R;
    using C = cx<R>;
    const HopParams& P = M.h;
    const uint32_t S = blockDim.x;
    const uint32_t n = P.g.vh;
    const uint32_t nchunk = (n + 63) >> 6;
    for (uint32_t b = blockIdx.x; b < M.nblk; b += gridDim.x) {
        const uint32_t blk = xcd_block(b, M.nblk, P.remap);
        const uint32_t base = block_first_site(P.sched, P.g, blk, S);
        const uint32_t ih = base + threadIdx.x;
        const bool valid = ih < n;
        Nbr nb;
        RawRec<LP, L12 ? 6 : 9, hop_nt<SP>()> lk[8];
        RawRec<SP, 12> ring[D + 1];
        if (valid) {
            const Site s = decode(P.g, ih, P.out_par);
            nb = neighbours(P.g, s);
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int mu = k >> 1;
                const bool fwd = (k & 1) == 0;
                lk[k].load(P.u + (size_t)(2 * mu + (fwd ? P.out_par : 1 - P.out_par)) * P.link_block, n,
                           fwd ? ih : nb.i[k]);
            }
#pragma unroll
            for (int k = 0; k < D; ++k) ring[k].load(P.in, n, nb.i[k]);
        }
        for (int r = 0; r < M.nrhs; ++r) {
            double nrm = 0.0, dre = 0.0, dim = 0.0;
            if (valid) {
                // keep the links as raw words across the loop: without this the
                // compiler hoists their conversion out of it and spills
#pragma unroll
                for (int k = 0; k < 8; ++k) lr_pin(lk[k]);
                const uint8_t* in = P.in + (size_t)r * P.spinor_bytes;
                // after the last right-hand side the prefetch re-reads this one
                // (cache hits, no branch inside the unrolled directions)
                const uint8_t* in_next = r + 1 < M.nrhs ? in + P.spinor_bytes : in;
                C acc[12];
#pragma unroll
                for (int k = 0; k < 12; ++k) acc[k] = czero<C>();
                lr_step<SP, LP, L12, DAG, CPH, D, 0>(P, in, in_next, nb, lk, ring, acc);
                if (P.y) hop_addends<SP>(P, (size_t)r, ih, acc);
                store_rec<SP, 12, C, mrhs_nt_store<SP>()>(P.out + (size_t)r * P.spinor_bytes, n, ih, acc);
                if (P.partial) hop_reduce<SP>(P, (size_t)r, ih, acc, nrm, dre, dim);
            }
            if (P.partial)
                hop_partials_out(P, (size_t)r, (base + (threadIdx.x & ~63u)) >> 6, nchunk, (threadIdx.x & 63) == 0, nrm,
                                 dre, dim);
        }
    }
}

// ---- links staged in LDS, right-hand sides across wavefronts --------------------
// A workgroup of W wavefronts owns 64 output sites.  The wavefronts first
// copy the raw words of the 64 sites' 8 links from memory into LDS (each
// wavefront some of the directions), then each walks its own right-hand
// sides (w, w + W, ...) with the single-rhs pipeline, taking the links from
// LDS.  Every link is read from memory once per launch, as in the
// link-resident form, but the links occupy LDS shared by W wavefronts
// instead of registers of each lane, so the register footprint is the
// single-rhs kernel's: this is the form that exists for FP64 (whose 8 links
// do not fit a lane's registers next to its pipeline), and a candidate for
// the other formats.  LDS holds the links as [direction][16-byte slot][site]
// (a tail of 4 or 8 bytes takes a whole slot), so the 64 lanes of a read
// touch 1 KiB of consecutive words.
template <int SP, int LP, bool L12> struct LwShape {
    using LRaw = RawRec<LP, L12 ? 6 : 9, hop_nt<SP>()>;
    static constexpr int NC = Rec<LP, L12 ? 6 : 9>::NFULL;
    static constexpr int TB = Rec<LP, L12 ? 6 : 9>::TAILB;
    static constexpr int NS = NC + (TB ? 1 : 0);     // 16-byte slots per link
    static constexpr int LDS_U4 = 8 * NS * 64;
};

template <int SP, int LP, bool L12>
__device__ __forceinline__ void lw_put(uint4* lds, int k, uint32_t lane,
                                       const typename LwShape<SP, LP, L12>::LRaw& r) {
    using Sh = LwShape<SP, LP, L12>;
#pragma unroll
    for (int p = 0; p < Sh::NC; ++p) lds[(k * Sh::NS + p) * 64 + lane] = r.w[p];
    if constexpr (Sh::TB == 8) lds[(k * Sh::NS + Sh::NC) * 64 + lane] = make_uint4(r.t8.x, r.t8.y, 0u, 0u);
    if constexpr (Sh::TB == 4) lds[(k * Sh::NS + Sh::NC) * 64 + lane] = make_uint4(r.t4, 0u, 0u, 0u);
}

template <int SP, int LP, bool L12>
__device__ __forceinline__ void lw_get(const uint4* lds, int k, uint32_t lane,
                                       typename LwShape<SP, LP, L12>::LRaw& r) {
    using Sh = LwShape<SP, LP, L12>;
#pragma unroll
    for (int p = 0; p < Sh::NC; ++p) r.w[p] = lds[(k * Sh::NS + p) * 64 + lane];
    if constexpr (Sh::TB == 8) {
        const uint4 v = lds[(k * Sh::NS + Sh::NC) * 64 + lane];
        r.t8 = make_uint2(v.x, v.y);
    }
    if constexpr (Sh::TB == 4) r.t4 = lds[(k * Sh::NS + Sh::NC) * 64 + lane].x;
}

template <int SP> constexpr int lw_depth() { return 1; }
// Most wavefronts per workgroup: FP64 keeps the single-rhs register budget
// (256 VGPRs, as the FP64 single-rhs hop), so at most 4; FP32 fits 3 waves
// per SIMD at up to 12; FP16 / BF16 at up to 8 (12 spills a little).
template <int SP> constexpr int lw_maxw() { return SP == P_F64 ? 4 : (SP == P_F32 ? 12 : 8); }
// Prefetch of the next right-hand side's first records across the epilogue
// (off for FP64: its records held through the epilogue spill).
template <int SP> constexpr bool lw_cross() { return LW_CROSS; }

template <int SP, int LP, bool L12> struct LwSlot {
    RawRec<SP, 12> sp;
    typename LwShape<SP, LP, L12>::LRaw ln;
};

// Ring of D+1 slots as in the link-resident form: the neighbour record and
// the link words of direction K + D are fetched while direction K is
// computed; the last D directions of one right-hand side fetch the first
// records of the next.
template <int SP, int LP, bool L12, bool DAG, bool CPH, int D, int K, class C>
__device__ __forceinline__ void lw_step(const HopParams& P, const uint4* lds, uint32_t lane, const uint8_t* in,
                                        const uint8_t* in_next, const Nbr& nb, LwSlot<SP, LP, L12> (&ring)[D + 1],
                                        C* acc) {
    constexpr int KN = (K + D) & 7;
    if constexpr (K + D < 8 || lw_cross<SP>()) {
        LwSlot<SP, LP, L12>& nx = ring[(K + D) % (D + 1)];
        nx.sp.load(K + D < 8 ? in : in_next, P.g.vh, nb.i[KN]);
        lw_get<SP, LP, L12>(lds, KN, lane, nx.ln);
    }
    __builtin_amdgcn_sched_barrier(0);
    lr_consume<SP, LP, L12, DAG, CPH, K>(P, nb, ring[K % (D + 1)].ln, ring[K % (D + 1)].sp, acc);
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (K + 1 < 8) lw_step<SP, LP, L12, DAG, CPH, D, K + 1>(P, lds, lane, in, in_next, nb, ring, acc);
}


template <int SP, int LP, bool L12, bool DAG, bool CPH, bool DOT>
__global__ void __launch_bounds__(64 * lw_maxw<SP>()) k_hop_lw(const MrhsParams M) {
    using R = typename Arith<SP>::R;
    using C = cx<R>;
    using Sh = LwShape<SP, LP, L12>;
    constexpr int D = lw_depth<SP>();
    __shared__ uint4 lds[Sh::LDS_U4];
    const HopParams& P = M.h;
    const uint32_t n = P.g.vh;
    const uint32_t nchunk = (n + 63) >> 6;
    const uint32_t lane = threadIdx.x;                    // blockDim.x == 64
    const int wv = __builtin_amdgcn_readfirstlane((int)threadIdx.y);
    const int W = (int)blockDim.y;
    // this grid row's right-hand sides [r0, r1): rows are separate sweeps
    const int r0 = (int)blockIdx.y * M.rhs_per_row;
    const int r1 = r0 + M.rhs_per_row < M.nrhs ? r0 + M.rhs_per_row : M.nrhs;
    for (uint32_t b = blockIdx.x; b < M.nblk; b += gridDim.x) {
        const uint32_t blk = xcd_block(b, M.nblk, P.remap);
        const uint32_t base = block_first_site(P.sched, P.g, blk, 64);
        const uint32_t ih = base + lane;
        const bool valid = ih < n;
        Nbr nb;
        if (valid) nb = neighbours(P.g, decode(P.g, ih, P.out_par));
        __syncthreads();                                  // the previous block's links are consumed
        if (valid) {
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                if (k % W != wv) continue;                // wave-uniform
                const int mu = k >> 1;
                const bool fwd = (k & 1) == 0;
                typename Sh::LRaw r;
                r.load(P.u + (size_t)(2 * mu + (fwd ? P.out_par : 1 - P.out_par)) * P.link_block, n,
                       fwd ? ih : nb.i[k]);
                lw_put<SP, LP, L12>(lds, k, lane, r);
            }
        }
        __syncthreads();
        LwSlot<SP, LP, L12> ring[D + 1];
        if (lw_cross<SP>() && valid && r0 + wv < r1) {
            const uint8_t* in0 = P.in + (size_t)(r0 + wv) * P.spinor_bytes;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                ring[k].sp.load(in0, n, nb.i[k]);
                lw_get<SP, LP, L12>(lds, k, lane, ring[k].ln);
            }
        }
        for (int r = r0 + wv; r < r1; r += W) {
            double nrm = 0.0, dre = 0.0, dim = 0.0;
            if (valid) {
                const uint8_t* in = P.in + (size_t)r * P.spinor_bytes;
                if constexpr (!lw_cross<SP>()) {
#pragma unroll
                    for (int k = 0; k < D; ++k) {
                        ring[k].sp.load(in, n, nb.i[k]);
                        lw_get<SP, LP, L12>(lds, k, lane, ring[k].ln);
                    }
                }
                const uint8_t* in_next = r + W < r1 ? in + (size_t)W * P.spinor_bytes : in;
                // an opaque copy of the lane index per right-hand side: the LDS
                // link words are invariant in this loop, and without it the
                // compiler hoists all 8 links' reads out of it into registers
                uint32_t lo = lane;
                asm volatile("" : "+v"(lo));
                C acc[12];
#pragma unroll
                for (int k = 0; k < 12; ++k) acc[k] = czero<C>();
                lw_step<SP, LP, L12, DAG, CPH, D, 0>(P, lds, lo, in, in_next, nb, ring, acc);
                if (P.y) hop_addends<SP>(P, (size_t)r, ih, acc);
                store_rec<SP, 12, C, mrhs_nt_store<SP>()>(P.out + (size_t)r * P.spinor_bytes, n, ih, acc);
                if (P.partial) hop_reduce<SP, DOT>(P, (size_t)r, ih, acc, nrm, dre, dim);
            }
            if (P.partial) hop_partials_out<DOT>(P, (size_t)r, base >> 6, nchunk, lane == 0, nrm, dre, dim);
        }
    }
}

// ---- link-resident form on packed FP16 pairs (FP16 spinors and links) --------
// The FP32 form above converts every FP16 word it reads (8 links and 8
// neighbour records per site and right-hand side) and spends 4 FP32
// instructions per complex multiply-add; measured, it issues VALU work on
// about 90 % of the cycles, so arithmetic, not memory, bounds it.  Here the
// values stay FP16 pairs (re, im) where they are read: the spin projection
// is one packed FP16 add per complex number, and the SU(3) products are
// v_dot2_f32_f16 (two FP16 products summed into an FP32 accumulator), two
// per complex multiply-add:
//     (U h).re = dot2((U.re, U.im), (h.re, -h.im)),  (U h).im = dot2(U, (h.im, h.re))
//     (U^dag h).re = dot2(U, h),                      (U^dag h).im = dot2(U, (h.im, -h.re))
// with accumulation and the reconstruction in FP32.  A site's 8 links are
// kept as 9 FP16 pairs each (a 12-real link's third row rebuilt once per
// site in FP32 and rounded to FP16; boundary phases folded in once per
// site).  The projected half spinor and the rebuilt row are rounded to FP16
// (relative 2^-11, the storage precision of the inputs); products and sums
// are FP32.
typedef _Float16 h2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ h2v h2v_of(uint32_t w) { return __builtin_bit_cast(h2v, w); }
__device__ __forceinline__ uint32_t u32_of(h2v v) { return __builtin_bit_cast(uint32_t, v); }
__device__ __forceinline__ float dot2(uint32_t a, uint32_t b, float c) {
    return __builtin_amdgcn_fdot2(h2v_of(a), h2v_of(b), c, false);
}
__device__ __forceinline__ uint32_t swap_pair(uint32_t w) { return __builtin_amdgcn_alignbit(w, w, 16); }

struct Link16 {
    uint32_t e[9];       // U_ab as FP16 pairs, row-major
};

// Link of direction k of the site (raw FP16 words), third row rebuilt for
// 12 reals, boundary phase ph folded in on edge hops (ph U forward,
// (ph U)^dag = conj(ph) U^dag backward, so the stored link is ph U either way).
template <bool L12, bool CPH>
__device__ __forceinline__ void link16_load(const uint8_t* base, uint32_t n, uint32_t i, bool edge, float2 ph,
                                            Link16& L) {
    RawRec<P_F16, L12 ? 6 : 9, true> r;
    r.load(base, n, i);
    constexpr int NW = L12 ? 6 : 9;
    uint32_t w[9];
#pragma unroll
    for (int p = 0; p < Rec<P_F16, NW>::NFULL; ++p) {
        w[4 * p] = r.w[p].x; w[4 * p + 1] = r.w[p].y; w[4 * p + 2] = r.w[p].z; w[4 * p + 3] = r.w[p].w;
    }
    if constexpr (Rec<P_F16, NW>::TAILB == 8) { w[4 * Rec<P_F16, NW>::NFULL] = r.t8.x; w[4 * Rec<P_F16, NW>::NFULL + 1] = r.t8.y; }
    if constexpr (Rec<P_F16, NW>::TAILB == 4) w[4 * Rec<P_F16, NW>::NFULL] = r.t4;
    if constexpr (L12) {
        float2 u[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) u[k] = h2_to_f2(w[k]);
        w[6] = f2_to_h2(conj_(sub(mul(u[1], u[5]), mul(u[2], u[4]))));
        w[7] = f2_to_h2(conj_(sub(mul(u[2], u[3]), mul(u[0], u[5]))));
        w[8] = f2_to_h2(conj_(sub(mul(u[0], u[4]), mul(u[1], u[3]))));
    }
    if constexpr (CPH) {
        const float2 f = edge ? ph : make_float2(1.f, 0.f);
#pragma unroll
        for (int k = 0; k < 9; ++k) L.e[k] = f2_to_h2(mul(f, h2_to_f2(w[k])));
    } else {
        // a real phase +-1: a sign flip of both halves where it is -1
        const uint32_t flip = (edge && ph.x < 0.f) ? 0x80008000u : 0u;
#pragma unroll
        for (int k = 0; k < 9; ++k) L.e[k] = w[k] ^ flip;
    }
}

// One direction on a neighbour record p (12 FP16 pairs, [spin][colour]):
// project with (1 - S gamma_mu), multiply by U (FWD) or U^dag, rebuild and
// accumulate in FP32 (the rules of hop_dir).
template <int MU, int S, bool FWD>
__device__ __forceinline__ void h16_dir(const uint32_t* p, const Link16& L, float2* acc) {
    uint32_t h[2][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const h2v p0 = h2v_of(p[c]), p1 = h2v_of(p[3 + c]), p2 = h2v_of(p[6 + c]), p3 = h2v_of(p[9 + c]);
        h2v h0, h1;
        if constexpr (MU == 0) {
            const h2v i3 = h2v{-p3.y, p3.x}, i2 = h2v{-p2.y, p2.x};
            h0 = S > 0 ? p0 + i3 : p0 - i3;
            h1 = S > 0 ? p1 + i2 : p1 - i2;
        } else if constexpr (MU == 1) {
            h0 = S > 0 ? p0 + p3 : p0 - p3;
            h1 = S > 0 ? p1 - p2 : p1 + p2;
        } else if constexpr (MU == 2) {
            const h2v i2 = h2v{-p2.y, p2.x}, i3 = h2v{-p3.y, p3.x};
            h0 = S > 0 ? p0 + i2 : p0 - i2;
            h1 = S > 0 ? p1 - i3 : p1 + i3;
        } else {
            h0 = S > 0 ? p2 : p0;
            h1 = S > 0 ? p3 : p1;
        }
        h[0][c] = u32_of(h0);
        h[1][c] = u32_of(h1);
    }
    float2 g[2][3];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        uint32_t ha[3], hb[3];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            if constexpr (FWD) {
                ha[b] = h[s][b] ^ 0x80000000u;                    // (h.re, -h.im)
                hb[b] = swap_pair(h[s][b]);                       // (h.im, h.re)
            } else {
                ha[b] = h[s][b];                                  // (h.re, h.im)
                hb[b] = swap_pair(h[s][b]) ^ 0x80000000u;         // (h.im, -h.re)
            }
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            float re = 0.f, im = 0.f;
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const uint32_t u = FWD ? L.e[3 * a + b] : L.e[3 * b + a];
                re = dot2(u, ha[b], re);
                im = dot2(u, hb[b], im);
            }
            g[s][a] = make_float2(re, im);
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float2 g0 = g[0][a], g1 = g[1][a];
        if constexpr (MU == 3) {
            const int o = S > 0 ? 6 : 0;
            acc[o + a].x = fmaf(2.f, g0.x, acc[o + a].x); acc[o + a].y = fmaf(2.f, g0.y, acc[o + a].y);
            acc[o + 3 + a].x = fmaf(2.f, g1.x, acc[o + 3 + a].x); acc[o + 3 + a].y = fmaf(2.f, g1.y, acc[o + 3 + a].y);
        } else {
            acc[a] = add(acc[a], g0);
            acc[3 + a] = add(acc[3 + a], g1);
            if constexpr (MU == 0) {
                acc[6 + a] = S > 0 ? sub(acc[6 + a], imul(g1)) : add(acc[6 + a], imul(g1));
                acc[9 + a] = S > 0 ? sub(acc[9 + a], imul(g0)) : add(acc[9 + a], imul(g0));
            } else if constexpr (MU == 1) {
                acc[6 + a] = S > 0 ? sub(acc[6 + a], g1) : add(acc[6 + a], g1);
                acc[9 + a] = S > 0 ? add(acc[9 + a], g0) : sub(acc[9 + a], g0);
            } else {
                acc[6 + a] = S > 0 ? sub(acc[6 + a], imul(g0)) : add(acc[6 + a], imul(g0));
                acc[9 + a] = S > 0 ? add(acc[9 + a], imul(g1)) : sub(acc[9 + a], imul(g1));
            }
        }
    }
}

__device__ __forceinline__ void rec16_words(const RawRec<P_F16, 12>& r, uint32_t* p) {
#pragma unroll
    for (int q = 0; q < 3; ++q) { p[4 * q] = r.w[q].x; p[4 * q + 1] = r.w[q].y; p[4 * q + 2] = r.w[q].z; p[4 * q + 3] = r.w[q].w; }
}

template <bool DAG, int D, int K>
__device__ __forceinline__ void h16_step(const HopParams& P, const uint8_t* in, const uint8_t* in_next,
                                         const Nbr& nb, const Link16 (&lk)[8], RawRec<P_F16, 12> (&ring)[D + 1],
                                         float2* acc) {
    constexpr int MU = K / 2;
    constexpr int SF = DAG ? -1 : 1;
    if constexpr (K + D < 8) ring[(K + D) % (D + 1)].load(in, P.g.vh, nb.i[K + D]);
    else ring[(K + D) % (D + 1)].load(in_next, P.g.vh, nb.i[K + D - 8]);
    __builtin_amdgcn_sched_barrier(0);
    uint32_t p[12];
    rec16_words(ring[K % (D + 1)], p);
    if constexpr ((K & 1) == 0) h16_dir<MU, SF, true>(p, lk[K], acc);
    else h16_dir<MU, -SF, false>(p, lk[K], acc);
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (K + 1 < 8) h16_step<DAG, D, K + 1>(P, in, in_next, nb, lk, ring, acc);
}

template <bool L12, bool DAG, bool CPH, int D>
__global__ void __launch_bounds__(256) k_hop_lr16(const MrhsParams M) {
    static_assert(8 % (D + 1) == 0, "ring size must divide the 8 directions");
    const HopParams& P = M.h;
    const uint32_t S = blockDim.x;
    const uint32_t n = P.g.vh;
    const uint32_t nchunk = (n + 63) >> 6;
    for (uint32_t b = blockIdx.x; b < M.nblk; b += gridDim.x) {
        const uint32_t blk = xcd_block(b, M.nblk, P.remap);
        const uint32_t base = block_first_site(P.sched, P.g, blk, S);
        const uint32_t ih = base + threadIdx.x;
        const bool valid = ih < n;
        Nbr nb;
        Link16 lk[8];
        RawRec<P_F16, 12> ring[D + 1];
        if (valid) {
            const Site s = decode(P.g, ih, P.out_par);
            nb = neighbours(P.g, s);
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int mu = k >> 1;
                const bool fwd = (k & 1) == 0;
                // ph U for both hops: the backward one multiplies by (ph U)^dag
                const float2 ph = make_float2((float)P.ph[mu][0], (float)P.ph[mu][1]);
                link16_load<L12, CPH>(P.u + (size_t)(2 * mu + (fwd ? P.out_par : 1 - P.out_par)) * P.link_block, n,
                                      fwd ? ih : nb.i[k], nb.edge[k], ph, lk[k]);
            }
#pragma unroll
            for (int k = 0; k < D; ++k) ring[k].load(P.in, n, nb.i[k]);
        }
        for (int r = 0; r < M.nrhs; ++r) {
            double nrm = 0.0, dre = 0.0, dim = 0.0;
            if (valid) {
                // keep the link words as they are across the loop
#pragma unroll
                for (int k = 0; k < 8; ++k)
#pragma unroll
                    for (int e = 0; e < 9; ++e) asm volatile("" : "+v"(lk[k].e[e]));
                const uint8_t* in = P.in + (size_t)r * P.spinor_bytes;
                const uint8_t* in_next = r + 1 < M.nrhs ? in + P.spinor_bytes : in;
                float2 acc[12];
#pragma unroll
                for (int k = 0; k < 12; ++k) acc[k] = make_float2(0.f, 0.f);
                h16_step<DAG, D, 0>(P, in, in_next, nb, lk, ring, acc);
                if (P.y) hop_addends<P_F16>(P, (size_t)r, ih, acc);
                store_rec<P_F16, 12, float2, mrhs_nt_store<P_F16>()>(P.out + (size_t)r * P.spinor_bytes, n, ih, acc);
                if (P.partial) hop_reduce<P_F16>(P, (size_t)r, ih, acc, nrm, dre, dim);
            }
            if (P.partial)
                hop_partials_out(P, (size_t)r, (base + (threadIdx.x & ~63u)) >> 6, nchunk, (threadIdx.x & 63) == 0, nrm,
                                 dre, dim);
        }
    }
}

// ------------------------------------------------------------------ host ----
static HopParams hop_params(const HopLaunch& h) {
    HopParams P;
    P.g = h.g;
    P.out_par = h.out_par;
    P.remap = hop_tune().remap;
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
    return P;
}

template <int SP, int LP, bool L12, int NR>
static hipError_t mrhs_nr(const HopLaunch& h, const MrhsParams& M, dim3 grid, dim3 block, hipStream_t s) {
    if (h.dagger)
        hipLaunchKernelGGL((k_hop_mrhs<SP, LP, L12, true, NR>), grid, block, 0, s, M);
    else
        hipLaunchKernelGGL((k_hop_mrhs<SP, LP, L12, false, NR>), grid, block, 0, s, M);
    return hipGetLastError();
}

template <int SP, int LP, bool L12>
static hipError_t mrhs_fmt(const HopLaunch& h, const MrhsParams& M, int nr, dim3 grid, dim3 block,
                           hipStream_t s) {
    switch (nr) {
        case 2: return mrhs_nr<SP, LP, L12, 2>(h, M, grid, block, s);
        case 3: return mrhs_nr<SP, LP, L12, 3>(h, M, grid, block, s);
        default: break;
    }
    if constexpr (SP != P_F64) {
        switch (nr) {
            case 4: return mrhs_nr<SP, LP, L12, 4>(h, M, grid, block, s);
            case 6: return mrhs_nr<SP, LP, L12, 6>(h, M, grid, block, s);
            default: break;
        }
    }
    return hipErrorInvalidValue;
}

template <int SP, int LP, bool L12, int D>
static hipError_t lr_depth(const HopLaunch& h, const MrhsParams& M, dim3 grid, dim3 block, hipStream_t s) {
    bool cph = false;
    for (int m = 0; m < 4; ++m) cph = cph || h.phase[m][1] != 0.0;
#define WEO_LR(DG, CP) hipLaunchKernelGGL((k_hop_lr<SP, LP, L12, DG, CP, D>), grid, block, 0, s, M)
    if (h.dagger) { if (cph) WEO_LR(true, true); else WEO_LR(true, false); }
    else { if (cph) WEO_LR(false, true); else WEO_LR(false, false); }
#undef WEO_LR
    return hipGetLastError();
}

template <int SP, int LP, bool L12>
static hipError_t lr_fmt(const HopLaunch& h, const MrhsParams& M, int depth, dim3 grid, dim3 block,
                         hipStream_t s) {
    return depth == 3 ? lr_depth<SP, LP, L12, 3>(h, M, grid, block, s)
                      : lr_depth<SP, LP, L12, 1>(h, M, grid, block, s);
}

template <bool L12, int D>
static hipError_t lr16_depth(const HopLaunch& h, const MrhsParams& M, dim3 grid, dim3 block, hipStream_t s) {
    bool cph = false;
    for (int m = 0; m < 4; ++m) cph = cph || h.phase[m][1] != 0.0;
#define WEO_LR16(DG, CP) hipLaunchKernelGGL((k_hop_lr16<L12, DG, CP, D>), grid, block, 0, s, M)
    if (h.dagger) { if (cph) WEO_LR16(true, true); else WEO_LR16(true, false); }
    else { if (cph) WEO_LR16(false, true); else WEO_LR16(false, false); }
#undef WEO_LR16
    return hipGetLastError();
}

// FP16 spinors with FP16 links: the packed-pair form (ring depth 1 or 3)
static hipError_t launch_hop_lr16(const HopLaunch& h, const MrhsParams& M, int depth, dim3 grid, dim3 block,
                                  hipStream_t s) {
    switch (h.fmt) {
        case FMT_H_H_18: return depth == 3 ? lr16_depth<false, 3>(h, M, grid, block, s)
                                           : lr16_depth<false, 1>(h, M, grid, block, s);
        case FMT_H_H_12: return depth == 3 ? lr16_depth<true, 3>(h, M, grid, block, s)
                                           : lr16_depth<true, 1>(h, M, grid, block, s);
        default: return hipErrorInvalidValue;
    }
}

bool lr16_supported(int fmt) { return fmt == FMT_H_H_18 || fmt == FMT_H_H_12; }

static hipError_t launch_hop_lr(const HopLaunch& h, const MrhsParams& M, int depth, dim3 grid, dim3 block,
                                hipStream_t s) {
    switch (h.fmt) {
        case FMT_S_S_18: return lr_fmt<P_F32, P_F32, false>(h, M, depth, grid, block, s);
        case FMT_S_S_12: return lr_fmt<P_F32, P_F32, true>(h, M, depth, grid, block, s);
        case FMT_H_H_18: return lr_fmt<P_F16, P_F16, false>(h, M, depth, grid, block, s);
        case FMT_H_H_12: return lr_fmt<P_F16, P_F16, true>(h, M, depth, grid, block, s);
        case FMT_B_H_18: return lr_fmt<P_BF16, P_F16, false>(h, M, depth, grid, block, s);
        case FMT_B_H_12: return lr_fmt<P_BF16, P_F16, true>(h, M, depth, grid, block, s);
        default: return hipErrorInvalidValue;       // FP64: not built (register file)
    }
}

bool lr_supported(int fmt) { return fmt_info(fmt).spinor_prec != P_F64; }

template <int SP, int LP, bool L12>
static hipError_t lw_fmt(const HopLaunch& h, const MrhsParams& M, dim3 grid, dim3 block, hipStream_t s) {
    bool cph = false;
    for (int m = 0; m < 4; ++m) cph = cph || h.phase[m][1] != 0.0;
#define WEO_LW(DG, CP, DT) hipLaunchKernelGGL((k_hop_lw<SP, LP, L12, DG, CP, DT>), grid, block, 0, s, M)
    if (h.dmode) {
        if (!h.partial) return hipErrorInvalidValue;
        if (h.dagger) { if (cph) WEO_LW(true, true, true); else WEO_LW(true, false, true); }
        else { if (cph) WEO_LW(false, true, true); else WEO_LW(false, false, true); }
    } else {
        if (h.dagger) { if (cph) WEO_LW(true, true, false); else WEO_LW(true, false, false); }
        else { if (cph) WEO_LW(false, true, false); else WEO_LW(false, false, false); }
    }
#undef WEO_LW
    return hipGetLastError();
}

static int lw_max_waves(int fmt) {
    switch (fmt_info(fmt).spinor_prec) {
        case P_F64: return lw_maxw<P_F64>();
        case P_F32: return lw_maxw<P_F32>();
        default: return lw_maxw<P_F16>();
    }
}

// LDS-staged form: W wavefronts of 64 sites per workgroup
static hipError_t launch_hop_lw(const HopLaunch& h, const MrhsParams& M, int W, dim3 grid, hipStream_t s) {
    if (W > lw_max_waves(h.fmt)) return hipErrorInvalidValue;
    const dim3 block(64, (unsigned)W);
    switch (h.fmt) {
        case FMT_D_D_18: return lw_fmt<P_F64, P_F64, false>(h, M, grid, block, s);
        case FMT_D_D_12: return lw_fmt<P_F64, P_F64, true>(h, M, grid, block, s);
        case FMT_S_S_18: return lw_fmt<P_F32, P_F32, false>(h, M, grid, block, s);
        case FMT_S_S_12: return lw_fmt<P_F32, P_F32, true>(h, M, grid, block, s);
        case FMT_H_H_18: return lw_fmt<P_F16, P_F16, false>(h, M, grid, block, s);
        case FMT_H_H_12: return lw_fmt<P_F16, P_F16, true>(h, M, grid, block, s);
        case FMT_B_H_18: return lw_fmt<P_BF16, P_F16, false>(h, M, grid, block, s);
        case FMT_B_H_12: return lw_fmt<P_BF16, P_F16, true>(h, M, grid, block, s);
        default: return hipErrorInvalidValue;
    }
}

bool lw_waves_ok(int w) { return w == 2 || w == 3 || w == 4 || w == 6 || w == 8 || w == 12; }

hipError_t launch_hop_mrhs(const HopLaunch& h, const MrhsCfg& c, hipStream_t s) {
    MrhsParams M;
    M.h = hop_params(h);
    M.rhs_per_row = h.nrhs;
    if (c.nr == kNrLw) {
        // LDS-staged: 64 sites per workgroup, c.s wavefronts
        if (!lw_waves_ok(c.s)) return hipErrorInvalidValue;
        M.h.sched = make_sched(h.g, c.bz, 64u);
        M.nrhs = h.nrhs;
        M.nblk = (h.g.vh + 63u) / 64u;
        // c.split = right-hand sides per sweep (0: all in one); each sweep
        // is a grid row and stages the links again
        M.rhs_per_row = c.split > 0 && c.split < h.nrhs ? c.split : h.nrhs;
        const unsigned rows = (unsigned)((h.nrhs + M.rhs_per_row - 1) / M.rhs_per_row);
        uint32_t nwg = M.nblk;
        if (c.persist) {
            const uint32_t cap = 8u * 256u;
            if (nwg > cap) nwg = cap;
            nwg = ((nwg + 7u) / 8u) * 8u;
        }
        return launch_hop_lw(h, M, c.s, dim3(nwg, rows), s);
    }
    M.h.sched = make_sched(h.g, c.bz, (uint32_t)c.s);
    if (c.nr < 0) {
        // link-resident: one lane per site, all rhs in turn; -nr is the ring depth
        M.nrhs = h.nrhs;
        M.nblk = (h.g.vh + (uint32_t)c.s - 1) / (uint32_t)c.s;
        uint32_t nwg = M.nblk;
        if (c.persist) {
            const uint32_t cap = 8u * 256u;
            if (nwg > cap) nwg = cap;
            nwg = ((nwg + 7u) / 8u) * 8u;
        }
        // nr = -1 / -3: FP32 arithmetic, ring depth 1 / 3; nr = -2 / -4: the
        // packed FP16 form, ring depth 1 / 3
        if (c.nr == -2 || c.nr == -4) return launch_hop_lr16(h, M, c.nr == -4 ? 3 : 1, dim3(nwg), dim3((unsigned)c.s), s);
        return launch_hop_lr(h, M, -c.nr, dim3(nwg), dim3((unsigned)c.s), s);
    }
    M.nrhs = h.nrhs;
    M.nblk = (h.g.vh + (uint32_t)c.s - 1) / (uint32_t)c.s;
    const int groups = (h.nrhs + c.nr - 1) / c.nr;
    int gy = c.split ? 1 : 256 / c.s;
    if (gy > groups) gy = groups;
    const dim3 block((unsigned)c.s, (unsigned)gy);
    uint32_t nwg = M.nblk;
    if (c.persist) {
        const uint32_t cap = 8u * 256u;
        if (nwg > cap) nwg = cap;
        nwg = ((nwg + 7u) / 8u) * 8u;
    }
    const dim3 grid(nwg, (unsigned)((groups + gy - 1) / gy));
    switch (h.fmt) {
        case FMT_D_D_18: return mrhs_fmt<P_F64, P_F64, false>(h, M, c.nr, grid, block, s);
        case FMT_D_D_12: return mrhs_fmt<P_F64, P_F64, true>(h, M, c.nr, grid, block, s);
        case FMT_S_S_18: return mrhs_fmt<P_F32, P_F32, false>(h, M, c.nr, grid, block, s);
        case FMT_S_S_12: return mrhs_fmt<P_F32, P_F32, true>(h, M, c.nr, grid, block, s);
        case FMT_H_H_18: return mrhs_fmt<P_F16, P_F16, false>(h, M, c.nr, grid, block, s);
        case FMT_H_H_12: return mrhs_fmt<P_F16, P_F16, true>(h, M, c.nr, grid, block, s);
        case FMT_B_H_18: return mrhs_fmt<P_BF16, P_F16, false>(h, M, c.nr, grid, block, s);
        case FMT_B_H_12: return mrhs_fmt<P_BF16, P_F16, true>(h, M, c.nr, grid, block, s);
        default: return hipErrorInvalidValue;
    }
}

namespace {

// dims, format, nrhs, epilogue (1: axpy, 2: norm partials)
using TuneKey = std::tuple<int, int, int, int, int, int, int>;

struct TuneEntry {
    MrhsCfg cfg;       // nr == 1: the single-rhs kernel
    float us;
};

std::mutex g_tune_mu;
std::map<TuneKey, TuneEntry> g_tune;

// The half-plane column walks (bz < 0) are not candidates: at 32^3x64 with
// 12 rhs they were never faster than the z strips (FP16/12 406 us against
// 399 us, FP32/12 728 against 725 us); weo_set_mrhs_shape still selects them.
std::vector<MrhsCfg> candidates(const HopLaunch& h) {
    std::vector<MrhsCfg> v;
    v.push_back({1, 0, 0, 0, 0});
    const bool wide = fmt_info(h.fmt).spinor_prec == P_F64;
    const bool dot = h.dmode != 0;      // the fused dot: single-rhs and LDS-staged kernels only
    if (lr_supported(h.fmt) && !dot)
        for (int s : {64, 128, 256})
            for (int persist : {0, 1})
                for (int bz : {0, 2, 4, 8}) {
                    if (bz && make_sched(h.g, bz, (uint32_t)s).bz != bz) continue;
                    for (int nr : {-1, -3}) v.push_back({nr, s, persist, bz, 0});
                    if (lr16_supported(h.fmt))
                        for (int nr : {-2, -4}) v.push_back({nr, s, persist, bz, 0});
                }
    for (int w : {2, 3, 4, 6, 8, 12}) {
        if (w > h.nrhs || w > lw_max_waves(h.fmt)) continue;
        for (int persist : {0, 1})
            for (int bz : {0, 2, 4, 8}) {
                if (bz && make_sched(h.g, bz, 64u).bz != bz) continue;
                for (int f : {0, 6}) {                // right-hand sides per sweep (0: all)
                    if (f && (f >= h.nrhs || f < w)) continue;
                    v.push_back({kNrLw, w, persist, bz, f});
                }
            }
    }
    const int nrs[] = {2, 3, 4, 6};
    for (int nr : nrs) {
        if (dot || nr > h.nrhs || (wide && nr > 3)) continue;
        for (int s : {64, 128, 256})
            for (int persist : {0, 1})
                for (int bz : {0, 2, 4, 8}) {
                    if (bz && make_sched(h.g, bz, (uint32_t)s).bz != bz) continue;
                    v.push_back({nr, s, persist, bz, 0});
                    const int groups = (h.nrhs + nr - 1) / nr;
                    if (groups > 1 && s < 256) v.push_back({nr, s, persist, bz, 1});
                }
    }
    return v;
}

hipError_t run_cfg(const HopLaunch& h, const MrhsCfg& c, hipStream_t s) {
    return c.nr == 1 ? launch_hop_single(h, s) : launch_hop_mrhs(h, c, s);
}

bool tuning_enabled() {
    const char* e = getenv("WEO_TUNE");
    return !(e && e[0] == '0');
}

bool tuning_verbose() {
    const char* e = getenv("WEO_TUNE_VERBOSE");
    return e && e[0] == '1';
}

// ---- persistent tuning cache ----------------------------------------------
// WILSON_EO_TUNE_CACHE names a text file that carries tuned shapes across
// processes: a header line naming the cache version and the GPU
// architecture, then one line per key
//   lx ly lz lt fmt nrhs epilogue  nr sites persist bz split  us
// A file with another header is ignored and rewritten on the next tuning.
// An entry is used only if its shape is among the current candidates for
// that key (so a stale or edited file can pick a slower shape, never an
// invalid launch).  New results are appended, one line per write.
constexpr int kTuneCacheVersion = 4;

const char* tune_cache_path() {
    const char* p = getenv("WILSON_EO_TUNE_CACHE");
    return p && p[0] ? p : nullptr;
}

std::map<TuneKey, TuneEntry> g_cached;       // entries read from the file
bool g_cache_loaded = false;
bool g_cache_header_ok = false;               // the file exists with our header

void cache_header(char* buf, size_t len) {
    int dev = 0;
    hipDeviceProp_t prop;
    const char* arch = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        arch = prop.gcnArchName;
    snprintf(buf, len, "# wilson_eo tuning cache %d %s", kTuneCacheVersion, arch);
}

// with g_tune_mu held
void load_cache_locked() {
    if (g_cache_loaded) return;
    g_cache_loaded = true;
    const char* path = tune_cache_path();
    if (!path) return;
    FILE* f = fopen(path, "r");
    if (!f) return;
    char want[256], line[512];
    cache_header(want, sizeof want);
    if (fgets(line, sizeof line, f)) {
        line[strcspn(line, "\r\n")] = 0;
        g_cache_header_ok = strcmp(line, want) == 0;
    }
    while (g_cache_header_ok && fgets(line, sizeof line, f)) {
        int v[12];
        float us = 0.f;
        if (sscanf(line, "%d %d %d %d %d %d %d %d %d %d %d %d %f", &v[0], &v[1], &v[2], &v[3], &v[4], &v[5],
                   &v[6], &v[7], &v[8], &v[9], &v[10], &v[11], &us) != 13)
            continue;
        TuneEntry e;
        e.cfg = {v[7], v[8], v[9], v[10], v[11]};
        e.us = us;
        g_cached[TuneKey{v[0], v[1], v[2], v[3], v[4], v[5], v[6]}] = e;
    }
    fclose(f);
}

// with g_tune_mu held
void append_cache_locked(const TuneKey& k, const TuneEntry& e) {
    const char* path = tune_cache_path();
    if (!path) return;
    FILE* f = fopen(path, g_cache_header_ok ? "a" : "w");
    if (!f) return;
    if (!g_cache_header_ok) {
        char hdr[256];
        cache_header(hdr, sizeof hdr);
        fprintf(f, "%s\n", hdr);
        g_cache_header_ok = true;
    }
    fprintf(f, "%d %d %d %d %d %d %d %d %d %d %d %d %.2f\n", std::get<0>(k), std::get<1>(k), std::get<2>(k),
            std::get<3>(k), std::get<4>(k), std::get<5>(k), std::get<6>(k), e.cfg.nr, e.cfg.s, e.cfg.persist,
            e.cfg.bz, e.cfg.split, e.us);
    fclose(f);
}

bool is_candidate(const HopLaunch& h, const MrhsCfg& c) {
    for (const MrhsCfg& d : candidates(h))
        if (d.nr == c.nr && d.s == c.s && d.persist == c.persist && d.bz == c.bz && d.split == c.split) return true;
    return false;
}

// Average microseconds of reps launches of shape c (after one warm-up).
hipError_t time_cfg(const HopLaunch& h, const MrhsCfg& c, hipStream_t s, hipEvent_t e0, hipEvent_t e1, int reps,
                    float* us) {
    hipError_t err = run_cfg(h, c, s);                            // warm-up
    if (err != hipSuccess) return err;
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < reps && err == hipSuccess; ++r) err = run_cfg(h, c, s);
    (void)hipEventRecord(e1, s);
    if (err != hipSuccess || (err = hipEventSynchronize(e1)) != hipSuccess) return err;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    *us = 1000.f * ms / reps;
    return hipSuccess;
}

// Every candidate timed briefly (3 launches), then the 4 fastest again over
// 12 launches each: single short timings vary by several per cent between
// neighbouring shapes, which had made the choice drift from run to run.
hipError_t tune(const HopLaunch& h, hipStream_t s, TuneEntry* best) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return hipErrorUnknown;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return hipErrorUnknown; }
    best->us = 1e30f;
    best->cfg = {1, 0, 0, 0, 0};
    hipError_t err = hipSuccess;
    std::vector<std::pair<float, MrhsCfg>> timed;
    for (const MrhsCfg& c : candidates(h)) {
        float us = 0.f;
        if ((err = time_cfg(h, c, s, e0, e1, 3, &us)) != hipSuccess) break;
        if (tuning_verbose())
            fprintf(stderr, "[weo tune] fmt %d nrhs %d: nr %d sites %d persist %d bz %d split %d -> %.1f us\n",
                    h.fmt, h.nrhs, c.nr, c.s, c.persist, c.bz, c.split, us);
        timed.push_back({us, c});
    }
    if (err == hipSuccess) {
        std::sort(timed.begin(), timed.end(), [](const std::pair<float, MrhsCfg>& a,
                                                 const std::pair<float, MrhsCfg>& b) { return a.first < b.first; });
        const size_t nfinal = timed.size() < 4 ? timed.size() : 4;
        for (size_t k = 0; k < nfinal; ++k) {
            float us = 0.f;
            if ((err = time_cfg(h, timed[k].second, s, e0, e1, 12, &us)) != hipSuccess) break;
            if (tuning_verbose())
                fprintf(stderr, "[weo tune] final: nr %d sites %d persist %d bz %d split %d -> %.1f us\n",
                        timed[k].second.nr, timed[k].second.s, timed[k].second.persist, timed[k].second.bz,
                        timed[k].second.split, us);
            if (us < best->us) { best->us = us; best->cfg = timed[k].second; }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return err;
}

}  // namespace

// Forced shape (weo_set_mrhs_shape); nr == 0 means autotune.
static MrhsCfg g_forced = {0, 0, 0, 0, 0};

int set_mrhs_shape(int nr, int sites, int persist, int bz, int split) {
    if (nr == 0 || nr == 1) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_forced = {nr, 0, 0, 0, 0};
        return 0;
    }
    if (nr == kNrLw) {
        if (!lw_waves_ok(sites) || (persist != 0 && persist != 1) || bz < -64 || bz > 64 || split < 0 ||
            split > 16)       // 16: the most right-hand sides of a launch
            return -1;
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_forced = {nr, sites, persist, bz, split};
        return 0;
    }
    if (nr < -4) return -1;
    if (split != 0 && split != 1) return -1;
    if (nr < 0) {
        if (sites != 64 && sites != 128 && sites != 256) return -1;
        if (persist != 0 && persist != 1) return -1;
        if (bz < -64 || bz > 64) return -1;
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_forced = {nr, sites, persist, bz, 0};
        return 0;
    }
    if (nr != 2 && nr != 3 && nr != 4 && nr != 6) return -1;
    if (sites != 64 && sites != 128 && sites != 256) return -1;
    if (persist != 0 && persist != 1) return -1;
    if (bz < -64 || bz > 64) return -1;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_forced = {nr, sites, persist, bz, split};
    return 0;
}

hipError_t launch_hop(const HopLaunch& h, hipStream_t s) {
    if (h.nrhs == 1) return launch_hop_single(h, s);
    MrhsCfg forced;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        forced = g_forced;
    }
    if (forced.nr == 1) return launch_hop_single(h, s);
    if (h.dmode && forced.nr != 0 && forced.nr != kNrLw) return launch_hop_single(h, s);   // no fused dot there
    if (forced.nr == kNrLw) {
        MrhsCfg c = forced;
        if (c.s > lw_max_waves(h.fmt)) c.s = lw_max_waves(h.fmt);      // the format's most wavefronts
        return launch_hop_mrhs(h, c, s);
    }
    if (forced.nr < 0) {
        if (!lr_supported(h.fmt)) return launch_hop_single(h, s);
        if ((forced.nr == -2 || forced.nr == -4) && !lr16_supported(h.fmt)) {
            MrhsCfg c = forced;
            c.nr = forced.nr == -4 ? -3 : -1;          // FP32 arithmetic for the other formats
            return launch_hop_mrhs(h, c, s);
        }
        return launch_hop_mrhs(h, forced, s);
    }
    if (forced.nr > 1) {
        MrhsCfg c = forced;
        const bool wide = fmt_info(h.fmt).spinor_prec == P_F64;
        if (wide && c.nr > 3) c.nr = 3;          // FP64 builds nr 2 and 3 only
        if (c.nr > h.nrhs) c.nr = h.nrhs;
        return c.nr <= 1 ? launch_hop_single(h, s) : launch_hop_mrhs(h, c, s);
    }
    const int epi = (h.y != nullptr ? 1 : 0) + (h.partial != nullptr ? 2 : 0) + (h.z != nullptr ? 4 : 0) +
                    (h.dmode != 0 ? 8 : 0);
    const TuneKey key{h.g.lx, h.g.ly, h.g.lz, h.g.lt, h.fmt, h.nrhs, epi};
    TuneEntry e;
    bool have = false;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) { e = it->second; have = true; }
    }
    if (!have && h.y != nullptr) {
        // an in-place axpy (y is out) cannot be timed by repeated launches:
        // each would add to the previous result.  Run it untuned.
        const size_t fb = (size_t)h.nrhs * spinor_field_bytes(h.g, h.fmt);
        const uintptr_t y = reinterpret_cast<uintptr_t>(h.y), o = reinterpret_cast<uintptr_t>(h.out);
        if (y < o + fb && o < y + fb) return launch_hop_single(h, s);
    }
    if (!have && tuning_enabled()) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        load_cache_locked();
        auto it = g_cached.find(key);
        if (it != g_cached.end() && is_candidate(h, it->second.cfg)) {
            e = it->second;
            g_tune[key] = e;
            have = true;
        }
    }
    if (!have) {
        if (tuning_enabled()) {
            const hipError_t err = tune(h, s, &e);
            if (err != hipSuccess) return err;
        } else {
            e.cfg = {h.nrhs >= 3 ? 3 : h.nrhs, 64, 0, 0, 0};
            e.us = 0.f;
        }
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[key] = e;
        if (tuning_enabled()) append_cache_locked(key, e);
    }
    return run_cfg(h, e.cfg, s);
}

// Text report of the tuned choices (one line per key) for diagnostics.
int tuning_report(char* buf, size_t len) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    size_t off = 0;
    for (const auto& kv : g_tune) {
        const TuneKey& k = kv.first;
        const TuneEntry& e = kv.second;
        const int n = snprintf(buf ? buf + off : nullptr, buf && off < len ? len - off : 0,
                               "{\"dims\":[%d,%d,%d,%d],\"fmt\":%d,\"nrhs\":%d,\"epilogue\":%d,\"nr\":%d,"
                               "\"sites\":%d,\"persist\":%d,\"bz\":%d,\"split\":%d,\"us\":%.2f}\n",
                               std::get<0>(k), std::get<1>(k), std::get<2>(k), std::get<3>(k), std::get<4>(k),
                               std::get<5>(k), std::get<6>(k), e.cfg.nr, e.cfg.s, e.cfg.persist, e.cfg.bz,
                               e.cfg.split, e.us);
        if (n > 0) off += (size_t)n;
    }
    return (int)off;
}

}  // namespace weo
