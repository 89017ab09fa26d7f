// Site-local diagonal blocks of a clover-type operator: with a clover term the
// diagonal blocks D_ee, D_oo of Eqs. (3)-(5) act site by site (Sec. 2).
//
// The site matrix commutes with gamma5, so in the gamma5 eigenbasis of the
// Dirac representation (gamma5 = -[[0, 1], [1, 0]] in 2 x 2 spin blocks) it is
// two 6 x 6 Hermitian blocks:
//     psi_A = (psi_up + psi_dn) / sqrt2  ->  B0 psi_A
//     psi_B = (psi_up - psi_dn) / sqrt2  ->  B1 psi_B
// (up = spins 0, 1; dn = spins 2, 3; 6-vectors ordered spin-major).
//
// Packed block record, 18 complex in the link precision: slots 0..2 hold the
// six real diagonal entries in pairs (d0, d1), (d2, d3), (d4, d5); slots 3..17
// the lower triangle B(i, j), i > j, row by row.  A clover field is
// [parity][block][plane][V/2], i.e. four one-parity record fields.
#pragma once

#include "weo_device.h"

namespace weo {

constexpr int kCloverSlots = 18;

// y = B x for a packed Hermitian 6 x 6 block.
template <class C>
__device__ __forceinline__ void herm6_mul(const C* blk, const C* x, C* y) {
    using R = decltype(C().x);
    const R d[6] = {blk[0].x, blk[0].y, blk[1].x, blk[1].y, blk[2].x, blk[2].y};
#pragma unroll
    for (int i = 0; i < 6; ++i) { y[i].x = d[i] * x[i].x; y[i].y = d[i] * x[i].y; }
    int k = 3;
#pragma unroll
    for (int i = 1; i < 6; ++i)
#pragma unroll
        for (int j = 0; j < i; ++j, ++k) {
            y[i] = fma_(blk[k], x[j], y[i]);     // B(i, j) x_j
            y[j] = fmac_(blk[k], x[i], y[j]);    // B(j, i) x_i = conj(B(i, j)) x_i
        }
}

// Load one packed block (link precision CP) as arithmetic type C.
template <int CP, class C>
__device__ __forceinline__ void load_block(const uint8_t* base, uint32_t n, uint32_t i, C* blk) {
    using CR = typename St<CP>::real;
    if constexpr (sizeof(CR) == sizeof(decltype(C().x))) {
        load_rec<CP, kCloverSlots>(base, n, i, blk);
    } else {
        cx<CR> w[kCloverSlots];
        load_rec<CP, kCloverSlots>(base, n, i, w);
#pragma unroll
        for (int k = 0; k < kCloverSlots; ++k) { blk[k].x = w[k].x; blk[k].y = w[k].y; }
    }
}

// v <- A v from the two block records already in registers.
template <int CP, class C, class RR>
__device__ __forceinline__ void clover_apply_raw(const RR& r0, const RR& r1, C* v) {
    using R = decltype(C().x);
    using CR = typename St<CP>::real;
    C a[6], b[6], ya[6], yb[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) { a[k] = add(v[k], v[6 + k]); b[k] = sub(v[k], v[6 + k]); }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        cx<CR> w[kCloverSlots];
        (q == 0 ? r0 : r1).unpack(w);
        C blk[kCloverSlots];
#pragma unroll
        for (int k = 0; k < kCloverSlots; ++k) { blk[k].x = (R)w[k].x; blk[k].y = (R)w[k].y; }
        herm6_mul(blk, q == 0 ? a : b, q == 0 ? ya : yb);
    }
    const R h = R(0.5);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        v[k].x = h * (ya[k].x + yb[k].x);
        v[k].y = h * (ya[k].y + yb[k].y);
        v[6 + k].x = h * (ya[k].x - yb[k].x);
        v[6 + k].y = h * (ya[k].y - yb[k].y);
    }
}

// v <- A v for the site matrix A of half-index i; par_base points at the
// parity's two block fields, block_bytes is the size of one of them.
template <int CP, class C>
__device__ __forceinline__ void clover_apply_site(const uint8_t* par_base, size_t block_bytes, uint32_t n,
                                                  uint32_t i, C* v) {
    using R = decltype(C().x);
    C a[6], b[6], ya[6], yb[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) { a[k] = add(v[k], v[6 + k]); b[k] = sub(v[k], v[6 + k]); }
    {
        C blk[kCloverSlots];
        load_block<CP>(par_base, n, i, blk);
        herm6_mul(blk, a, ya);
    }
    {
        C blk[kCloverSlots];
        load_block<CP>(par_base + block_bytes, n, i, blk);
        herm6_mul(blk, b, yb);
    }
    const R h = R(0.5);     // the two 1/sqrt2 of the basis change
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        v[k].x = h * (ya[k].x + yb[k].x);
        v[k].y = h * (ya[k].y + yb[k].y);
        v[6 + k].x = h * (ya[k].x - yb[k].x);
        v[6 + k].y = h * (ya[k].y - yb[k].y);
    }
}

}  // namespace weo
