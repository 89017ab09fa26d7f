// Device-side building blocks of libwilson_eo: complex arithmetic, storage
// traits of the packed field formats, record loads/stores, lattice geometry.
//
// Packed layout (all fields): a field is a set of "records", one per site of
// one parity, each record a fixed number NC of complex numbers (12 for a
// spinor in [spin][colour] order, 9 or 6 for a link in row-major order).  The
// records of V/2 sites are stored as structure-of-arrays "planes" of 16-byte
// chunks: plane p holds bytes [16p, 16p+16) of every record, consecutive
// sites adjacent, so that one wavefront reading plane p for 64 consecutive
// sites issues one fully coalesced 1 KiB request.  When the record size is
// not a multiple of 16 bytes the remaining 8 or 4 bytes form a narrower tail
// plane after the full planes.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "weo_geom.h"

namespace weo {

__host__ __device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv& f) {
#if defined(__HIP_DEVICE_COMPILE__)
    return (__umulhi(n, f.m) + n) >> f.s;
#else
    return host_fdiv(n, f);
#endif
}

enum : int { P_F64 = 0, P_F32 = 1, P_F16 = 2, P_BF16 = 3 };

// ---------------------------------------------------------------- complex --
// Complex numbers are float2 / double2 (x = re, y = im).  The helpers are
// templates on the vector type so that one body serves both precisions.
template <class R> struct cx_t;
template <> struct cx_t<float> { using type = float2; };
template <> struct cx_t<double> { using type = double2; };
template <class R> using cx = typename cx_t<R>::type;

template <class V> __device__ __forceinline__ V mk(decltype(V().x) a, decltype(V().x) b) { V r; r.x = a; r.y = b; return r; }
template <class V> __device__ __forceinline__ V czero() { V r; r.x = 0; r.y = 0; return r; }
template <class V> __device__ __forceinline__ V add(V a, V b) { V r; r.x = a.x + b.x; r.y = a.y + b.y; return r; }
template <class V> __device__ __forceinline__ V sub(V a, V b) { V r; r.x = a.x - b.x; r.y = a.y - b.y; return r; }
// a * b
template <class V> __device__ __forceinline__ V mul(V a, V b) {
    V r; r.x = a.x * b.x - a.y * b.y; r.y = a.x * b.y + a.y * b.x; return r;
}
// acc + a * b
template <class V> __device__ __forceinline__ V fma_(V a, V b, V acc) {
    acc.x = fma(a.x, b.x, acc.x); acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y); acc.y = fma(a.y, b.x, acc.y);
    return acc;
}
// acc + conj(a) * b
template <class V> __device__ __forceinline__ V fmac_(V a, V b, V acc) {
    acc.x = fma(a.x, b.x, acc.x); acc.x = fma(a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y); acc.y = fma(-a.y, b.x, acc.y);
    return acc;
}
// conj(a) * b
template <class V> __device__ __forceinline__ V mulc(V a, V b) {
    V r; r.x = a.x * b.x + a.y * b.y; r.y = a.x * b.y - a.y * b.x; return r;
}
// i * a
template <class V> __device__ __forceinline__ V imul(V a) { V r; r.x = -a.y; r.y = a.x; return r; }
template <class V, class R> __device__ __forceinline__ V scal(R s, V a) { V r; r.x = s * a.x; r.y = s * a.y; return r; }
template <class V> __device__ __forceinline__ V conj_(V a) { V r; r.x = a.x; r.y = -a.y; return r; }

// ------------------------------------------------------- storage traits ----
// cbytes: bytes of one stored complex number; real: arithmetic type.
template <int P> struct St;

template <> struct St<P_F64> {
    using real = double;
    static constexpr int cbytes = 16;
    __device__ static __forceinline__ void unpack16(const uint4& w, double2* v) {
        v[0].x = __hiloint2double((int)w.y, (int)w.x);
        v[0].y = __hiloint2double((int)w.w, (int)w.z);
    }
    __device__ static __forceinline__ uint4 pack16(const double2* v) {
        uint4 w;
        w.x = (uint32_t)__double2loint(v[0].x); w.y = (uint32_t)__double2hiint(v[0].x);
        w.z = (uint32_t)__double2loint(v[0].y); w.w = (uint32_t)__double2hiint(v[0].y);
        return w;
    }
};

template <> struct St<P_F32> {
    using real = float;
    static constexpr int cbytes = 8;
    __device__ static __forceinline__ void unpack16(const uint4& w, float2* v) {
        v[0] = make_float2(__uint_as_float(w.x), __uint_as_float(w.y));
        v[1] = make_float2(__uint_as_float(w.z), __uint_as_float(w.w));
    }
    __device__ static __forceinline__ void unpack8(const uint2& w, float2* v) {
        v[0] = make_float2(__uint_as_float(w.x), __uint_as_float(w.y));
    }
    __device__ static __forceinline__ uint4 pack16(const float2* v) {
        return make_uint4(__float_as_uint(v[0].x), __float_as_uint(v[0].y),
                          __float_as_uint(v[1].x), __float_as_uint(v[1].y));
    }
    __device__ static __forceinline__ uint2 pack8(const float2* v) {
        return make_uint2(__float_as_uint(v[0].x), __float_as_uint(v[0].y));
    }
};

// IEEE binary16, round to nearest even on conversion.
__device__ __forceinline__ float2 h2_to_f2(uint32_t w) {
    __half2 h = *reinterpret_cast<__half2*>(&w);
    return __half22float2(h);
}
__device__ __forceinline__ uint32_t f2_to_h2(float2 f) {
    __half2 h = __floats2half2_rn(f.x, f.y);
    return *reinterpret_cast<uint32_t*>(&h);
}

template <> struct St<P_F16> {
    using real = float;
    static constexpr int cbytes = 4;
    __device__ static __forceinline__ void unpack16(const uint4& w, float2* v) {
        v[0] = h2_to_f2(w.x); v[1] = h2_to_f2(w.y); v[2] = h2_to_f2(w.z); v[3] = h2_to_f2(w.w);
    }
    __device__ static __forceinline__ void unpack8(const uint2& w, float2* v) {
        v[0] = h2_to_f2(w.x); v[1] = h2_to_f2(w.y);
    }
    __device__ static __forceinline__ void unpack4(uint32_t w, float2* v) { v[0] = h2_to_f2(w); }
    __device__ static __forceinline__ uint4 pack16(const float2* v) {
        return make_uint4(f2_to_h2(v[0]), f2_to_h2(v[1]), f2_to_h2(v[2]), f2_to_h2(v[3]));
    }
    __device__ static __forceinline__ uint2 pack8(const float2* v) {
        return make_uint2(f2_to_h2(v[0]), f2_to_h2(v[1]));
    }
    __device__ static __forceinline__ uint32_t pack4(const float2* v) { return f2_to_h2(v[0]); }
};

// bfloat16: the upper 16 bits of an IEEE binary32; conversion rounds to
// nearest even, NaN stays NaN.
__device__ __forceinline__ uint32_t f_to_bf16(float f) {
    const uint32_t u = __float_as_uint(f);
    const uint32_t rne = (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
    const uint32_t qnan = (u >> 16) | 0x40u;
    return ((u & 0x7fffffffu) > 0x7f800000u) ? qnan : rne;   // a select, no branch
}
__device__ __forceinline__ float2 bf2_to_f2(uint32_t w) {
    return make_float2(__uint_as_float(w << 16), __uint_as_float(w & 0xffff0000u));
}
__device__ __forceinline__ uint32_t f2_to_bf2(float2 f) {
    return f_to_bf16(f.x) | (f_to_bf16(f.y) << 16);
}

template <> struct St<P_BF16> {
    using real = float;
    static constexpr int cbytes = 4;
    __device__ static __forceinline__ void unpack16(const uint4& w, float2* v) {
        v[0] = bf2_to_f2(w.x); v[1] = bf2_to_f2(w.y); v[2] = bf2_to_f2(w.z); v[3] = bf2_to_f2(w.w);
    }
    __device__ static __forceinline__ void unpack8(const uint2& w, float2* v) {
        v[0] = bf2_to_f2(w.x); v[1] = bf2_to_f2(w.y);
    }
    __device__ static __forceinline__ void unpack4(uint32_t w, float2* v) { v[0] = bf2_to_f2(w); }
    __device__ static __forceinline__ uint4 pack16(const float2* v) {
        return make_uint4(f2_to_bf2(v[0]), f2_to_bf2(v[1]), f2_to_bf2(v[2]), f2_to_bf2(v[3]));
    }
    __device__ static __forceinline__ uint2 pack8(const float2* v) {
        return make_uint2(f2_to_bf2(v[0]), f2_to_bf2(v[1]));
    }
    __device__ static __forceinline__ uint32_t pack4(const float2* v) { return f2_to_bf2(v[0]); }
};

// ------------------------------------------------------ record load/store --
// A record of NC complex numbers of site i.  ``base`` is the start of the
// field (its first plane), ``n`` the number of sites per plane.  Plane bases
// are wave-uniform; the per-lane offset is a 32-bit byte offset, which lets
// the compiler use scalar-base + vector-offset addressing (every plane of the
// largest field is far below 4 GiB).
template <int P, int NC> struct Rec {
    static constexpr int CB = St<P>::cbytes;
    static constexpr int K = 16 / CB;                 // complex per 16-byte chunk
    static constexpr int NFULL = (NC * CB) / 16;      // full planes
    static constexpr int TAILB = (NC * CB) % 16;      // bytes in the tail plane
    static constexpr int BYTES = NC * CB;
};

typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));

// Plain or streaming (non-temporal: the line is not kept in the caches for
// reuse) loads of 16, 8 and 4 bytes.
template <bool NT> __device__ __forceinline__ uint4 ld16(const uint8_t* p) {
    if constexpr (NT) {
        const u32x4_t w = __builtin_nontemporal_load(reinterpret_cast<const u32x4_t*>(p));
        return make_uint4(w.x, w.y, w.z, w.w);
    } else {
        return *reinterpret_cast<const uint4*>(p);
    }
}
template <bool NT> __device__ __forceinline__ uint2 ld8(const uint8_t* p) {
    if constexpr (NT) {
        const u32x2_t w = __builtin_nontemporal_load(reinterpret_cast<const u32x2_t*>(p));
        return make_uint2(w.x, w.y);
    } else {
        return *reinterpret_cast<const uint2*>(p);
    }
}
template <bool NT> __device__ __forceinline__ uint32_t ld4(const uint8_t* p) {
    if constexpr (NT) return __builtin_nontemporal_load(reinterpret_cast<const uint32_t*>(p));
    else return *reinterpret_cast<const uint32_t*>(p);
}

template <int P, int NC, bool NT = false, class V>
__device__ __forceinline__ void load_rec(const uint8_t* __restrict__ base, uint32_t n, uint32_t i, V* v) {
    using T = Rec<P, NC>;
    const size_t pb = (size_t)n * 16;
#pragma unroll
    for (int p = 0; p < T::NFULL; ++p) {
        const uint4 w = ld16<NT>(base + p * pb + (uint32_t)(i * 16u));
        St<P>::unpack16(w, v + p * T::K);
    }
    if constexpr (T::TAILB == 8) {
        const uint2 w = ld8<NT>(base + T::NFULL * pb + (uint32_t)(i * 8u));
        St<P>::unpack8(w, v + T::NFULL * T::K);
    } else if constexpr (T::TAILB == 4) {
        const uint32_t w = ld4<NT>(base + T::NFULL * pb + (uint32_t)(i * 4u));
        St<P>::unpack4(w, v + T::NFULL * T::K);
    }
}

// A record held as the raw words of its planes, so that loads can be issued
// well before the values are needed without keeping unpacked copies live.
template <int P, int NC, bool NT = false> struct RawRec {
    using T = Rec<P, NC>;
    uint4 w[T::NFULL > 0 ? T::NFULL : 1];
    uint2 t8;
    uint32_t t4;
    __device__ __forceinline__ void load(const uint8_t* __restrict__ base, uint32_t n, uint32_t i) {
        const size_t pb = (size_t)n * 16;
#pragma unroll
        for (int p = 0; p < T::NFULL; ++p) w[p] = ld16<NT>(base + p * pb + (uint32_t)(i * 16u));
        if constexpr (T::TAILB == 8) t8 = ld8<NT>(base + T::NFULL * pb + (uint32_t)(i * 8u));
        if constexpr (T::TAILB == 4) t4 = ld4<NT>(base + T::NFULL * pb + (uint32_t)(i * 4u));
    }
    template <class V> __device__ __forceinline__ void unpack(V* v) const {
#pragma unroll
        for (int p = 0; p < T::NFULL; ++p) St<P>::unpack16(w[p], v + p * T::K);
        if constexpr (T::TAILB == 8) St<P>::unpack8(t8, v + T::NFULL * T::K);
        if constexpr (T::TAILB == 4) St<P>::unpack4(t4, v + T::NFULL * T::K);
    }
};

// The values a record holds after a store in precision P (round trip through
// the storage words in registers), for norms of what was actually written.
template <int P, int NC, class V>
__device__ __forceinline__ void round_rec(const V* in, V* out) {
    using T = Rec<P, NC>;
#pragma unroll
    for (int p = 0; p < T::NFULL; ++p) St<P>::unpack16(St<P>::pack16(in + p * T::K), out + p * T::K);
    if constexpr (T::TAILB == 8) St<P>::unpack8(St<P>::pack8(in + T::NFULL * T::K), out + T::NFULL * T::K);
    if constexpr (T::TAILB == 4) St<P>::unpack4(St<P>::pack4(in + T::NFULL * T::K), out + T::NFULL * T::K);
}

template <int P, int NC, class V, bool NT = false>
__device__ __forceinline__ void store_rec(uint8_t* __restrict__ base, uint32_t n, uint32_t i, const V* v) {
    using T = Rec<P, NC>;
    const size_t pb = (size_t)n * 16;
#pragma unroll
    for (int p = 0; p < T::NFULL; ++p) {
        const uint4 w = St<P>::pack16(v + p * T::K);
        if constexpr (NT) {
            u32x4_t x;
            x.x = w.x; x.y = w.y; x.z = w.z; x.w = w.w;
            __builtin_nontemporal_store(x, reinterpret_cast<u32x4_t*>(base + p * pb + (uint32_t)(i * 16u)));
        } else {
            *reinterpret_cast<uint4*>(base + p * pb + (uint32_t)(i * 16u)) = w;
        }
    }
    if constexpr (T::TAILB == 8) {
        *reinterpret_cast<uint2*>(base + T::NFULL * pb + (uint32_t)(i * 8u)) = St<P>::pack8(v + T::NFULL * T::K);
    } else if constexpr (T::TAILB == 4) {
        *reinterpret_cast<uint32_t*>(base + T::NFULL * pb + (uint32_t)(i * 4u)) = St<P>::pack4(v + T::NFULL * T::K);
    }
}

// Bytes of one field of n records.
template <int P, int NC> constexpr size_t field_bytes(uint32_t n) { return (size_t)n * Rec<P, NC>::BYTES; }

// ------------------------------------------------------------- geometry ----
// Geom and FastDiv are shared with host code (weo_geom.h).
// Coordinates of half index ih of parity par.
struct Site {
    uint32_t ih;
    int xh, x, y, z, t;
};
__host__ __device__ __forceinline__ Site decode(const Geom& g, uint32_t ih, int par) {
    Site s;
    s.ih = ih;
    const uint32_t r = fdiv(ih, g.d_lxh);
    s.xh = (int)(ih - r * (uint32_t)g.lxh);
    const uint32_t r2 = fdiv(r, g.d_ly);
    s.y = (int)(r - r2 * (uint32_t)g.ly);
    const uint32_t t = fdiv(r2, g.d_lz);
    s.z = (int)(r2 - t * (uint32_t)g.lz);
    s.t = (int)t;
    s.x = 2 * s.xh + ((s.y + s.z + s.t + par) & 1);
    return s;
}

// Half indices (in the opposite parity) of the 8 neighbours and whether the
// hop crosses the lattice edge.  Index 2*mu is x + mu-hat, 2*mu+1 is x - mu-hat.
struct Nbr {
    uint32_t i[8];
    bool edge[8];
};
__host__ __device__ __forceinline__ Nbr neighbours(const Geom& g, const Site& s) {
    Nbr n;
    const uint32_t row = s.ih - (uint32_t)s.xh;
    {
        const bool e = (s.x == g.lx - 1);
        n.i[0] = row + (uint32_t)((e ? 0 : s.x + 1) >> 1);
        n.edge[0] = e;
        const bool f = (s.x == 0);
        n.i[1] = row + (uint32_t)((f ? g.lx - 1 : s.x - 1) >> 1);
        n.edge[1] = f;
    }
    {
        const bool e = (s.y == g.ly - 1), f = (s.y == 0);
        n.i[2] = e ? s.ih - (uint32_t)((g.ly - 1) * g.sy) : s.ih + (uint32_t)g.sy;
        n.i[3] = f ? s.ih + (uint32_t)((g.ly - 1) * g.sy) : s.ih - (uint32_t)g.sy;
        n.edge[2] = e; n.edge[3] = f;
    }
    {
        const bool e = (s.z == g.lz - 1), f = (s.z == 0);
        n.i[4] = e ? s.ih - (uint32_t)((g.lz - 1) * g.sz) : s.ih + (uint32_t)g.sz;
        n.i[5] = f ? s.ih + (uint32_t)((g.lz - 1) * g.sz) : s.ih - (uint32_t)g.sz;
        n.edge[4] = e; n.edge[5] = f;
    }
    {
        const bool e = (s.t == g.lt - 1), f = (s.t == 0);
        n.i[6] = e ? s.ih - (uint32_t)((g.lt - 1) * g.st) : s.ih + (uint32_t)g.st;
        n.i[7] = f ? s.ih + (uint32_t)((g.lt - 1) * g.st) : s.ih - (uint32_t)g.st;
        n.edge[6] = e; n.edge[7] = f;
    }
    return n;
}

// Order in which workgroups visit the lattice.  bz = 0: lexicographic
// (x fastest, then y, z, t).  bz > 0: the (z, t) planes are visited in
// strips of bz consecutive z values, all t for one strip before the next
// strip, so the input records a site shares with its +-t neighbours are
// touched again within a window of about bz planes instead of a whole
// t-slice (this matters when many right-hand sides multiply the working set).
// Needs plane % S == 0 (S = sites per workgroup) and lz % bz == 0.
// bz < 0: the same with each (x, y) plane cut into two halves along y, all
// strips of the first half before the second: a column of half planes
// times |bz| z values walks t, which halves the window between +-t reuses
// for one more halo along y.  Needs plane % (2 S) == 0 and lz % |bz| == 0.
using Sched = SchedHost;    // built on the host by make_sched (weo_geom.h)

__host__ __device__ __forceinline__ uint32_t block_first_site(const Sched& s, const Geom& g, uint32_t blk,
                                                              uint32_t S) {
    if (s.bz == 0) return blk * S;
    if (s.bz < 0) {
        const uint32_t q = fdiv(blk, s.d_bpp);
        const uint32_t c = blk - q * s.d_bpp.d;        // block within the half plane
        const uint32_t q2 = fdiv(q, s.d_bz);
        const uint32_t zi = q - q2 * s.d_bz.d;
        const uint32_t q3 = fdiv(q2, s.d_lt);
        const uint32_t t = q2 - q3 * s.d_lt.d;
        const uint32_t half = fdiv(q3, s.d_nzb);
        const uint32_t zb = q3 - half * s.d_nzb.d;
        const uint32_t z = zb * s.d_bz.d + zi;
        return (half * s.d_bpp.d + c) * S + s.plane * (z + (uint32_t)g.lz * t);
    }
    const uint32_t q = fdiv(blk, s.d_bpp);
    const uint32_t c = blk - q * s.d_bpp.d;
    const uint32_t q2 = fdiv(q, s.d_bz);
    const uint32_t zi = q - q2 * s.d_bz.d;
    const uint32_t zb = fdiv(q2, s.d_lt);
    const uint32_t t = q2 - zb * s.d_lt.d;
    const uint32_t z = zb * s.d_bz.d + zi;
    return c * S + s.plane * (z + (uint32_t)g.lz * t);
}

// Sum over the 64 lanes of a wavefront (result in every lane).
__device__ __forceinline__ double wave_sum64(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Workgroup index remap: the hardware deals consecutive workgroups round-robin
// to the 8 XCDs (each with its own L2).  Map them so that XCD k works on one
// contiguous range of the lattice, keeping stencil neighbours in one L2.
__host__ __device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t nb, int remap) {
    if (!remap) return b;
    const uint32_t k = b & 7u, j = b >> 3, q = nb >> 3, r = nb & 7u;
    return k * q + (k < r ? k : r) + j;
}

}  // namespace weo
