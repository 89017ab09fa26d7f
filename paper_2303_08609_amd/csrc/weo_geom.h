// Plain-data descriptions shared by host and device code of libwilson_eo.
#pragma once

#include <stdint.h>
#include <stddef.h>

namespace weo {

// Division by a runtime constant d (1 <= d < 2^31) for dividends n < 2^31:
// q = (umulhi(n, m) + n) >> s with s = ceil(log2 d) and
// m = floor(2^32 (2^s - d) / d) + 1 (round-up reciprocal, Granlund and
// Montgomery, PLDI 1994).
struct FastDiv {
    uint32_t d, m, s;
};

inline FastDiv make_fastdiv(uint32_t d) {
    FastDiv f;
    f.d = d;
    uint32_t s = 0;
    while ((1ull << s) < d) ++s;
    f.s = s;
    f.m = (uint32_t)((((1ull << 32) * ((1ull << s) - d)) / d) + 1);
    return f;
}

inline uint32_t host_fdiv(uint32_t n, const FastDiv& f) {
    const uint32_t hi = (uint32_t)(((uint64_t)n * f.m) >> 32);
    return (hi + n) >> f.s;
}

struct Geom {
    int lx, ly, lz, lt;     // extents
    int lxh;                // lx / 2
    uint32_t vh;            // sites per parity
    int sy, sz, st;         // half-index strides of y, z, t: lxh, lxh*ly, lxh*ly*lz
    FastDiv d_lxh, d_ly, d_lz;
};

inline Geom make_geom(const int dims[4]) {
    Geom g;
    g.lx = dims[0]; g.ly = dims[1]; g.lz = dims[2]; g.lt = dims[3];
    g.lxh = g.lx / 2;
    g.sy = g.lxh;
    g.sz = g.lxh * g.ly;
    g.st = g.lxh * g.ly * g.lz;
    g.vh = (uint32_t)((uint64_t)g.st * g.lt);
    g.d_lxh = make_fastdiv((uint32_t)g.lxh);
    g.d_ly = make_fastdiv((uint32_t)g.ly);
    g.d_lz = make_fastdiv((uint32_t)g.lz);
    return g;
}

// Schedule descriptor for block_first_site (weo_device.h); bz = 0 when the
// requested strip height does not fit the lattice or the workgroup size.
struct SchedHost {
    int bz;             // 0: lexicographic; > 0: z strips; < 0: half-plane columns
    uint32_t plane;
    FastDiv d_bpp;      // blocks per plane (strips) or per half plane (columns)
    FastDiv d_bz, d_lt;
    FastDiv d_nzb;      // strips of |bz| planes along z (columns)
};

// bz > 0 needs plane % S == 0, bz < 0 plane % (2 S) == 0; both need
// lz % |bz| == 0.  Otherwise the schedule is lexicographic (bz = 0).
inline SchedHost make_sched(const Geom& g, int bz, uint32_t sites_per_block) {
    SchedHost s;
    s.plane = (uint32_t)g.lxh * (uint32_t)g.ly;
    s.bz = 0;
    const uint32_t S = sites_per_block;
    const int az = bz < 0 ? -bz : bz;
    const uint32_t parts = bz < 0 ? 2u : 1u;
    if (bz != 0 && S > 0 && s.plane % (parts * S) == 0 && g.lz % az == 0) s.bz = bz;
    s.d_bpp = make_fastdiv(s.bz ? s.plane / (parts * S) : 1);
    s.d_bz = make_fastdiv(s.bz ? (uint32_t)az : 1);
    s.d_lt = make_fastdiv((uint32_t)g.lt);
    s.d_nzb = make_fastdiv(s.bz ? (uint32_t)(g.lz / az) : 1);
    return s;
}

// Built storage formats.  id = 2 * combo + (link12 ? 1 : 0).
enum FmtId : int {
    FMT_D_D_18 = 0, FMT_D_D_12 = 1,     // F64 spinor, F64 links
    FMT_S_S_18 = 2, FMT_S_S_12 = 3,     // F32 spinor, F32 links
    FMT_H_H_18 = 4, FMT_H_H_12 = 5,     // F16 spinor, F16 links
    FMT_B_H_18 = 6, FMT_B_H_12 = 7,     // BF16 spinor, F16 links
    FMT_COUNT = 8
};

}  // namespace weo
