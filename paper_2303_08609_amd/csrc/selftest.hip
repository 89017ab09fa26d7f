// Host-side self-test of the index arithmetic the kernels use (no GPU needed):
// fast division, site decoding, the 8 neighbour half indices with their edge
// flags, and the XCD workgroup remap.  Each is compared with a direct
// computation from lattice coordinates.
#include <stdint.h>

#include <vector>

#include "../../include/wilson_eo.h"
#include "weo_device.h"

namespace weo {

static int check_fastdiv() {
    for (uint32_t d = 1; d <= 200; ++d) {
        const FastDiv f = make_fastdiv(d);
        for (uint32_t n = 0; n < (1u << 16); ++n)
            if (fdiv(n, f) != n / d) return 1;
        for (uint32_t n = (1u << 31) - 70000; n < (1u << 31); n += 7)
            if (fdiv(n, f) != n / d) return 2;
    }
    return 0;
}

static uint32_t half_index(const Geom& g, int x, int y, int z, int t) {
    return (uint32_t)(x >> 1) + (uint32_t)g.lxh * ((uint32_t)y + (uint32_t)g.ly * ((uint32_t)z + (uint32_t)g.lz * (uint32_t)t));
}

static int check_geometry(const int dims[4]) {
    const Geom g = make_geom(dims);
    const int L[4] = {g.lx, g.ly, g.lz, g.lt};
    for (int par = 0; par < 2; ++par) {
        for (uint32_t ih = 0; ih < g.vh; ++ih) {
            const Site s = decode(g, ih, par);
            if (((s.x + s.y + s.z + s.t) & 1) != par) return 10;
            if (half_index(g, s.x, s.y, s.z, s.t) != ih) return 11;
            const Nbr nb = neighbours(g, s);
            for (int mu = 0; mu < 4; ++mu) {
                for (int dir = 0; dir < 2; ++dir) {
                    int c[4] = {s.x, s.y, s.z, s.t};
                    c[mu] += dir == 0 ? 1 : -1;
                    bool edge = false;
                    if (c[mu] == L[mu]) { c[mu] = 0; edge = true; }
                    if (c[mu] < 0) { c[mu] = L[mu] - 1; edge = true; }
                    const uint32_t want = half_index(g, c[0], c[1], c[2], c[3]);
                    if (nb.i[2 * mu + dir] != want) return 12;
                    if (nb.i[2 * mu + dir] >= g.vh) return 13;
                    if (nb.edge[2 * mu + dir] != edge) return 14;
                }
            }
        }
    }
    return 0;
}

static int check_remap() {
    for (uint32_t nb = 1; nb < 3000; nb += (nb < 64 ? 1 : 37)) {
        std::vector<char> seen(nb, 0);
        for (uint32_t b = 0; b < nb; ++b) {
            const uint32_t l = xcd_block(b, nb, 1);
            if (l >= nb || seen[l]) return 20;
            seen[l] = 1;
        }
    }
    return 0;
}

// Every site is visited exactly once under each workgroup schedule.
static int check_sched(const int dims[4]) {
    const Geom g = make_geom(dims);
    for (uint32_t S : {64u, 128u, 256u}) {
        for (int bz : {0, 2, 4, 8, -1, -2, -4, -8, -16}) {
            const Sched sc = make_sched(g, bz, S);
            if (bz && sc.bz == 0) continue;
            const uint32_t nblk = (g.vh + S - 1) / S;
            std::vector<char> seen(g.vh, 0);
            for (uint32_t b = 0; b < nblk; ++b) {
                const uint32_t f = block_first_site(sc, g, b, S);
                for (uint32_t t = 0; t < S; ++t) {
                    const uint32_t ih = f + t;
                    if (ih >= g.vh) {
                        if (sc.bz) return 31;     // blocked schedules have no ragged tail
                        continue;
                    }
                    if (seen[ih]) return 30;
                    seen[ih] = 1;
                }
            }
            for (uint32_t i = 0; i < g.vh; ++i)
                if (!seen[i]) return 32;
        }
    }
    return 0;
}

}  // namespace weo

extern "C" int weo_selftest(void) {
    using namespace weo;
    int rc = check_fastdiv();
    if (rc) return rc;
    const int shapes[][4] = {{2, 2, 2, 2}, {4, 4, 4, 4}, {4, 6, 2, 8}, {6, 4, 8, 2},
                             {10, 6, 4, 6}, {16, 16, 16, 32}, {24, 12, 10, 6}, {32, 32, 32, 64},
                             {48, 48, 48, 96}};
    for (const auto& d : shapes)
        if ((rc = check_geometry(d))) return rc;
    for (const auto& d : shapes)
        if ((rc = check_sched(d))) return rc;
    return check_remap();
}
