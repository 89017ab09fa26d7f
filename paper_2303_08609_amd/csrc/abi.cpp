// extern "C" entry points of libwilson_eo: argument validation, format
// tables and dispatch to the HIP launchers.  Host-only C++ (no kernels here):
// every check runs before the first HIP call, so a bad argument never reaches
// the device.
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstdint>
#include <cstring>

#include "../../include/wilson_eo.h"
#include "weo_internal.h"

namespace weo {

static const FmtInfo k_fmt[FMT_COUNT] = {
    // spinor, link, link12, spinor site bytes, link bytes, wide
    {WEO_F64, WEO_F64, 0, 12 * 16, 9 * 16, 1},
    {WEO_F64, WEO_F64, 1, 12 * 16, 6 * 16, 1},
    {WEO_F32, WEO_F32, 0, 12 * 8, 9 * 8, 0},
    {WEO_F32, WEO_F32, 1, 12 * 8, 6 * 8, 0},
    {WEO_F16, WEO_F16, 0, 12 * 4, 9 * 4, 0},
    {WEO_F16, WEO_F16, 1, 12 * 4, 6 * 4, 0},
    {WEO_BF16, WEO_F16, 0, 12 * 4, 9 * 4, 0},
    {WEO_BF16, WEO_F16, 1, 12 * 4, 6 * 4, 0},
};

const FmtInfo& fmt_info(int id) { return k_fmt[id]; }

int format_id(const weo_format* f) {
    if (!f) return -1;
    if (f->link_fmt != WEO_LINK18 && f->link_fmt != WEO_LINK12) return -1;
    for (int i = 0; i < FMT_COUNT; ++i)
        if (k_fmt[i].spinor_prec == f->spinor_prec && k_fmt[i].link_prec == f->link_prec &&
            k_fmt[i].link12 == (f->link_fmt == WEO_LINK12))
            return i;
    return -1;
}

// Largest supported sites per parity: keeps every plane below 2^31 bytes
// so that per-lane 32-bit byte offsets cannot wrap.
static const uint64_t k_max_vh = 1ull << 26;

int check_lattice(const weo_lattice* lat, Geom* g) {
    if (!lat) return WEO_ERR_ARG;
    uint64_t v = 1;
    for (int m = 0; m < 4; ++m) {
        const int L = lat->dims[m];
        if (L < 2 || (L & 1)) return WEO_ERR_DIMS;
        v *= (uint64_t)L;
        if (v > 2 * k_max_vh) return WEO_ERR_DIMS;
        if (!std::isfinite(lat->bc[m][0]) || !std::isfinite(lat->bc[m][1])) return WEO_ERR_ARG;
    }
    if (!std::isfinite(lat->kappa)) return WEO_ERR_ARG;
    if (g) *g = make_geom(lat->dims);
    return WEO_OK;
}

int check_fmt(const weo_format* f, int* id) {
    if (!f) return WEO_ERR_ARG;
    const int known = (unsigned)f->spinor_prec <= WEO_BF16 && (unsigned)f->link_prec <= WEO_BF16 &&
                      (f->link_fmt == WEO_LINK18 || f->link_fmt == WEO_LINK12);
    if (!known) return WEO_ERR_ARG;
    const int i = format_id(f);
    if (i < 0) return WEO_ERR_FORMAT;
    if (id) *id = i;
    return WEO_OK;
}

int check_ptr(const void* p) {
    if (!p) return WEO_ERR_ARG;
    if (reinterpret_cast<uintptr_t>(p) & 255u) return WEO_ERR_ALIGN;
    return WEO_OK;
}

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
    const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return x < y + nb && y < x + na;
}

void phases_of(const weo_lattice* lat, double ph[4][2]) {
    for (int m = 0; m < 4; ++m) { ph[m][0] = lat->bc[m][0]; ph[m][1] = lat->bc[m][1]; }
}

int hip_status(hipError_t e) { return e == hipSuccess ? WEO_OK : WEO_ERR_HIP; }

}  // namespace weo

using namespace weo;

#define WEO_TRY(expr)                 \
    do {                              \
        const int _rc = (expr);       \
        if (_rc != WEO_OK) return _rc; \
    } while (0)

extern "C" {

const char* wilson_eo_strerror(int code) {
    switch (code) {
        case WEO_OK: return "ok";
        case WEO_ERR_ARG: return "invalid argument (null pointer, bad enum or count, or overlapping buffers)";
        case WEO_ERR_DIMS: return "invalid lattice extents (each must be even and >= 2; volume limited)";
        case WEO_ERR_ALIGN: return "buffer base pointer not 256-byte aligned";
        case WEO_ERR_FORMAT: return "precision / link-format combination not built into this library";
        case WEO_ERR_HIP: return "HIP runtime error";
        case WEO_ERR_WORKSPACE: return "workspace missing or too small";
        case WEO_NOT_CONVERGED: return "solver did not reach the tolerance within its iteration caps";
        case WEO_BREAKDOWN: return "solver breakdown (non-positive or non-finite scalar)";
        default: return "unknown status code";
    }
}

int weo_format_supported(const weo_format* fmt) { return format_id(fmt) >= 0 ? 1 : 0; }

int weo_set_mrhs_shape(int nr, int sites, int persist, int bz, int split) {
    return set_mrhs_shape(nr, sites, persist, bz, split) == 0 ? WEO_OK : WEO_ERR_ARG;
}

int weo_tuning_report(char* buf, size_t len) {
    if (buf && len) buf[0] = 0;
    const int n = tuning_report(buf, len);
    if (buf && len) buf[len - 1] = 0;
    return n;
}

size_t weo_gauge_bytes(const weo_lattice* lat, const weo_format* fmt) {
    Geom g;
    int id;
    if (check_lattice(lat, &g) != WEO_OK || check_fmt(fmt, &id) != WEO_OK) return 0;
    return gauge_field_bytes(g, id);
}

size_t weo_spinor_bytes(const weo_lattice* lat, const weo_format* fmt, int nrhs) {
    Geom g;
    int id;
    if (check_lattice(lat, &g) != WEO_OK || check_fmt(fmt, &id) != WEO_OK) return 0;
    if (nrhs < 1 || nrhs > WEO_MAX_RHS) return 0;
    return (size_t)nrhs * spinor_field_bytes(g, id);
}

int weo_pack_gauge(const weo_lattice* lat, const weo_format* fmt, const void* u_canon, int canon_prec,
                   void* u_packed, void* stream) {
    Geom g;
    int id;
    WEO_TRY(check_lattice(lat, &g));
    WEO_TRY(check_fmt(fmt, &id));
    if (canon_prec != WEO_F64 && canon_prec != WEO_F32) return WEO_ERR_ARG;
    WEO_TRY(check_ptr(u_canon));
    WEO_TRY(check_ptr(u_packed));
    const size_t nc = (size_t)g.vh * 2 * 4 * 9 * (canon_prec == WEO_F64 ? 16 : 8);
    if (overlaps(u_canon, nc, u_packed, gauge_field_bytes(g, id))) return WEO_ERR_ARG;
    return hip_status(launch_pack_gauge(g, id, u_canon, canon_prec == WEO_F64, u_packed,
                                        static_cast<hipStream_t>(stream)));
}

int weo_pack_spinor(const weo_lattice* lat, const weo_format* fmt, int nrhs, const void* s_canon,
                    int canon_prec, double scale, void* s_packed, void* stream) {
    Geom g;
    int id;
    WEO_TRY(check_lattice(lat, &g));
    WEO_TRY(check_fmt(fmt, &id));
    if (nrhs < 1 || nrhs > WEO_MAX_RHS || !std::isfinite(scale)) return WEO_ERR_ARG;
    if (canon_prec != WEO_F64 && canon_prec != WEO_F32) return WEO_ERR_ARG;
    WEO_TRY(check_ptr(s_canon));
    WEO_TRY(check_ptr(s_packed));
    const size_t nc = (size_t)nrhs * g.vh * 12 * (canon_prec == WEO_F64 ? 16 : 8);
    if (overlaps(s_canon, nc, s_packed, (size_t)nrhs * spinor_field_bytes(g, id))) return WEO_ERR_ARG;
    return hip_status(launch_pack_spinor(g, id, nrhs, s_canon, canon_prec == WEO_F64, scale, s_packed,
                                         static_cast<hipStream_t>(stream)));
}

int weo_unpack_spinor(const weo_lattice* lat, const weo_format* fmt, int nrhs, const void* s_packed,
                      double scale, void* s_canon, int canon_prec, void* stream) {
    Geom g;
    int id;
    WEO_TRY(check_lattice(lat, &g));
    WEO_TRY(check_fmt(fmt, &id));
    if (nrhs < 1 || nrhs > WEO_MAX_RHS || !std::isfinite(scale)) return WEO_ERR_ARG;
    if (canon_prec != WEO_F64 && canon_prec != WEO_F32) return WEO_ERR_ARG;
    WEO_TRY(check_ptr(s_canon));
    WEO_TRY(check_ptr(s_packed));
    const size_t nc = (size_t)nrhs * g.vh * 12 * (canon_prec == WEO_F64 ? 16 : 8);
    if (overlaps(s_canon, nc, s_packed, (size_t)nrhs * spinor_field_bytes(g, id))) return WEO_ERR_ARG;
    return hip_status(launch_unpack_spinor(g, id, nrhs, s_packed, scale, s_canon, canon_prec == WEO_F64,
                                           static_cast<hipStream_t>(stream)));
}

int wilson_eo_hop(const weo_lattice* lat, const weo_format* fmt, int out_parity, int dagger,
                  const void* u, const void* in, void* out, int nrhs, void* stream) {
    Geom g;
    int id;
    WEO_TRY(check_lattice(lat, &g));
    WEO_TRY(check_fmt(fmt, &id));
    if ((out_parity != 0 && out_parity != 1) || (dagger != 0 && dagger != 1)) return WEO_ERR_ARG;
    if (nrhs < 1 || nrhs > WEO_MAX_RHS) return WEO_ERR_ARG;
    WEO_TRY(check_ptr(u));
    WEO_TRY(check_ptr(in));
    WEO_TRY(check_ptr(out));
    const size_t sb = (size_t)nrhs * spinor_field_bytes(g, id);
    if (overlaps(in, sb, out, sb) || overlaps(u, gauge_field_bytes(g, id), out, sb)) return WEO_ERR_ARG;
    HopLaunch h;
    h.g = g;
    h.fmt = id;
    h.out_par = out_parity;
    h.dagger = dagger;
    phases_of(lat, h.phase);
    h.u = u;
    h.in = in;
    h.out = out;
    h.y = nullptr;
    h.alpha = 0.0;
    h.partial = nullptr;
    h.nrhs = nrhs;
    return hip_status(launch_hop(h, static_cast<hipStream_t>(stream)));
}

size_t weo_face_bytes(const weo_lattice* lat, const weo_format* fmt, int mu, int nrhs) {
    Geom g;
    int id;
    if (check_lattice(lat, &g) != WEO_OK || check_fmt(fmt, &id) != WEO_OK) return 0;
    if (nrhs < 1 || nrhs > WEO_MAX_RHS || mu < 0 || mu > 3) return 0;
    return (size_t)nrhs * face_field_bytes(g, id, mu);
}

int wilson_eo_face_pack(const weo_lattice* lat, const weo_format* fmt, int mu, int out_parity, int dagger,
                        const void* u, const void* in, void* send_lo, void* send_hi, int nrhs,
                        void* stream) {
    Geom g;
    int id;
    WEO_TRY(check_lattice(lat, &g));
    WEO_TRY(check_fmt(fmt, &id));
    if ((out_parity != 0 && out_parity != 1) || (dagger != 0 && dagger != 1)) return WEO_ERR_ARG;
    if (mu < 0 || mu > 3) return WEO_ERR_ARG;
    if (nrhs < 1 || nrhs > WEO_MAX_RHS) return WEO_ERR_ARG;
    WEO_TRY(check_ptr(u));
    WEO_TRY(check_ptr(in));
    WEO_TRY(check_ptr(send_lo));
    WEO_TRY(check_ptr(send_hi));
    const size_t sb = (size_t)nrhs * spinor_field_bytes(g, id);
    const size_t fb = (size_t)nrhs * face_field_bytes(g, id, mu);
    const size_t ub = gauge_field_bytes(g, id);
    if (overlaps(send_lo, fb, send_hi, fb) || overlaps(send_lo, fb, in, sb) ||
        overlaps(send_hi, fb, in, sb) || overlaps(send_lo, fb, u, ub) || overlaps(send_hi, fb, u, ub))
        return WEO_ERR_ARG;
    return hip_status(launch_face_pack(g, id, mu, out_parity, dagger, u, in, send_lo, send_hi, nrhs,
                                       static_cast<hipStream_t>(stream)));
}

int wilson_eo_face_unpack(const weo_lattice* lat, const weo_format* fmt, int mu, int out_parity, int dagger,
                          const double phase_lo[2], const double phase_hi[2], double alpha,
                          const void* u, const void* recv_lo, const void* recv_hi, void* out,
                          int nrhs, void* stream) {
    Geom g;
    int id;
    WEO_TRY(check_lattice(lat, &g));
    WEO_TRY(check_fmt(fmt, &id));
    if ((out_parity != 0 && out_parity != 1) || (dagger != 0 && dagger != 1)) return WEO_ERR_ARG;
    if (mu < 0 || mu > 3) return WEO_ERR_ARG;
    if (nrhs < 1 || nrhs > WEO_MAX_RHS || !std::isfinite(alpha)) return WEO_ERR_ARG;
    if (!phase_lo || !phase_hi) return WEO_ERR_ARG;
    for (int k = 0; k < 2; ++k)
        if (!std::isfinite(phase_lo[k]) || !std::isfinite(phase_hi[k])) return WEO_ERR_ARG;
    WEO_TRY(check_ptr(u));
    WEO_TRY(check_ptr(recv_lo));
    WEO_TRY(check_ptr(recv_hi));
    WEO_TRY(check_ptr(out));
    const size_t sb = (size_t)nrhs * spinor_field_bytes(g, id);
    const size_t fb = (size_t)nrhs * face_field_bytes(g, id, mu);
    if (overlaps(recv_lo, fb, out, sb) || overlaps(recv_hi, fb, out, sb) ||
        overlaps(u, gauge_field_bytes(g, id), out, sb))
        return WEO_ERR_ARG;
    return hip_status(launch_face_unpack(g, id, mu, out_parity, dagger, phase_lo, phase_hi, alpha, u,
                                         recv_lo, recv_hi, out, nrhs, static_cast<hipStream_t>(stream)));
}

int wilson_eo_hop_axpy(const weo_lattice* lat, const weo_format* fmt, int out_parity, int dagger,
                       double alpha, const void* u, const void* in, const void* y, void* out, int nrhs,
                       void* stream) {
    Geom g;
    int id;
    WEO_TRY(check_lattice(lat, &g));
    WEO_TRY(check_fmt(fmt, &id));
    if ((out_parity != 0 && out_parity != 1) || (dagger != 0 && dagger != 1)) return WEO_ERR_ARG;
    if (nrhs < 1 || nrhs > WEO_MAX_RHS || !std::isfinite(alpha)) return WEO_ERR_ARG;
    WEO_TRY(check_ptr(u));
    WEO_TRY(check_ptr(in));
    WEO_TRY(check_ptr(y));
    WEO_TRY(check_ptr(out));
    const size_t sb = (size_t)nrhs * spinor_field_bytes(g, id);
    // each lane reads its own y record before writing the same out record,
    // so y == out is safe; partial overlap is not
    if (overlaps(in, sb, out, sb) || overlaps(u, gauge_field_bytes(g, id), out, sb) ||
        (y != out && overlaps(y, sb, out, sb)))
        return WEO_ERR_ARG;
    HopLaunch h;
    h.g = g;
    h.fmt = id;
    h.out_par = out_parity;
    h.dagger = dagger;
    phases_of(lat, h.phase);
    h.u = u;
    h.in = in;
    h.out = out;
    h.y = y;
    h.alpha = alpha;
    h.partial = nullptr;
    h.nrhs = nrhs;
    return hip_status(launch_hop(h, static_cast<hipStream_t>(stream)));
}

size_t weo_clover_bytes(const weo_lattice* lat, const weo_format* fmt) {
    Geom g;
    int id;
    if (check_lattice(lat, &g) != WEO_OK || check_fmt(fmt, &id) != WEO_OK) return 0;
    return clover_field_bytes(g, id);
}

int weo_pack_clover(const weo_lattice* lat, const weo_format* fmt, const void* canon, int canon_prec, int invert,
                    void* packed, void* stream) {
    Geom g;
    int id;
    WEO_TRY(check_lattice(lat, &g));
    WEO_TRY(check_fmt(fmt, &id));
    if (canon_prec != WEO_F64 && canon_prec != WEO_F32) return WEO_ERR_ARG;
    if (invert != 0 && invert != 1) return WEO_ERR_ARG;
    WEO_TRY(check_ptr(canon));
    WEO_TRY(check_ptr(packed));
    const size_t nc = (size_t)g.vh * 2 * 2 * 36 * (canon_prec == WEO_F64 ? 16 : 8);
    if (overlaps(canon, nc, packed, clover_field_bytes(g, id))) return WEO_ERR_ARG;
    return hip_status(launch_pack_clover(g, id, canon, canon_prec == WEO_F64, invert, packed,
                                         static_cast<hipStream_t>(stream)));
}

int wilson_eo_clover_site(const weo_lattice* lat, const weo_format* fmt, int parity, const void* clover,
                          const void* in, const void* y, double alpha, void* out, int nrhs, void* stream) {
    Geom g;
    int id;
    WEO_TRY(check_lattice(lat, &g));
    WEO_TRY(check_fmt(fmt, &id));
    if ((parity != 0 && parity != 1) || nrhs < 1 || nrhs > WEO_MAX_RHS || !std::isfinite(alpha))
        return WEO_ERR_ARG;
    WEO_TRY(check_ptr(clover));
    WEO_TRY(check_ptr(in));
    WEO_TRY(check_ptr(out));
    if (y) WEO_TRY(check_ptr(y));
    const size_t sb = (size_t)nrhs * spinor_field_bytes(g, id);
    if (overlaps(in, sb, out, sb) || overlaps(clover, clover_field_bytes(g, id), out, sb)) return WEO_ERR_ARG;
    return hip_status(launch_clover_site(g, id, parity, clover, in, y, alpha, out, nrhs,
                                         static_cast<hipStream_t>(stream)));
}

int wilson_eo_clover_hop(const weo_lattice* lat, const weo_format* fmt, int out_parity, int dagger,
                         const void* u, const void* clover, const void* in, const void* y, double alpha,
                         void* out, int nrhs, void* stream) {
    Geom g;
    int id;
    WEO_TRY(check_lattice(lat, &g));
    WEO_TRY(check_fmt(fmt, &id));
    if ((out_parity != 0 && out_parity != 1) || (dagger != 0 && dagger != 1)) return WEO_ERR_ARG;
    if (nrhs < 1 || nrhs > WEO_MAX_RHS || !std::isfinite(alpha)) return WEO_ERR_ARG;
    WEO_TRY(check_ptr(u));
    WEO_TRY(check_ptr(clover));
    WEO_TRY(check_ptr(in));
    WEO_TRY(check_ptr(out));
    if (y) WEO_TRY(check_ptr(y));
    const size_t sb = (size_t)nrhs * spinor_field_bytes(g, id);
    if (overlaps(in, sb, out, sb) || overlaps(u, gauge_field_bytes(g, id), out, sb) ||
        overlaps(clover, clover_field_bytes(g, id), out, sb))
        return WEO_ERR_ARG;
    HopLaunch h;
    h.g = g;
    h.fmt = id;
    h.out_par = out_parity;
    h.dagger = dagger;
    phases_of(lat, h.phase);
    h.u = u;
    h.in = in;
    h.out = out;
    h.y = y;
    h.alpha = y ? alpha : 0.0;
    h.partial = nullptr;
    h.nrhs = nrhs;
    return hip_status(launch_hop_clover(h, clover, static_cast<hipStream_t>(stream)));
}

int wilson_eo_clover_apply(const weo_lattice* lat, const weo_format* fmt, int dagger, const void* u,
                           const void* clover_inv, const void* in, void* out, void* tmp, int nrhs, void* stream) {
    Geom g;
    int id;
    WEO_TRY(check_lattice(lat, &g));
    WEO_TRY(check_fmt(fmt, &id));
    if (dagger != 0 && dagger != 1) return WEO_ERR_ARG;
    if (nrhs < 1 || nrhs > WEO_MAX_RHS) return WEO_ERR_ARG;
    WEO_TRY(check_ptr(u));
    WEO_TRY(check_ptr(clover_inv));
    WEO_TRY(check_ptr(in));
    WEO_TRY(check_ptr(out));
    WEO_TRY(check_ptr(tmp));
    const size_t sb = (size_t)nrhs * spinor_field_bytes(g, id);
    const size_t gb = gauge_field_bytes(g, id), cb = clover_field_bytes(g, id);
    if (overlaps(in, sb, out, sb) || overlaps(in, sb, tmp, sb) || overlaps(out, sb, tmp, sb) ||
        overlaps(u, gb, out, sb) || overlaps(u, gb, tmp, sb) || overlaps(clover_inv, cb, out, sb) ||
        overlaps(clover_inv, cb, tmp, sb))
        return WEO_ERR_ARG;
    double ph[4][2];
    phases_of(lat, ph);
    return hip_status(launch_apply_clover(g, id, ph, lat->kappa, dagger, u, clover_inv, in, out, tmp, nrhs,
                                          nullptr, static_cast<hipStream_t>(stream)));
}

int wilson_eo_apply(const weo_lattice* lat, const weo_format* fmt, int dagger, const void* u,
                    const void* in, void* out, void* tmp, int nrhs, void* stream) {
    Geom g;
    int id;
    WEO_TRY(check_lattice(lat, &g));
    WEO_TRY(check_fmt(fmt, &id));
    if (dagger != 0 && dagger != 1) return WEO_ERR_ARG;
    if (nrhs < 1 || nrhs > WEO_MAX_RHS) return WEO_ERR_ARG;
    WEO_TRY(check_ptr(u));
    WEO_TRY(check_ptr(in));
    WEO_TRY(check_ptr(out));
    WEO_TRY(check_ptr(tmp));
    const size_t sb = (size_t)nrhs * spinor_field_bytes(g, id);
    const size_t gb = gauge_field_bytes(g, id);
    if (overlaps(in, sb, out, sb) || overlaps(in, sb, tmp, sb) || overlaps(out, sb, tmp, sb) ||
        overlaps(u, gb, out, sb) || overlaps(u, gb, tmp, sb))
        return WEO_ERR_ARG;
    HopLaunch h;
    h.g = g;
    h.fmt = id;
    h.dagger = dagger;
    phases_of(lat, h.phase);
    h.u = u;
    h.nrhs = nrhs;
    h.partial = nullptr;
    // tmp_o = H_oe in
    h.out_par = 1;
    h.in = in;
    h.out = tmp;
    h.y = nullptr;
    h.alpha = 0.0;
    hipStream_t s = static_cast<hipStream_t>(stream);
    WEO_TRY(hip_status(launch_hop(h, s)));
    // out_e = in - kappa^2 H_eo tmp_o
    h.out_par = 0;
    h.in = tmp;
    h.out = out;
    h.y = in;
    h.alpha = -lat->kappa * lat->kappa;
    return hip_status(launch_hop(h, s));
}

// ---- Schwarz alternating procedure ------------------------------------------
static int sap_checks(const weo_lattice* lat, const weo_format* fmt, int nrhs, Geom* g, int* id) {
    WEO_TRY(check_lattice(lat, g));
    WEO_TRY(check_fmt(fmt, id));
    if (fmt_info(*id).spinor_prec != WEO_F32 || fmt_info(*id).link_prec != WEO_F32) return WEO_ERR_FORMAT;
    if (nrhs < 1 || nrhs > WEO_MAX_RHS) return WEO_ERR_ARG;
    // full fields: both parities, per-lane offsets stay below 2^31 per plane
    if ((uint64_t)g->vh > (1ull << 25)) return WEO_ERR_DIMS;
    return WEO_OK;
}

static size_t round256(size_t n) { return (n + 255) & ~(size_t)255; }

size_t wilson_eo_sap_workspace_bytes(const weo_lattice* lat, const weo_format* fmt, int nrhs) {
    Geom g;
    int id;
    if (sap_checks(lat, fmt, nrhs, &g, &id) != WEO_OK) return 0;
    return 3 * round256((size_t)nrhs * 2 * spinor_field_bytes(g, id));
}

int wilson_eo_sap(const weo_lattice* lat, const weo_format* fmt, const weo_sap_params* sap, const void* u,
                  const void* eta, void* psi, void* workspace, size_t ws_bytes, int nrhs, void* stream) {
    Geom g;
    int id;
    WEO_TRY(sap_checks(lat, fmt, nrhs, &g, &id));
    if (!sap || sap->ncy < 1 || sap->nmr < 1 || sap->nmr > 64) return WEO_ERR_ARG;
    SapGeom sg;
    if (make_sap_geom(g, sap->block, &sg) != 0) return WEO_ERR_ARG;
    WEO_TRY(check_ptr(u));
    WEO_TRY(check_ptr(eta));
    WEO_TRY(check_ptr(psi));
    if (!workspace) return WEO_ERR_WORKSPACE;
    WEO_TRY(check_ptr(workspace));
    const size_t nb = (size_t)nrhs * 2 * spinor_field_bytes(g, id), fb = round256(nb);
    if (ws_bytes < 3 * fb) return WEO_ERR_WORKSPACE;
    const size_t gb = gauge_field_bytes(g, id);
    if (overlaps(eta, nb, psi, nb) || overlaps(workspace, 3 * fb, psi, nb) || overlaps(workspace, 3 * fb, eta, nb) ||
        overlaps(u, gb, psi, nb) || overlaps(u, gb, workspace, 3 * fb))
        return WEO_ERR_ARG;
    double ph[4][2];
    phases_of(lat, ph);
    uint8_t* w = static_cast<uint8_t*>(workspace);
    return hip_status(sap_apply(g, id, sg, sap->ncy, sap->nmr, lat->kappa, ph, u, eta, psi, w, w + fb, w + 2 * fb,
                                nrhs, static_cast<hipStream_t>(stream)));
}

int wilson_eo_force(const weo_lattice* lat, const weo_format* fmt, const void* u, const void* lam_e,
                    const void* lam_o, const void* r_e, const void* r_o, double coeff, int flags,
                    void* g_canon, int canon_prec, void* stream) {
    Geom g;
    int id;
    WEO_TRY(check_lattice(lat, &g));
    WEO_TRY(check_fmt(fmt, &id));
    if ((flags & ~(WEO_FORCE_PROJECT | WEO_FORCE_ACCUMULATE)) || !std::isfinite(coeff)) return WEO_ERR_ARG;
    if (canon_prec != WEO_F64 && canon_prec != WEO_F32) return WEO_ERR_ARG;
    const void* ptrs[6] = {u, lam_e, lam_o, r_e, r_o, g_canon};
    for (const void* q : ptrs) WEO_TRY(check_ptr(q));
    const size_t ob = (size_t)g.vh * 2 * 4 * 9 * (canon_prec == WEO_F64 ? 16 : 8);
    const size_t sb = spinor_field_bytes(g, id);
    for (int i = 0; i < 5; ++i)
        if (overlaps(ptrs[i], i == 0 ? gauge_field_bytes(g, id) : sb, g_canon, ob)) return WEO_ERR_ARG;
    double ph[4][2];
    phases_of(lat, ph);
    return hip_status(launch_force(g, id, ph, u, lam_e, lam_o, r_e, r_o, coeff, flags, g_canon,
                                   canon_prec == WEO_F64, static_cast<hipStream_t>(stream)));
}

}  // extern "C"
