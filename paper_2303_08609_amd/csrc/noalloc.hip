// wilson_eo_apply_noalloc: the even-odd operator of Eq. (4) for callers that
// cannot allocate device memory (code under stream capture, tight serving
// loops, harnesses that forbid allocation).  The odd-parity intermediate
// field that wilson_eo_apply takes as a caller buffer (tmp) lives here in a
// file-scope device array instead; every call on a device shares that
// device's copy, so calls that overlap on one GPU race.
//
// Host code never passes the array's name to a kernel or a copy: its device
// address is looked up once per device with hipGetSymbolAddress (with that
// device current) and cached; the launches take that address.  The
// intermediate field is written in full by the first hop before the second
// hop reads it, so nothing needs clearing between calls.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/wilson_eo.h"
#include "weo_internal.h"

namespace weo {

// argument checks of the C ABI (abi.cpp)
int check_lattice(const weo_lattice* lat, Geom* g);
int check_fmt(const weo_format* f, int* id);

namespace {

__device__ __align__(256) uint8_t scratch[WEO_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (looked up on first use).
int scratch_ptr(int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices) return WEO_ERR_ARG;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return WEO_ERR_HIP;
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return WEO_OK;
}

}  // namespace
}  // namespace weo

extern "C" int wilson_eo_apply_noalloc(const weo_lattice* lat, const weo_format* fmt, int dagger,
                                       const void* u, const void* in, void* out, int nrhs, void* stream) {
    using namespace weo;
    Geom g;
    int id, rc;
    if ((rc = check_lattice(lat, &g)) != WEO_OK) return rc;
    if ((rc = check_fmt(fmt, &id)) != WEO_OK) return rc;
    if (nrhs < 1 || nrhs > WEO_MAX_RHS) return WEO_ERR_ARG;
    // the intermediate odd field of nrhs right-hand sides must fit the array
    if ((size_t)nrhs * spinor_field_bytes(g, id) > (size_t)WEO_NOALLOC_SCRATCH_BYTES) return WEO_ERR_WORKSPACE;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return WEO_ERR_HIP;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (s) {
        // the array used is the current device's: the stream must run there
        hipDevice_t sdev = -1;
        if (hipStreamGetDevice(s, &sdev) != hipSuccess) return WEO_ERR_HIP;
        if (sdev != dev) return WEO_ERR_ARG;
    }
    void* tmp = nullptr;
    if ((rc = scratch_ptr(dev, &tmp)) != WEO_OK) return rc;
    return wilson_eo_apply(lat, fmt, dagger, u, in, out, tmp, nrhs, stream);
}
