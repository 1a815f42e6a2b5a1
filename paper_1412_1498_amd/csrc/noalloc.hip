// noalloc.hip -- gf_quality_noalloc: F (eq. 1) and theta (eqs. 2-3) of one
// lattice without a context and without any allocation, for callers that
// cannot allocate device memory (code under HIP graph capture, tight serving
// loops, harnesses that forbid it).
//
// The only scratch the reduction needs is one partial pair per quality tile.
// It lives in the file-scope device array `scratch` below, of a fixed size:
// every GPU the library runs on holds its own copy from the time the code
// object is loaded until the process ends. Its device address is looked up
// once per device (hipGetSymbolAddress, with that device current) and kept;
// host code uses only that address. Every tile writes its partial pair on
// every call, so nothing has to start at zero; but all calls on one GPU share
// the array, so calls that overlap in time on one GPU (different streams,
// threads) race on it and must be ordered by the caller.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <mutex>
#include <string>
#include <vector>

#include "gf.h"
#include "gf_internal.hpp"

namespace gf {

// Largest lattice: NOALLOC_MAX_TILES quality tiles of QTILE / 2 half sites,
// i.e. V <= 2^24 sites (48^4 and 48^3 x 96 fit); 1 MiB of scratch.
constexpr int NOALLOC_MAX_TILES = 1 << 16;

static __device__ __align__(256) double scratch[2 * NOALLOC_MAX_TILES];

namespace {

std::mutex scratch_mtx;
std::vector<double *> scratch_ptr;  // per device, nullptr until looked up

thread_local std::string last_error;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    last_error = buf;
    return code;
}

// Device address of `scratch` on the current device.
int device_scratch(double **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(GF_EDEVICE, "hipGetDevice failed: %s", hipGetErrorString(e));
    std::lock_guard<std::mutex> lock(scratch_mtx);
    if ((int)scratch_ptr.size() <= dev) scratch_ptr.resize(dev + 1, nullptr);
    if (!scratch_ptr[dev]) {
        double *p = nullptr;
        e = hipGetSymbolAddress((void **)&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(GF_EDEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                        hipGetErrorString(e));
        scratch_ptr[dev] = p;
    }
    *out = scratch_ptr[dev];
    return GF_OK;
}

}  // namespace

const char *noalloc_last_error() { return last_error.c_str(); }

}  // namespace gf

using namespace gf;

extern "C" int gf_quality_noalloc(const void *U, const int dims[4], int gauge, int prec, int storage,
                                  void *stream, double *out) {
    last_error.clear();
    if (!dims) return fail(GF_EINVAL, "dims is NULL");
    long long V = 1;
    for (int i = 0; i < 4; i++) {
        if (dims[i] < 2 || dims[i] % 2 != 0)
            return fail(GF_EINVAL, "dims[%d] = %d: every lattice dimension must be even and >= 2", i, dims[i]);
        V *= dims[i];
    }
    if (4 * V >= (1LL << 31)) return fail(GF_EINVAL, "lattice volume %lld too large", V);
    if (gauge != GF_LANDAU && gauge != GF_COULOMB) return fail(GF_EINVAL, "gauge = %d", gauge);
    if (prec != GF_F64 && prec != GF_F32) return fail(GF_EINVAL, "prec = %d", prec);
    if (storage != GF_STORE_18 && storage != GF_STORE_12 && storage != GF_STORE_8)
        return fail(GF_EINVAL, "storage = %d", storage);
    if (!U || (reinterpret_cast<uintptr_t>(U) & 15) != 0)
        return fail(GF_EINVAL, "U must be a non-NULL device pointer, at least 16-byte aligned");
    if (!out || (reinterpret_cast<uintptr_t>(out) & 7) != 0)
        return fail(GF_EINVAL, "out must be a non-NULL device pointer to 2 doubles, 8-byte aligned");
    const int nelem = storage == GF_STORE_12 ? 6 : storage == GF_STORE_8 ? 4 : 9;
    CfgDesc d{};
    d.g = make_geom(dims, nelem);
    d.U = const_cast<void *>(U);
    d.omega = 1.0;
    d.gauge = gauge;
    d.tile0 = 0;
    d.qtile0 = 0;
    d.nqtiles = (d.g.Vh + QTILE / 2 - 1) / (QTILE / 2);
    if (d.nqtiles > NOALLOC_MAX_TILES)
        return fail(GF_EINVAL,
                    "lattice of %lld sites exceeds the allocation-free limit of %lld sites (%d reduction tiles)",
                    V, (long long)NOALLOC_MAX_TILES * QTILE, NOALLOC_MAX_TILES);
    double *partials = nullptr;
    int rc = device_scratch(&partials);
    if (rc != GF_OK) return rc;
    const hipError_t e = launch_quality_one(prec, nelem, d, partials, out, (hipStream_t)stream);
    if (e != hipSuccess) return fail(GF_EDEVICE, "launch failed: %s", hipGetErrorString(e));
    return GF_OK;
}
