// gn_noalloc.hip -- the damped solve (G + mu I) delta = -g for callers that
// cannot allocate device memory: no handle, no hipMalloc, no library routine
// that allocates.  Its scratch (status word, diagonal-block inverses of the
// factor, the vectors of the two substitutions) is one file-scope device
// array, `scratch`, that every call on a GPU shares with every other call on
// that GPU; it keeps the last call's contents, and calls that overlap on one
// GPU race on it.  The kernels are those of gn_solve; the factorisation runs
// on the caller's stream only (no look-ahead stream).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>
#include <string>

#include "gn.h"
#include "gn_internal.h"

using namespace gn;

namespace {

constexpr int64_t kMaxOrder = GN_SOLVE_NOALLOC_MAX_ORDER;
constexpr int64_t kBlock = 128;                                   // diagonal block of the factor
constexpr int64_t kStatusDoubles = 32;                            // 256 bytes
constexpr int64_t kTmpDoubles = 64 * 64;
constexpr int64_t kLinvDoubles = (kMaxOrder + kBlock - 1) / kBlock * kBlock * kBlock;
constexpr int64_t kScratchDoubles = kStatusDoubles + kTmpDoubles + 2 * kMaxOrder + kLinvDoubles;
static_assert(sizeof(DevStatus) <= kStatusDoubles * sizeof(double), "status word does not fit its slot");
static_assert(kTmpDoubles % 32 == 0 && kMaxOrder % 32 == 0, "slots keep 256-byte alignment");

constexpr int kMaxDevices = 64;
double *g_scratch[kMaxDevices] = {};   // device address of `scratch` on each device (set once)
std::mutex g_mutex;
thread_local std::string g_err;

gn_status nerr(gn_status s, const char *fmt, long long v = 0) {
    char buf[256];
    snprintf(buf, sizeof buf, fmt, v);
    g_err = buf;
    return s;
}

}  // namespace

// 17.1 MB per GPU for order 16384: 128 inverse blocks of 128 x 128, two
// vectors, the status word and the diagonal factor's spill tile.
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

// Device address of `scratch` on the current device, looked up once per
// device with that device current.  In host code the array's name is only a
// host-side stand-in; kernels get this address.
gn_status scratch_on_device(double **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return nerr(GN_EDEVICE, "hipGetDevice failed (%lld)", (long long)e);
    if (dev < 0 || dev >= kMaxDevices) return nerr(GN_EDEVICE, "device index %lld out of range", dev);
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return nerr(GN_EDEVICE, "hipGetSymbolAddress(scratch) failed (%lld)", (long long)e);
        g_scratch[dev] = static_cast<double *>(p);
    }
    *out = g_scratch[dev];
    return GN_OK;
}

}  // namespace

const char *gn::noalloc_last_error() { return g_err.c_str(); }

#define NA_HIP(expr)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess) return nerr(GN_EDEVICE, "HIP error %lld", (long long)e_);  \
    } while (0)

extern "C" gn_status gn_solve_noalloc(void *stream, double *d_G, int64_t p, int64_t ldG, double mu,
                                      const double *d_g, double *d_delta, int64_t *h_info) {
    if (!d_G || !d_g || !d_delta) return nerr(GN_EINVAL, "null device pointer");
    if (p < 1) return nerr(GN_EINVAL, "order p = %lld < 1", (long long)p);
    if (p > kMaxOrder)
        return nerr(GN_EINVAL, "order p = %lld exceeds the scratch limit GN_SOLVE_NOALLOC_MAX_ORDER", (long long)p);
    if (ldG < p) return nerr(GN_EINVAL, "ldG = %lld < p", (long long)ldG);
    if (!(mu >= 0.0)) return nerr(GN_EINVAL, "mu must be >= 0");
    if (chol_linv_size(p) > kLinvDoubles || chol_tmp_size() > kTmpDoubles)
        return nerr(GN_EDEVICE, "scratch layout does not match the factorisation");
    double *base = nullptr;
    gn_status s = scratch_on_device(&base);
    if (s != GN_OK) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    DevStatus *status = reinterpret_cast<DevStatus *>(base);
    double *tmp = base + kStatusDoubles;
    double *y = tmp + kTmpDoubles;
    double *z = y + kMaxOrder;
    double *linv = z + kMaxOrder;
    // the status word is the only part that must start cleared (a fill kernel)
    NA_HIP(launch_reset_status(st, status));
    NA_HIP(launch_cholesky(st, nullptr, nullptr, nullptr, d_G, p, ldG, mu, 0, linv, tmp, status));
    NA_HIP(launch_copy_strided(st, d_g, p, 1, y, 1, -1.0));
    NA_HIP(launch_solve_lower(st, d_G, p, ldG, linv, y, z, status));
    NA_HIP(launch_solve_upper(st, d_G, p, ldG, linv, z, d_delta, status));
    NA_HIP(launch_check_finite(st, d_delta, p, status));
    DevStatus ds;
    NA_HIP(hipMemcpyAsync(&ds, status, sizeof ds, hipMemcpyDeviceToHost, st));
    NA_HIP(hipStreamSynchronize(st));
    if (h_info) *h_info = ds.chol_info;
    if (ds.flag) return nerr(GN_ENOTPD, "Cholesky pivot %lld is not positive", (long long)ds.chol_info);
    if (ds.nonfinite) return nerr(GN_ENONFINITE, "non-finite update");
    g_err.clear();
    return GN_OK;
}
