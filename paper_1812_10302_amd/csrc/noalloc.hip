// dtws_dtw_band without a context and without any allocation, for callers that cannot allocate
// device memory.  The only scratch memory the banded-DTW stage needs beyond its inputs and outputs
// is the prepared query (normalised, sentinel-padded, its envelope in visiting order); here it lives
// in one file-scope device array per GPU, whose device address is looked up once per device with
// hipGetSymbolAddress (host code never passes the array's own name to a kernel).
#include <mutex>

#include "dtws_internal.h"

namespace dtws {
namespace {

constexpr int kNaMaxM = 2048;
constexpr int kNaMaxBand = kDiagMaxBand;
constexpr int64_t kNaQstride = 2 * (int64_t)kQPad + kNaMaxM;           // floats of the padded query
constexpr size_t kNaQpadBytes = sizeof(float) * kNaQstride;
constexpr size_t kNaQhatBytes = sizeof(double) * kNaMaxM;
constexpr size_t kNaSortedBytes = sizeof(float) * kNaMaxM;               // per envelope / sorted array (5)
constexpr size_t kNaOrderBytes = sizeof(int32_t) * kNaMaxM;
constexpr size_t kScratchBytes = kNaQpadBytes + kNaQhatBytes + 5 * kNaSortedBytes + kNaOrderBytes;
static_assert(kNaQpadBytes % 8 == 0 && kNaQhatBytes % 8 == 0, "the FP64 query starts 8-byte aligned");

// The query scratch of every call on this device (about 105 KB, held until the process ends).
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kNaMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kNaMaxDevices] = {nullptr};   // device address of `scratch` on each device
int g_num_cu[kNaMaxDevices] = {0};

// Device address of the scratch array on the current device, looked up on the first call there.
int scratch_of(int *device, void **ptr, int *num_cu) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return DTWS_ENODEV;
    if (dev >= kNaMaxDevices) return DTWS_EINVAL;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return DTWS_EHIP;
        }
        int cu = 0;
        if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu <= 0) cu = 256;
        g_ptr[dev] = p;
        g_num_cu[dev] = cu;
    }
    *device = dev;
    *ptr = g_ptr[dev];
    *num_cu = g_num_cu[dev];
    return DTWS_OK;
}

}  // namespace
}  // namespace dtws

using namespace dtws;

extern "C" {

DTWS_API int dtws_dtw_band_noalloc(const float *T, int64_t n, const float *Q, int32_t m, int32_t r,
                                   const int64_t *starts, int64_t count, float abandon_at, float *dist, void *stream) {
    if (!T || !Q || !starts || !dist || m < 2 || m > kNaMaxM || n < m || r < 0 || count < 0) return DTWS_EINVAL;
    if (r > m - 1) r = m - 1;
    if (r > kNaMaxBand) return DTWS_EINVAL;
    if (count == 0) return DTWS_OK;
    int dev = 0, num_cu = 0;
    void *base = nullptr;
    const int rc = scratch_of(&dev, &base, &num_cu);
    if (rc != DTWS_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    uint8_t *p = (uint8_t *)base;
    QueryBufs b{};
    b.qpad = (float *)p;
    p += kNaQpadBytes;
    b.qhat64 = (double *)p;
    p += kNaQhatBytes;
    b.qsorted = (float *)p;
    p += kNaSortedBytes;
    b.Usorted = (float *)p;
    p += kNaSortedBytes;
    b.Lsorted = (float *)p;
    p += kNaSortedBytes;
    b.order = (int32_t *)p;
    p += kNaOrderBytes;
    b.Unat = (float *)p;
    p += kNaSortedBytes;
    b.Lnat = (float *)p;
    if (launch_query_prep(Q, m, r, b, s) != hipSuccess) return DTWS_EHIP;
    DtwArgs d{};
    d.T = T;
    d.m = m;
    d.r = r;
    d.w = 2 * r + 1;
    d.qpad = b.qpad;
    d.starts64 = starts;
    d.count = count;
    d.n = n;
    d.single = -1;
    d.abandon_at = abandon_at;
    d.nb_cap = kNearBestCap;
    d.dist_out = dist;
    // the schedule dtws_dtw_band picks by default: one wave per candidate for small counts and for
    // bands beyond the register kernel, else one lane per candidate (no global DP rows: r <= 1023)
    const bool wave = 2 * r + 1 > 16 * kMaxChunks || count <= 16384;
    hipError_t e;
    if (wave) {
        const int64_t blocks = (count + 1) / 2;
        e = launch_dtw_diag_list(d, false, (int)(blocks < num_cu * 8 ? blocks : num_cu * 8), s);
    } else {
        e = launch_dtw(d, false, count, num_cu, nullptr, 0, s);
    }
    return e == hipSuccess ? DTWS_OK : DTWS_EHIP;
}

}  // extern "C"
