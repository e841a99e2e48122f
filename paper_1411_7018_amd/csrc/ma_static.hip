// The residual and its norm without allocation (ma_residual_noalloc,
// include/ma.h), for callers that cannot allocate device memory: code under
// hipGraph capture, tight serving loops, harnesses that forbid hipMalloc.
//
// It runs the kernels of ma_residual (the residual r = F - det D^2 u at the
// interior nodes with one partial sum of r^2 per block, then a fixed-order
// reduction of the partials) with the partials in `scratch`, a file-scope
// device array of fixed size instead of a solver's allocation.  Each device
// holds its own copy of the array, at its own address: the first call on a
// device looks that address up (hipGetSymbolAddress) with the device
// current and keeps it; every kernel then takes that pointer, never the
// array's name (which in host code is only a stand-in).  All calls on one
// device share the array, so calls that overlap on one device race.
#include "ma.h"
#include "ma_internal.h"
#include "ma_runtime.h"

#include <cmath>
#include <mutex>
#include <string>

namespace mafas {

namespace {

// Largest grid: the partials of n = MA_NOALLOC_MAX_N (8 x 128 x 511 blocks)
// plus the reduced sum.
constexpr int kMaxN = MA_NOALLOC_MAX_N;
constexpr size_t kScratchDoubles = 524288;   // 4 MiB per device
static_assert(kScratchDoubles >= 1 + (kMaxN - 1 + 63) / 64 * ((kMaxN - 1 + 3) / 4) *
                                         size_t(kMaxN - 1),
              "scratch holds the partials of the largest grid");

static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
double *g_ptr[kMaxDevices] = {};

// the device address of this device's scratch (looked up once per device)
hipError_t scratch_ptr(double **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    if (dev < 0 || dev >= kMaxDevices)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        g_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_ptr[dev];
    return hipSuccess;
}

// l2 = sqrt(sum * h * h * h), the expression ma_residual evaluates on the host
__global__ void k_l2(const double *__restrict__ sum, double h, double *__restrict__ l2)
{
    if (threadIdx.x == 0)
        *l2 = sqrt(sum[0] * h * h * h);
}

ma_status fail(ma_status st, const std::string &why)
{
    set_global_error(why);
    return st;
}

} // namespace

} // namespace mafas

using namespace mafas;

extern "C" ma_status ma_residual_noalloc(int n, const double *u, const double *f,
                                         double *r_or_null, double *l2_dev, void *hip_stream)
{
    if (n < 2 || n > kMaxN)
        return fail(MA_ERR_ARG, "ma_residual_noalloc: n must be in 2.." +
                                    std::to_string(kMaxN) + " (its static scratch is sized for "
                                    "n = " + std::to_string(kMaxN) + ")");
    if (!u || !f || !l2_dev)
        return fail(MA_ERR_ARG, "ma_residual_noalloc: u, f and l2_dev must be device pointers");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    double *sp = nullptr;
    hipError_t e = scratch_ptr(&sp);
    if (e != hipSuccess)
        return fail(MA_ERR_DEVICE, std::string("ma_residual_noalloc: scratch: ") +
                                       hipGetErrorString(e));
    double *sum = sp;
    double *partials = sp + 1;
    const size_t cnt = residual_partials(n);
    if (r_or_null) {
        const size_t pts = size_t(n + 1) * size_t(n + 1) * size_t(n + 1);
        if ((e = launch_fill(st, pts, 0.0, r_or_null)) != hipSuccess)
            return fail(MA_ERR_DEVICE, hipGetErrorString(e));
    }
    if ((e = launch_residual(st, OP_MA, n, u, f, r_or_null, partials)) != hipSuccess ||
        (e = launch_reduce(st, partials, cnt, sum)) != hipSuccess)
        return fail(MA_ERR_DEVICE, hipGetErrorString(e));
    hipLaunchKernelGGL(k_l2, dim3(1), dim3(64), 0, st, sum, 1.0 / double(n), l2_dev);
    if ((e = hipGetLastError()) != hipSuccess)
        return fail(MA_ERR_DEVICE, hipGetErrorString(e));
    return MA_OK;
}
