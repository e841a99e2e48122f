// Storage of the FP32/FP64 mixed-precision form (outer FP64 defect
// correction).  The arithmetic lives in ma_mixed_device.h and runs inside
// the batched engine:
//   outer loop, FP64: r64 = f - S(u64) on the finest grid, its L2 norm, and
//   u64 += delta;
//   inner problem, FP32 FAS V-cycles on the correction delta,
//       T(delta) = det(H + D^2 delta) - det(H) = r64,   H = D^2 u64,
//   with coarse H_l = D^2_l (injection of u64).
#include "ma_runtime.h"

using namespace mafas;

namespace {
__global__ void k_zero32(float *__restrict__ dst, size_t count)
{
    const size_t q = blockIdx.x * size_t(blockDim.x) + threadIdx.x;
    if (q < count)
        dst[q] = 0.0f;
}
} // namespace

// FP32 d, b, w, r per level and an FP64 injected copy of u on coarse levels.
size_t mafas::mixed_bytes(const ma_params *p)
{
    int ns[32];
    const int L = ma_levels(p->n, ns, 32);
    size_t b = 0;
    for (int l = 0; l < L; ++l) {
        const size_t c = npts(ns[l]);
        b += 4 * c * sizeof(float);
        if (l > 0)
            b += c * sizeof(double);
    }
    return b;
}

ma_status ma_solver::mixed_allocate()
{
    int ns[32];
    const int L = ma_levels(p.n, ns, 32);
    mx.resize(L);
    auto falloc = [&](float **q, size_t count) -> ma_status {
        const hipError_t e = hipMalloc(reinterpret_cast<void **>(q), count * sizeof(float));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            *q = nullptr;
            return fail(MA_ERR_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
        }
        mixed_owned.push_back(*q);
        hipLaunchKernelGGL(k_zero32, dim3((count + 255) / 256), dim3(256), 0, stream, *q, count);
        return hipGetLastError() == hipSuccess ? MA_OK
                                               : fail(MA_ERR_DEVICE, "zeroing FP32 storage");
    };
    for (int l = 0; l < L; ++l) {
        MixedLevel &m = mx[l];
        m.n = ns[l];
        const size_t c = npts(m.n);
        MA_TRY(falloc(&m.d, c));
        MA_TRY(falloc(&m.b, c));
        MA_TRY(falloc(&m.w, c));
        MA_TRY(falloc(&m.r, c));
        if (l > 0)
            MA_TRY(alloc(&m.U, c));
    }
    return MA_OK;
}

void ma_solver::mixed_release()
{
    for (void *q : mixed_owned)
        (void)hipFree(q);
    mixed_owned.clear();
}
