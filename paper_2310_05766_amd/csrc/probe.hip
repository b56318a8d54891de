// Measurement aid, not part of the method: the device's rate for scattered
// 64-bit atomicMin, the operation that bounds the key-volume paths (vertical
// interpolation and free-space carving), on the same kind of footprint (a
// key volume of hundreds of MiB) or on an L2-resident one.
#include "internal.hpp"

namespace tsdf {

namespace {

__device__ __forceinline__ uint64_t mix64(uint64_t x)
{
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdull;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ull;
    x ^= x >> 33;
    return x;
}

__global__ __launch_bounds__(256) void k_atomic_probe(unsigned long long *keys, uint64_t span, int32_t per_lane)
{
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t x = mix64(t * 0x9E3779B97F4A7C15ull + 1);
    for (int32_t k = 0; k < per_lane; ++k) {
        const uint64_t h = mix64(x + (uint64_t)k);
        atomicMin(&keys[h % span], (unsigned long long)mix64(h));
    }
}

}  // namespace

}  // namespace tsdf

using namespace tsdf;

extern "C" tsdf_status tsdf_atomic_probe(void *keys_dev, int64_t n_keys, int32_t waves, int32_t per_lane,
                                         int32_t pattern, void *hip_stream, float *ms_out)
{
    constexpr int64_t kL2Keys = (int64_t)1 << 19;  // 4 MiB
    if (!keys_dev || !ms_out || waves < 4 || waves % 4 != 0 || per_lane < 1 || (pattern != 0 && pattern != 1))
        return TSDF_EINVAL;
    if (n_keys < (pattern == 1 ? kL2Keys : 1)) return TSDF_EINVAL;
    const uint64_t span = pattern == 1 ? (uint64_t)kL2Keys : (uint64_t)n_keys;
    hipStream_t s = (hipStream_t)hip_stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess) return TSDF_EDEVICE;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return TSDF_EDEVICE;
    }
    tsdf_status st = TSDF_OK;
    if (hipEventRecord(e0, s) != hipSuccess) st = TSDF_EDEVICE;
    if (st == TSDF_OK) {
        hipLaunchKernelGGL(k_atomic_probe, dim3((uint32_t)(waves / 4)), dim3(256), 0, s,
                           (unsigned long long *)keys_dev, span, per_lane);
        if (hipGetLastError() != hipSuccess || hipEventRecord(e1, s) != hipSuccess ||
            hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(ms_out, e0, e1) != hipSuccess)
            st = TSDF_EDEVICE;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}
