// Measurement aid for the benchmark, built as a library of its own
// (libtsdf_probe.so) and not part of the TSDF library: the device's rate for
// scattered 64-bit atomicMin, the operation that bounds the key-volume paths
// (vertical interpolation and free-space carving), on the same kind of
// footprint (a key volume of hundreds of MiB) or on an L2-resident one.
//
// int probe_atomic_min_rate(void *keys_dev, int64_t n_keys, int32_t waves,
//                           int32_t per_lane, int32_t pattern,
//                           void *hip_stream, float *ms_out)
// waves (a multiple of 4) wavefronts of 64 lanes each apply per_lane
// atomicMins to pseudo-random keys of the caller's device buffer of n_keys
// uint64, whose contents it overwrites: pattern 0 spreads them over the whole
// buffer, pattern 1 over its first 2^19 keys (4 MiB; needs n_keys >= 2^19).
// Synchronous: times the launch with events on hip_stream and writes the
// milliseconds to ms_out. Returns 0, -1 for bad arguments, -3 for a HIP
// error.
#include <hip/hip_runtime.h>
#include <stdint.h>

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

extern "C" int probe_atomic_min_rate(void *keys_dev, int64_t n_keys, int32_t waves, int32_t per_lane,
                                     int32_t pattern, void *hip_stream, float *ms_out)
{
    constexpr int kEinval = -1, kEdevice = -3;
    constexpr int64_t kL2Keys = (int64_t)1 << 19;  // 4 MiB
    if (!keys_dev || !ms_out || waves < 4 || waves % 4 != 0 || per_lane < 1 || (pattern != 0 && pattern != 1))
        return kEinval;
    if (n_keys < (pattern == 1 ? kL2Keys : 1)) return kEinval;
    const uint64_t span = pattern == 1 ? (uint64_t)kL2Keys : (uint64_t)n_keys;
    hipStream_t s = (hipStream_t)hip_stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess) return kEdevice;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return kEdevice;
    }
    int st = 0;
    if (hipEventRecord(e0, s) != hipSuccess) st = kEdevice;
    if (st == 0) {
        hipLaunchKernelGGL(k_atomic_probe, dim3((uint32_t)(waves / 4)), dim3(256), 0, s,
                           (unsigned long long *)keys_dev, span, per_lane);
        if (hipGetLastError() != hipSuccess || hipEventRecord(e1, s) != hipSuccess ||
            hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(ms_out, e0, e1) != hipSuccess)
            st = kEdevice;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}
