// Plain per-scan integration (FeatSense, arXiv 2310.05766, Sec. VI).
//
// k_candidates is the paper's min-tsdf step: every ray walks its band and
// offers each resident voxel a packed key (|s|, point index, s); a 64-bit
// atomicMin keeps the smallest, so the per-scan volume V does not depend on
// the order in which rays arrive (the paper's atomicCAS retry loop admits
// several results on ties; the packed key admits exactly one). The first ray
// to reach a voxel (atomicMin returned EMPTY) appends its slot to the
// touched list, wave-aggregated.
//
// k_merge is the paper's averaging step, Eq. (1) and Eq. (2) with one unit
// of weight per scan, applied to the touched voxels only; it empties their
// keys again, and its last block publishes the scan's counters.
#include "internal.hpp"

namespace tsdf {

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Wave-aggregated append: each active lane with pred set gets a distinct
// index; one atomic per wave.
__device__ __forceinline__ uint32_t wave_append(uint32_t *counter, bool pred)
{
    const uint64_t mask = __ballot(pred);
    const uint32_t leader = (uint32_t)__ffsll((unsigned long long)mask) - 1u;
    uint32_t base = 0;
    if (mask != 0 && lane_id() == leader) base = atomicAdd(counter, (uint32_t)__popcll(mask));
    base = __shfl(base, (int)(mask != 0 ? leader : 0));
    const uint64_t below = mask & ((1ull << lane_id()) - 1ull);
    return base + (uint32_t)__popcll(below);
}

__global__ __launch_bounds__(kBlock) void k_candidates(ScanParams P, uint64_t *__restrict__ keys,
                                                       uint32_t *__restrict__ touched,
                                                       DevCounters *__restrict__ ctr)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    uint32_t valid = 0, visits = 0;
    Ray R;
    Walk W;
    bool active = false;
    if (i < P.n) {
        const float *p = P.xyz + 3 * i;
        int32_t q[3];
        if (quantise(p[0], p[1], p[2], P, q) && make_ray(q, P, R)) {
            valid = 1;
            active = true;
            walk_init(R, W);
        }
    }
    while (active) {
        const int64_t slot = window_slot(W.g, P);
        bool first = false;
        if (slot >= 0) {
            const int32_t s = voxel_sdf(W.n, R, P.tau);
            const uint64_t key = pack_key(s, (uint32_t)i);
            const uint64_t old = atomicMin((unsigned long long *)&keys[slot], (unsigned long long)key);
            first = (old == kEmptyKey);
            ++visits;
        }
        const uint32_t pos = wave_append(&ctr->touched, first);
        if (first) touched[pos] = (uint32_t)slot;
        active = walk_next(W);
    }
    // block totals, then one global atomic per block
    __shared__ uint32_t s_valid, s_visits;
    if (threadIdx.x == 0) { s_valid = 0; s_visits = 0; }
    __syncthreads();
    if (valid) atomicAdd(&s_valid, valid);
    if (visits) atomicAdd(&s_visits, visits);
    __syncthreads();
    if (threadIdx.x == 0) {
        if (s_valid) atomicAdd(&ctr->valid, s_valid);
        if (s_visits) atomicAdd(&ctr->visits, s_visits);
    }
}

// rdiv(n, d) for |n| < 2^30 + 2^15, 0 < d <= 32768, ties away from zero.
__device__ __forceinline__ int32_t rdiv_small(int32_t n, int32_t d)
{
    const uint32_t a = (uint32_t)(n < 0 ? -n : n);
    const uint32_t k = (2u * a + (uint32_t)d) / (2u * (uint32_t)d);
    return n < 0 ? -(int32_t)k : (int32_t)k;
}

__global__ __launch_bounds__(kBlock) void k_merge(uint64_t *__restrict__ keys, const uint32_t *__restrict__ touched,
                                                  DevCounters *__restrict__ ctr, int16_t *__restrict__ sdf,
                                                  int16_t *__restrict__ w, int32_t w_max)
{
    const uint32_t n = __atomic_load_n(&ctr->touched, __ATOMIC_RELAXED);
    for (uint32_t j = blockIdx.x * kBlock + threadIdx.x; j < n; j += gridDim.x * kBlock) {
        const uint32_t slot = touched[j];
        const uint64_t key = keys[slot];
        keys[slot] = kEmptyKey;
        const int32_t v = (int16_t)(uint16_t)(key & 0xffffu);
        const int32_t gw = w[slot];
        const int32_t gv = sdf[slot];
        sdf[slot] = (int16_t)rdiv_small(gv * gw + v, gw + 1);
        w[slot] = (int16_t)(gw + 1 < w_max ? gw + 1 : w_max);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const uint32_t ticket = atomicAdd(&ctr->done, 1u);
        if (ticket == gridDim.x - 1) {
            __threadfence();
            ctr->last[0] = __atomic_load_n(&ctr->touched, __ATOMIC_RELAXED);
            ctr->last[1] = __atomic_load_n(&ctr->valid, __ATOMIC_RELAXED);
            ctr->last[2] = __atomic_load_n(&ctr->visits, __ATOMIC_RELAXED);
            ctr->touched = 0;
            ctr->valid = 0;
            ctr->visits = 0;
            ctr->done = 0;
            __threadfence();
        }
    }
}

__global__ void k_fill_u64(uint64_t *p, int64_t n, uint64_t v)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
        p[j] = v;
}

__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t v)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
        p[j] = v;
}

}  // namespace

ScratchLayout ScratchLayout::of(int64_t nvox)
{
    ScratchLayout L;
    auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
    L.keys_off = 0;
    L.touched_off = up(L.keys_off + (size_t)nvox * sizeof(uint64_t));
    L.counters_off = up(L.touched_off + (size_t)nvox * sizeof(uint32_t));
    L.total = up(L.counters_off + sizeof(DevCounters));
    return L;
}

hipError_t launch_candidates(const ScanParams &P, uint64_t *keys, uint32_t *touched, DevCounters *ctr,
                             hipStream_t stream)
{
    if (P.n <= 0) return hipSuccess;
    const int64_t blocks = (P.n + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_candidates, dim3((uint32_t)blocks), dim3(kBlock), 0, stream, P, keys, touched, ctr);
    return hipGetLastError();
}

hipError_t launch_merge(uint64_t *keys, const uint32_t *touched, DevCounters *ctr, int16_t *sdf, int16_t *w,
                        int32_t w_max, hipStream_t stream)
{
    // 2048 blocks cover the touched list with a grid-stride loop; the list
    // length is only known on the device.
    hipLaunchKernelGGL(k_merge, dim3(2048), dim3(kBlock), 0, stream, keys, touched, ctr, sdf, w, w_max);
    return hipGetLastError();
}

hipError_t launch_fill_u64(uint64_t *p, int64_t n, uint64_t v, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_fill_u64, dim3((uint32_t)blocks), dim3(256), 0, stream, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_fill_u32, dim3((uint32_t)blocks), dim3(256), 0, stream, p, n, v);
    return hipGetLastError();
}

}  // namespace tsdf
