// Vertical interpolation between scan lines (FeatSense, arXiv 2310.05766,
// Sec. VI, Eq. (3) and Eq. (4)): every band voxel of a ray also gives its
// value to the voxels along the interpolation vector int = d x (d x up),
// up to the height h = delta_z * len above and below the ray, where len is
// the voxel's distance along the ray. The filled voxels of one band voxel
// are the exact floor-set of the segment [c - e, c + e] around its centre c,
// with e = h int / |int| in fixed point; each receives the band voxel's key,
// and the per-scan minimum over all keys (band and fill, all rays) decides.
//
// A fill reaches across tiles, so this form does not use the tiled engine:
// one thread walks one ray's band and each band voxel's fill segment and
// resolves keys with 64-bit atomicMin on a key volume over the window (8
// bytes per voxel, all EMPTY between scans) and marks the key's run of 64
// slots as touched (one byte per run, a plain store); a second kernel, one
// wave per 64 runs, merges the keys of touched runs (Eq. (1), Eq. (2)) and
// empties them again.
//
// Free-space carving uses the same key volume and merge: a ray longer than
// tau also walks [o, S] from the sensor to the start of its band (the long
// walk, clipped to the window), whose voxels take the ray's key like band
// voxels.
//
// A carving visit reads the key first and issues the atomic only when it
// would lower it (keys only fall during a scan, so a stale read at worst
// costs an atomic), and marks the run only when it read EMPTY: the path is
// bound by how many scattered 64-bit atomics and stores the L2 takes per
// second.
//
// Integer ranges (all exact): d = rdiv(1024 D, r) has |d| <= 1026, the up
// vector U is in 1/1024 units, so |int| < 2^31 and int . int < 2^62; a fill
// applies to rays of r < 2^30 (|D|^2 < 2^62); h is capped at 65535 (64
// voxels), so a fill segment spans |2 e_a| < 2^17 per axis, the range the
// exact walk is built for.
#include "internal.hpp"

namespace tsdf {

namespace {

constexpr int kInterpBlock = 256;

// rdiv(n, d) for d > 0: to nearest, ties away from zero (64-bit integers).
__device__ __forceinline__ int64_t rdiv64(int64_t n, int64_t d)
{
    const uint64_t a = (uint64_t)(n < 0 ? -n : n);
    const uint64_t k = (2 * a + (uint64_t)d) / (2 * (uint64_t)d);
    return n < 0 ? -(int64_t)k : (int64_t)k;
}

__device__ __forceinline__ int64_t floor_mod64(int64_t a, int64_t b)
{
    const int64_t m = a % b;
    return m < 0 ? m + b : m;
}

// Eq. (1) with one unit of weight, Eq. (2) (|g w + v| <= tau (w + 1)).
__device__ __forceinline__ void merge_key(int16_t &sdf, int16_t &w, uint64_t key, int32_t w_max)
{
    const int64_t v = (int16_t)(uint16_t)(key & 0xffffu);
    const int64_t gw = w, gv = sdf;
    sdf = (int16_t)rdiv64(gv * gw + v, gw + 1);
    w = (int16_t)(gw + 1 < w_max ? gw + 1 : w_max);
}

__device__ __forceinline__ void block_add(uint64_t v, unsigned long long *dst)
{
    __shared__ unsigned long long s_sum;
    if (threadIdx.x == 0) s_sum = 0;
    __syncthreads();
    if (v) atomicAdd(&s_sum, (unsigned long long)v);
    __syncthreads();
    if (threadIdx.x == 0 && s_sum) atomicAdd(dst, s_sum);
}

__global__ __launch_bounds__(kInterpBlock) void k_interp_scan(InterpScan P)
{
    const int64_t i = (int64_t)blockIdx.x * kInterpBlock + threadIdx.x;
    uint64_t valid = 0, visits = 0;
    int32_t q[3];
    Ray R;
    if (i < P.n && quantise(P.xyz[3 * i], P.xyz[3 * i + 1], P.xyz[3 * i + 2], P.rp, q) && make_ray(q, P.rp, R)) {
        valid = 1;
        const int64_t rr = (int64_t)R.r;
        int64_t Di[3], v[3] = {0, 0, 0}, nv = 0, dd = 0;
        for (int a = 0; a < 3; ++a) Di[a] = (int64_t)R.D[a];
        const bool fills = P.dq > 0 && rr < ((int64_t)1 << 30);
        if (fills) {
            int64_t d[3], w[3];
            for (int a = 0; a < 3; ++a) {
                d[a] = rdiv64(1024 * Di[a], rr);
                dd += Di[a] * Di[a];
            }
            w[0] = d[1] * P.up[2] - d[2] * P.up[1];
            w[1] = d[2] * P.up[0] - d[0] * P.up[2];
            w[2] = d[0] * P.up[1] - d[1] * P.up[0];
            v[0] = d[1] * w[2] - d[2] * w[1];
            v[1] = d[2] * w[0] - d[0] * w[2];
            v[2] = d[0] * w[1] - d[1] * w[0];
            nv = (int64_t)isqrt_u64((uint64_t)(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]));
        }
        Walk W;
        walk_init(R, W);
        do {
            const int32_t s = voxel_sdf(W.n, R, P.rp.tau);
            const unsigned long long key = pack_key(s, (uint32_t)i);
            // the fill segment of this band voxel: [c - e, c + e]
            int64_t e[3] = {0, 0, 0};
            if (fills && nv > 0) {
                // (c - o) . D = (q - o) . D - (q - c) . D, the walk's n
                const int64_t len = rdiv64(dd - (int64_t)W.n, rr);
                if (len > 0) {
                    int64_t h = rdiv64(P.dq * len, (int64_t)1 << 20);
                    h = h < 65535 ? h : 65535;
                    for (int a = 0; a < 3; ++a) e[a] = rdiv64(h * v[a], nv);
                }
            }
            Ray F;  // a segment only: the fill walk needs no distances
            for (int a = 0; a < 3; ++a) {
                const int32_t c = 1024 * W.g[a] + 512;
                F.S[a] = c - (int32_t)e[a];
                F.E[a] = c + (int32_t)e[a];
                F.q[a] = 0;
                F.D[a] = 0.0;
            }
            Walk FW;
            walk_init(F, FW);
            do {
                bool inside = true;
                for (int a = 0; a < 3; ++a)
                    inside = inside && FW.g[a] >= P.origin[a] && FW.g[a] < P.origin[a] + P.dims[a];
                if (inside) {
                    const int64_t slot =
                        (floor_mod64(FW.g[0], P.dims[0]) * P.dims[1] + floor_mod64(FW.g[1], P.dims[1])) * P.dims[2] +
                        floor_mod64(FW.g[2], P.dims[2]);
                    atomicMin(&P.keys[slot], key);
                    P.touched[slot >> 6] = 1;
                    ++visits;
                }
            } while (walk_next(FW));
        } while (walk_next(W));
    }
    block_add(valid, &P.counters[0]);
    block_add(visits, &P.counters[1]);
}

// Slot of a window voxel: floor_mod(g_a, dims_a) per axis, z fastest.
__device__ __forceinline__ int64_t window_slot(const InterpScan &P, const int32_t g[3])
{
    int64_t sl = 0;
    for (int a = 0; a < 3; ++a) {
        int32_t v = g[a] - P.origin[a] + P.ring0[a];
        v -= v >= P.dims[a] ? P.dims[a] : 0;
        sl = sl * P.dims[a] + v;
    }
    return sl;
}

// One candidate: the atomic only when it would lower the key read, the
// run's mark only by a thread that read EMPTY (the first atomic on a slot in
// a scan comes from such a thread: no key can be read before one is written).
__device__ __forceinline__ void offer_key(const InterpScan &P, int64_t sl, uint64_t key)
{
    unsigned long long *k = &P.keys[sl];
    const unsigned long long seen = *k;
    if (seen > key) {
        atomicMin(k, (unsigned long long)key);
        if (seen == kEmptyKey) P.touched[sl >> 6] = 1;
    }
}

// Free-space walks of neighbouring points (consecutive indices: neighbouring
// columns of one scan line) that start in the same voxel visit the voxels
// they share at the same step, so the wave walks in lockstep and a lane
// whose left neighbour holds the same slot with a smaller key leaves the
// candidate to it (that neighbour offers it, or is covered the same way by
// a smaller key further left). A lane whose walk has ended still shows the
// last candidate it held, which was offered.
__global__ __launch_bounds__(kInterpBlock) void k_carve_scan(InterpScan P)
{
    const int64_t i = (int64_t)blockIdx.x * kInterpBlock + threadIdx.x;
    const int lane = (int)(threadIdx.x & 63u);
    uint64_t valid = 0, visits = 0;
    int32_t q[3];
    Ray R;
    int32_t lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        lo[a] = P.origin[a];
        hi[a] = P.origin[a] + P.dims[a];
    }
    const bool ray = i < P.n && quantise(P.xyz[3 * i], P.xyz[3 * i + 1], P.xyz[3 * i + 2], P.rp, q) &&
                     make_ray(q, P.rp, R);
    FreeWalk F;
    bool act = ray && R.r > (double)P.rp.tau && free_walk_init(R, P.rp, lo, hi, F);
    int64_t sl = -1;
    uint64_t key = 0;
    while (__any(act)) {
        if (act) {
            sl = window_slot(P, F.W.g);
            key = free_walk_key(F, R, P.rp.tau, (uint32_t)i);
        }
        const int64_t left_sl = __shfl_up(sl, 1);
        const uint64_t left_key = __shfl_up(key, 1);
        if (act) {
            if (!(lane > 0 && left_sl == sl && left_key <= key)) offer_key(P, sl, key);
            ++visits;
            act = free_walk_next(F);
        }
    }
    if (ray) {
        valid = 1;
        Walk W;
        walk_init(R, W);
        do {
            bool inside = true;
            for (int a = 0; a < 3; ++a) inside = inside && W.g[a] >= lo[a] && W.g[a] < hi[a];
            if (inside) {
                offer_key(P, window_slot(P, W.g), pack_key(voxel_sdf(W.n, R, P.rp.tau), (uint32_t)i));
                ++visits;
            }
        } while (walk_next(W));
    }
    block_add(valid, &P.counters[0]);
    block_add(visits, &P.counters[1]);
}

// One wave per group of 64 runs of 64 slots: the wave reads the group's 64
// touched bytes at once and clears them, then merges the touched runs one
// after the other, each run's keys read before the previous run is written
// back (a run's keys, then its voxels: two dependent reads per run).
__global__ __launch_bounds__(256) void k_interp_merge(InterpScan P, int64_t nvox)
{
    uint64_t updated = 0;
    const int64_t nruns = (nvox + 63) / 64;
    const int64_t ngroups = (nruns + 63) / 64;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
    const int64_t waves = (int64_t)gridDim.x * blockDim.x / 64;
    const int lane = (int)(threadIdx.x & 63u);
    for (int64_t gi = wave; gi < ngroups; gi += waves) {
        const int64_t b0 = gi * 64;
        const bool t = b0 + lane < nruns && P.touched[b0 + lane] != 0;
        if (t) P.touched[b0 + lane] = 0;
        uint64_t mask = __ballot(t);  // the same for the whole wave
        if (!mask) continue;
        int64_t j = (b0 + __builtin_ctzll(mask)) * 64 + lane;
        unsigned long long key = j < nvox ? P.keys[j] : kEmptyKey;
        for (;;) {
            mask &= mask - 1;
            int64_t jn = 0;
            unsigned long long keyn = kEmptyKey;
            if (mask) {
                jn = (b0 + __builtin_ctzll(mask)) * 64 + lane;
                if (jn < nvox) keyn = P.keys[jn];
            }
            if (key != kEmptyKey) {
                merge_key(P.sdf[j], P.w[j], key, P.w_max);
                P.keys[j] = kEmptyKey;
                ++updated;
            }
            if (!mask) break;
            j = jn;
            key = keyn;
        }
    }
    block_add(updated, &P.counters[2]);
}

}  // namespace

hipError_t launch_interp(const InterpScan &P, int64_t nvox, hipStream_t stream)
{
    if (P.n > 0) {
        const int64_t blocks = (P.n + kInterpBlock - 1) / kInterpBlock;
        if (P.carve)
            hipLaunchKernelGGL(k_carve_scan, dim3((uint32_t)blocks), dim3(kInterpBlock), 0, stream, P);
        else
            hipLaunchKernelGGL(k_interp_scan, dim3((uint32_t)blocks), dim3(kInterpBlock), 0, stream, P);
    }
    // four waves per block, one group of 64 runs per wave
    int64_t mblocks = ((nvox + 63) / 64 + 255) / 256;
    if (mblocks > 8192) mblocks = 8192;
    hipLaunchKernelGGL(k_interp_merge, dim3((uint32_t)(mblocks > 0 ? mblocks : 1)), dim3(256), 0, stream, P, nvox);
    return hipGetLastError();
}

}  // namespace tsdf
