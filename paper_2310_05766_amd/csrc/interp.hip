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
// slots as touched (one byte per run, a plain store: an atomic that returns
// the old key, to mark only on the first candidate, is slower); a second
// kernel, one wave per 64 runs, merges the keys of touched runs (Eq. (1),
// Eq. (2)) and empties them again.
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
constexpr int kCarveChunkLog2 = 3;

// rdiv(n, d) = sign(n) floor((2|n| + d) / 2d), to nearest with ties away
// from zero, for a divisor 0 < d < 2^32 fixed per ray (given as 2d and
// 1 / 2d correctly rounded) and |n| < 2^61 with a quotient below 2^31: the
// float64 estimate is within one of the quotient, and one exact 64-bit
// correction each way fixes it (no integer division). Here, once per ray:
// d = r < 2^30 with n = 1024 D_a (the fills of each band voxel take the
// float64 forms band_len and fill_offset).
__device__ __forceinline__ int64_t rdiv_by(int64_t n, uint64_t d2, double inv_d2)
{
    const uint64_t a = (uint64_t)(n < 0 ? -n : n);
    const uint64_t num = 2 * a + (d2 >> 1);
    uint64_t k = (uint64_t)((double)num * inv_d2);
    k -= k * d2 > num ? 1u : 0u;
    k += (k + 1) * d2 <= num ? 1u : 0u;
    return n < 0 ? -(int64_t)k : (int64_t)k;
}

// Slot of a voxel inside the window: floor_mod(g_a, dims_a) per axis, z
// fastest.
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

// Eq. (1) with one unit of weight, Eq. (2) (|g w + v| <= tau (w + 1)).
__device__ __forceinline__ void merge_key(int16_t &sdf, int16_t &w, uint64_t key, int32_t w_max)
{
    const int64_t v = (int16_t)(uint16_t)(key & 0xffffu);
    const int64_t gw = w, gv = sdf;
    sdf = (int16_t)rdiv_small((int32_t)(gv * gw + v), (int32_t)(gw + 1));
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
    uint64_t valid = 0, visits = 0, atomics = 0;
    int32_t q[3];
    Ray R;
    if (i < P.n && quantise(P.xyz[3 * i], P.xyz[3 * i + 1], P.xyz[3 * i + 2], P.rp, q) && make_ray(q, P.rp, R)) {
        valid = 1;
        const int64_t rr = (int64_t)R.r;
        int64_t Di[3], v[3] = {0, 0, 0}, nv = 0, dd = 0;
        double vd[3] = {0.0, 0.0, 0.0}, nvh = 0.0, tt = 0.0;
        for (int a = 0; a < 3; ++a) Di[a] = (int64_t)R.D[a];
        const bool fills = P.dq > 0 && rr < ((int64_t)1 << 30);
        const uint64_t r2 = 2 * (uint64_t)rr;
        const double inv_r2 = 1.0 / (double)r2;
        uint64_t nv2 = 0;
        double inv_nv2 = 0.0;
        if (fills) {
            int64_t d[3], w[3];
            for (int a = 0; a < 3; ++a) {
                d[a] = rdiv_by(1024 * Di[a], r2, inv_r2);
                dd += Di[a] * Di[a];
            }
            w[0] = d[1] * P.up[2] - d[2] * P.up[1];
            w[1] = d[2] * P.up[0] - d[0] * P.up[2];
            w[2] = d[0] * P.up[1] - d[1] * P.up[0];
            v[0] = d[1] * w[2] - d[2] * w[1];
            v[1] = d[2] * w[0] - d[0] * w[2];
            v[2] = d[0] * w[1] - d[1] * w[0];
            nv = (int64_t)isqrt_u64((uint64_t)(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]));
            nv2 = 2 * (uint64_t)nv;
            inv_nv2 = nv > 0 ? 1.0 / (double)nv2 : 0.0;
            for (int a = 0; a < 3; ++a) vd[a] = (double)v[a];
            nvh = (double)nv + 0.5;
            tt = (double)(dd - rr * rr);  // |D|^2 - r^2, in [0, 2r]
        }
        Walk W;
        walk_init(R, W);
        const double taud = (double)P.rp.tau, rh = R.r + 0.5;
        const uint32_t ihi = (uint32_t)i >> 16, ilo = (uint32_t)i << 16;
        do {
            // a voxel of the band walk: band_key is pack_key(voxel_sdf(...))
            const unsigned long long key = band_key(W.n, rh, R.inv_r2, taud, ihi, ilo);
            // the fill segment of this band voxel: [c - e, c + e]
            int64_t e[3] = {0, 0, 0};
            if (fills && nv > 0) {
                // len = rdiv((c - o) . D, r), (c - o) . D = |D|^2 - n
                const double len = band_len(W.n, tt, R);
                if (len > 0.0) {
                    // h = rdiv(dq len, 2^20): dq len < 2^51 is exact, the
                    // scaling by 2^-20 too
                    const double h = fmin(floor(__fma_rn((double)P.dq, len, 524288.0) * 0x1p-20), 65535.0);
                    for (int a = 0; a < 3; ++a) e[a] = fill_offset(h * vd[a], nvh, inv_nv2);
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
                    const int64_t slot = window_slot(P, FW.g);
                    atomicMin(&P.keys[slot], key);
                    P.touched[slot >> 6] = 1;
                    ++visits;
                    ++atomics;
                }
            } while (walk_next(FW));
        } while (walk_next(W));
    }
    block_add(valid, &P.counters[0]);
    block_add(visits, &P.counters[1]);
    block_add(atomics, &P.counters[3]);
}

// One candidate: the atomic only when it would lower the key read, the
// run's mark only by a thread that read EMPTY (the first atomic on a slot in
// a scan comes from such a thread: no key can be read before one is written).
// Returns 1 when it issued the atomic.
__device__ __forceinline__ uint32_t offer_key(const InterpScan &P, int64_t sl, uint64_t key)
{
    unsigned long long *k = &P.keys[sl];
    const unsigned long long seen = *k;
    if (seen > key) {
        atomicMin(k, (unsigned long long)key);
        if (seen == kEmptyKey) P.touched[sl >> 6] = 1;
        return 1;
    }
    return 0;
}

// Free-space walks of neighbouring points (consecutive indices: neighbouring
// columns of one scan line) that start in the same voxel visit the voxels
// they share at the same step, so the wave walks in lockstep and a lane
// whose left neighbour holds the same slot with a smaller key leaves the
// candidate to it (that neighbour offers it, or is covered the same way by
// a smaller key further left). A lane whose walk has ended still shows the
// last candidate it held, which was offered.
// Free-space walks differ a lot in length (a wave runs as long as its longest
// lane), so each ray's free segment is cut into chunks: chunk c walks only
// the slab of voxels [(k0 + c) C, (k0 + c + 1) C) along the segment's longest
// axis, slabs of C = 2^kCarveChunkLog2 voxels in global coordinates counted
// from the slab k0 that holds the segment's lowest voxel inside the window.
// A wave holds one chunk of 64 consecutive rays, and consecutive waves take
// the chunks of one group of rays in turn (wave w: rays 64 (w / nch) + lane,
// chunk w mod nch), which spreads the atomics near the sensor, where all rays
// meet, over the whole launch instead of its first waves. Chunk 0 also walks
// the band. Four waves per SIMD: held to five, the walk state spills.
__global__ __launch_bounds__(kInterpBlock) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_carve_scan(InterpScan P,
                                                                                                      int64_t nch,
                                                                                                      int64_t block0)
{
    // block0: this launch's first block of the whole grid (the grid may be
    // split over several launches)
    const int64_t t = (block0 + (int64_t)blockIdx.x) * kInterpBlock + threadIdx.x;
    const int64_t w = t >> 6;
    const int64_t i = (w / nch) * 64 + (t & 63);
    const int32_t chunk = (int32_t)(w % nch);
    const int lane = (int)(threadIdx.x & 63u);
    uint64_t valid = 0, visits = 0, atomics = 0;
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
    bool act = false;
    if (ray && R.r > (double)P.rp.tau) {
        // the free segment [o, S]: its longest axis and its voxel range there
        int da = 0;
        int64_t best = -1;
        for (int a = 0; a < 3; ++a) {
            const int64_t L = (int64_t)R.S[a] - P.rp.o[a];
            const int64_t m = L < 0 ? -L : L;
            if (m > best) {
                best = m;
                da = a;
            }
        }
        const int32_t g0 = P.rp.o[da] >> 10, g1 = R.S[da] >> 10;
        int32_t gmin = g0 < g1 ? g0 : g1, gmax = g0 < g1 ? g1 : g0;
        gmin = gmin > lo[da] ? gmin : lo[da];
        gmax = gmax < hi[da] - 1 ? gmax : hi[da] - 1;
        const int32_t k = (gmin >> kCarveChunkLog2) + chunk;  // arithmetic shift: floor division
        const int32_t slo = k * (1 << kCarveChunkLog2), shi = slo + (1 << kCarveChunkLog2);
        if (gmin <= gmax && slo <= gmax) {
            lo[da] = lo[da] > slo ? lo[da] : slo;
            hi[da] = hi[da] < shi ? hi[da] : shi;
            act = lo[da] < hi[da] && free_walk_init(R, P.rp, lo, hi, F);
        }
        for (int a = 0; a < 3; ++a) {
            lo[a] = P.origin[a];
            hi[a] = P.origin[a] + P.dims[a];
        }
    }
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
            if (!(lane > 0 && left_sl == sl && left_key <= key)) atomics += offer_key(P, sl, key);
            ++visits;
            act = free_walk_next(F);
        }
    }
    if (ray && chunk == 0) {
        valid = 1;
        Walk W;
        walk_init(R, W);
        do {
            bool inside = true;
            for (int a = 0; a < 3; ++a) inside = inside && W.g[a] >= lo[a] && W.g[a] < hi[a];
            if (inside) {
                atomics += offer_key(P, window_slot(P, W.g), pack_key(voxel_sdf(W.n, R, P.rp.tau), (uint32_t)i));
                ++visits;
            }
        } while (walk_next(W));
    }
    block_add(valid, &P.counters[0]);
    block_add(visits, &P.counters[1]);
    block_add(atomics, &P.counters[3]);
}

// One wave per group of 64 runs of 64 slots: the wave reads the group's 64
// touched bytes at once and clears them, then merges the touched runs
// kMergeBatch at a time: the batch's keys are all requested together, then
// the voxels of its touched slots, so that a wave waits on two dependent
// reads per batch instead of per run.
constexpr int kMergeBatch = 8;

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
        while (mask) {
            int64_t j[kMergeBatch];
            unsigned long long key[kMergeBatch];
#pragma unroll
            for (int b = 0; b < kMergeBatch; ++b) {
                j[b] = 0;
                key[b] = kEmptyKey;
                if (mask) {
                    j[b] = (b0 + __builtin_ctzll(mask)) * 64 + lane;
                    mask &= mask - 1;
                    if (j[b] < nvox) key[b] = P.keys[j[b]];
                }
            }
            int16_t sv[kMergeBatch], wv[kMergeBatch];
#pragma unroll
            for (int b = 0; b < kMergeBatch; ++b) {
                sv[b] = 0;
                wv[b] = 0;
                if (key[b] != kEmptyKey) {
                    sv[b] = P.sdf[j[b]];
                    wv[b] = P.w[j[b]];
                }
            }
#pragma unroll
            for (int b = 0; b < kMergeBatch; ++b) {
                if (key[b] == kEmptyKey) continue;
                merge_key(sv[b], wv[b], key[b], P.w_max);
                P.sdf[j[b]] = sv[b];
                P.w[j[b]] = wv[b];
                P.keys[j[b]] = kEmptyKey;
                ++updated;
            }
        }
    }
    block_add(updated, &P.counters[2]);
}

}  // namespace

hipError_t launch_interp(const InterpScan &P, int64_t nvox, hipStream_t stream)
{
    if (P.n > 0) {
        const int64_t blocks = (P.n + kInterpBlock - 1) / kInterpBlock;
        if (P.carve) {
            // chunks of a ray: as many slabs as the window's longest side
            // spans, plus one for a slab boundary inside it
            int32_t dmax = P.dims[0] > P.dims[1] ? P.dims[0] : P.dims[1];
            dmax = dmax > P.dims[2] ? dmax : P.dims[2];
            const int64_t nchunk = ((int64_t)dmax + (1 << kCarveChunkLog2) - 1) / (1 << kCarveChunkLog2) + 1;
            // blocks * nchunk blocks in launches of at most 2^23 blocks
            // (2^31 work-items), so that no grid exceeds a launch's limits
            const int64_t total = blocks * nchunk, per = (int64_t)1 << 23;
            for (int64_t b0 = 0; b0 < total; b0 += per) {
                const int64_t nb = total - b0 < per ? total - b0 : per;
                hipLaunchKernelGGL(k_carve_scan, dim3((uint32_t)nb), dim3(kInterpBlock), 0, stream, P, nchunk, b0);
            }
        } else
            hipLaunchKernelGGL(k_interp_scan, dim3((uint32_t)blocks), dim3(kInterpBlock), 0, stream, P);
    }
    // four waves per block, one group of 64 runs per wave
    int64_t mblocks = ((nvox + 63) / 64 + 255) / 256;
    if (mblocks > 8192) mblocks = 8192;
    hipLaunchKernelGGL(k_interp_merge, dim3((uint32_t)(mblocks > 0 ? mblocks : 1)), dim3(256), 0, stream, P, nvox);
    return hipGetLastError();
}

}  // namespace tsdf
