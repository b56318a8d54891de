// Batched integration (FeatSense, arXiv 2310.05766, Sec. VI): any number of
// registered scans, into any number of maps, in one pass of five kernels.
//
// Each map window is cut into tiles of 2^lt voxels per axis (window-relative
// coordinates). The per-scan volume V of the min-tsdf step never reaches HBM:
// a workgroup owns one tile, keeps its candidate keys (|s|, point index, s)
// in LDS and resolves them with ds_min_u64 (order independent, one winner per
// voxel), then applies the averaging step, Eq. (1) and Eq. (2), to the tile.
// When several scans of one map share a batch, the tile's SDF and weights
// stay in LDS while its workgroup applies those scans one after another, in
// submission order, and go back to HBM once.
//
//   k_bin<count>  every ray walks its band on the grid of tiles (the exact
//                 walk with tile-sized cells) and counts one entry per tile;
//                 keys are (sequence slot, tile), merged per block in an LDS
//                 table so that each block sends one atomic per distinct key
//   k_alloc       a run of the entry buffer per (sequence slot, tile), runs of
//                 one tile consecutive in sequence order; list of busy tiles
//   k_bin<fill>   the same walk, writing point indices into the runs
//   k_tile        per busy tile, per sequence slot in order: every ray jumps
//                 to its first voxel in the tile (exact crossing counts) and
//                 walks the tile; candidates meet in LDS; then the merge
//   k_stats       per-scan counts, when asked for
#include <string.h>

#include "internal.hpp"

namespace tsdf {

namespace {

constexpr int kAllocBlock = 512;

__device__ __forceinline__ uint32_t lane() { return __lane_id(); }

// A map array seen as global memory: through a generic pointer the compiler
// must assume it may alias the LDS buffers, and it then waits for every map
// load before the LDS store that follows it.
typedef __attribute__((address_space(1))) int16_t glob_i16;
__device__ __forceinline__ glob_i16 *glob(int16_t *p) { return (glob_i16 *)p; }

template <int kLog2>
__device__ __forceinline__ uint32_t hash_slot(uint32_t key)
{
    return (key * 2654435761u) >> (32 - kLog2);
}

// Second half of an entry record: what the tile pass needs of the ray
// beyond its point, r = isqrt(|D|^2) and the band offsets off = E - q (both
// exact: r < 2^32, |off_a| <= tau < 2^15), and the voxel crossings per axis
// (each < 2^7) up to the event that entered the tile.
__device__ __forceinline__ uint4 entry_ray(const Ray &R, uint32_t cpack)
{
    const uint32_t o0 = (uint32_t)(R.E[0] - R.q[0]) & 0xffffu, o1 = (uint32_t)(R.E[1] - R.q[1]) & 0xffffu,
                   o2 = (uint32_t)(R.E[2] - R.q[2]) & 0xffffu;
    return make_uint4((uint32_t)R.r, o0 | o1 << 16, o2 | (cpack & 0xffffu) << 16, cpack >> 16);
}

// kInline (counting pass only): the batch is one scan whose descriptors are
// I, not yet in memory.
template <bool kFill, int kBinBlock, bool kInline>
__global__ __launch_bounds__(kBinBlock) void k_bin(BatchArrays B, InlineDesc I)
{
    // the block's (sequence slot, tile) keys: a hash table of two slots per
    // point of the block (a block of 256 OS1-128 points meets about 100
    // tiles), so that clearing and flushing it stays cheap; keys that find it
    // full go straight to their runs
    constexpr int kHashLog2 = kBinBlock == 128 ? 8 : (kBinBlock == 256 ? 9 : 10);
    constexpr uint32_t kHashSlots = 1u << kHashLog2;
    static_assert(kHashSlots == 2 * kBinBlock && kHashSlots <= 1024, "slots fit the 10-bit field below");
    __shared__ uint32_t h_key[kHashSlots];  // key + 1; 0 = free
    __shared__ uint32_t h_cnt[kHashSlots];
    __shared__ uint32_t h_base[kFill ? kHashSlots : 1];
    // per emitted entry: hash slot | crossing counts (7 bits per axis) << 10, and rank
    __shared__ uint32_t s_slot[kFill ? kMaxEmit * kBinBlock : 1];
    __shared__ uint16_t s_rank[kFill ? kMaxEmit * kBinBlock : 1];
    __shared__ uint32_t s_valid;
    // a one-scan batch's descriptors come with the counting launch, which
    // stores them for the kernels after it
    constexpr bool inl = !kFill && kInline;
    const BatchHdr H = inl ? I.hdr : *B.hdr;
    if (inl && blockIdx.x == 0 && threadIdx.x == 0) {
        *B.hdr = I.hdr;
        B.maps[0] = I.map;
        B.scans[0] = I.scan;
        B.seq_sensor[0] = make_int4(I.scan.rp.o[0], I.scan.rp.o[1], I.scan.rp.o[2], I.scan.rp.tau);
    }
    if (!kFill && blockIdx.x == 0 && threadIdx.x == 0) {
        // the allocation counters of the previous batch are done with (the
        // grid always has a block 0, also for a batch without points)
        B.ctl->n_nonempty = 0;
        B.ctl->n_light = 0;
        B.ctl->entries = 0;
        B.ctl->overflow = 0;
        for (int q = 0; q < kQueues; ++q) B.ctl->work[q * kQueueStride] = 0;
    }
    if (blockIdx.x >= H.nblocks) return;
    for (uint32_t j = threadIdx.x; j < kHashSlots; j += kBinBlock) {
        h_key[j] = 0;
        h_cnt[j] = 0;
    }
    if (threadIdx.x == 0) s_valid = 0;
    __syncthreads();

    // (a one-scan batch's block table is written here, for the fill)
    if (inl && threadIdx.x == 0) B.block_scan[blockIdx.x] = 0u;
    const uint32_t s = inl ? 0u : B.block_scan[blockIdx.x];
    const ScanDev &SD = inl ? I.scan : B.scans[s];
    const MapDev &MD = inl ? I.map : B.maps[SD.map];
    const int64_t i = (int64_t)(blockIdx.x - SD.block0) * kBinBlock + threadIdx.x;
    const RayParams rp = SD.rp;
    Ray R;
    Walk W, Wv;  // the walk on the tile grid; the voxel walk's start (fill)
    bool active = false;
    int32_t q[3] = {0, 0, 0};
    if (i < SD.n) {
        const float *p = SD.xyz + 3 * i;
        if (quantise(p[0], p[1], p[2], rp, q) && make_ray(q, rp, R)) {
            active = true;
            // the tiles of the band's voxels are the cells of the same exact
            // walk on the grid of tiles (floor of a floor division)
            const int32_t lc[3] = {10 + H.lt[0], 10 + H.lt[1], 10 + H.lt[2]};
            const int32_t base[3] = {1024 * MD.origin[0], 1024 * MD.origin[1], 1024 * MD.origin[2]};
            walk_init_cells(R, W, lc, base);
            if (kFill) walk_init(R, Wv);
        }
    }
    const uint32_t valid = active ? 1u : 0u;
    const uint32_t key0 = (uint32_t)SD.seq * H.gtiles + MD.tile_base;
    // the map's tile counts in registers: loads through MD inside the walk
    // would be repeated after every atomic (they may alias)
    const uint32_t nt0 = (uint32_t)__builtin_amdgcn_readfirstlane(MD.nt[0]);
    const uint32_t nt1 = (uint32_t)__builtin_amdgcn_readfirstlane(MD.nt[1]);
    const uint32_t nt2 = (uint32_t)__builtin_amdgcn_readfirstlane(MD.nt[2]);
    int ne = 0;
    uint32_t listed = 0;  // fill: bit k set when entry k was listed in LDS (not sent straight to its run)
    double t_in = -1.0;  // event that entered the current tile (none for the first)
    int typ_in = 0;
    while (active) {
        if ((uint32_t)W.g[0] < nt0 && (uint32_t)W.g[1] < nt1 && (uint32_t)W.g[2] < nt2) {
            const uint32_t key =
                key0 + ((uint32_t)W.g[0] * nt1 + (uint32_t)W.g[1]) * nt2 + (uint32_t)W.g[2];
            uint32_t h = hash_slot<kHashLog2>(key), slot = 0xffffu;
            for (uint32_t probe = 0; probe < kHashSlots; ++probe) {
                const uint32_t old = atomicCAS(&h_key[h], 0u, key + 1u);
                if (old == 0u || old == key + 1u) {
                    slot = h;
                    break;
                }
                h = (h + 1u) & (kHashSlots - 1u);
            }
            // voxel crossings of each axis up to the event that entered
            // this tile: the tile pass resumes the voxel walk there
            uint32_t cpack = 0;
            if (kFill && t_in >= 0.0) {
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    cpack |= (uint32_t)crossings_upto(Wv.T[a], Wv.dT[a], Wv.step[a] > 0 ? 0 : 1, t_in, typ_in)
                             << (8 * a);
            }
            if (slot != 0xffffu && (!kFill || ne < kMaxEmit)) {
                const uint32_t rank = atomicAdd(&h_cnt[slot], 1u);
                if (kFill) {
                    s_slot[ne * kBinBlock + threadIdx.x] = slot | counts_8to7(cpack) << 10;
                    s_rank[ne * kBinBlock + threadIdx.x] = (uint16_t)rank;
                    listed |= 1u << ne;
                }
            } else if (kFill) {  // table full or very long band: straight to the tile's run
                const uint32_t pos = atomicAdd(&B.cursor[key], 1u);
                if (pos < H.cap) {
                    B.entries[pos] = make_uint4((uint32_t)i, (uint32_t)q[0], (uint32_t)q[1], (uint32_t)q[2]);
                    B.entries2[pos] = entry_ray(R, cpack);
                } else {
                    atomicOr(&B.ctl->overflow, 1u);
                }
            } else {
                atomicAdd(&B.counts[key], 1u);
            }
            ++ne;
        }
        active = walk_next_event(W, t_in, typ_in);
    }
    if (!kFill && valid) atomicAdd(&s_valid, 1u);
    __syncthreads();
    // one global atomic per distinct key of this block
    for (uint32_t j = threadIdx.x; j < kHashSlots; j += kBinBlock) {
        const uint32_t k1 = h_key[j];
        const uint32_t c = h_cnt[j];
        if (k1 == 0u || c == 0u) continue;
        if (kFill) h_base[j] = atomicAdd(&B.cursor[k1 - 1u], c);
        else atomicAdd(&B.counts[k1 - 1u], c);
    }
    if (!kFill) {
        if (threadIdx.x == 0) B.valid_part[blockIdx.x] = s_valid;
        return;
    }
    __syncthreads();
    // each record carries the point's fixed-point position, so the tile pass
    // needs neither the point nor the pose again
    const uint4 rec = make_uint4((uint32_t)i, (uint32_t)q[0], (uint32_t)q[1], (uint32_t)q[2]);
    // the entries listed in LDS: an entry that found the table full went
    // straight to its run and left its LDS place unwritten
    const int nl = ne < kMaxEmit ? ne : kMaxEmit;
    for (int k = 0; k < nl; ++k) {
        if (!((listed >> k) & 1u)) continue;
        const uint32_t sc = s_slot[k * kBinBlock + threadIdx.x];
        const uint32_t pos = h_base[sc & 1023u] + s_rank[k * kBinBlock + threadIdx.x];
        if (pos < H.cap) {
            B.entries[pos] = rec;
            B.entries2[pos] = entry_ray(R, counts_7to8(sc >> 10));
        } else {
            atomicOr(&B.ctl->overflow, 1u);
        }
    }
}

// Map slot of a global tile: the last map whose first tile is <= g.
__device__ __forceinline__ int32_t map_of_tile(const BatchArrays &B, int32_t nmaps, uint32_t g)
{
    int32_t lo = 0, hi = nmaps - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (B.maps[mid].tile_base <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Runs of the entry buffer: one per (sequence slot, tile), a tile's runs
// consecutive in sequence order; the tile is listed as busy. Runs may lie in
// any order, so they are handed out by atomic allocation, one atomic per
// block and counter (same-address device atomics serialise; a block prefix
// keeps them few). Four lanes share a tile, each summing a quarter of its
// sequence slots, so that the chains of count loads stay short.
constexpr int kAllocTiles = kAllocBlock / 4;
constexpr int kAllocPer = kMaxSeq / 4;  // sequence slots per lane, at most
// A tile with this many entries or more is listed first: the persistent tile
// pass then starts the longest tiles early instead of ending on one of them.
constexpr uint32_t kHeavyTile = 2048;

__global__ __launch_bounds__(kAllocBlock) void k_alloc(BatchArrays B)
{
    __shared__ uint32_t s_w[3][kAllocBlock / 64];  // per wave: entries, heavy tiles, light tiles
    __shared__ uint32_t s_base[3];
    const BatchHdr H = *B.hdr;
    if (blockIdx.x * kAllocTiles >= H.gtiles) return;
    const uint32_t t = blockIdx.x * kAllocTiles + threadIdx.x / 4;
    const uint32_t part = threadIdx.x & 3u, wave = threadIdx.x / 64;
    const int per = (H.S + 3) / 4;  // at most kAllocPer
    const int s_lo = (int)part * per, s_hi = min(H.S, s_lo + per);
    // this part's counts, kept for the runs: every load is issued (at a
    // clamped, valid index) before any is used, so all are in flight together
    uint32_t cs[kAllocPer];
    const uint32_t tc = min(t, H.gtiles - 1u);
#pragma unroll
    for (int j = 0; j < kAllocPer; ++j) cs[j] = B.counts[(uint32_t)min(s_lo + j, H.S - 1) * H.gtiles + tc];
#pragma unroll
    for (int j = 0; j < kAllocPer; ++j) cs[j] = (t < H.gtiles && s_lo + j < s_hi) ? cs[j] : 0u;
    uint32_t c = 0;
    uint64_t busy = 0;  // this part's busy sequence slots
#pragma unroll
    for (int j = 0; j < kAllocPer; ++j) {
        c += cs[j];
        busy |= cs[j] ? 1ull << (s_lo + j) : 0ull;
    }
    // the tile's busy slots: the four parts' masks together
#pragma unroll
    for (int x = 1; x < 4; x <<= 1) {
        const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)busy, x);
        const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(busy >> 32), x);
        busy |= (uint64_t)lo | (uint64_t)hi << 32;
    }
    // inclusive prefix of the four parts of a tile, and the tile's total
    uint32_t pq = c;
    {
        uint32_t a = (uint32_t)__shfl_up((int)pq, 1);
        if (part >= 1) pq += a;
        a = (uint32_t)__shfl_up((int)pq, 2);
        if (part >= 2) pq += a;
    }
    const uint32_t tile_c = (uint32_t)__shfl((int)pq, (int)(lane() | 3u));
    // inclusive prefix over the wave's tiles (counted on each tile's last lane)
    const bool heavy = tile_c >= kHeavyTile;
    uint32_t pc = part == 3u ? tile_c : 0u, pn = (part == 3u && heavy) ? 1u : 0u;
    uint32_t pl = (part == 3u && tile_c && !heavy) ? 1u : 0u;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t a = (uint32_t)__shfl_up((int)pc, off);
        const uint32_t b = (uint32_t)__shfl_up((int)pn, off);
        const uint32_t d = (uint32_t)__shfl_up((int)pl, off);
        if (lane() >= (uint32_t)off) {
            pc += a;
            pn += b;
            pl += d;
        }
    }
    pc = (uint32_t)__shfl((int)pc, (int)(lane() | 3u));
    pn = (uint32_t)__shfl((int)pn, (int)(lane() | 3u));
    pl = (uint32_t)__shfl((int)pl, (int)(lane() | 3u));
    if (lane() == 63) {
        s_w[0][wave] = pc;
        s_w[1][wave] = pn;
        s_w[2][wave] = pl;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        // lane a: exclusive prefix of counter a over the waves, then one
        // atomic for the block; the three atomics leave as one instruction
        const int a = (int)threadIdx.x;
        uint32_t sum = 0;
        for (int k = 0; k < kAllocBlock / 64; ++k) {
            const uint32_t v = s_w[a][k];
            s_w[a][k] = sum;
            sum += v;
        }
        uint32_t *ctr = a == 0 ? &B.ctl->entries : (a == 1 ? &B.ctl->n_nonempty : &B.ctl->n_light);
        s_base[a] = sum ? atomicAdd(ctr, sum) : 0u;
    }
    __syncthreads();
    if (tile_c) {
        // this part's first run: after the wave's earlier tiles and the
        // tile's earlier parts
        uint32_t off = s_base[0] + s_w[0][wave] + (pc - tile_c) + (pq - c);
#pragma unroll
        for (int j = 0; j < kAllocPer; ++j) {
            if (!cs[j]) continue;  // runs of empty slots are never read (nor slots past S)
            const uint32_t k = (uint32_t)(s_lo + j) * H.gtiles + t;
            B.offsets[k] = off;
            B.cursor[k] = off;
            off += cs[j];
        }
        if (part == 0u) {
            const uint32_t slot =
                heavy ? s_base[1] + s_w[1][wave] + pn - 1u : H.gtiles - 1u - (s_base[2] + s_w[2][wave] + pl - 1u);
            B.jobs[slot] = make_uint4(t, (uint32_t)map_of_tile(B, H.nmaps, t), (uint32_t)busy, (uint32_t)(busy >> 32));
        }
    }
}

// Eq. (1) with one unit of weight, Eq. (2), on a voxel state held in 32-bit
// registers (the stored int16 values, sign-extended once).
__device__ __forceinline__ void merge_one(int32_t &sdf, int32_t &w, uint64_t key, int32_t w_max)
{
    const int32_t v = tile_key_sdf(key);
    sdf = rdiv_small(__mul24(sdf, w) + v, w + 1);  // |sdf|, w < 2^15: a 24-bit product
    w = w + 1 < w_max ? w + 1 : w_max;
}

__device__ __forceinline__ void merge_one(int16_t &sdf, int16_t &w, uint64_t key, int32_t w_max)
{
    int32_t s = sdf, ww = w;
    merge_one(s, ww, key, w_max);
    sdf = (int16_t)s;
    w = (int16_t)ww;
}

constexpr int kMaxGroup = 8;

// Merge the touched voxels of one run of 8 z-consecutive voxels straight
// into HBM (one busy sequence slot on the tile).
__device__ __forceinline__ uint32_t merge_run_direct(uint64_t *kr, const MapDev &MD, int64_t row, int32_t rz0)
{
    uint64_t kk[8];
    bool any = false;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        kk[j] = kr[j];
        any |= kk[j] != kEmptyKey;
    }
    if (!any) return 0;
    uint32_t updated = 0;
    if (MD.vec_ok) {
        // 8 int16 of sdf and of w in one 16-byte access each
        int32_t sz = rz0 + MD.ring0[2];
        sz -= sz >= MD.dims[2] ? MD.dims[2] : 0;
        int4 sv = *reinterpret_cast<const int4 *>(MD.sdf + row + sz);
        int4 wv = *reinterpret_cast<const int4 *>(MD.w + row + sz);
        int16_t *sp = reinterpret_cast<int16_t *>(&sv);
        int16_t *wp = reinterpret_cast<int16_t *>(&wv);
#pragma unroll
        for (int j = 0; j < 8; ++j)
            if (kk[j] != kEmptyKey) {
                merge_one(sp[j], wp[j], kk[j], MD.w_max);
                kr[j] = kEmptyKey;
                ++updated;
            }
        *reinterpret_cast<int4 *>(MD.sdf + row + sz) = sv;
        *reinterpret_cast<int4 *>(MD.w + row + sz) = wv;
    } else {
        for (int j = 0; j < 8; ++j) {
            if (kk[j] == kEmptyKey) continue;
            int32_t sz = rz0 + j + MD.ring0[2];
            sz -= sz >= MD.dims[2] ? MD.dims[2] : 0;
            merge_one(MD.sdf[row + sz], MD.w[row + sz], kk[j], MD.w_max);
            kr[j] = kEmptyKey;
            ++updated;
        }
    }
    return updated;
}

// Slot of window-relative voxel r of a map.
__device__ __forceinline__ int64_t slot_of_rel(const MapDev &MD, int32_t rx, int32_t ry, int32_t rz)
{
    int32_t sx = rx + MD.ring0[0], sy = ry + MD.ring0[1], sz = rz + MD.ring0[2];
    sx -= sx >= MD.dims[0] ? MD.dims[0] : 0;
    sy -= sy >= MD.dims[1] ? MD.dims[1] : 0;
    sz -= sz >= MD.dims[2] ? MD.dims[2] : 0;
    return ((int64_t)sx * MD.dims[1] + sy) * MD.dims[2] + sz;
}

// Values every lane of a workgroup holds alike, moved to scalar registers
// (the compiler cannot tell that values read from LDS or memory are uniform,
// and keeps them, and all derived from them, in vector registers otherwise).
__device__ __forceinline__ uint32_t uniform(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }

// LDS byte address of a shared-memory pointer, and back: an address kept
// in one integer register needs no base added per access.
typedef __attribute__((address_space(3))) unsigned long long lds_u64;

__device__ __forceinline__ uint32_t lds_address(uint64_t *p) { return (uint32_t)(uintptr_t)(lds_u64 *)p; }
__device__ __forceinline__ unsigned long long *lds_pointer(int32_t a)
{
    return (unsigned long long *)(lds_u64 *)(uintptr_t)(uint32_t)a;
}
__device__ __forceinline__ int32_t uniform(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
template <typename T>
__device__ __forceinline__ T *uniform(T *p)
{
    const uint64_t a = (uint64_t)p;
    return (T *)((uint64_t)uniform((uint32_t)a) | (uint64_t)uniform((uint32_t)(a >> 32)) << 32);
}

__device__ __forceinline__ MapDev uniform_map(const MapDev &m)
{
    MapDev u;
    u.sdf = uniform(m.sdf);
    u.w = uniform(m.w);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        u.dims[a] = uniform(m.dims[a]);
        u.origin[a] = uniform(m.origin[a]);
        u.ring0[a] = uniform(m.ring0[a]);
        u.nt[a] = uniform(m.nt[a]);
    }
    u.ntot = uniform(m.ntot);
    u.tile_base = uniform(m.tile_base);
    u.tau = uniform(m.tau);
    u.w_max = uniform(m.w_max);
    u.vec_ok = uniform(m.vec_ok);
    u.pad = 0;
    return u;
}

// Persistent tile pass. Workgroup b first takes busy tile b, then pulls
// further tiles from queue b % nq, nq = min(8, workgroups) (one queue per
// XCD keeps same-address atomics spread; with fewer than 8 workgroups each
// queue still has one, so every job is reached). A tile's job record holds
// its map and its busy sequence slots, so that the runs and the map record
// of a tile are requested together, and a group's sensors come from a table
// indexed by (map, sequence slot). Per tile, the busy sequence slots are
// taken in groups of G: the candidates of a group's runs are computed
// together, one LDS key buffer per slot, then each voxel applies the group's
// scans in submission order. A tile busy in several slots keeps its SDF and
// weights in LDS.
// At most 96 VGPRs: five waves per SIMD, the most this kernel holds without
// spilling.
template <int kTileBlock, bool kStats>
__global__ __launch_bounds__(kTileBlock) __attribute__((amdgpu_waves_per_eu(5))) void k_tile(BatchArrays B)
{
    extern __shared__ uint64_t s_keys[];  // G * tvox keys, then the cached tile: tvox sdf, tvox w
    // per busy slot of the tile, in sequence order: first entry, entries,
    // sequence slot; per slot of the current group: sensor (o, tau)
    __shared__ uint32_t s_beg[kMaxSeq], s_cnt[kMaxSeq];
    __shared__ uint8_t s_list[kMaxSeq];
    __shared__ int4 s_sens[kMaxGroup];
    __shared__ uint32_t s_vis[kMaxGroup], s_upd[kMaxGroup];
    __shared__ uint32_t s_job;
    const BatchHdr H = *B.hdr;
    const int32_t lsum = H.lt[0] + H.lt[1] + H.lt[2];
    const uint32_t tvox = 1u << lsum;
    const int32_t G = H.G;
    int16_t *c_sdf = reinterpret_cast<int16_t *>(s_keys + (size_t)G * tvox);
    int16_t *c_w = c_sdf + tvox;
    // heavy tiles first (from the list's start), then the others (from its end)
    const uint32_t nheavy = B.ctl->n_nonempty, nne = nheavy + B.ctl->n_light;
    const uint32_t ez = 1u << H.lt[2], ey = 1u << H.lt[1];
    const int32_t sh[3] = {H.lt[1] + H.lt[2], H.lt[2], 0};  // LDS index shift per axis
    const int32_t shb[3] = {sh[0] + 3, sh[1] + 3, 3};          // the same, in bytes of 8-byte keys
    uint32_t job = blockIdx.x;
    if (job >= nne) return;
    const uint32_t nq = gridDim.x < (uint32_t)kQueues ? gridDim.x : (uint32_t)kQueues;
    const uint32_t queue = blockIdx.x % nq;
    for (uint32_t v = threadIdx.x; v < (uint32_t)G * tvox; v += kTileBlock) s_keys[v] = kEmptyKey;
    while (job < nne) {
        const uint32_t at = job < nheavy ? job : H.gtiles - 1u - (job - nheavy);
        const uint4 jb = B.jobs[at];
        const uint32_t g = uniform(jb.x);
        const int32_t mb = uniform((int32_t)jb.y);
        const uint64_t busy = (uint64_t)uniform(jb.z) | (uint64_t)uniform(jb.w) << 32;
        const int nbusy = __popcll(busy);
        // the busy slots' runs and sensors, all in flight together, listed in
        // order, so that groups of G hold busy slots only
        if (threadIdx.x < 64u && ((busy >> threadIdx.x) & 1ull)) {
            const uint32_t k = threadIdx.x * H.gtiles + g;
            const int p = __popcll(busy & ((1ull << threadIdx.x) - 1ull));
            s_cnt[p] = B.counts[k];
            s_beg[p] = B.offsets[k];
            s_list[p] = (uint8_t)threadIdx.x;
        }
        const MapDev MD = uniform_map(B.maps[mb]);
        const uint32_t t = g - MD.tile_base;
        const uint32_t tz = t % (uint32_t)MD.nt[2];
        const uint32_t txy = t / (uint32_t)MD.nt[2];
        const int32_t t0[3] = {(int32_t)(txy / (uint32_t)MD.nt[1]) << H.lt[0],
                               (int32_t)(txy % (uint32_t)MD.nt[1]) << H.lt[1], (int32_t)tz << H.lt[2]};
        // the tile's voxel box, clipped to the window, in global coordinates
        int32_t blo[3], bhi[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            blo[a] = MD.origin[a] + t0[a];
            bhi[a] = MD.origin[a] + min(t0[a] + (1 << H.lt[a]), MD.dims[a]);
        }
        __syncthreads();
        const bool cached = nbusy > 1;
        if (cached) {
            for (uint32_t v = threadIdx.x; v < tvox; v += kTileBlock) {
                const int32_t rz = (int32_t)(v & (ez - 1)) + t0[2];
                const int32_t ry = (int32_t)((v >> H.lt[2]) & (ey - 1)) + t0[1];
                const int32_t rx = (int32_t)(v >> (H.lt[1] + H.lt[2])) + t0[0];
                if (rx >= MD.dims[0] || ry >= MD.dims[1] || rz >= MD.dims[2]) continue;
                const int64_t slot = slot_of_rel(MD, rx, ry, rz);
                const int16_t sv = glob(MD.sdf)[slot], wv = glob(MD.w)[slot];
                c_sdf[v] = sv;
                c_w[v] = wv;
            }
        }
        for (int j0 = 0; j0 < nbusy; j0 += G) {
            // a group: busy slots j0 .. j0 + ng - 1 of the list, in order
            const int ng = min(G, nbusy - j0);
            // inclusive prefix of the group's run lengths (uniform: scalar
            // registers), so that an entry finds its run by comparisons
            uint32_t pre[kMaxGroup];
            uint32_t gsum = 0;
#pragma unroll
            for (int r = 0; r < kMaxGroup; ++r) {
                if (r < ng) gsum += s_cnt[j0 + r];
                pre[r] = uniform(gsum);
            }
            gsum = uniform(gsum);
            if (threadIdx.x < (uint32_t)ng) {
                s_vis[threadIdx.x] = 0;
                s_upd[threadIdx.x] = 0;
                s_sens[threadIdx.x] = B.seq_sensor[mb * H.S + (int32_t)s_list[j0 + threadIdx.x]];
            }
            __syncthreads();
            for (uint32_t e = threadIdx.x; e < gsum; e += kTileBlock) {
                // which run of the group entry e belongs to (the group's
                // runs are all non-empty: pre rises strictly up to gsum)
                int r = 0;
                uint32_t base = 0;
#pragma unroll
                for (int k = 0; k < kMaxGroup - 1; ++k) {
                    const bool past = e >= pre[k];
                    r += past ? 1 : 0;
                    base = past ? pre[k] : base;
                }
                const uint32_t ee = e - base;
                const uint32_t beg = s_beg[j0 + r];
                // the run lies inside the entry buffer unless the fill overflowed
                if (beg + ee >= H.cap) continue;
                const uint4 ra = B.entries[beg + ee];
                const uint4 rb = B.entries2[beg + ee];
                const uint32_t i = ra.x;
                const int4 sens = s_sens[r];
                const int32_t o[3] = {sens.x, sens.y, sens.z};
                const int32_t tau = sens.w;
                const int32_t q[3] = {(int32_t)ra.y, (int32_t)ra.z, (int32_t)ra.w};
                const int32_t off[3] = {(int16_t)(rb.y & 0xffffu), (int16_t)(rb.y >> 16), (int16_t)(rb.z & 0xffffu)};
                const int32_t c[3] = {(int32_t)((rb.z >> 16) & 0xffu), (int32_t)(rb.z >> 24), (int32_t)(rb.w & 0xffu)};
                // resume the walk right after the event that entered the
                // tile, set down on its first voxel in the box; the voxels
                // of the walk inside the box are one run (the walk carries
                // the key's LDS address itself)
                Ray R;
                BoxWalk V;
                if (!box_walk_resume(q, off, rb.x, c, o, tau, blo, bhi, shb, lds_address(s_keys + (size_t)r * tvox), R,
                                     V))
                    continue;
                const double taud = (double)tau, rh = R.r + 0.5;
                const uint32_t ihi = i >> 16, ilo = i << 16;
                uint32_t visits = 0;
                do {
                    atomicMin(lds_pointer(V.lv), (unsigned long long)tile_key(V.n, rh, R.inv_r2, taud, ihi, ilo));
                    ++visits;
                } while (box_walk_next(V));
                if (kStats && visits) atomicAdd(&s_vis[r], visits);
            }
            __syncthreads();
            if (cached) {
                // each voxel applies the group's scans in submission order,
                // its cached state held in registers across them
                uint32_t upd[kMaxGroup];
#pragma unroll
                for (int r = 0; r < kMaxGroup; ++r) upd[r] = 0;
                for (uint32_t v = threadIdx.x; v < tvox; v += kTileBlock) {
                    int32_t vs = 0, vw = 0;
                    bool touched = false;
#pragma unroll
                    for (int r = 0; r < kMaxGroup; ++r) {
                        if (r >= ng) break;
                        uint64_t *kp = &s_keys[(size_t)r * tvox + v];
                        const uint64_t key = *kp;
                        if (key == kEmptyKey) continue;
                        if (!touched) {
                            vs = c_sdf[v];
                            vw = c_w[v];
                            touched = true;
                        }
                        merge_one(vs, vw, key, MD.w_max);
                        *kp = kEmptyKey;
                        ++upd[r];
                    }
                    if (touched) {
                        c_sdf[v] = (int16_t)vs;
                        c_w[v] = (int16_t)vw;
                    }
                }
                if (kStats)
                    for (int r = 0; r < ng; ++r)
                        if (upd[r]) atomicAdd(&s_upd[r], upd[r]);
            } else {
                // a single busy slot: merge straight into HBM, runs of 8
                const int rb = 0;
                uint32_t updated = 0;
                for (uint32_t v0 = threadIdx.x * 8u; v0 < tvox; v0 += kTileBlock * 8u) {
                    const int32_t rz0 = (int32_t)(v0 & (ez - 1)) + t0[2];
                    const int32_t ry = (int32_t)((v0 >> H.lt[2]) & (ey - 1)) + t0[1];
                    const int32_t rx = (int32_t)(v0 >> (H.lt[1] + H.lt[2])) + t0[0];
                    if (rx >= MD.dims[0] || ry >= MD.dims[1] || rz0 >= MD.dims[2]) continue;  // no key there
                    int32_t sx = rx + MD.ring0[0], sy = ry + MD.ring0[1];
                    sx -= sx >= MD.dims[0] ? MD.dims[0] : 0;
                    sy -= sy >= MD.dims[1] ? MD.dims[1] : 0;
                    const int64_t row = ((int64_t)sx * MD.dims[1] + sy) * MD.dims[2];
                    updated += merge_run_direct(&s_keys[(size_t)rb * tvox + v0], MD, row, rz0);
                }
                if (kStats && updated) atomicAdd(&s_upd[rb], updated);
            }
            __syncthreads();
            if (threadIdx.x < (uint32_t)ng) {
                const uint32_t k = (uint32_t)s_list[j0 + threadIdx.x] * H.gtiles + g;  // sequence slot, tile
                B.counts[k] = 0;  // ready for the next batch
                if (kStats) {
                    B.tile_vis[k] = s_vis[threadIdx.x];
                    B.tile_upd[k] = s_upd[threadIdx.x];
                }
            }
        }
        if (cached) {
            for (uint32_t v = threadIdx.x; v < tvox; v += kTileBlock) {
                const int32_t rz = (int32_t)(v & (ez - 1)) + t0[2];
                const int32_t ry = (int32_t)((v >> H.lt[2]) & (ey - 1)) + t0[1];
                const int32_t rx = (int32_t)(v >> (H.lt[1] + H.lt[2])) + t0[0];
                if (rx >= MD.dims[0] || ry >= MD.dims[1] || rz >= MD.dims[2]) continue;
                const int64_t slot = slot_of_rel(MD, rx, ry, rz);
                glob(MD.sdf)[slot] = c_sdf[v];
                glob(MD.w)[slot] = c_w[v];
            }
        }
        // next tile from this workgroup's queue
        if (threadIdx.x == 0)
            s_job = gridDim.x + queue + nq * atomicAdd(&B.ctl->work[queue * kQueueStride], 1u);
        __syncthreads();
        job = uniform(s_job);
    }
}

// Per-scan counts (one workgroup per scan): voxels updated and visits over
// the scan's (sequence slot, tile) records, which it clears again, and
// points with a ray over the scan's binning blocks.
__global__ __launch_bounds__(256) void k_stats(BatchArrays B)
{
    __shared__ uint32_t s_sum[3][256];
    const BatchHdr H = *B.hdr;
    const uint32_t s = blockIdx.x;
    if (!H.want_stats || s >= (uint32_t)H.nscans) return;
    const ScanDev &SD = B.scans[s];
    const MapDev &MD = B.maps[SD.map];
    uint32_t vis = 0, upd = 0, val = 0;
    const uint32_t k0 = (uint32_t)SD.seq * H.gtiles + MD.tile_base;
    for (uint32_t t = threadIdx.x; t < MD.ntot; t += 256) {
        vis += B.tile_vis[k0 + t];
        upd += B.tile_upd[k0 + t];
        B.tile_vis[k0 + t] = 0;
        B.tile_upd[k0 + t] = 0;
    }
    const uint32_t nb = (uint32_t)((SD.n + H.bin_block - 1) / H.bin_block);
    for (uint32_t b = threadIdx.x; b < nb; b += 256) val += B.valid_part[SD.block0 + b];
    s_sum[0][threadIdx.x] = upd;
    s_sum[1][threadIdx.x] = val;
    s_sum[2][threadIdx.x] = vis;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < (uint32_t)off)
            for (int j = 0; j < 3; ++j) s_sum[j][threadIdx.x] += s_sum[j][threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        B.scan_stats[4 * s + 0] = s_sum[0][0];
        B.scan_stats[4 * s + 1] = s_sum[1][0];
        B.scan_stats[4 * s + 2] = s_sum[2][0];
        B.scan_stats[4 * s + 3] = B.ctl->overflow;
    }
}

__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t v)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
        p[j] = v;
}

}  // namespace

// Entries one point can emit: the tiles its band segment's walk visits.
int32_t max_tiles_per_ray(int32_t tau, const int32_t lt[3]) { return band_tiles_bound(tau, lt); }

namespace {

template <int kBB>
void launch_bin(bool fill, uint32_t bins, const BatchArrays &B, const InlineDesc &I, hipStream_t stream)
{
    if (fill) hipLaunchKernelGGL((k_bin<true, kBB, false>), dim3(bins), dim3(kBB), 0, stream, B, I);
    else if (I.on) hipLaunchKernelGGL((k_bin<false, kBB, true>), dim3(bins), dim3(kBB), 0, stream, B, I);
    else hipLaunchKernelGGL((k_bin<false, kBB, false>), dim3(bins), dim3(kBB), 0, stream, B, I);
}

void launch_bin_any(bool fill, uint32_t bins, uint32_t block, const BatchArrays &B, const InlineDesc &I,
                    hipStream_t stream)
{
    if (block == 128) launch_bin<128>(fill, bins, B, I, stream);
    else if (block == 512) launch_bin<512>(fill, bins, B, I, stream);
    else launch_bin<256>(fill, bins, B, I, stream);
}

}  // namespace

bool launch_blocks_ok(int32_t bin_block, int32_t tile_block)
{
    return (bin_block == 128 || bin_block == 256 || bin_block == 512) && (tile_block == 256 || tile_block == 512);
}

hipError_t launch_batch(const BatchArrays &B, const LaunchCaps &caps, hipStream_t stream, hipEvent_t ev_start,
                        hipEvent_t ev_binned, hipEvent_t ev_tiles, const InlineDesc *inl)
{
    hipError_t e;
    if (ev_start && (e = hipEventRecord(ev_start, stream)) != hipSuccess) return e;
    const uint32_t bins = caps.blocks > 0 ? caps.blocks : 1u;
    InlineDesc none;
    memset(&none, 0, sizeof(none));
    launch_bin_any(false, bins, caps.bin_block, B, inl ? *inl : none, stream);
    hipLaunchKernelGGL(k_alloc, dim3((caps.gtiles + kAllocTiles - 1) / kAllocTiles), dim3(kAllocBlock), 0, stream,
                       B);
    launch_bin_any(true, bins, caps.bin_block, B, none, stream);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (ev_binned && (e = hipEventRecord(ev_binned, stream)) != hipSuccess) return e;
    // the per-scan counts are a template switch: without them the walk and
    // the merges carry no counters
    const dim3 tg((uint32_t)caps.tile_grid);
    if (caps.tile_block == 512) {
        if (caps.stats) hipLaunchKernelGGL((k_tile<512, true>), tg, dim3(512), caps.tile_lds, stream, B);
        else hipLaunchKernelGGL((k_tile<512, false>), tg, dim3(512), caps.tile_lds, stream, B);
    } else {
        if (caps.stats) hipLaunchKernelGGL((k_tile<256, true>), tg, dim3(256), caps.tile_lds, stream, B);
        else hipLaunchKernelGGL((k_tile<256, false>), tg, dim3(256), caps.tile_lds, stream, B);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (ev_tiles && (e = hipEventRecord(ev_tiles, stream)) != hipSuccess) return e;
    if (caps.stats) hipLaunchKernelGGL(k_stats, dim3(caps.scans > 0 ? caps.scans : 1u), dim3(256), 0, stream, B);
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
