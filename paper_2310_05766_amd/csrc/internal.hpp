// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "../../include/tsdf.h"
#include "ray.hpp"

namespace tsdf {

// ---------------------------------------------------------------------------
// Batched integration engine (batch.hip). Every integration, a single scan
// included, is a batch: scans (any maps, several per map allowed) whose rays
// are binned by (map tile, position of the scan among its map's scans in the
// batch); one workgroup per tile then applies the map's scans to that tile in
// submission order.
// ---------------------------------------------------------------------------

constexpr int kBinBlock = 256;   // default binning threads per block (one ray each); 128 and 512 also run
constexpr int kTileBlockDefault = 256;  // default tile workgroup size; 512 also runs
constexpr int kMaxEmit = 6;      // tiles per ray listed in LDS before taking positions (more go
                                  // straight to their runs)
constexpr int32_t kMaxTileGrid = 65536;
constexpr int32_t kMaxSeq = 64;  // scans of one map in one batch

struct MapDev {
    int16_t *sdf, *w;
    int32_t dims[3], origin[3], ring0[3];
    int32_t nt[3];
    uint32_t ntot;       // tiles of this map
    uint32_t tile_base;  // first global tile id of this map
    int32_t tau, w_max;
    int32_t vec_ok;      // 16-byte runs possible (see k_tile)
    int32_t pad;
};

struct ScanDev {
    RayParams rp;        // pose, scale, sensor position, tau
    const float *xyz;
    int64_t n;
    int32_t map;         // map slot in the batch
    int32_t seq;         // position among this map's scans in the batch
    uint32_t block0;     // first binning block of this scan
    uint32_t pad;
};

struct BatchHdr {
    int32_t lt[3];
    int32_t S;           // sequence slots per tile (most scans of one map)
    int32_t G;           // sequence slots whose candidates a tile workgroup holds at once
    int32_t nmaps, nscans;
    uint32_t gtiles;     // sum of the maps' tile counts
    uint32_t nblocks;    // binning blocks of this batch
    uint32_t cap;        // entry capacity
    uint32_t want_stats;
    uint32_t bin_block;  // binning threads per block (one ray each)
    uint32_t pad;
};

// The descriptors of a batch of one scan, handed to the first binning
// kernel as arguments: it reads them from there and stores them for the
// kernels after it, so that no copy precedes the launch (on = 0: the
// descriptors are in device memory already).
struct InlineDesc {
    BatchHdr hdr;
    MapDev map;
    ScanDev scan;
    uint32_t on;
    uint32_t pad[3];
};

constexpr int kQueues = 8;  // tile job queues, one per XCD (workgroup b runs on XCD b % 8)
// Words between two queue counters: each counter on a 128-byte line of its
// own, so that atomics on different queues do not meet in one line.
constexpr int kQueueStride = 32;

struct BatchCtl {
    uint32_t n_nonempty;  // busy tiles with heavy work, listed from the list's start
    uint32_t entries, overflow;
    uint32_t n_light;     // the other busy tiles, listed from the list's end
    uint32_t pad[28];
    uint32_t work[kQueues * kQueueStride];  // next job of queue q: work[q * kQueueStride]
};

// Device addresses of one engine (all inside buffers the engine owns).
struct BatchArrays {
    BatchHdr *hdr;
    MapDev *maps;
    ScanDev *scans;
    uint32_t *block_scan;  // [nblocks] scan of each binning block
    int4 *seq_sensor;      // [nmaps * S] sensor position (fixed point) and tau of the scan at (map, seq)
    uint32_t *counts;      // [S * gtiles] entries per (seq, tile), seq-major; zero between batches
    uint32_t *offsets;     // [S * gtiles] start of each run
    uint32_t *cursor;      // [S * gtiles] fill position
    uint32_t *tile_vis;    // [S * gtiles] visits per (seq, tile), when stats are wanted
    uint32_t *tile_upd;    // [S * gtiles] voxels updated per (seq, tile)
    uint4 *jobs;           // [gtiles] busy tiles: (global tile, map slot, busy sequence slots as a 64-bit mask)
    uint4 *entries;        // [cap] (point index, q.x, q.y, q.z), by tile then seq
    uint4 *entries2;       // [cap] (r, packed band offsets, crossing counts at tile entry)
    uint32_t *valid_part;  // [nblocks] points with a ray per binning block
    uint32_t *scan_stats;  // [nscans * 4] updated, valid, visits, overflow
    BatchCtl *ctl;
};

// Upper bound of the tiles one ray's band can fall in.
int32_t max_tiles_per_ray(int32_t tau, const int32_t lt[3]);

// Grid sizes of one launch. Every grid is sized from these capacities and
// the kernels read the batch's real sizes from the header, so a captured
// graph serves every batch that fits them.
struct LaunchCaps {
    uint32_t blocks;      // binning blocks
    uint32_t gtiles;      // global tiles
    uint32_t scans;       // scans
    int32_t tile_grid;    // tile workgroups
    uint32_t tile_lds;    // dynamic LDS bytes of a tile workgroup
    uint32_t bin_block;   // binning threads per block: 128, 256 or 512
    uint32_t tile_block;  // tile workgroup size: 256 or 512
    uint32_t stats;       // per-scan counts wanted: k_stats runs only then
};

// The block sizes the kernels are built for.
bool launch_blocks_ok(int32_t bin_block, int32_t tile_block);

// Events recorded (when non-null) after binning and after the tile pass,
// for per-stage timing. inl (when non-null, with on = 1): the descriptors of
// a one-scan batch, stored by the first kernel instead of copied before.
hipError_t launch_batch(const BatchArrays &B, const LaunchCaps &caps, hipStream_t stream, hipEvent_t ev_start,
                        hipEvent_t ev_binned, hipEvent_t ev_tiles, const InlineDesc *inl = nullptr);
hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t stream);

// One scan through the global key volume (interp.hip): with vertical
// interpolation between scan lines (dq > 0), or with free-space carving.
struct InterpScan {
    RayParams rp;
    const float *xyz;  // device points
    int64_t n;
    int64_t dq;        // delta_z of Eq. (3) in 1/2^20 units (0 with carving)
    int64_t up[3];     // the sensor's up vector in 1/1024 units
    int32_t carve;     // walk each ray longer than tau from the sensor as well
    int32_t origin[3], dims[3];
    int32_t ring0[3];  // floor_mod(origin, dims): the slot of the window's first voxel
    int16_t *sdf, *w;
    int32_t w_max;
    unsigned long long *keys;      // [nx*ny*nz] per-scan keys, all EMPTY between scans
    uint8_t *touched;              // [ceil(nx*ny*nz / 64)] runs of 64 slots with a key, all 0 between scans
    unsigned long long *counters;  // valid points, visits, voxels updated, 64-bit atomics issued (added to)
};
hipError_t launch_interp(const InterpScan &P, int64_t nvox, hipStream_t stream);

// Point-to-TSDF registration sums (register.hip).
constexpr int kRegSums = 29;  // H upper triangle (21), J^T r (6), sum r^2, points used
struct RegArgs {
    double M[12];      // pose rows 0..2
    const float *xyz;  // device points
    int64_t n;
    const int16_t *sdf, *w;
    int32_t dims[3], origin[3];
    int32_t tau;
    double vs;
};
int64_t reg_blocks(int64_t n);
hipError_t launch_reg_sums(const RegArgs &A, double *partials, hipStream_t stream);

// Surface extraction of a box of the window (mesh.hip).
struct MeshArgs {
    const int16_t *sdf, *w;
    int32_t dims[3];  // the window (slot = floor_mod(g, dims))
    int32_t lo[3];    // first cube's voxel
    int64_t n[3];     // cubes per axis
    int64_t ncubes;
    double vs;        // voxel size, metres
};
int64_t mesh_blocks(int64_t ncubes);
hipError_t launch_mesh_count(const MeshArgs &A, uint32_t *block_tris, hipStream_t stream);
hipError_t launch_mesh_emit(const MeshArgs &A, const uint64_t *block_base, float *out, hipStream_t stream);

// ---------------------------------------------------------------------------
// Host-side store of 64^3-voxel chunks that left the window.
// ---------------------------------------------------------------------------
constexpr int kChunk = 64;
constexpr int64_t kChunkVox = (int64_t)kChunk * kChunk * kChunk;

struct ChunkKey {
    int32_t x, y, z;
    bool operator==(const ChunkKey &o) const { return x == o.x && y == o.y && z == o.z; }
};
struct ChunkKeyHash {
    size_t operator()(const ChunkKey &k) const
    {
        uint64_t h = (uint64_t)(uint32_t)k.x * 0x9E3779B97F4A7C15ull;
        h ^= (uint64_t)(uint32_t)k.y * 0xC2B2AE3D27D4EB4Full + (h << 6) + (h >> 2);
        h ^= (uint64_t)(uint32_t)k.z * 0x165667B19E3779F9ull + (h << 6) + (h >> 2);
        return (size_t)h;
    }
};
// A chunk of the host store: kChunkVox sdf values then kChunkVox weights,
// [x][y][z] z fastest, in pinned host memory (a buffer of the map's chunk
// pool), so that a whole chunk crosses the host link in one copy.
struct Chunk {
    int16_t *buf = nullptr;
    int16_t *sdf() const { return buf; }
    int16_t *w() const { return buf + kChunkVox; }
};

// A box of voxels copied between the window and a dense staging buffer:
// global box [lo, lo + ext), staged at `off` (elements) as [x][y][z].
struct BoxXfer {
    int32_t lo[3];
    int32_t ext[3];
    int64_t off;
};
// Slot of a global voxel: floor_mod(g, dims) per axis.
// pack: stage <- window (and, with clear, the window voxels are reset to 0);
// unpack: window <- stage, or <- 0 when stage_sdf is null.
hipError_t launch_pack_boxes(const BoxXfer *boxes_dev, int32_t nboxes, int64_t max_box_vox, int16_t *sdf,
                             int16_t *w, const int32_t dims[3], int16_t *stage_sdf, int16_t *stage_w, bool clear,
                             hipStream_t stream);
// Whole chunks of a window whose dims are multiples of 64 (chunks_dev[j].lo:
// the chunk's global origin), staged chunk by chunk in the store's layout
// (stage + j * 2 * kChunkVox: sdf, then w). pack clears the window voxels and
// sets flags[j] (zero beforehand) when chunk j holds a non-zero voxel.
hipError_t launch_pack_chunks(const BoxXfer *chunks_dev, int32_t nchunks, int16_t *sdf, int16_t *w,
                              const int32_t dims[3], int16_t *stage, uint32_t *flags, hipStream_t stream);
hipError_t launch_unpack_chunks(const BoxXfer *chunks_dev, int32_t nchunks, int16_t *sdf, int16_t *w,
                                const int32_t dims[3], const int16_t *stage, hipStream_t stream);
hipError_t launch_unpack_boxes(const BoxXfer *boxes_dev, int32_t nboxes, int64_t max_box_vox, int16_t *sdf,
                               int16_t *w, const int32_t dims[3], const int16_t *stage_sdf,
                               const int16_t *stage_w, hipStream_t stream);

}  // namespace tsdf
