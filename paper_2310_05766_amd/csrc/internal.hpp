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

// Counters a scan accumulates on the device, and the finished scan's copy.
struct DevCounters {
    uint32_t touched;   // voxels whose candidate left EMPTY (== voxels updated)
    uint32_t valid;     // points with a ray
    uint32_t visits;    // (ray, resident voxel) candidates
    uint32_t done;      // blocks of the merge that finished
    uint32_t last[4];   // touched, valid, visits of the last finished scan
};

// Scratch of the plain per-scan path: a window-sized candidate array of
// 64-bit keys (EMPTY between scans), the list of touched slots, counters.
struct ScratchLayout {
    size_t keys_off, touched_off, counters_off, total;
    static ScratchLayout of(int64_t nvox);
};

// Host-side store of 64^3-voxel chunks that left the window.
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
struct Chunk {
    std::vector<int16_t> sdf, w;  // kChunkVox each, [x][y][z] z fastest
};

// Launchers (integrate.hip, shift.hip). All enqueue on `stream`.
hipError_t launch_candidates(const ScanParams &P, uint64_t *keys, uint32_t *touched, DevCounters *ctr,
                             hipStream_t stream);
hipError_t launch_merge(uint64_t *keys, const uint32_t *touched, DevCounters *ctr, int16_t *sdf, int16_t *w,
                        int32_t w_max, hipStream_t stream);
hipError_t launch_fill_u64(uint64_t *p, int64_t n, uint64_t v, hipStream_t stream);
hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t stream);

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
hipError_t launch_unpack_boxes(const BoxXfer *boxes_dev, int32_t nboxes, int64_t max_box_vox, int16_t *sdf,
                               int16_t *w, const int32_t dims[3], const int16_t *stage_sdf,
                               const int16_t *stage_w, hipStream_t stream);

}  // namespace tsdf
