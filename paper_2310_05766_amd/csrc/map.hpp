// The map object behind the C ABI's opaque tsdf_map, shared by the
// library's translation units (runtime.hip holds its calls).
#pragma once

#include <atomic>
#include <memory>

#include "engine.hpp"

struct tsdf_map {
    tsdf_map_desc d;
    int64_t nvox = 0;
    double scale = 0.0;
    int16_t *sdf = nullptr, *w = nullptr;
    bool own_arrays = false;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int device = 0;
    int32_t lt[3] = {0, 0, 0};  // integration tiling; {0, 0, 0}: chosen per call
    int32_t tile_grid = 0;      // 0: as many workgroups as fit the device
    int32_t bin_block = 0;      // binning threads per block; 0: the default
    int32_t tile_block = 0;     // tile workgroup size; 0: the default
    std::unique_ptr<tsdf::Engine> engine;  // single-scan integration on the map's stream
    // vertical interpolation between scan lines, or free-space carving (their
    // own path through a key volume over the window, interp.hip)
    int64_t interp_dq = 0;                     // delta_z of Eq. (3), 1/2^20 units; 0: off
    bool carve = false;                        // rays longer than tau walked from the sensor
    unsigned long long *interp_keys = nullptr;  // [nvox], EMPTY between scans
    uint8_t *interp_touched = nullptr;          // [ceil(nvox / 64)], 0 between scans
    unsigned long long *interp_ctr = nullptr;   // device counters (3)
    unsigned long long *interp_ctr_host = nullptr;
    float *interp_pts = nullptr;                // device copy of host points
    int64_t interp_pts_cap = 0;                 // points
    // shift / readback staging
    int16_t *stage_dev = nullptr;  // [2][stage_cap]
    int16_t *stage_host = nullptr;
    int64_t stage_cap = 0;  // voxels per array
    tsdf::BoxXfer *boxes_dev = nullptr;
    tsdf::BoxXfer *boxes_host = nullptr;
    int32_t boxes_cap = 0;
    // whole-chunk shifts: device staging of kShiftChunks chunks leaving and
    // kShiftChunks entering, per-chunk non-zero flags (device, pinned host),
    // chunk lists (pinned host, device), and a second stream for the copies
    // into the window, so that both directions of the host link run together
    int16_t *cstage_dev = nullptr;
    uint32_t *cflags_dev = nullptr, *cflags_host = nullptr;
    tsdf::BoxXfer *clist_host = nullptr, *clist_dev = nullptr;
    hipStream_t copy_stream = nullptr;
    hipEvent_t copy_done = nullptr;
    // the store's chunk buffers: pinned host slabs cut into 1 MiB chunks
    std::vector<void *> pool_slabs;
    std::vector<int16_t *> pool_free;
    // per-kernel event timing (pack, unpack)
    bool prof_on = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_ev[TSDF_KERNEL_COUNT];
    std::vector<hipEvent_t> ev_pool;
    // state
    bool poisoned = false;
    std::atomic<int> busy{0};
    std::unordered_map<tsdf::ChunkKey, tsdf::Chunk, tsdf::ChunkKeyHash> store;
};

namespace tsdf {

// One host thread per map: a call holds the map's busy flag while it runs.
struct Guard {
    tsdf_map *m;
    bool ok;
    explicit Guard(tsdf_map *mm) : m(mm), ok(false)
    {
        int expected = 0;
        ok = m->busy.compare_exchange_strong(expected, 1);
    }
    ~Guard()
    {
        if (ok) m->busy.store(0);
    }
};


// Tiles of 2^lt voxels: every lt in [2, 6], the z edge at least 8 (merge
// runs), 2^9..2^12 voxels per tile (12 bytes of LDS per voxel).
// Tilings used while a map has none set: scan-by-scan calls do best with
// few, large tiles (per-tile fixed costs dominate one scan's work); batches
// with many scans per tile do best with 8^3 tiles.
inline constexpr int32_t kPlainTiling[3] = {4, 4, 3};
inline constexpr int32_t kBatchTiling[3] = {3, 3, 3};

inline const int32_t *tiling_for(const tsdf_map *m, bool batch)
{
    if (m->lt[0] != 0) return m->lt;
    return batch ? kBatchTiling : kPlainTiling;
}

// The launch shape of an integration on this map (a batch takes its first
// scan's map's).
inline LaunchShape launch_shape(const tsdf_map *m, bool batch)
{
    LaunchShape sh;
    const int32_t *lt = tiling_for(m, batch);
    for (int a = 0; a < 3; ++a) sh.lt[a] = lt[a];
    sh.tile_grid = m->tile_grid;
    sh.bin_block = m->bin_block > 0 ? m->bin_block : kBinBlock;
    sh.tile_block = m->tile_block > 0 ? m->tile_block : kTileBlockDefault;
    return sh;
}

}  // namespace tsdf
