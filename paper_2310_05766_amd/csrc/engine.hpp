// Host side of the batched integration engine: device tables and buffers,
// staging of host points, ordering against the maps' streams, timing.
#pragma once

#include "internal.hpp"

namespace tsdf {

// What the engine needs to know of a map.
struct MapRef {
    const void *id;  // identity (the tsdf_map)
    int16_t *sdf, *w;
    int32_t dims[3], origin[3];
    double scale;  // 1024 / voxel size
    int32_t tau, w_max;
    hipStream_t stream;
};

// How a batch is cut up and launched: tiles of 2^lt voxels, tile_grid
// persistent tile workgroups (0: as many as fit), and the block sizes.
struct LaunchShape {
    int32_t lt[3];
    int32_t tile_grid;
    int32_t bin_block;   // 128, 256 or 512
    int32_t tile_block;  // 256 or 512
};

struct ScanRef {
    int32_t map;  // index into the maps vector
    const float *xyz;
    int64_t n;
    bool host;  // xyz is host memory
    const double *pose;
};

// Tile arrays of one map used on its own (one scan per batch), for maps
// built on caller-owned memory: the size for the finest allowed tiling.
size_t single_map_array_bytes(const int32_t dims[3]);

class Engine {
public:
    Engine(hipStream_t stream, int device);
    ~Engine();
    Engine(const Engine &) = delete;
    Engine &operator=(const Engine &) = delete;

    // Use caller-owned memory for the tile arrays (fixed capacity).
    void adopt_arrays(void *p, size_t bytes);

    // Integrate the scans (in order per map). stats: one entry per scan or
    // null. Returns TSDF_EINVAL before doing anything for bad arguments.
    tsdf_status run(const std::vector<MapRef> &maps, const std::vector<ScanRef> &scans, const LaunchShape &shape,
                    tsdf_scan_stats *stats);

    hipStream_t stream() const { return stream_; }
    bool poisoned() const { return poisoned_; }

    // per-stage timing (events on the engine's stream)
    void profile(bool on);
    // capture each launch shape once in a hipGraph and replay it
    static void set_graphs(bool on);
    static bool graphs();
    // stage 0: binning (count, runs, fill), 1: tile pass, 2: per-scan counts,
    // 3: the whole launch
    tsdf_status profile_read(int stage, double *ms, int64_t *n);

private:
    tsdf_status run_chunk(const std::vector<MapRef> &maps, const std::vector<ScanRef> &scans, size_t b, size_t e,
                          const LaunchShape &shape, tsdf_scan_stats *stats);
    tsdf_status grow(void **p, size_t *cap, size_t need, bool zero, bool host_pinned = false);
    tsdf_status fail();

    hipStream_t stream_;
    int device_;
    bool poisoned_ = false;
    int num_cu_ = 256;
    // descriptor tables: pinned host staging and device copies, both
    // double-buffered; a batch's tables go to the device on copy_stream_,
    // while the previous batch's kernels still run on stream_
    void *desc_dev_[2] = {nullptr, nullptr};
    size_t desc_cap_[2] = {0, 0};
    void *desc_host_[2] = {nullptr, nullptr};
    size_t desc_host_cap_[2] = {0, 0};
    hipEvent_t desc_ev_[2] = {nullptr, nullptr};    // staging k copied to device k (copy_stream_)
    bool desc_ev_live_[2] = {false, false};
    hipEvent_t desc_used_[2] = {nullptr, nullptr};  // kernels reading device k done (stream_)
    bool desc_used_live_[2] = {false, false};
    int desc_cur_ = 0;
    hipStream_t copy_stream_ = nullptr;
    // the tables of one-scan batches, which their first kernel writes (on
    // stream_ only: no copy, no event)
    void *inline_dev_ = nullptr;
    size_t inline_cap_ = 0;
    // tile arrays: counts | offsets | cursor | tile_vis | tile_upd (c_cap each), jobs (g_cap)
    void *arr_ = nullptr;
    size_t arr_bytes_ = 0;
    bool arr_external_ = false;
    size_t c_cap_ = 0, g_cap_ = 0;
    void *entries_ = nullptr;
    size_t entries_cap_ = 0;  // bytes
    void *valid_ = nullptr;
    size_t valid_cap_ = 0;  // bytes
    void *stats_ = nullptr;
    size_t stats_cap_ = 0;  // bytes
    void *ctl_ = nullptr;
    // host points staging
    void *pts_dev_ = nullptr;
    size_t pts_dev_cap_ = 0;
    void *pts_host_[2] = {nullptr, nullptr};
    size_t pts_host_cap_[2] = {0, 0};
    hipEvent_t pts_ev_[2] = {nullptr, nullptr};
    bool pts_ev_live_[2] = {false, false};
    int pts_cur_ = 0;
    // cross-stream ordering
    hipEvent_t order_ev_ = nullptr;
    // captured launches, keyed by buffers and (bucketed) grid sizes
    struct GraphEntry {
        BatchArrays B;
        LaunchCaps caps;
        hipGraphExec_t exec;
    };
    std::vector<GraphEntry> graphs_;
    hipError_t launch(const BatchArrays &B, const LaunchCaps &caps);
    // timing
    bool prof_on_ = false;
    std::vector<hipEvent_t> ev_pool_;
    std::vector<std::array<hipEvent_t, 4>> prof_ev_;
};

}  // namespace tsdf
