// C ABI of the TSDF library: map objects, argument checks, the batched
// integration engine's front door, the host chunk store behind the
// local-map shift, readback.
// (FeatSense, arXiv 2310.05766, Sec. VI for integration, Sec. I for the
// shifted local map and the store of what leaves it.)
#include <math.h>
#include <string.h>

#include <algorithm>
#include <memory>
#include <new>

#include "map.hpp"

using namespace tsdf;

namespace {

tsdf_status fail_device(tsdf_map *m)
{
    if (m) m->poisoned = true;
    return TSDF_EDEVICE;
}

#define HIPCHK(m, call)                                  \
    do {                                                 \
        if ((call) != hipSuccess) return fail_device(m); \
    } while (0)

hipEvent_t take_event(tsdf_map *m)
{
    if (!m->ev_pool.empty()) {
        hipEvent_t e = m->ev_pool.back();
        m->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Bracket a launch with events on the map's stream when profiling is on.
hipError_t prof_start(tsdf_map *m, int id)
{
    if (!m->prof_on) return hipSuccess;
    hipEvent_t a = take_event(m), b = take_event(m);
    if (!a || !b) return hipErrorOutOfMemory;
    m->prof_ev[id].push_back({a, b});
    return hipEventRecord(a, m->stream);
}

hipError_t prof_stop(tsdf_map *m, int id)
{
    if (!m->prof_on) return hipSuccess;
    return hipEventRecord(m->prof_ev[id].back().second, m->stream);
}

void prof_clear(tsdf_map *m)
{
    for (int k = 0; k < TSDF_KERNEL_COUNT; ++k) {
        for (auto &p : m->prof_ev[k]) {
            m->ev_pool.push_back(p.first);
            m->ev_pool.push_back(p.second);
        }
        m->prof_ev[k].clear();
    }
}

int64_t floor_div64(int64_t a, int64_t b)
{
    int64_t q = a / b;
    if ((a % b != 0) && (a < 0)) --q;
    return q;
}

int64_t floor_mod64(int64_t a, int64_t b) { return a - floor_div64(a, b) * b; }

bool desc_ok(const tsdf_map_desc *d)
{
    if (!d) return false;
    int64_t nv = 1;
    for (int a = 0; a < 3; ++a) {
        if (d->dims[a] < 1) return false;
        nv *= d->dims[a];
        // points are kept only within 2^30 fixed-point units (2^20 voxels)
        // of the global origin, so a window beyond that could never be hit
        if ((int64_t)d->origin[a] + d->dims[a] > (int64_t)1 << 20 || (int64_t)d->origin[a] < -((int64_t)1 << 20))
            return false;
    }
    if (nv >= ((int64_t)1 << 31)) return false;
    if (!(d->voxel_size_m > 0.0) || !isfinite(d->voxel_size_m)) return false;
    if (d->tau_q10 < 1 || d->tau_q10 > 32767) return false;
    if (d->w_max < 1 || d->w_max > 32767) return false;
    return true;
}

int64_t nvox_of(const tsdf_map_desc *d) { return (int64_t)d->dims[0] * d->dims[1] * d->dims[2]; }

bool tiling_ok(const int32_t lt[3])
{
    int sum = 0;
    for (int a = 0; a < 3; ++a) {
        if (lt[a] < 2 || lt[a] > 6) return false;
        sum += lt[a];
    }
    return lt[2] >= 3 && sum >= 9 && sum <= 12;
}

MapRef map_ref(const tsdf_map *m)
{
    MapRef r;
    r.id = m;
    r.sdf = m->sdf;
    r.w = m->w;
    for (int a = 0; a < 3; ++a) {
        r.dims[a] = m->d.dims[a];
        r.origin[a] = m->d.origin[a];
    }
    r.scale = m->scale;
    r.tau = m->d.tau_q10;
    r.w_max = m->d.w_max;
    r.stream = m->stream;
    return r;
}

tsdf_status ensure_stage(tsdf_map *m, int64_t vox, int32_t boxes)
{
    if (vox > m->stage_cap) {
        HIPCHK(m, hipStreamSynchronize(m->stream));
        if (m->stage_dev) HIPCHK(m, hipFree(m->stage_dev));
        if (m->stage_host) HIPCHK(m, hipHostFree(m->stage_host));
        m->stage_dev = nullptr;
        m->stage_host = nullptr;
        m->stage_cap = 0;
        if (hipMalloc(&m->stage_dev, (size_t)vox * 2 * sizeof(int16_t)) != hipSuccess) return TSDF_ENOMEM;
        if (hipHostMalloc((void **)&m->stage_host, (size_t)vox * 2 * sizeof(int16_t), hipHostMallocDefault) !=
            hipSuccess)
            return TSDF_ENOMEM;
        m->stage_cap = vox;
    }
    if (boxes > m->boxes_cap) {
        HIPCHK(m, hipStreamSynchronize(m->stream));
        if (m->boxes_dev) HIPCHK(m, hipFree(m->boxes_dev));
        if (m->boxes_host) HIPCHK(m, hipHostFree(m->boxes_host));
        m->boxes_dev = nullptr;
        m->boxes_host = nullptr;
        m->boxes_cap = 0;
        if (hipMalloc(&m->boxes_dev, (size_t)boxes * sizeof(BoxXfer)) != hipSuccess) return TSDF_ENOMEM;
        if (hipHostMalloc((void **)&m->boxes_host, (size_t)boxes * sizeof(BoxXfer), hipHostMallocDefault) !=
            hipSuccess)
            return TSDF_ENOMEM;
        m->boxes_cap = boxes;
    }
    return TSDF_OK;
}

// Chunks of the host store come from pinned slabs of kPoolSlab chunks, so
// that a whole chunk is one DMA copy to or from the device; a freed chunk
// goes back to the pool (slabs are returned when the map is destroyed).
constexpr int kPoolSlab = 16;

int16_t *chunk_take(tsdf_map *m)
{
    if (m->pool_free.empty()) {
        void *p = nullptr;
        const size_t bytes = (size_t)kPoolSlab * 2 * kChunkVox * sizeof(int16_t);
        if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) return nullptr;
        m->pool_slabs.push_back(p);
        for (int k = kPoolSlab - 1; k >= 0; --k) m->pool_free.push_back((int16_t *)p + (size_t)k * 2 * kChunkVox);
    }
    int16_t *b = m->pool_free.back();
    m->pool_free.pop_back();
    return b;
}

void chunk_give(tsdf_map *m, Chunk &c)
{
    if (c.buf) m->pool_free.push_back(c.buf);
    c.buf = nullptr;
}

// Staging of whole-chunk shifts: kShiftChunks chunks out and kShiftChunks in
// per round trip (one chunk layer of a 512 x 512 x 128 window).
constexpr int kShiftChunks = 16;

tsdf_status ensure_chunk_stage(tsdf_map *m)
{
    if (m->cstage_dev && m->cflags_dev && m->cflags_host && m->clist_dev && m->clist_host && m->copy_stream &&
        m->copy_done)
        return TSDF_OK;
    if (m->cstage_dev) return TSDF_ENOMEM;  // an earlier attempt failed part way
    const size_t bytes = (size_t)2 * kShiftChunks * 2 * kChunkVox * sizeof(int16_t);
    if (hipMalloc(&m->cstage_dev, bytes) != hipSuccess) {
        m->cstage_dev = nullptr;
        return TSDF_ENOMEM;
    }
    bool ok = hipMalloc(&m->cflags_dev, kShiftChunks * sizeof(uint32_t)) == hipSuccess;
    ok = ok && hipHostMalloc((void **)&m->cflags_host, kShiftChunks * sizeof(uint32_t), hipHostMallocDefault) ==
                   hipSuccess;
    ok = ok && hipMalloc(&m->clist_dev, 2 * kShiftChunks * sizeof(BoxXfer)) == hipSuccess;
    ok = ok && hipHostMalloc((void **)&m->clist_host, 2 * kShiftChunks * sizeof(BoxXfer), hipHostMallocDefault) ==
                   hipSuccess;
    ok = ok && hipStreamCreateWithFlags(&m->copy_stream, hipStreamNonBlocking) == hipSuccess;  // default priority
    ok = ok && hipEventCreateWithFlags(&m->copy_done, hipEventDisableTiming) == hipSuccess;
    return ok ? TSDF_OK : TSDF_ENOMEM;
}

void release(tsdf_map *m)
{
    if (!m) return;
    if (m->stream) (void)hipStreamSynchronize(m->stream);
    m->engine.reset();
    if (m->own_arrays) {
        if (m->sdf) (void)hipFree(m->sdf);
        if (m->w) (void)hipFree(m->w);
    }
    if (m->stage_dev) (void)hipFree(m->stage_dev);
    if (m->stage_host) (void)hipHostFree(m->stage_host);
    if (m->boxes_dev) (void)hipFree(m->boxes_dev);
    if (m->boxes_host) (void)hipHostFree(m->boxes_host);
    if (m->interp_keys) (void)hipFree(m->interp_keys);
    if (m->interp_touched) (void)hipFree(m->interp_touched);
    if (m->interp_ctr) (void)hipFree(m->interp_ctr);
    if (m->interp_ctr_host) (void)hipHostFree(m->interp_ctr_host);
    if (m->interp_pts) (void)hipFree(m->interp_pts);
    if (m->copy_stream) (void)hipStreamSynchronize(m->copy_stream);
    if (m->cstage_dev) (void)hipFree(m->cstage_dev);
    if (m->cflags_dev) (void)hipFree(m->cflags_dev);
    if (m->cflags_host) (void)hipHostFree(m->cflags_host);
    if (m->clist_dev) (void)hipFree(m->clist_dev);
    if (m->clist_host) (void)hipHostFree(m->clist_host);
    if (m->copy_done) (void)hipEventDestroy(m->copy_done);
    if (m->copy_stream) (void)hipStreamDestroy(m->copy_stream);
    m->store.clear();
    for (void *p : m->pool_slabs) (void)hipHostFree(p);
    prof_clear(m);
    for (hipEvent_t e : m->ev_pool) (void)hipEventDestroy(e);
    if (m->own_stream && m->stream) (void)hipStreamDestroy(m->stream);
    delete m;
}

tsdf_status init_map(tsdf_map *m, void *arrays, size_t array_bytes)
{
    m->nvox = nvox_of(&m->d);
    m->scale = 1024.0 / m->d.voxel_size_m;
    m->engine.reset(new (std::nothrow) Engine(m->stream, m->device));
    if (!m->engine) return TSDF_ENOMEM;
    if (m->engine->poisoned()) return fail_device(m);
    if (arrays) m->engine->adopt_arrays(arrays, array_bytes);
    HIPCHK(m, hipStreamSynchronize(m->stream));
    return TSDF_OK;
}

tsdf_map *new_map(const tsdf_map_desc *d, void *hip_stream, tsdf_status *st)
{
    tsdf_map *m = new (std::nothrow) tsdf_map();
    if (!m) {
        *st = TSDF_ENOMEM;
        return nullptr;
    }
    m->d = *d;
    if (hipGetDevice(&m->device) != hipSuccess) {
        delete m;
        *st = TSDF_EDEVICE;
        return nullptr;
    }
    if (hip_stream) {
        m->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&m->stream, hipStreamNonBlocking) != hipSuccess) {
            delete m;
            *st = TSDF_EDEVICE;
            return nullptr;
        }
        m->own_stream = true;
    }
    *st = TSDF_OK;
    return m;
}

// Engines for tsdf_integrate_batch, one per stream. The table is never
// destroyed: at process exit the HIP runtime may already be gone, and the
// operating system takes the memory back anyway.
std::mutex g_engines_mu;
std::unordered_map<hipStream_t, std::unique_ptr<Engine>> &engines()
{
    static auto *t = new std::unordered_map<hipStream_t, std::unique_ptr<Engine>>();
    return *t;
}

Engine *engine_of(hipStream_t s)
{
    std::lock_guard<std::mutex> lk(g_engines_mu);
    auto it = engines().find(s);
    return it == engines().end() ? nullptr : it->second.get();
}

// Drop the batch engine of a stream (its work is waited for first).
void drop_engine(hipStream_t s)
{
    std::unique_ptr<Engine> e;
    {
        std::lock_guard<std::mutex> lk(g_engines_mu);
        auto it = engines().find(s);
        if (it == engines().end()) return;
        e = std::move(it->second);
        engines().erase(it);
    }
}

// Box arithmetic over global voxel coordinates.
struct Box {
    int32_t lo[3], hi[3];  // [lo, hi)
    bool empty() const { return lo[0] >= hi[0] || lo[1] >= hi[1] || lo[2] >= hi[2]; }
    int64_t count() const { return empty() ? 0 : (int64_t)(hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2]); }
};

Box window_box(const int32_t origin[3], const int32_t dims[3])
{
    Box b;
    for (int a = 0; a < 3; ++a) {
        b.lo[a] = origin[a];
        b.hi[a] = origin[a] + dims[a];
    }
    return b;
}

Box intersect(const Box &x, const Box &y)
{
    Box b;
    for (int a = 0; a < 3; ++a) {
        b.lo[a] = std::max(x.lo[a], y.lo[a]);
        b.hi[a] = std::min(x.hi[a], y.hi[a]);
    }
    return b;
}

// A \ B for two boxes of equal extent, as up to three disjoint boxes.
std::vector<Box> difference(const Box &A, const Box &B)
{
    std::vector<Box> out;
    Box rest = A;  // the part of A not yet split off
    for (int a = 0; a < 3; ++a) {
        // part of rest whose coordinate a is outside [B.lo, B.hi)
        Box lo_part = rest, hi_part = rest;
        lo_part.hi[a] = std::min(rest.hi[a], B.lo[a]);
        hi_part.lo[a] = std::max(rest.lo[a], B.hi[a]);
        if (!lo_part.empty()) out.push_back(lo_part);
        if (!hi_part.empty()) out.push_back(hi_part);
        rest.lo[a] = std::max(rest.lo[a], B.lo[a]);
        rest.hi[a] = std::min(rest.hi[a], B.hi[a]);
        if (rest.empty()) break;
    }
    return out;
}

// Split a box along the global 64-voxel chunk grid.
void chunk_pieces(const Box &b, std::vector<Box> &out)
{
    if (b.empty()) return;
    for (int64_t cx = floor_div64(b.lo[0], kChunk); cx * kChunk < b.hi[0]; ++cx)
        for (int64_t cy = floor_div64(b.lo[1], kChunk); cy * kChunk < b.hi[1]; ++cy)
            for (int64_t cz = floor_div64(b.lo[2], kChunk); cz * kChunk < b.hi[2]; ++cz) {
                Box p;
                const int64_t c[3] = {cx, cy, cz};
                for (int a = 0; a < 3; ++a) {
                    p.lo[a] = (int32_t)std::max<int64_t>(b.lo[a], c[a] * kChunk);
                    p.hi[a] = (int32_t)std::min<int64_t>(b.hi[a], (c[a] + 1) * kChunk);
                }
                if (!p.empty()) out.push_back(p);
            }
}

ChunkKey key_of(const int32_t g[3])
{
    return ChunkKey{(int32_t)floor_div64(g[0], kChunk), (int32_t)floor_div64(g[1], kChunk),
                    (int32_t)floor_div64(g[2], kChunk)};
}

inline int64_t chunk_off(int32_t x, int32_t y, int32_t z)
{
    return ((int64_t)floor_mod64(x, kChunk) * kChunk + floor_mod64(y, kChunk)) * kChunk + floor_mod64(z, kChunk);
}

// Run `fn(pieces_batch, staged_total)` over batches of chunk pieces whose
// total size fits the staging buffers; pieces are staged back to back.
template <class Fn>
tsdf_status for_batches(tsdf_map *m, const std::vector<Box> &pieces, Fn fn)
{
    const int64_t cap = std::max<int64_t>(m->stage_cap, 16 * kChunkVox);
    tsdf_status st0 = ensure_stage(m, cap, 4096);
    if (st0 != TSDF_OK) return st0;
    size_t i = 0;
    while (i < pieces.size()) {
        std::vector<Box> batch;
        int64_t total = 0;
        while (i < pieces.size() && (batch.empty() || total + pieces[i].count() <= cap) &&
               batch.size() < (size_t)4096) {
            total += pieces[i].count();
            batch.push_back(pieces[i]);
            ++i;
        }
        int64_t off = 0, maxv = 0;
        for (size_t k = 0; k < batch.size(); ++k) {
            BoxXfer &x = m->boxes_host[k];
            for (int a = 0; a < 3; ++a) {
                x.lo[a] = batch[k].lo[a];
                x.ext[a] = batch[k].hi[a] - batch[k].lo[a];
            }
            x.off = off;
            off += batch[k].count();
            maxv = std::max(maxv, batch[k].count());
        }
        tsdf_status st = fn(batch, (int32_t)batch.size(), off, maxv);
        if (st != TSDF_OK) return st;
    }
    return TSDF_OK;
}

// Device -> host: pieces of the window into host arrays via staging.
tsdf_status stage_out(tsdf_map *m, int32_t nb, int64_t total, int64_t maxv, bool clear)
{
    int16_t *dsdf = m->stage_dev, *dw = m->stage_dev + m->stage_cap;
    HIPCHK(m, hipMemcpyAsync(m->boxes_dev, m->boxes_host, (size_t)nb * sizeof(BoxXfer), hipMemcpyHostToDevice,
                             m->stream));
    HIPCHK(m, prof_start(m, TSDF_KERNEL_PACK));
    HIPCHK(m, launch_pack_boxes(m->boxes_dev, nb, maxv, m->sdf, m->w, m->d.dims, dsdf, dw, clear, m->stream));
    HIPCHK(m, prof_stop(m, TSDF_KERNEL_PACK));
    HIPCHK(m, hipMemcpyAsync(m->stage_host, dsdf, (size_t)total * sizeof(int16_t), hipMemcpyDeviceToHost,
                             m->stream));
    HIPCHK(m, hipMemcpyAsync(m->stage_host + m->stage_cap, dw, (size_t)total * sizeof(int16_t),
                             hipMemcpyDeviceToHost, m->stream));
    HIPCHK(m, hipStreamSynchronize(m->stream));
    return TSDF_OK;
}

bool all_zero(const int16_t *a, const int16_t *b, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        if (a[i] | b[i]) return false;
    return true;
}


}  // namespace

extern "C" {

const char *tsdf_status_string(tsdf_status s)
{
    switch (s) {
    case TSDF_OK: return "ok";
    case TSDF_EINVAL: return "invalid argument";
    case TSDF_ENOMEM: return "out of memory";
    case TSDF_EDEVICE: return "device error (map poisoned)";
    case TSDF_ERANGE: return "size out of range";
    case TSDF_EBUSY: return "map busy";
    }
    return "unknown status";
}

size_t tsdf_scratch_bytes(const tsdf_map_desc *d)
{
    if (!desc_ok(d)) return 0;
    return single_map_array_bytes(d->dims);
}

tsdf_status tsdf_map_create(const tsdf_map_desc *d, void *hip_stream, tsdf_map **out)
{
    if (!desc_ok(d) || !out) return TSDF_EINVAL;
    *out = nullptr;
    tsdf_status st;
    tsdf_map *m = new_map(d, hip_stream, &st);
    if (!m) return st;
    const int64_t nv = nvox_of(d);
    m->own_arrays = true;
    if (hipMalloc(&m->sdf, (size_t)nv * sizeof(int16_t)) != hipSuccess ||
        hipMalloc(&m->w, (size_t)nv * sizeof(int16_t)) != hipSuccess) {
        release(m);
        return TSDF_ENOMEM;
    }
    // every voxel starts at (0, 0): unknown (not inside any captured graph)
    if (hipMemsetAsync(m->sdf, 0, (size_t)nv * sizeof(int16_t), m->stream) != hipSuccess ||
        hipMemsetAsync(m->w, 0, (size_t)nv * sizeof(int16_t), m->stream) != hipSuccess) {
        release(m);
        return TSDF_EDEVICE;
    }
    st = init_map(m, nullptr, 0);
    if (st != TSDF_OK) {
        release(m);
        return st;
    }
    *out = m;
    return TSDF_OK;
}

tsdf_status tsdf_map_create_in(const tsdf_map_desc *d, void *sdf_dev, void *w_dev, void *scratch_dev,
                               size_t scratch_bytes, void *hip_stream, tsdf_map **out)
{
    if (!desc_ok(d) || !out || !sdf_dev || !w_dev || !scratch_dev) return TSDF_EINVAL;
    if (scratch_bytes < tsdf_scratch_bytes(d)) return TSDF_EINVAL;
    *out = nullptr;
    tsdf_status st;
    tsdf_map *m = new_map(d, hip_stream, &st);
    if (!m) return st;
    m->sdf = (int16_t *)sdf_dev;
    m->w = (int16_t *)w_dev;
    // the caller's scratch holds the tile arrays; zero them once
    if (launch_fill_u32((uint32_t *)scratch_dev, (int64_t)(scratch_bytes / 4), 0u, m->stream) != hipSuccess) {
        release(m);
        return TSDF_EDEVICE;
    }
    st = init_map(m, scratch_dev, scratch_bytes);
    if (st != TSDF_OK) {
        release(m);
        return st;
    }
    *out = m;
    return TSDF_OK;
}

tsdf_status tsdf_map_destroy(tsdf_map *m)
{
    if (!m) return TSDF_EINVAL;
    // a batch engine running on the stream this map owns goes with it
    if (m->own_stream) drop_engine(m->stream);
    release(m);
    return TSDF_OK;
}

// Whether the map's scans take the key-volume path (interp.hip).
static bool keyvol_path(const tsdf_map *m) { return m->interp_dq > 0 || m->carve; }

// One scan through the key-volume path, on the map's stream.
static tsdf_status integrate_interp(tsdf_map *m, const float *xyz, int64_t n, bool host, const double pose[16],
                             tsdf_scan_stats *stats)
{
    for (int k = 0; k < 12; ++k)
        if (!std::isfinite(pose[k])) return TSDF_EINVAL;
    InterpScan P;
    for (int k = 0; k < 12; ++k) P.rp.M[k] = pose[k];
    P.rp.scale = m->scale;
    for (int a = 0; a < 3; ++a) {
        const double o = nearbyint(pose[4 * a + 3] * m->scale);
        if (!(fabs(o) < 1073741824.0)) return TSDF_EINVAL;
        P.rp.o[a] = (int32_t)o;
        P.up[a] = (int64_t)nearbyint(pose[4 * a + 2] * 1024.0);
        P.origin[a] = m->d.origin[a];
        P.dims[a] = m->d.dims[a];
        const int32_t r0 = m->d.origin[a] % m->d.dims[a];
        P.ring0[a] = r0 < 0 ? r0 + m->d.dims[a] : r0;
    }
    P.rp.tau = m->d.tau_q10;
    P.n = n;
    P.dq = m->interp_dq;
    P.carve = m->carve ? 1 : 0;
    P.sdf = m->sdf;
    P.w = m->w;
    P.w_max = m->d.w_max;
    P.keys = m->interp_keys;
    P.touched = m->interp_touched;
    P.counters = m->interp_ctr;
    P.xyz = xyz;
    if (host && n > 0) {
        if (n > m->interp_pts_cap) {
            HIPCHK(m, hipStreamSynchronize(m->stream));
            if (m->interp_pts) HIPCHK(m, hipFree(m->interp_pts));
            m->interp_pts = nullptr;
            m->interp_pts_cap = 0;
            if (hipMalloc(&m->interp_pts, (size_t)n * 3 * sizeof(float)) != hipSuccess) return TSDF_ENOMEM;
            m->interp_pts_cap = n;
        }
        // synchronous from pageable memory: the caller may reuse xyz at once
        HIPCHK(m, hipMemcpyAsync(m->interp_pts, xyz, (size_t)n * 3 * sizeof(float), hipMemcpyHostToDevice,
                                 m->stream));
        HIPCHK(m, hipStreamSynchronize(m->stream));
        P.xyz = m->interp_pts;
    }
    // the first three counters are per scan; the atomics counter (fourth)
    // adds up until tsdf_map_key_atomics reads it
    HIPCHK(m, launch_fill_u32((uint32_t *)m->interp_ctr, 6, 0u, m->stream));
    HIPCHK(m, launch_interp(P, m->nvox, m->stream));
    if (stats) {
        HIPCHK(m, hipMemcpyAsync(m->interp_ctr_host, m->interp_ctr, 3 * sizeof(unsigned long long),
                                 hipMemcpyDeviceToHost, m->stream));
        HIPCHK(m, hipStreamSynchronize(m->stream));
        stats->points_in = n;
        stats->points_valid = (int64_t)m->interp_ctr_host[0];
        stats->visits = (int64_t)m->interp_ctr_host[1];
        stats->voxels_updated = (int64_t)m->interp_ctr_host[2];
    }
    return TSDF_OK;
}

// The key volume (all EMPTY), its touched-run bytes and counters, once.
static tsdf_status ensure_key_volume(tsdf_map *m)
{
    if (m->interp_keys) return TSDF_OK;
    if (hipMalloc(&m->interp_keys, (size_t)m->nvox * sizeof(unsigned long long)) != hipSuccess) {
        m->interp_keys = nullptr;
        return TSDF_ENOMEM;
    }
    const int64_t runs = (m->nvox + 63) / 64;
    const size_t touched_bytes = (size_t)((runs + 3) / 4 * 4);
    if (hipMalloc(&m->interp_ctr, 4 * sizeof(unsigned long long)) != hipSuccess) m->interp_ctr = nullptr;
    if (hipHostMalloc(&m->interp_ctr_host, 4 * sizeof(unsigned long long), hipHostMallocDefault) != hipSuccess)
        m->interp_ctr_host = nullptr;
    if (hipMalloc(&m->interp_touched, touched_bytes) != hipSuccess) m->interp_touched = nullptr;
    if (!m->interp_ctr || !m->interp_ctr_host || !m->interp_touched) {
        if (m->interp_ctr) (void)hipFree(m->interp_ctr);
        if (m->interp_ctr_host) (void)hipHostFree(m->interp_ctr_host);
        if (m->interp_touched) (void)hipFree(m->interp_touched);
        (void)hipFree(m->interp_keys);
        m->interp_ctr = nullptr;
        m->interp_ctr_host = nullptr;
        m->interp_touched = nullptr;
        m->interp_keys = nullptr;
        return TSDF_ENOMEM;
    }
    HIPCHK(m, launch_fill_u32((uint32_t *)m->interp_keys, m->nvox * 2, 0xffffffffu, m->stream));
    HIPCHK(m, launch_fill_u32((uint32_t *)m->interp_touched, (int64_t)(touched_bytes / 4), 0u, m->stream));
    HIPCHK(m, launch_fill_u32((uint32_t *)m->interp_ctr, 8, 0u, m->stream));
    return TSDF_OK;
}

tsdf_status tsdf_map_set_interpolation(tsdf_map *m, double vfov_deg, int32_t hlines)
{
    if (!m) return TSDF_EINVAL;
    int64_t dq = 0;
    if (vfov_deg != 0.0) {
        // Eq. (3): delta_z = tan(rad(vfov / hlines)), below 1
        if (!(vfov_deg > 0.0) || !std::isfinite(vfov_deg) || hlines < 1) return TSDF_EINVAL;
        const double step = vfov_deg / (double)hlines;
        if (!(step < 45.0)) return TSDF_EINVAL;
        dq = (int64_t)llrint(tan(step * (M_PI / 180.0)) * 1048576.0);
    }
    Guard g(m);
    if (!g.ok) return TSDF_EBUSY;
    if (m->poisoned) return TSDF_EDEVICE;
    if (dq > 0 && m->carve) return TSDF_EINVAL;  // not together with carving
    if (dq > 0) {
        const tsdf_status st = ensure_key_volume(m);
        if (st != TSDF_OK) return st;
    }
    m->interp_dq = dq;
    return TSDF_OK;
}

// Normal equations of the registration at pose M, on device points xyz
// (the map's stream; synchronous): sums in block order.
static tsdf_status reg_sums_dev(tsdf_map *m, const float *xyz, int64_t n, const double M[16], double *partials,
                                std::vector<double> &host, double sums[kRegSums])
{
    RegArgs A;
    for (int k = 0; k < 12; ++k) A.M[k] = M[k];
    A.xyz = xyz;
    A.n = n;
    A.sdf = m->sdf;
    A.w = m->w;
    for (int a = 0; a < 3; ++a) {
        A.dims[a] = m->d.dims[a];
        A.origin[a] = m->d.origin[a];
    }
    A.tau = m->d.tau_q10;
    A.vs = m->d.voxel_size_m;
    for (int k = 0; k < kRegSums; ++k) sums[k] = 0.0;
    const int64_t nb = reg_blocks(n);
    if (nb == 0) return TSDF_OK;
    HIPCHK(m, launch_reg_sums(A, partials, m->stream));
    HIPCHK(m, hipMemcpyAsync(host.data(), partials, (size_t)nb * kRegSums * sizeof(double), hipMemcpyDeviceToHost,
                             m->stream));
    HIPCHK(m, hipStreamSynchronize(m->stream));
    for (int64_t b = 0; b < nb; ++b)
        for (int k = 0; k < kRegSums; ++k) sums[k] += host[(size_t)(b * kRegSums + k)];
    return TSDF_OK;
}

// (H + lambda I) d = -g by Cholesky; then the pose exp([theta]x) applied on
// the left with translation rho (d = (rho, theta)). false when H + lambda I
// is not positive definite.
static bool reg_update(const double sums[kRegSums], double lambda, const double M[16], double out[16], double d[6])
{
    double H[6][6], L[6][6] = {{0}}, y[6];
    for (int a = 0, k = 0; a < 6; ++a)
        for (int b = a; b < 6; ++b, ++k) H[a][b] = H[b][a] = sums[k];
    for (int a = 0; a < 6; ++a) H[a][a] += lambda;
    for (int i = 0; i < 6; ++i) {
        for (int j = 0; j < i; ++j) {
            double s = H[i][j];
            for (int q = 0; q < j; ++q) s -= L[i][q] * L[j][q];
            L[i][j] = s / L[j][j];
        }
        double s = H[i][i];
        for (int q = 0; q < i; ++q) s -= L[i][q] * L[i][q];
        if (!(s > 0.0)) return false;
        L[i][i] = sqrt(s);
    }
    for (int i = 0; i < 6; ++i) {
        double s = -sums[21 + i];
        for (int q = 0; q < i; ++q) s -= L[i][q] * y[q];
        y[i] = s / L[i][i];
    }
    for (int i = 5; i >= 0; --i) {
        double s = y[i];
        for (int q = i + 1; q < 6; ++q) s -= L[q][i] * d[q];
        d[i] = s / L[i][i];
    }
    const double ax = d[3], ay = d[4], az = d[5];
    const double ang = sqrt(ax * ax + ay * ay + az * az);
    const double a = ang > 1e-12 ? sin(ang) / ang : 1.0;
    const double b = ang > 1e-12 ? (1.0 - cos(ang)) / (ang * ang) : 0.5;
    // exp(K) = I + a K + b K^2, K = [theta]x
    const double K[3][3] = {{0.0, -az, ay}, {az, 0.0, -ax}, {-ay, ax, 0.0}};
    double R[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double k2 = 0.0;
            for (int q = 0; q < 3; ++q) k2 += K[i][q] * K[q][j];
            R[i][j] = (i == j ? 1.0 : 0.0) + a * K[i][j] + b * k2;
        }
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 4; ++j) {
            double s = j == 3 ? d[i] : 0.0;
            for (int q = 0; q < 3; ++q) s += R[i][q] * M[4 * q + j];
            out[4 * i + j] = s;
        }
    }
    out[12] = out[13] = out[14] = 0.0;
    out[15] = 1.0;
    return true;
}

// Device copy of a scan's points for the registration calls.
static tsdf_status reg_points(tsdf_map *m, const float *xyz, int64_t n, bool host, const float **dev)
{
    *dev = xyz;
    if (!host || n == 0) return TSDF_OK;
    if (n > m->interp_pts_cap) {
        HIPCHK(m, hipStreamSynchronize(m->stream));
        if (m->interp_pts) HIPCHK(m, hipFree(m->interp_pts));
        m->interp_pts = nullptr;
        m->interp_pts_cap = 0;
        if (hipMalloc(&m->interp_pts, (size_t)n * 3 * sizeof(float)) != hipSuccess) return TSDF_ENOMEM;
        m->interp_pts_cap = n;
    }
    HIPCHK(m, hipMemcpyAsync(m->interp_pts, xyz, (size_t)n * 3 * sizeof(float), hipMemcpyHostToDevice, m->stream));
    HIPCHK(m, hipStreamSynchronize(m->stream));
    *dev = m->interp_pts;
    return TSDF_OK;
}

tsdf_status tsdf_register_sums(tsdf_map *m, const float *xyz, int64_t n_points, tsdf_ptr_kind kind,
                               const double pose[16], double sums[29])
{
    if (!m || !pose || !sums || n_points < 0 || (n_points > 0 && !xyz)) return TSDF_EINVAL;
    if (kind != TSDF_PTR_HOST && kind != TSDF_PTR_DEVICE) return TSDF_EINVAL;
    for (int k = 0; k < 12; ++k)
        if (!std::isfinite(pose[k])) return TSDF_EINVAL;
    Guard g(m);
    if (!g.ok) return TSDF_EBUSY;
    if (m->poisoned) return TSDF_EDEVICE;
    const float *dev;
    tsdf_status st = reg_points(m, xyz, n_points, kind == TSDF_PTR_HOST, &dev);
    if (st != TSDF_OK) return st;
    const int64_t nb = reg_blocks(n_points);
    double *partials = nullptr;
    if (nb > 0 && hipMalloc(&partials, (size_t)nb * kRegSums * sizeof(double)) != hipSuccess) return TSDF_ENOMEM;
    std::vector<double> host((size_t)nb * kRegSums);
    st = reg_sums_dev(m, dev, n_points, pose, partials, host, sums);
    if (partials) (void)hipFree(partials);
    return st;
}

tsdf_status tsdf_register_scan(tsdf_map *m, const float *xyz, int64_t n_points, tsdf_ptr_kind kind,
                               const double init_pose[16], int32_t iterations, double damping, double pose_out[16],
                               tsdf_register_info *info)
{
    if (!m || !init_pose || !pose_out || n_points < 0 || (n_points > 0 && !xyz) || iterations < 0 ||
        !(damping >= 0.0) || !std::isfinite(damping))
        return TSDF_EINVAL;
    if (kind != TSDF_PTR_HOST && kind != TSDF_PTR_DEVICE) return TSDF_EINVAL;
    for (int k = 0; k < 12; ++k)
        if (!std::isfinite(init_pose[k])) return TSDF_EINVAL;
    Guard g(m);
    if (!g.ok) return TSDF_EBUSY;
    if (m->poisoned) return TSDF_EDEVICE;
    const float *dev;
    tsdf_status st = reg_points(m, xyz, n_points, kind == TSDF_PTR_HOST, &dev);
    if (st != TSDF_OK) return st;
    const int64_t nb = reg_blocks(n_points);
    double *partials = nullptr;
    if (nb > 0 && hipMalloc(&partials, (size_t)nb * kRegSums * sizeof(double)) != hipSuccess) return TSDF_ENOMEM;
    std::vector<double> host((size_t)nb * kRegSums);
    double M[16], sums[kRegSums], d[6] = {0, 0, 0, 0, 0, 0}, step = 0.0;
    memcpy(M, init_pose, sizeof(M));
    int32_t it = 0;
    for (; it < iterations && st == TSDF_OK; ++it) {
        st = reg_sums_dev(m, dev, n_points, M, partials, host, sums);
        if (st != TSDF_OK || sums[28] < 6.0) break;
        double Mn[16];
        if (!reg_update(sums, damping, M, Mn, d)) break;
        memcpy(M, Mn, sizeof(M));
        step = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + d[3] * d[3] + d[4] * d[4] + d[5] * d[5]);
    }
    if (st == TSDF_OK) st = reg_sums_dev(m, dev, n_points, M, partials, host, sums);
    if (partials) (void)hipFree(partials);
    if (st != TSDF_OK) return st;
    memcpy(pose_out, M, sizeof(M));
    if (info) {
        info->points_used = (int64_t)sums[28];
        info->cost = sums[27];
        info->last_step = step;
        info->steps = it;
    }
    return TSDF_OK;
}

tsdf_status tsdf_mesh(tsdf_map *m, const int32_t lo[3], const int32_t hi[3], float *tris, int64_t max_tris,
                      int64_t *n_tris)
{
    if (!m || !lo || !hi || !n_tris || max_tris < 0 || (max_tris > 0 && !tris)) return TSDF_EINVAL;
    for (int a = 0; a < 3; ++a)
        if (hi[a] < lo[a] || lo[a] < m->d.origin[a] || (int64_t)hi[a] > (int64_t)m->d.origin[a] + m->d.dims[a])
            return TSDF_EINVAL;
    Guard g(m);
    if (!g.ok) return TSDF_EBUSY;
    if (m->poisoned) return TSDF_EDEVICE;
    MeshArgs A;
    A.sdf = m->sdf;
    A.w = m->w;
    A.ncubes = 1;
    for (int a = 0; a < 3; ++a) {
        A.dims[a] = m->d.dims[a];
        A.lo[a] = lo[a];
        A.n[a] = std::max<int64_t>(0, (int64_t)hi[a] - lo[a] - 1);
        A.ncubes *= A.n[a];
    }
    A.vs = m->d.voxel_size_m;
    *n_tris = 0;
    if (A.ncubes == 0) return TSDF_OK;
    const int64_t nb = mesh_blocks(A.ncubes);
    uint32_t *bt = nullptr;
    uint64_t *bb = nullptr;
    float *out = nullptr;
    std::vector<uint32_t> counts((size_t)nb);
    std::vector<uint64_t> base((size_t)nb);
    tsdf_status st = TSDF_OK;
    auto done = [&](tsdf_status r) {
        if (bt) (void)hipFree(bt);
        if (bb) (void)hipFree(bb);
        if (out) (void)hipFree(out);
        return r;
    };
    if (hipMalloc(&bt, (size_t)nb * sizeof(uint32_t)) != hipSuccess) return done(TSDF_ENOMEM);
    if (launch_mesh_count(A, bt, m->stream) != hipSuccess ||
        hipMemcpyAsync(counts.data(), bt, (size_t)nb * sizeof(uint32_t), hipMemcpyDeviceToHost, m->stream) !=
            hipSuccess ||
        hipStreamSynchronize(m->stream) != hipSuccess)
        return done(fail_device(m));
    uint64_t total = 0;
    for (int64_t b = 0; b < nb; ++b) {
        base[(size_t)b] = total;
        total += counts[(size_t)b];
    }
    *n_tris = (int64_t)total;
    if (!tris || total == 0) return done(TSDF_OK);  // a query of the count
    if ((uint64_t)max_tris < total) return done(TSDF_ERANGE);
    if (hipMalloc(&bb, (size_t)nb * sizeof(uint64_t)) != hipSuccess ||
        hipMalloc(&out, (size_t)total * 9 * sizeof(float)) != hipSuccess)
        return done(TSDF_ENOMEM);
    if (hipMemcpyAsync(bb, base.data(), (size_t)nb * sizeof(uint64_t), hipMemcpyHostToDevice, m->stream) !=
            hipSuccess ||
        launch_mesh_emit(A, bb, out, m->stream) != hipSuccess ||
        hipMemcpyAsync(tris, out, (size_t)total * 9 * sizeof(float), hipMemcpyDeviceToHost, m->stream) !=
            hipSuccess ||
        hipStreamSynchronize(m->stream) != hipSuccess)
        st = fail_device(m);
    return done(st);
}

tsdf_status tsdf_map_get_interpolation(const tsdf_map *m, int64_t *delta_q20)
{
    if (!m || !delta_q20) return TSDF_EINVAL;
    *delta_q20 = m->interp_dq;
    return TSDF_OK;
}

tsdf_status tsdf_map_set_carving(tsdf_map *m, int32_t on)
{
    if (!m || (on != 0 && on != 1)) return TSDF_EINVAL;
    Guard g(m);
    if (!g.ok) return TSDF_EBUSY;
    if (m->poisoned) return TSDF_EDEVICE;
    if (on && m->interp_dq > 0) return TSDF_EINVAL;  // not together with interpolation
    if (on) {
        const tsdf_status st = ensure_key_volume(m);
        if (st != TSDF_OK) return st;
    }
    m->carve = on != 0;
    return TSDF_OK;
}

tsdf_status tsdf_map_key_atomics(tsdf_map *m, int64_t *issued)
{
    if (!m || !issued) return TSDF_EINVAL;
    Guard g(m);
    if (!g.ok) return TSDF_EBUSY;
    if (m->poisoned) return TSDF_EDEVICE;
    *issued = 0;
    if (!m->interp_ctr) return TSDF_OK;  // no key volume yet: nothing issued
    HIPCHK(m, hipMemcpyAsync(m->interp_ctr_host + 3, m->interp_ctr + 3, sizeof(unsigned long long),
                             hipMemcpyDeviceToHost, m->stream));
    HIPCHK(m, hipStreamSynchronize(m->stream));
    *issued = (int64_t)m->interp_ctr_host[3];
    HIPCHK(m, launch_fill_u32((uint32_t *)(m->interp_ctr + 3), 2, 0u, m->stream));
    return TSDF_OK;
}

tsdf_status tsdf_map_get_carving(const tsdf_map *m, int32_t *on)
{
    if (!m || !on) return TSDF_EINVAL;
    *on = m->carve ? 1 : 0;
    return TSDF_OK;
}

tsdf_status tsdf_integrate_scan(tsdf_map *m, const float *xyz, int64_t n_points, tsdf_ptr_kind kind,
                                const double pose[16], tsdf_scan_stats *stats)
{
    if (!m || !pose || n_points < 0 || n_points > 0xffffffffLL || (n_points > 0 && !xyz)) return TSDF_EINVAL;
    if (kind != TSDF_PTR_HOST && kind != TSDF_PTR_DEVICE) return TSDF_EINVAL;
    Guard g(m);
    if (!g.ok) return TSDF_EBUSY;
    if (m->poisoned) return TSDF_EDEVICE;
    if (keyvol_path(m)) return integrate_interp(m, xyz, n_points, kind == TSDF_PTR_HOST, pose, stats);
    std::vector<MapRef> maps{map_ref(m)};
    std::vector<ScanRef> scans{ScanRef{0, xyz, n_points, kind == TSDF_PTR_HOST, pose}};
    tsdf_status st = m->engine->run(maps, scans, launch_shape(m, false), stats);
    if (st == TSDF_EDEVICE) m->poisoned = true;
    return st;
}

tsdf_status tsdf_integrate_batch(const tsdf_scan_desc *scans, int32_t count, tsdf_ptr_kind kind, void *hip_stream,
                                 tsdf_scan_stats *stats)
{
    if (count < 0 || (count > 0 && !scans)) return TSDF_EINVAL;
    if (kind != TSDF_PTR_HOST && kind != TSDF_PTR_DEVICE) return TSDF_EINVAL;
    if (count == 0) return TSDF_OK;
    // Scans of maps with vertical interpolation or carving take their own path, one by
    // one in order on their map's stream, between events on the batch
    // stream; the others go through the batched engine as one batch. (Maps
    // are independent, so the two groups may run in either order.)
    bool any_interp = false;
    for (int32_t k = 0; k < count; ++k) {
        if (!scans[k].map) return TSDF_EINVAL;
        any_interp = any_interp || keyvol_path(scans[k].map);
    }
    if (any_interp) {
        hipStream_t bs = hip_stream ? (hipStream_t)hip_stream : scans[0].map->stream;
        std::vector<tsdf_scan_desc> rest;
        std::vector<int32_t> rest_at;
        for (int32_t k = 0; k < count; ++k) {
            tsdf_map *m = scans[k].map;
            if (!keyvol_path(m)) {
                rest.push_back(scans[k]);
                rest_at.push_back(k);
                continue;
            }
            Guard g(m);
            if (!g.ok) return TSDF_EBUSY;
            if (m->poisoned) return TSDF_EDEVICE;
            hipEvent_t before = take_event(m), after = take_event(m);
            if (!before || !after) return fail_device(m);
            HIPCHK(m, hipEventRecord(before, bs));
            HIPCHK(m, hipStreamWaitEvent(m->stream, before, 0));
            tsdf_status st = integrate_interp(m, scans[k].xyz, scans[k].n_points, kind == TSDF_PTR_HOST,
                                              scans[k].pose, stats ? &stats[k] : nullptr);
            if (st != TSDF_OK) return st;
            HIPCHK(m, hipEventRecord(after, m->stream));
            HIPCHK(m, hipStreamWaitEvent(bs, after, 0));
            m->ev_pool.push_back(before);
            m->ev_pool.push_back(after);
        }
        if (rest.empty()) return TSDF_OK;
        std::vector<tsdf_scan_stats> rst(stats ? rest.size() : 0);
        tsdf_status st = tsdf_integrate_batch(rest.data(), (int32_t)rest.size(), kind, (void *)bs,
                                              stats ? rst.data() : nullptr);
        if (st == TSDF_OK && stats)
            for (size_t j = 0; j < rest.size(); ++j) stats[rest_at[j]] = rst[j];
        return st;
    }
    std::vector<MapRef> maps;
    std::vector<ScanRef> refs;
    std::unordered_map<const tsdf_map *, int32_t> idx;
    std::vector<std::unique_ptr<Guard>> guards;
    for (int32_t k = 0; k < count; ++k) {
        tsdf_map *m = scans[k].map;
        if (!m) return TSDF_EINVAL;
        auto it = idx.find(m);
        if (it == idx.end()) {
            guards.emplace_back(new Guard(m));
            if (!guards.back()->ok) return TSDF_EBUSY;
            if (m->poisoned) return TSDF_EDEVICE;
            it = idx.emplace(m, (int32_t)maps.size()).first;
            maps.push_back(map_ref(m));
        }
        refs.push_back(ScanRef{it->second, scans[k].xyz, scans[k].n_points, kind == TSDF_PTR_HOST, scans[k].pose});
    }
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : maps[0].stream;
    Engine *eng;
    {
        std::lock_guard<std::mutex> lk(g_engines_mu);
        auto &slot = engines()[s];
        if (!slot) {
            int dev = 0;
            if (hipGetDevice(&dev) != hipSuccess) return TSDF_EDEVICE;
            slot.reset(new (std::nothrow) Engine(s, dev));
            if (!slot) return TSDF_ENOMEM;
        }
        eng = slot.get();
    }
    const tsdf_map *first = scans[0].map;
    tsdf_status st = eng->run(maps, refs, launch_shape(first, true), stats);
    if (st == TSDF_EDEVICE)
        for (int32_t k = 0; k < count; ++k) scans[k].map->poisoned = true;
    return st;
}

tsdf_status tsdf_shift(tsdf_map *m, const int32_t new_origin[3])
{
    if (!m || !new_origin) return TSDF_EINVAL;
    for (int a = 0; a < 3; ++a)
        if ((int64_t)new_origin[a] + m->d.dims[a] > (int64_t)1 << 20 || (int64_t)new_origin[a] < -((int64_t)1 << 20))
            return TSDF_EINVAL;
    Guard g(m);
    if (!g.ok) return TSDF_EBUSY;
    if (m->poisoned) return TSDF_EDEVICE;
    const Box oldw = window_box(m->d.origin, m->d.dims);
    const Box neww = window_box(new_origin, m->d.dims);
    std::vector<Box> leaving, entering, lp, ep;
    leaving = difference(oldw, neww);
    entering = difference(neww, oldw);
    for (auto &b : leaving) chunk_pieces(b, lp);
    for (auto &b : entering) chunk_pieces(b, ep);

    // Whole chunks cross the host link as one copy each, in the store's own
    // layout, when every (x, y) row of the window holds a chunk's z-run
    // contiguously (dims multiples of 64, 16-byte aligned arrays); other
    // pieces go through the general staging path. Entering voxels take the
    // slots that leaving voxels free, so every write into the window comes
    // after every read: leaving chunks and pieces first, then entering ones.
    const bool chunked = m->d.dims[0] % kChunk == 0 && m->d.dims[1] % kChunk == 0 && m->d.dims[2] % kChunk == 0 &&
                         (uintptr_t)m->sdf % 16 == 0 && (uintptr_t)m->w % 16 == 0;
    std::vector<Box> lfull, lpart, efull, epart;
    for (auto &b : lp) (chunked && b.count() == kChunkVox ? lfull : lpart).push_back(b);
    for (auto &b : ep) {
        if (!m->store.count(key_of(b.lo))) continue;  // never stored: its slots were cleared on leaving
        (chunked && b.count() == kChunkVox ? efull : epart).push_back(b);
    }
    tsdf_status st = TSDF_OK;
    if (!lfull.empty() || !efull.empty()) {
        st = ensure_chunk_stage(m);
        if (st != TSDF_OK) return st;
    }
    int16_t *cs_out = m->cstage_dev, *cs_in = m->cstage_dev + (size_t)kShiftChunks * 2 * kChunkVox;
    const size_t chunk_bytes = (size_t)2 * kChunkVox * sizeof(int16_t);
    // the first round of entering chunks goes to the device on the copy
    // stream right away, while the leaving chunks are packed and copied out
    auto copy_in = [&](size_t e0) -> tsdf_status {
        const size_t n = std::min<size_t>(kShiftChunks, efull.size() - e0);
        for (size_t j = 0; j < n; ++j) {
            const Chunk &c = m->store.find(key_of(efull[e0 + j].lo))->second;
            HIPCHK(m, hipMemcpyAsync(cs_in + j * 2 * kChunkVox, c.buf, chunk_bytes, hipMemcpyHostToDevice,
                                     m->copy_stream));
        }
        HIPCHK(m, hipEventRecord(m->copy_done, m->copy_stream));
        return TSDF_OK;
    };
    if (!efull.empty() && (st = copy_in(0)) != TSDF_OK) return st;

    // 1. whole leaving chunks: pack (and clear) on the device, flags of the
    //    chunks that hold an observed voxel, one copy out per such chunk
    for (size_t l0 = 0; l0 < lfull.size(); l0 += kShiftChunks) {
        const int32_t n = (int32_t)std::min<size_t>(kShiftChunks, lfull.size() - l0);
        for (int32_t j = 0; j < n; ++j) {
            BoxXfer &x = m->clist_host[j];
            for (int a = 0; a < 3; ++a) {
                x.lo[a] = lfull[l0 + j].lo[a];
                x.ext[a] = kChunk;
            }
            x.off = 0;
        }
        HIPCHK(m, hipMemcpyAsync(m->clist_dev, m->clist_host, (size_t)n * sizeof(BoxXfer), hipMemcpyHostToDevice,
                                 m->stream));
        HIPCHK(m, launch_fill_u32(m->cflags_dev, n, 0u, m->stream));
        HIPCHK(m, prof_start(m, TSDF_KERNEL_PACK));
        HIPCHK(m, launch_pack_chunks(m->clist_dev, n, m->sdf, m->w, m->d.dims, cs_out, m->cflags_dev, m->stream));
        HIPCHK(m, prof_stop(m, TSDF_KERNEL_PACK));
        HIPCHK(m, hipMemcpyAsync(m->cflags_host, m->cflags_dev, (size_t)n * sizeof(uint32_t), hipMemcpyDeviceToHost,
                                 m->stream));
        HIPCHK(m, hipStreamSynchronize(m->stream));
        for (int32_t j = 0; j < n; ++j) {
            const ChunkKey ck = key_of(lfull[l0 + j].lo);
            auto it = m->store.find(ck);
            if (!m->cflags_host[j]) {
                // nothing observed: nothing to keep (a stored chunk whose voxels
                // were all resident holds zeros only)
                if (it != m->store.end()) {
                    chunk_give(m, it->second);
                    m->store.erase(it);
                }
                continue;
            }
            if (it == m->store.end()) {
                Chunk c;
                c.buf = chunk_take(m);
                if (!c.buf) return TSDF_ENOMEM;
                it = m->store.emplace(ck, c).first;
            }
            HIPCHK(m, hipMemcpyAsync(it->second.buf, cs_out + (size_t)j * 2 * kChunkVox, chunk_bytes,
                                     hipMemcpyDeviceToHost, m->stream));
        }
        HIPCHK(m, hipStreamSynchronize(m->stream));
    }

    // 2. other leaving pieces: pack (and clear) -> host staging -> store
    st = for_batches(m, lpart, [&](const std::vector<Box> &batch, int32_t nb, int64_t total, int64_t maxv) {
        tsdf_status s = stage_out(m, nb, total, maxv, true);
        if (s != TSDF_OK) return s;
        const int16_t *hs = m->stage_host, *hw = m->stage_host + m->stage_cap;
        for (int32_t k = 0; k < nb; ++k) {
            const Box &b = batch[k];
            const int64_t off = m->boxes_host[k].off;
            const int64_t cnt = b.count();
            const ChunkKey ck = key_of(b.lo);
            auto it = m->store.find(ck);
            if (it == m->store.end()) {
                if (all_zero(hs + off, hw + off, cnt)) continue;  // nothing observed: nothing to keep
                Chunk c;
                c.buf = chunk_take(m);
                if (!c.buf) return TSDF_ENOMEM;
                memset(c.buf, 0, (size_t)2 * kChunkVox * sizeof(int16_t));
                it = m->store.emplace(ck, c).first;
            }
            Chunk &c = it->second;
            const int32_t ey = b.hi[1] - b.lo[1], ez = b.hi[2] - b.lo[2];
            for (int32_t x = b.lo[0]; x < b.hi[0]; ++x)
                for (int32_t y = b.lo[1]; y < b.hi[1]; ++y) {
                    const int64_t src = off + ((int64_t)(x - b.lo[0]) * ey + (y - b.lo[1])) * ez;
                    const int64_t dst = chunk_off(x, y, b.lo[2]);
                    memcpy(c.sdf() + dst, hs + src, (size_t)ez * sizeof(int16_t));
                    memcpy(c.w() + dst, hw + src, (size_t)ez * sizeof(int16_t));
                }
        }
        return TSDF_OK;
    });
    if (st != TSDF_OK) return st;

    // 3. whole entering chunks held by the store: already on their way to the
    //    device (copy stream); unpacked once there, then dropped from the store
    for (size_t e0 = 0; e0 < efull.size(); e0 += kShiftChunks) {
        const int32_t n = (int32_t)std::min<size_t>(kShiftChunks, efull.size() - e0);
        if (e0 > 0 && (st = copy_in(e0)) != TSDF_OK) return st;
        BoxXfer *list = m->clist_host + kShiftChunks;
        for (int32_t j = 0; j < n; ++j) {
            for (int a = 0; a < 3; ++a) {
                list[j].lo[a] = efull[e0 + j].lo[a];
                list[j].ext[a] = kChunk;
            }
            list[j].off = 0;
        }
        HIPCHK(m, hipMemcpyAsync(m->clist_dev + kShiftChunks, list, (size_t)n * sizeof(BoxXfer),
                                 hipMemcpyHostToDevice, m->stream));
        HIPCHK(m, hipStreamWaitEvent(m->stream, m->copy_done, 0));
        HIPCHK(m, prof_start(m, TSDF_KERNEL_UNPACK));
        HIPCHK(m, launch_unpack_chunks(m->clist_dev + kShiftChunks, n, m->sdf, m->w, m->d.dims, cs_in, m->stream));
        HIPCHK(m, prof_stop(m, TSDF_KERNEL_UNPACK));
        HIPCHK(m, hipStreamSynchronize(m->stream));
        for (int32_t j = 0; j < n; ++j) {
            auto it = m->store.find(key_of(efull[e0 + j].lo));
            chunk_give(m, it->second);
            m->store.erase(it);
        }
    }

    // 4. other entering pieces held by the store: store -> host staging -> unpack
    st = for_batches(m, epart, [&](const std::vector<Box> &batch, int32_t nb, int64_t total, int64_t maxv) {
        int16_t *hs = m->stage_host, *hw = m->stage_host + m->stage_cap;
        for (int32_t k = 0; k < nb; ++k) {
            const Box &b = batch[k];
            const int64_t off = m->boxes_host[k].off;
            auto it = m->store.find(key_of(b.lo));
            Chunk &c = it->second;
            const int32_t ey = b.hi[1] - b.lo[1], ez = b.hi[2] - b.lo[2];
            for (int32_t x = b.lo[0]; x < b.hi[0]; ++x)
                for (int32_t y = b.lo[1]; y < b.hi[1]; ++y) {
                    const int64_t dst = off + ((int64_t)(x - b.lo[0]) * ey + (y - b.lo[1])) * ez;
                    const int64_t src = chunk_off(x, y, b.lo[2]);
                    memcpy(hs + dst, c.sdf() + src, (size_t)ez * sizeof(int16_t));
                    memcpy(hw + dst, c.w() + src, (size_t)ez * sizeof(int16_t));
                    // popped: the store no longer holds these voxels
                    memset(c.sdf() + src, 0, (size_t)ez * sizeof(int16_t));
                    memset(c.w() + src, 0, (size_t)ez * sizeof(int16_t));
                }
            if (b.count() == kChunkVox) {
                chunk_give(m, c);
                m->store.erase(it);
            }
        }
        int16_t *dsdf = m->stage_dev, *dw = m->stage_dev + m->stage_cap;
        HIPCHK(m, hipMemcpyAsync(m->boxes_dev, m->boxes_host, (size_t)nb * sizeof(BoxXfer), hipMemcpyHostToDevice,
                                 m->stream));
        HIPCHK(m, hipMemcpyAsync(dsdf, hs, (size_t)total * sizeof(int16_t), hipMemcpyHostToDevice, m->stream));
        HIPCHK(m, hipMemcpyAsync(dw, hw, (size_t)total * sizeof(int16_t), hipMemcpyHostToDevice, m->stream));
        HIPCHK(m, prof_start(m, TSDF_KERNEL_UNPACK));
        HIPCHK(m, launch_unpack_boxes(m->boxes_dev, nb, maxv, m->sdf, m->w, m->d.dims, dsdf, dw, m->stream));
        HIPCHK(m, prof_stop(m, TSDF_KERNEL_UNPACK));
        HIPCHK(m, hipStreamSynchronize(m->stream));
        return TSDF_OK;
    });
    if (st != TSDF_OK) return st;
    for (int a = 0; a < 3; ++a) m->d.origin[a] = new_origin[a];
    return TSDF_OK;
}

tsdf_status tsdf_readback(tsdf_map *m, const int32_t lo[3], const int32_t hi[3], int16_t *sdf_out, int16_t *w_out)
{
    if (!m || !lo || !hi || !sdf_out || !w_out) return TSDF_EINVAL;
    for (int a = 0; a < 3; ++a)
        if (hi[a] < lo[a]) return TSDF_EINVAL;
    Guard g(m);
    if (!g.ok) return TSDF_EBUSY;
    if (m->poisoned) return TSDF_EDEVICE;
    Box req;
    for (int a = 0; a < 3; ++a) {
        req.lo[a] = lo[a];
        req.hi[a] = hi[a];
    }
    if (req.empty()) return TSDF_OK;
    const int64_t ny = hi[1] - lo[1], nz = hi[2] - lo[2];
    // stored or unseen voxels first
    std::vector<Box> pieces;
    chunk_pieces(req, pieces);
    for (const Box &b : pieces) {
        auto it = m->store.find(key_of(b.lo));
        for (int32_t x = b.lo[0]; x < b.hi[0]; ++x)
            for (int32_t y = b.lo[1]; y < b.hi[1]; ++y) {
                const int64_t dst = ((int64_t)(x - lo[0]) * ny + (y - lo[1])) * nz + (b.lo[2] - lo[2]);
                const size_t nb = (size_t)(b.hi[2] - b.lo[2]) * sizeof(int16_t);
                if (it == m->store.end()) {
                    memset(sdf_out + dst, 0, nb);
                    memset(w_out + dst, 0, nb);
                } else {
                    const int64_t src = chunk_off(x, y, b.lo[2]);
                    memcpy(sdf_out + dst, it->second.sdf() + src, nb);
                    memcpy(w_out + dst, it->second.w() + src, nb);
                }
            }
    }
    // then the resident part, from the device
    const Box res = intersect(req, window_box(m->d.origin, m->d.dims));
    std::vector<Box> rp;
    chunk_pieces(res, rp);
    return for_batches(m, rp, [&](const std::vector<Box> &batch, int32_t nb, int64_t total, int64_t maxv) {
        tsdf_status s = stage_out(m, nb, total, maxv, false);
        if (s != TSDF_OK) return s;
        const int16_t *hs = m->stage_host, *hw = m->stage_host + m->stage_cap;
        for (int32_t k = 0; k < nb; ++k) {
            const Box &b = batch[k];
            const int64_t off = m->boxes_host[k].off;
            const int32_t ey = b.hi[1] - b.lo[1], ez = b.hi[2] - b.lo[2];
            for (int32_t x = b.lo[0]; x < b.hi[0]; ++x)
                for (int32_t y = b.lo[1]; y < b.hi[1]; ++y) {
                    const int64_t src = off + ((int64_t)(x - b.lo[0]) * ey + (y - b.lo[1])) * ez;
                    const int64_t dst = ((int64_t)(x - lo[0]) * ny + (y - lo[1])) * nz + (b.lo[2] - lo[2]);
                    memcpy(sdf_out + dst, hs + src, (size_t)ez * sizeof(int16_t));
                    memcpy(w_out + dst, hw + src, (size_t)ez * sizeof(int16_t));
                }
        }
        return TSDF_OK;
    });
}

tsdf_status tsdf_batch_profile(void *hip_stream, int32_t on)
{
    Engine *e = engine_of((hipStream_t)hip_stream);
    if (!e) return TSDF_EINVAL;
    e->profile(on != 0);
    return TSDF_OK;
}

tsdf_status tsdf_batch_profile_read(void *hip_stream, int32_t stage, double *total_ms, int64_t *launches)
{
    Engine *e = engine_of((hipStream_t)hip_stream);
    if (!e || stage < 0 || stage > 3 || !total_ms || !launches) return TSDF_EINVAL;
    return e->profile_read(stage, total_ms, launches);
}

tsdf_status tsdf_set_graph_launch(int32_t on)
{
    Engine::set_graphs(on != 0);
    return TSDF_OK;
}

tsdf_status tsdf_batch_release(void *hip_stream)
{
    drop_engine((hipStream_t)hip_stream);
    return TSDF_OK;
}

tsdf_status tsdf_map_origin(const tsdf_map *m, int32_t origin[3])
{
    if (!m || !origin) return TSDF_EINVAL;
    for (int a = 0; a < 3; ++a) origin[a] = m->d.origin[a];
    return TSDF_OK;
}

tsdf_status tsdf_map_device_arrays(const tsdf_map *m, void **sdf_dev, void **w_dev, void **hip_stream)
{
    if (!m) return TSDF_EINVAL;
    if (sdf_dev) *sdf_dev = m->sdf;
    if (w_dev) *w_dev = m->w;
    if (hip_stream) *hip_stream = m->stream;
    return TSDF_OK;
}

tsdf_status tsdf_recentre_origin(const tsdf_map *m, const double pose[16], int64_t radius_q10, int32_t chunk,
                                 int32_t force, int32_t new_origin[3], int32_t *due)
{
    if (!m || !pose || !new_origin || !due || chunk < 1 || radius_q10 < 0) return TSDF_EINVAL;
    int64_t o[3];
    for (int a = 0; a < 3; ++a) {
        const double r = nearbyint(pose[4 * a + 3] * m->scale);
        if (!(fabs(r) < 1073741824.0)) return TSDF_EINVAL;
        o[a] = (int64_t)r;
    }
    __int128 d2 = 0;
    for (int a = 0; a < 3; ++a) {
        const __int128 c = (__int128)1024 * ((int64_t)m->d.origin[a] + m->d.dims[a] / 2);
        const __int128 dd = (__int128)o[a] - c;
        d2 += dd * dd;
    }
    *due = (force || d2 > (__int128)radius_q10 * radius_q10) ? 1 : 0;
    for (int a = 0; a < 3; ++a) {
        const int64_t sv = floor_div64(o[a], 1024);
        new_origin[a] = (int32_t)(chunk * floor_div64(sv + chunk / 2, chunk) - m->d.dims[a] / 2);
    }
    return TSDF_OK;
}

tsdf_status tsdf_store_info(const tsdf_map *m, int64_t *chunks, int64_t *bytes)
{
    if (!m) return TSDF_EINVAL;
    if (chunks) *chunks = (int64_t)m->store.size();
    if (bytes) *bytes = (int64_t)m->store.size() * kChunkVox * 2 * (int64_t)sizeof(int16_t);
    return TSDF_OK;
}

tsdf_status tsdf_profile_enable(tsdf_map *m, int32_t on)
{
    if (!m) return TSDF_EINVAL;
    Guard g(m);
    if (!g.ok) return TSDF_EBUSY;
    if (m->poisoned) return TSDF_EDEVICE;
    HIPCHK(m, hipStreamSynchronize(m->stream));
    prof_clear(m);
    m->prof_on = on != 0;
    m->engine->profile(on != 0);
    return TSDF_OK;
}

tsdf_status tsdf_profile_read(tsdf_map *m, int32_t kernel, double *total_ms, int64_t *launches)
{
    if (!m || kernel < 0 || kernel >= TSDF_KERNEL_COUNT || !total_ms || !launches) return TSDF_EINVAL;
    Guard g(m);
    if (!g.ok) return TSDF_EBUSY;
    if (m->poisoned) return TSDF_EDEVICE;
    if (kernel == TSDF_KERNEL_BIN || kernel == TSDF_KERNEL_TILE) {
        tsdf_status st = m->engine->profile_read(kernel == TSDF_KERNEL_BIN ? 0 : 1, total_ms, launches);
        if (st == TSDF_EDEVICE) m->poisoned = true;
        return st;
    }
    HIPCHK(m, hipStreamSynchronize(m->stream));
    double tot = 0.0;
    for (auto &p : m->prof_ev[kernel]) {
        float ms = 0.f;
        HIPCHK(m, hipEventElapsedTime(&ms, p.first, p.second));
        tot += ms;
    }
    *total_ms = tot;
    *launches = (int64_t)m->prof_ev[kernel].size();
    return TSDF_OK;
}

const char *tsdf_kernel_name(int32_t kernel)
{
    switch (kernel) {
    case TSDF_KERNEL_BIN: return "k_bin";
    case TSDF_KERNEL_TILE: return "k_tile";
    case TSDF_KERNEL_PACK: return "k_pack";
    case TSDF_KERNEL_UNPACK: return "k_unpack";
    default: return "unknown";
    }
}

tsdf_status tsdf_map_set_tiling(tsdf_map *m, const int32_t log2_tile[3], int32_t tile_workgroups)
{
    if (!m || !log2_tile || tile_workgroups < 0 || tile_workgroups > kMaxTileGrid) return TSDF_EINVAL;
    const bool automatic = log2_tile[0] == 0 && log2_tile[1] == 0 && log2_tile[2] == 0;
    if (!automatic && !tiling_ok(log2_tile)) return TSDF_EINVAL;
    Guard g(m);
    if (!g.ok) return TSDF_EBUSY;
    if (m->poisoned) return TSDF_EDEVICE;
    for (int a = 0; a < 3; ++a) m->lt[a] = log2_tile[a];
    m->tile_grid = tile_workgroups;
    return TSDF_OK;
}

tsdf_status tsdf_map_set_blocks(tsdf_map *m, int32_t bin_block, int32_t tile_block)
{
    if (!m) return TSDF_EINVAL;
    const int32_t bb = bin_block > 0 ? bin_block : kBinBlock;
    const int32_t tb = tile_block > 0 ? tile_block : kTileBlockDefault;
    if (bin_block < 0 || tile_block < 0 || !launch_blocks_ok(bb, tb)) return TSDF_EINVAL;
    Guard g(m);
    if (!g.ok) return TSDF_EBUSY;
    m->bin_block = bin_block;
    m->tile_block = tile_block;
    return TSDF_OK;
}

tsdf_status tsdf_map_get_blocks(const tsdf_map *m, int32_t *bin_block, int32_t *tile_block)
{
    if (!m || !bin_block || !tile_block) return TSDF_EINVAL;
    *bin_block = m->bin_block > 0 ? m->bin_block : kBinBlock;
    *tile_block = m->tile_block > 0 ? m->tile_block : kTileBlockDefault;
    return TSDF_OK;
}

tsdf_status tsdf_map_get_tiling(const tsdf_map *m, int32_t log2_tile[3], int32_t *tile_workgroups)
{
    if (!m || !log2_tile || !tile_workgroups) return TSDF_EINVAL;
    for (int a = 0; a < 3; ++a) log2_tile[a] = m->lt[a];
    *tile_workgroups = m->tile_grid;
    return TSDF_OK;
}

tsdf_status tsdf_map_synchronize(tsdf_map *m)
{
    if (!m) return TSDF_EINVAL;
    if (m->poisoned) return TSDF_EDEVICE;
    HIPCHK(m, hipStreamSynchronize(m->stream));
    return TSDF_OK;
}

}  // extern "C"
