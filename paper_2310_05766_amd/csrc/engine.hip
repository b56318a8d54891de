// Host side of the batched integration engine (see batch.hip for the
// kernels). One engine serves one HIP stream; it owns the descriptor tables,
// the tile arrays, the entry buffer and the staging of host points, growing
// them when a batch needs more.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <array>

#include "engine.hpp"

namespace tsdf {

namespace {

constexpr size_t kAlign = 256;
size_t up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

// Fixed layout of the descriptor tables for given capacities.
struct DescLayout {
    size_t hdr, maps, scans, block_scan, seq_sensor, total;
    static DescLayout of(size_t cap_maps, size_t cap_scans, size_t cap_blocks)
    {
        DescLayout L;
        L.hdr = 0;
        L.maps = up(sizeof(BatchHdr));
        L.scans = up(L.maps + cap_maps * sizeof(MapDev));
        L.block_scan = up(L.scans + cap_scans * sizeof(ScanDev));
        L.seq_sensor = up(L.block_scan + cap_blocks * sizeof(uint32_t));
        L.total = up(L.seq_sensor + cap_maps * kMaxSeq * sizeof(int4));
        return L;
    }
};

int64_t floor_mod64(int64_t a, int64_t b)
{
    int64_t r = a % b;
    return r < 0 ? r + b : r;
}

int32_t ntiles_axis(int32_t n, int32_t lt) { return (n + (1 << lt) - 1) >> lt; }

std::atomic<bool> g_graphs{true};

uint32_t pow2_at_least(uint32_t v)
{
    uint32_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

}  // namespace

void Engine::set_graphs(bool on) { g_graphs.store(on); }
bool Engine::graphs() { return g_graphs.load(); }

hipError_t Engine::launch(const BatchArrays &B, const LaunchCaps &caps)
{
    for (const GraphEntry &g : graphs_)
        if (memcmp(&g.B, &B, sizeof(B)) == 0 && memcmp(&g.caps, &caps, sizeof(caps)) == 0)
            return hipGraphLaunch(g.exec, stream_);
    // capture this shape: the kernels read every batch size from the device
    // header, so the graph serves every later batch with these buffers and
    // grid sizes
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipError_t e = hipStreamBeginCapture(stream_, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t le = launch_batch(B, caps, stream_, nullptr, nullptr, nullptr);
    e = hipStreamEndCapture(stream_, &graph);
    if (le != hipSuccess) return le;
    if (e != hipSuccess) return e;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return e;
    if (graphs_.size() >= 8) {
        (void)hipGraphExecDestroy(graphs_.front().exec);
        graphs_.erase(graphs_.begin());
    }
    graphs_.push_back(GraphEntry{B, caps, exec});
    return hipGraphLaunch(exec, stream_);
}

size_t single_map_array_bytes(const int32_t dims[3])
{
    // finest allowed tiles: edges 4, 4, 8
    const size_t g = (size_t)ntiles_axis(dims[0], 2) * ntiles_axis(dims[1], 2) * ntiles_axis(dims[2], 3);
    return up(5 * g * sizeof(uint32_t)) + up(g * sizeof(uint4));
}

Engine::Engine(hipStream_t stream, int device) : stream_(stream), device_(device)
{
    int cu = 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cu > 0)
        num_cu_ = cu;
    for (int k = 0; k < 2; ++k) {
        if (hipEventCreateWithFlags(&desc_ev_[k], hipEventDisableTiming) != hipSuccess) poisoned_ = true;
        if (hipEventCreateWithFlags(&desc_used_[k], hipEventDisableTiming) != hipSuccess) poisoned_ = true;
        if (hipEventCreateWithFlags(&pts_ev_[k], hipEventDisableTiming) != hipSuccess) poisoned_ = true;
    }
    if (hipEventCreateWithFlags(&order_ev_, hipEventDisableTiming) != hipSuccess) poisoned_ = true;
    if (hipMalloc(&ctl_, sizeof(BatchCtl)) != hipSuccess) poisoned_ = true;
    else if (launch_fill_u32((uint32_t *)ctl_, sizeof(BatchCtl) / 4, 0u, stream_) != hipSuccess) poisoned_ = true;
}

Engine::~Engine()
{
    (void)hipStreamSynchronize(stream_);
    if (copy_stream_) {
        (void)hipStreamSynchronize(copy_stream_);
        (void)hipStreamDestroy(copy_stream_);
    }
    for (int k = 0; k < 2; ++k) {
        if (desc_host_[k]) (void)hipHostFree(desc_host_[k]);
        if (pts_host_[k]) (void)hipHostFree(pts_host_[k]);
        if (desc_ev_[k]) (void)hipEventDestroy(desc_ev_[k]);
        if (desc_used_[k]) (void)hipEventDestroy(desc_used_[k]);
        if (desc_dev_[k]) (void)hipFree(desc_dev_[k]);
        desc_dev_[k] = nullptr;
        if (pts_ev_[k]) (void)hipEventDestroy(pts_ev_[k]);
    }
    if (order_ev_) (void)hipEventDestroy(order_ev_);
    for (GraphEntry &g : graphs_) (void)hipGraphExecDestroy(g.exec);
    for (void *p : {inline_dev_, entries_, valid_, stats_, ctl_, pts_dev_})
        if (p) (void)hipFree(p);
    if (arr_ && !arr_external_) (void)hipFree(arr_);
    for (auto &t : prof_ev_)
        for (hipEvent_t e : t) ev_pool_.push_back(e);
    for (hipEvent_t e : ev_pool_) (void)hipEventDestroy(e);
}

tsdf_status Engine::fail()
{
    poisoned_ = true;
    return TSDF_EDEVICE;
}

#define ECHK(call)                              \
    do {                                        \
        if ((call) != hipSuccess) return fail(); \
    } while (0)

void Engine::adopt_arrays(void *p, size_t bytes)
{
    arr_ = p;
    arr_bytes_ = bytes;
    arr_external_ = true;
}

tsdf_status Engine::grow(void **p, size_t *cap, size_t need, bool zero, bool host_pinned)
{
    if (need <= *cap) return TSDF_OK;
    size_t ncap = std::max(need, *cap + *cap / 2);
    ncap = up(ncap);
    ECHK(hipStreamSynchronize(stream_));
    if (copy_stream_) ECHK(hipStreamSynchronize(copy_stream_));
    if (*p) {
        if (host_pinned) ECHK(hipHostFree(*p));
        else ECHK(hipFree(*p));
    }
    *p = nullptr;
    *cap = 0;
    if (host_pinned) {
        if (hipHostMalloc(p, ncap, hipHostMallocDefault) != hipSuccess) return TSDF_ENOMEM;
    } else {
        if (hipMalloc(p, ncap) != hipSuccess) return TSDF_ENOMEM;
        if (zero) ECHK(launch_fill_u32((uint32_t *)*p, (int64_t)(ncap / 4), 0u, stream_));
    }
    *cap = ncap;
    return TSDF_OK;
}

void Engine::profile(bool on)
{
    (void)hipStreamSynchronize(stream_);
    for (auto &t : prof_ev_)
        for (hipEvent_t e : t) ev_pool_.push_back(e);
    prof_ev_.clear();
    prof_on_ = on;
}

tsdf_status Engine::profile_read(int stage, double *ms, int64_t *n)
{
    ECHK(hipStreamSynchronize(stream_));
    double tot = 0.0;
    for (auto &t : prof_ev_) {
        float x = 0.f;
        const int a = stage == 3 ? 0 : stage, b = stage == 3 ? 3 : stage + 1;
        ECHK(hipEventElapsedTime(&x, t[a], t[b]));
        tot += x;
    }
    *ms = tot;
    *n = (int64_t)prof_ev_.size();
    return TSDF_OK;
}

tsdf_status Engine::run(const std::vector<MapRef> &maps, const std::vector<ScanRef> &scans, const LaunchShape &shape,
                        tsdf_scan_stats *stats)
{
    if (poisoned_) return TSDF_EDEVICE;
    if (!launch_blocks_ok(shape.bin_block, shape.tile_block)) return TSDF_EINVAL;
    // every argument first: nothing is touched for an invalid batch
    for (const ScanRef &s : scans) {
        if (s.map < 0 || (size_t)s.map >= maps.size() || !s.pose || s.n < 0 || s.n > 0xffffffffLL ||
            (s.n > 0 && !s.xyz))
            return TSDF_EINVAL;
        for (int k = 0; k < 12; ++k)
            if (!isfinite(s.pose[k])) return TSDF_EINVAL;
        const MapRef &m = maps[s.map];
        for (int a = 0; a < 3; ++a) {
            const double r = nearbyint(s.pose[4 * a + 3] * m.scale);
            if (!(fabs(r) < 1073741824.0)) return TSDF_EINVAL;
        }
    }
    // chunks in which no map has more than kMaxSeq scans
    size_t b = 0;
    while (b < scans.size()) {
        std::vector<int32_t> per(maps.size(), 0);
        size_t e = b;
        while (e < scans.size() && per[scans[e].map] < kMaxSeq) per[scans[e++].map]++;
        tsdf_status st = run_chunk(maps, scans, b, e, shape, stats ? stats + b : nullptr);
        if (st != TSDF_OK) return st;
        b = e;
    }
    return TSDF_OK;
}

tsdf_status Engine::run_chunk(const std::vector<MapRef> &maps, const std::vector<ScanRef> &scans, size_t b,
                              size_t e, const LaunchShape &shape, tsdf_scan_stats *stats)
{
    const int32_t *lt = shape.lt;
    const uint32_t bb = (uint32_t)shape.bin_block;
    const size_t nscans = e - b;
    // map slots in order of first appearance, and each scan's sequence slot
    std::vector<int32_t> slot_of(maps.size(), -1), seq(nscans), used;
    std::vector<int32_t> nseq;
    for (size_t k = 0; k < nscans; ++k) {
        const int32_t m = scans[b + k].map;
        if (slot_of[m] < 0) {
            slot_of[m] = (int32_t)used.size();
            used.push_back(m);
            nseq.push_back(0);
        }
        seq[k] = nseq[slot_of[m]]++;
    }
    const int32_t nmaps = (int32_t)used.size();
    int32_t S = 1;
    for (int32_t v : nseq) S = std::max(S, v);
    uint64_t gtiles = 0;
    int32_t tau_max = 1;
    std::vector<MapDev> md(nmaps);
    for (int32_t j = 0; j < nmaps; ++j) {
        const MapRef &m = maps[used[j]];
        MapDev &d = md[j];
        d.sdf = m.sdf;
        d.w = m.w;
        d.ntot = 1;
        for (int a = 0; a < 3; ++a) {
            d.dims[a] = m.dims[a];
            d.origin[a] = m.origin[a];
            d.ring0[a] = (int32_t)floor_mod64(m.origin[a], m.dims[a]);
            d.nt[a] = ntiles_axis(m.dims[a], lt[a]);
            d.ntot *= (uint32_t)d.nt[a];
        }
        d.tile_base = (uint32_t)gtiles;
        gtiles += d.ntot;
        d.tau = m.tau;
        d.w_max = m.w_max;
        d.vec_ok = (m.dims[2] % 8 == 0) && (d.ring0[2] % 8 == 0) && ((uintptr_t)m.sdf % 16 == 0) &&
                   ((uintptr_t)m.w % 16 == 0);
        d.pad = 0;
        tau_max = std::max(tau_max, m.tau);
    }
    const uint64_t C = (uint64_t)S * gtiles;
    if (C >= ((uint64_t)1 << 31)) return TSDF_ERANGE;
    // binning blocks, points, entries
    uint64_t nblocks = 0, npoints = 0, nhost = 0;
    std::vector<uint32_t> block0(nscans);
    for (size_t k = 0; k < nscans; ++k) {
        const ScanRef &s = scans[b + k];
        block0[k] = (uint32_t)nblocks;
        nblocks += (uint64_t)((s.n + bb - 1) / bb);
        npoints += (uint64_t)s.n;
        if (s.host) nhost += (uint64_t)s.n;
    }
    const uint64_t need_entries = npoints * (uint64_t)max_tiles_per_ray(tau_max, lt) + 1024;
    if (need_entries >= ((uint64_t)1 << 32) || nblocks >= ((uint64_t)1 << 31)) return TSDF_ERANGE;

    // capacities (growing waits for the stream)
    const size_t cap_maps = std::max<size_t>(nmaps, 1), cap_scans = std::max<size_t>(nscans, 1),
                 cap_blocks = std::max<size_t>(nblocks, 1);
    const DescLayout L = DescLayout::of(cap_maps, cap_scans, cap_blocks);
    tsdf_status st;
    // a batch of one scan hands its descriptors to the first kernel, which
    // stores them in a table of their own: no copy and no graph (the
    // arguments change per call); larger batches copy the tables first
    const bool one = nscans == 1 && nmaps == 1;
    if (one) {
        if ((st = grow(&inline_dev_, &inline_cap_, L.total, false)) != TSDF_OK) return st;
    } else if ((st = grow(&desc_dev_[desc_cur_], &desc_cap_[desc_cur_], L.total, false)) != TSDF_OK) {
        return st;
    }
    {
        // tile arrays: counts | offsets | cursor | tile_vis | tile_upd, then
        // the busy-tile list; counts and records are zero between batches,
        // so a new layout starts from zeroed memory
        const size_t need_c = std::max<size_t>(C, 1), need_g = std::max<size_t>(gtiles, 1);
        if (need_c > c_cap_ || need_g > g_cap_) {
            size_t nc = need_c, ng = need_g;
            if (!arr_external_) {
                nc = std::max(need_c, c_cap_ + c_cap_ / 2);
                ng = std::max(need_g, g_cap_ + g_cap_ / 2);
            }
            const size_t bytes = up(5 * nc * sizeof(uint32_t)) + up(ng * sizeof(uint4));
            if (arr_external_) {
                if (bytes > arr_bytes_) return TSDF_ERANGE;
                ECHK(hipStreamSynchronize(stream_));
            } else if ((st = grow(&arr_, &arr_bytes_, bytes, false)) != TSDF_OK) {
                return st;
            }
            ECHK(launch_fill_u32((uint32_t *)arr_, (int64_t)(bytes / 4), 0u, stream_));
            c_cap_ = nc;
            g_cap_ = ng;
        }
    }
    if ((st = grow(&entries_, &entries_cap_, need_entries * 2 * sizeof(uint4), false)) != TSDF_OK) return st;
    if ((st = grow(&valid_, &valid_cap_, cap_blocks * sizeof(uint32_t), false)) != TSDF_OK) return st;
    if ((st = grow(&stats_, &stats_cap_, cap_scans * 4 * sizeof(uint32_t), false)) != TSDF_OK) return st;

    // host points: pinned staging, one copy to the device
    std::vector<const float *> xyz(nscans);
    if (nhost > 0) {
        const size_t bytes = nhost * 3 * sizeof(float);
        if ((st = grow(&pts_dev_, &pts_dev_cap_, bytes, false)) != TSDF_OK) return st;
        const int k = pts_cur_;
        if (pts_ev_live_[k]) ECHK(hipEventSynchronize(pts_ev_[k]));
        pts_ev_live_[k] = false;
        if ((st = grow(&pts_host_[k], &pts_host_cap_[k], bytes, false, true)) != TSDF_OK) return st;
        size_t off = 0;
        for (size_t j = 0; j < nscans; ++j) {
            const ScanRef &s = scans[b + j];
            if (!s.host) {
                xyz[j] = s.xyz;
                continue;
            }
            memcpy((char *)pts_host_[k] + off * 12, s.xyz, (size_t)s.n * 12);
            xyz[j] = (const float *)((char *)pts_dev_ + off * 12);
            off += (size_t)s.n;
        }
        ECHK(hipMemcpyAsync(pts_dev_, pts_host_[k], bytes, hipMemcpyHostToDevice, stream_));
        ECHK(hipEventRecord(pts_ev_[k], stream_));
        pts_ev_live_[k] = true;
        pts_cur_ ^= 1;
    } else {
        for (size_t j = 0; j < nscans; ++j) xyz[j] = scans[b + j].xyz;
    }

    // descriptor tables
    const int dk = desc_cur_;
    if (desc_ev_live_[dk]) ECHK(hipEventSynchronize(desc_ev_[dk]));
    desc_ev_live_[dk] = false;
    if ((st = grow(&desc_host_[dk], &desc_host_cap_[dk], L.total, false, true)) != TSDF_OK) return st;
    char *h = (char *)desc_host_[dk];
    BatchHdr *hdr = (BatchHdr *)(h + L.hdr);
    for (int a = 0; a < 3; ++a) hdr->lt[a] = lt[a];
    hdr->S = S;
    hdr->nmaps = nmaps;
    hdr->nscans = (int32_t)nscans;
    hdr->gtiles = (uint32_t)gtiles;
    hdr->nblocks = (uint32_t)nblocks;
    hdr->cap = (uint32_t)std::min<size_t>(entries_cap_ / (2 * sizeof(uint4)), 0xffffffffu);
    hdr->want_stats = stats ? 1u : 0u;
    hdr->bin_block = bb;
    hdr->pad = 0;
    memcpy(h + L.maps, md.data(), nmaps * sizeof(MapDev));
    ScanDev *sd = (ScanDev *)(h + L.scans);
    uint32_t *bs = (uint32_t *)(h + L.block_scan);
    int4 *ss = (int4 *)(h + L.seq_sensor);
    for (size_t j = 0; j < (size_t)nmaps * S; ++j) ss[j] = make_int4(0, 0, 0, 0);
    for (size_t k = 0; k < nscans; ++k) {
        const ScanRef &s = scans[b + k];
        const MapRef &m = maps[s.map];
        ScanDev &d = sd[k];
        for (int q = 0; q < 12; ++q) d.rp.M[q] = s.pose[q];
        d.rp.scale = m.scale;
        for (int a = 0; a < 3; ++a) d.rp.o[a] = (int32_t)nearbyint(s.pose[4 * a + 3] * m.scale);
        d.rp.tau = m.tau;
        d.xyz = xyz[k];
        d.n = s.n;
        d.map = slot_of[s.map];
        d.seq = seq[k];
        d.block0 = block0[k];
        d.pad = 0;
        const uint32_t nb = (uint32_t)((s.n + bb - 1) / bb);
        for (uint32_t q = 0; q < nb; ++q) bs[block0[k] + q] = (uint32_t)k;
        ss[d.map * S + d.seq] = make_int4(d.rp.o[0], d.rp.o[1], d.rp.o[2], d.rp.tau);
    }
    LaunchCaps caps;
    caps.blocks = (uint32_t)nblocks;
    caps.gtiles = (uint32_t)gtiles;
    caps.scans = (uint32_t)nscans;
    caps.bin_block = bb;
    caps.tile_block = (uint32_t)shape.tile_block;
    caps.stats = stats ? 1u : 0u;
    {
        // LDS of a tile workgroup: G key buffers (8 bytes per voxel) and the
        // cached tile (4 bytes per voxel); G as large as ~32 KB per 256
        // threads allows, so that the workgroups a CU holds (the kernel's
        // register budget allows five waves per SIMD: five workgroups of
        // 256, two of 512) fit its 160 KB; the persistent grid fills the CUs
        const size_t tvox = (size_t)1 << (lt[0] + lt[1] + lt[2]);
        const int64_t budget = (int64_t)(32 * 1024) * (shape.tile_block / 256);
        const int64_t gfit = (budget / (int64_t)tvox - 4) / 8;
        const int32_t G = (int32_t)std::max<int64_t>(1, std::min<int64_t>({gfit, 8, (int64_t)S}));
        hdr->G = G;
        caps.tile_lds = (uint32_t)((8 * (size_t)G + 4) * tvox);
        const int by_waves = 20 / (shape.tile_block / 64);  // five waves per SIMD, four SIMDs
        const int per_cu =
            (int)std::max<size_t>(1, std::min<size_t>((size_t)by_waves, (160 * 1024) / caps.tile_lds));
        caps.tile_grid = shape.tile_grid > 0 ? shape.tile_grid : num_cu_ * per_cu;
    }
    InlineDesc I;
    memset(&I, 0, sizeof(I));
    if (one) {
        I.hdr = *hdr;
        I.map = md[0];
        I.scan = sd[0];
        I.on = 1;
    } else {
        // on the copy stream, after the kernels that last read this device
        // copy: the copy runs while the previous batch's kernels do, and the
        // batch's kernels wait only for its end. The stream is made for the
        // first batch of several scans (default priority, like every stream
        // of the library): engines of one-scan calls hold no extra stream.
        if (!copy_stream_) {
            if (hipStreamCreateWithFlags(&copy_stream_, hipStreamNonBlocking) != hipSuccess) {
                copy_stream_ = nullptr;
                return fail();
            }
        }
        if (desc_used_live_[dk]) ECHK(hipStreamWaitEvent(copy_stream_, desc_used_[dk], 0));
        ECHK(hipMemcpyAsync(desc_dev_[dk], h, L.total, hipMemcpyHostToDevice, copy_stream_));
        ECHK(hipEventRecord(desc_ev_[dk], copy_stream_));
        desc_ev_live_[dk] = true;
        ECHK(hipStreamWaitEvent(stream_, desc_ev_[dk], 0));
    }

    BatchArrays B;
    char *dd = (char *)(one ? inline_dev_ : desc_dev_[dk]);
    B.hdr = (BatchHdr *)(dd + L.hdr);
    B.maps = (MapDev *)(dd + L.maps);
    B.scans = (ScanDev *)(dd + L.scans);
    B.block_scan = (uint32_t *)(dd + L.block_scan);
    B.seq_sensor = (int4 *)(dd + L.seq_sensor);
    uint32_t *arr = (uint32_t *)arr_;
    B.counts = arr;
    B.offsets = arr + c_cap_;
    B.cursor = arr + 2 * c_cap_;
    B.tile_vis = arr + 3 * c_cap_;
    B.tile_upd = arr + 4 * c_cap_;
    B.jobs = (uint4 *)((char *)arr_ + up(5 * c_cap_ * 4));
    B.entries = (uint4 *)entries_;
    B.entries2 = B.entries + entries_cap_ / (2 * sizeof(uint4));
    B.valid_part = (uint32_t *)valid_;
    B.scan_stats = (uint32_t *)stats_;
    B.ctl = (BatchCtl *)ctl_;

    // order after earlier work on each map's own stream
    for (int32_t j = 0; j < nmaps; ++j) {
        const MapRef &m = maps[used[j]];
        if (m.stream != stream_) {
            ECHK(hipEventRecord(order_ev_, m.stream));
            ECHK(hipStreamWaitEvent(stream_, order_ev_, 0));
        }
    }
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    if (prof_on_) {
        for (int k = 0; k < 4; ++k) {
            if (!ev_pool_.empty()) {
                ev[k] = ev_pool_.back();
                ev_pool_.pop_back();
            } else if (hipEventCreate(&ev[k]) != hipSuccess) {
                return fail();
            }
        }
        prof_ev_.push_back({ev[0], ev[1], ev[2], ev[3]});
    }
    if (one || prof_on_ || !graphs()) {
        ECHK(launch_batch(B, caps, stream_, ev[0], ev[1], ev[2], one ? &I : nullptr));
        if (ev[3]) ECHK(hipEventRecord(ev[3], stream_));
    } else {
        // grid sizes rounded up to powers of two, so that few shapes exist
        LaunchCaps gc = caps;
        gc.blocks = pow2_at_least(std::max<uint32_t>(caps.blocks, 1));
        gc.gtiles = pow2_at_least(std::max<uint32_t>(caps.gtiles, 1));
        gc.scans = pow2_at_least(std::max<uint32_t>(caps.scans, 1));
        ECHK(launch(B, gc));
    }
    if (!one) {
        // the next copy into this device table waits for these kernels
        ECHK(hipEventRecord(desc_used_[dk], stream_));
        desc_used_live_[dk] = true;
        desc_cur_ ^= 1;
    }
    // later work on each map's stream waits for this batch
    for (int32_t j = 0; j < nmaps; ++j) {
        const MapRef &m = maps[used[j]];
        if (m.stream != stream_) {
            ECHK(hipEventRecord(order_ev_, stream_));
            ECHK(hipStreamWaitEvent(m.stream, order_ev_, 0));
        }
    }
    if (stats) {
        std::vector<uint32_t> host(nscans * 4);
        ECHK(hipMemcpyAsync(host.data(), stats_, nscans * 4 * sizeof(uint32_t), hipMemcpyDeviceToHost, stream_));
        ECHK(hipStreamSynchronize(stream_));
        for (size_t k = 0; k < nscans; ++k) {
            if (host[4 * k + 3]) return fail();  // entry buffer overflow: cannot happen by its sizing
            stats[k].points_in = scans[b + k].n;
            stats[k].points_valid = host[4 * k + 1];
            stats[k].visits = host[4 * k + 2];
            stats[k].voxels_updated = host[4 * k + 0];
        }
    }
    return TSDF_OK;
}

}  // namespace tsdf
