// Integration of one scan with every device buffer of the batch engine taken
// from one fixed, file-scope device array instead of allocations: for
// callers that cannot allocate (code under graph capture, tight serving
// loops, harnesses that forbid hipMalloc). The kernels are the batch
// engine's (batch.hip); only where their tables live differs.
//
// The array is per device (each GPU that runs the library holds its own copy
// for the life of the process) and shared by every call on that device: a
// call clears what its kernels need at zero before using it, and calls that
// overlap on one device race.
#include <math.h>

#include <mutex>

#include "map.hpp"

namespace tsdf {

namespace {

// The array's size, the most any call can use: enough for one OS1-128-shaped
// scan (131,072 points, tau of 5 voxels) on a 512 x 512 x 256 window at the
// default tiling (about 47 MiB of entry records and tables).
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;

__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

// Writes the batch header and the one map and scan record from the kernel's
// arguments, and clears the counters, the per-tile counts and the per-tile
// statistics that the engine's kernels expect at zero.
__global__ __launch_bounds__(256) void k_noalloc_setup(BatchArrays B, BatchHdr hdr, MapDev md, ScanDev sd,
                                                      uint32_t gtiles, uint32_t nblocks)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t stride = gridDim.x * blockDim.x;
    if (t == 0) {
        *B.hdr = hdr;
        B.maps[0] = md;
        B.scans[0] = sd;
        B.seq_sensor[0] = make_int4(sd.rp.o[0], sd.rp.o[1], sd.rp.o[2], sd.rp.tau);
    }
    uint32_t *ctl = reinterpret_cast<uint32_t *>(B.ctl);
    for (uint32_t j = t; j < (uint32_t)(sizeof(BatchCtl) / 4); j += stride) ctl[j] = 0;
    for (uint32_t j = t; j < nblocks; j += stride) B.block_scan[j] = 0;
    for (uint32_t j = t; j < gtiles; j += stride) {
        B.counts[j] = 0;
        B.tile_vis[j] = 0;
        B.tile_upd[j] = 0;
    }
    for (uint32_t j = t; j < 4; j += stride) B.scan_stats[j] = 0;
}

int g_cu[kMaxDevices] = {};  // compute units per device

hipError_t noalloc_scratch(int device, void **ptr)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[device]) {
        // the device address of this device's copy of the array (the array's
        // name in host code is only a host-side stand-in)
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_ptr[device] = p;
    }
    *ptr = g_ptr[device];
    return hipSuccess;
}

size_t noalloc_layout(void *base, uint32_t nblocks, uint32_t gtiles, uint32_t cap, BatchArrays *B)
{
    char *p = (char *)base;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *q = p ? p + off : nullptr;
        off = align_up(off + bytes);
        return q;
    };
    BatchArrays A;
    A.ctl = (BatchCtl *)take(sizeof(BatchCtl));
    A.hdr = (BatchHdr *)take(sizeof(BatchHdr));
    A.maps = (MapDev *)take(sizeof(MapDev));
    A.scans = (ScanDev *)take(sizeof(ScanDev));
    A.seq_sensor = (int4 *)take(sizeof(int4));
    A.block_scan = (uint32_t *)take((size_t)nblocks * 4);
    A.counts = (uint32_t *)take((size_t)gtiles * 4);
    A.offsets = (uint32_t *)take((size_t)gtiles * 4);
    A.cursor = (uint32_t *)take((size_t)gtiles * 4);
    A.tile_vis = (uint32_t *)take((size_t)gtiles * 4);
    A.tile_upd = (uint32_t *)take((size_t)gtiles * 4);
    A.jobs = (uint4 *)take((size_t)gtiles * sizeof(uint4));
    A.valid_part = (uint32_t *)take((size_t)nblocks * 4);
    A.scan_stats = (uint32_t *)take(4 * 4);
    A.entries = (uint4 *)take((size_t)cap * sizeof(uint4));
    A.entries2 = (uint4 *)take((size_t)cap * sizeof(uint4));
    if (B) *B = A;
    return off;
}

hipError_t launch_noalloc_setup(const BatchArrays &B, const BatchHdr &hdr, const MapDev &md, const ScanDev &sd,
                                hipStream_t stream)
{
    uint32_t n = hdr.gtiles > hdr.nblocks ? hdr.gtiles : hdr.nblocks;
    n = n > (uint32_t)(sizeof(BatchCtl) / 4) ? n : (uint32_t)(sizeof(BatchCtl) / 4);
    uint32_t blocks = (n + 255) / 256;
    blocks = blocks > 1024 ? 1024 : blocks;
    hipLaunchKernelGGL(k_noalloc_setup, dim3(blocks), dim3(256), 0, stream, B, hdr, md, sd, hdr.gtiles,
                       hdr.nblocks);
    return hipGetLastError();
}

int64_t floor_mod(int64_t a, int64_t b)
{
    const int64_t r = a % b;
    return r < 0 ? r + b : r;
}

}  // namespace

}  // namespace tsdf

using namespace tsdf;

extern "C" tsdf_status tsdf_integrate_scan_noalloc(tsdf_map *m, const float *xyz_dev, int64_t n_points,
                                                   const double world_T_sensor[16], tsdf_scan_stats *stats)
{
    if (!m || !world_T_sensor || n_points < 0 || n_points > 0xffffffffLL || (n_points > 0 && !xyz_dev))
        return TSDF_EINVAL;
    for (int k = 0; k < 12; ++k)
        if (!isfinite(world_T_sensor[k])) return TSDF_EINVAL;
    int32_t o[3];
    for (int a = 0; a < 3; ++a) {
        const double r = nearbyint(world_T_sensor[4 * a + 3] * m->scale);
        if (!(fabs(r) < 1073741824.0)) return TSDF_EINVAL;
        o[a] = (int32_t)r;
    }
    Guard g(m);
    if (!g.ok) return TSDF_EBUSY;
    if (m->poisoned) return TSDF_EDEVICE;
    if (m->interp_dq > 0 || m->carve) return TSDF_EINVAL;  // the key-volume paths allocate their volume

    // the same tables the batch engine builds for a batch of this one scan
    const LaunchShape shape = launch_shape(m, false);
    const int32_t *lt = shape.lt;
    MapDev md;
    md.sdf = m->sdf;
    md.w = m->w;
    md.ntot = 1;
    for (int a = 0; a < 3; ++a) {
        md.dims[a] = m->d.dims[a];
        md.origin[a] = m->d.origin[a];
        md.ring0[a] = (int32_t)floor_mod(m->d.origin[a], m->d.dims[a]);
        md.nt[a] = (m->d.dims[a] + (1 << lt[a]) - 1) >> lt[a];
        md.ntot *= (uint32_t)md.nt[a];
    }
    md.tile_base = 0;
    md.tau = m->d.tau_q10;
    md.w_max = m->d.w_max;
    md.vec_ok = (m->d.dims[2] % 8 == 0) && (md.ring0[2] % 8 == 0) && ((uintptr_t)m->sdf % 16 == 0) &&
                ((uintptr_t)m->w % 16 == 0);
    md.pad = 0;
    ScanDev sd;
    for (int k = 0; k < 12; ++k) sd.rp.M[k] = world_T_sensor[k];
    sd.rp.scale = m->scale;
    for (int a = 0; a < 3; ++a) sd.rp.o[a] = o[a];
    sd.rp.tau = m->d.tau_q10;
    sd.xyz = xyz_dev;
    sd.n = n_points;
    sd.map = 0;
    sd.seq = 0;
    sd.block0 = 0;
    sd.pad = 0;
    const uint64_t nblocks = (uint64_t)((n_points + shape.bin_block - 1) / shape.bin_block);
    const uint64_t cap = (uint64_t)n_points * (uint64_t)max_tiles_per_ray(m->d.tau_q10, lt) + 1024;
    if (cap >= ((uint64_t)1 << 32)) return TSDF_ERANGE;
    const size_t need = noalloc_layout(nullptr, (uint32_t)nblocks, md.ntot, (uint32_t)cap, nullptr);
    if (need > kNoAllocScratchBytes) return TSDF_ERANGE;

    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) return TSDF_EDEVICE;
    if (prev != m->device && hipSetDevice(m->device) != hipSuccess) return TSDF_EDEVICE;
    tsdf_status st = TSDF_OK;
    do {
        void *base = nullptr;
        if (noalloc_scratch(m->device, &base) != hipSuccess) {
            st = TSDF_EDEVICE;
            break;
        }
        if (!g_cu[m->device]) {
            int cu = 0;
            if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, m->device) != hipSuccess ||
                cu <= 0) {
                st = TSDF_EDEVICE;
                break;
            }
            g_cu[m->device] = cu;
        }
        BatchArrays B;
        noalloc_layout(base, (uint32_t)nblocks, md.ntot, (uint32_t)cap, &B);
        BatchHdr hdr;
        for (int a = 0; a < 3; ++a) hdr.lt[a] = lt[a];
        hdr.S = 1;
        hdr.G = 1;
        hdr.nmaps = 1;
        hdr.nscans = 1;
        hdr.gtiles = md.ntot;
        hdr.nblocks = (uint32_t)nblocks;
        hdr.cap = (uint32_t)cap;
        hdr.want_stats = stats ? 1u : 0u;
        hdr.bin_block = (uint32_t)shape.bin_block;
        hdr.pad = 0;
        LaunchCaps caps;
        caps.blocks = (uint32_t)nblocks;
        caps.gtiles = md.ntot;
        caps.scans = 1;
        caps.bin_block = (uint32_t)shape.bin_block;
        caps.tile_block = (uint32_t)shape.tile_block;
        caps.stats = stats ? 1u : 0u;
        const size_t tvox = (size_t)1 << (lt[0] + lt[1] + lt[2]);
        caps.tile_lds = (uint32_t)((8 + 4) * tvox);
        const int by_waves = 20 / (shape.tile_block / 64);
        const int per_cu =
            (int)std::max<size_t>(1, std::min<size_t>((size_t)by_waves, (160 * 1024) / caps.tile_lds));
        caps.tile_grid = m->tile_grid > 0 ? m->tile_grid : g_cu[m->device] * per_cu;
        if (launch_noalloc_setup(B, hdr, md, sd, m->stream) != hipSuccess ||
            launch_batch(B, caps, m->stream, nullptr, nullptr, nullptr) != hipSuccess) {
            st = TSDF_EDEVICE;
            break;
        }
        if (stats) {
            uint32_t host[4] = {0, 0, 0, 0};
            if (hipMemcpyAsync(host, B.scan_stats, sizeof(host), hipMemcpyDeviceToHost, m->stream) != hipSuccess ||
                hipStreamSynchronize(m->stream) != hipSuccess || host[3]) {
                st = TSDF_EDEVICE;  // an entry overflow cannot happen by the sizing above
                break;
            }
            stats->points_in = n_points;
            stats->points_valid = host[1];
            stats->visits = host[2];
            stats->voxels_updated = host[0];
        }
    } while (false);
    if (prev != m->device) (void)hipSetDevice(prev);
    if (st == TSDF_EDEVICE) m->poisoned = true;
    return st;
}
