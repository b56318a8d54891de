// Streaming copies between the resident window and dense staging buffers:
// the device side of the local-map shift (FeatSense, arXiv 2310.05766,
// Sec. I: what leaves the local map is written out, what re-enters it is
// loaded) and of readback. A window voxel g lives at slot floor_mod(g, dims),
// so a shift never moves voxels that stay resident; only the leaving and
// entering boxes are copied.
//
// Each box is a global voxel box [lo, lo + ext) staged as dense [x][y][z].
// One block row (blockIdx.y) per box; threads run along z, the contiguous
// axis of both layouts, so loads and stores are coalesced runs.
#include "internal.hpp"

namespace tsdf {

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ int32_t fmod_pos(int32_t a, int32_t n)
{
    int32_t r = a % n;
    return r < 0 ? r + n : r;
}

__global__ __launch_bounds__(kBlock) void k_pack(const BoxXfer *__restrict__ boxes, int16_t *__restrict__ sdf,
                                                 int16_t *__restrict__ w, int32_t nx, int32_t ny, int32_t nz,
                                                 int16_t *__restrict__ stage_sdf, int16_t *__restrict__ stage_w,
                                                 int clear)
{
    const BoxXfer b = boxes[blockIdx.y];
    const int64_t total = (int64_t)b.ext[0] * b.ext[1] * b.ext[2];
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < total; j += (int64_t)gridDim.x * kBlock) {
        const int32_t z = (int32_t)(j % b.ext[2]);
        const int64_t xy = j / b.ext[2];
        const int32_t y = (int32_t)(xy % b.ext[1]);
        const int32_t x = (int32_t)(xy / b.ext[1]);
        const int64_t slot = ((int64_t)fmod_pos(b.lo[0] + x, nx) * ny + fmod_pos(b.lo[1] + y, ny)) * nz +
                             fmod_pos(b.lo[2] + z, nz);
        stage_sdf[b.off + j] = sdf[slot];
        stage_w[b.off + j] = w[slot];
        if (clear) {
            sdf[slot] = 0;
            w[slot] = 0;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_unpack(const BoxXfer *__restrict__ boxes, int16_t *__restrict__ sdf,
                                                   int16_t *__restrict__ w, int32_t nx, int32_t ny, int32_t nz,
                                                   const int16_t *__restrict__ stage_sdf,
                                                   const int16_t *__restrict__ stage_w)
{
    const BoxXfer b = boxes[blockIdx.y];
    const int64_t total = (int64_t)b.ext[0] * b.ext[1] * b.ext[2];
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < total; j += (int64_t)gridDim.x * kBlock) {
        const int32_t z = (int32_t)(j % b.ext[2]);
        const int64_t xy = j / b.ext[2];
        const int32_t y = (int32_t)(xy % b.ext[1]);
        const int32_t x = (int32_t)(xy / b.ext[1]);
        const int64_t slot = ((int64_t)fmod_pos(b.lo[0] + x, nx) * ny + fmod_pos(b.lo[1] + y, ny)) * nz +
                             fmod_pos(b.lo[2] + z, nz);
        sdf[slot] = stage_sdf ? stage_sdf[b.off + j] : (int16_t)0;
        w[slot] = stage_w ? stage_w[b.off + j] : (int16_t)0;
    }
}

// Whole 64^3 chunks of a window whose dims are multiples of 64, so that a
// chunk's voxels occupy 64 contiguous slots along z in every (x, y) row of
// the window. Chunk j (global voxel origin c0, a multiple of 64 on each axis)
// is staged at stage + j * 2 * kChunkVox as its sdf block then its w block,
// both [x][y][z] in chunk order: the host store's own layout, so a chunk
// crosses the host link as one contiguous copy. Each thread moves 8 voxels
// (16 bytes) of each array per step. k_pack_chunks also clears the window
// voxels and sets flag[j] when any voxel of chunk j is non-zero.
constexpr int kChunkUnits = kChunk * kChunk * kChunk / 8;  // 16-byte units per array

__device__ __forceinline__ int64_t chunk_row_slot(const BoxXfer &b, int32_t u, int32_t nx, int32_t ny, int32_t nz)
{
    const int32_t x = u >> 9, y = (u >> 3) & 63, zq = u & 7;
    // slots of the chunk's rows: floor_mod(c0 + i, n) = floor_mod(c0, n) + i (n a multiple of 64)
    const int32_t sx = fmod_pos(b.lo[0], nx) + x, sy = fmod_pos(b.lo[1], ny) + y;
    const int32_t sz = fmod_pos(b.lo[2], nz) + 8 * zq;
    return ((int64_t)sx * ny + sy) * nz + sz;
}

__global__ __launch_bounds__(kBlock) void k_pack_chunks(const BoxXfer *__restrict__ boxes, int16_t *__restrict__ sdf,
                                                        int16_t *__restrict__ w, int32_t nx, int32_t ny, int32_t nz,
                                                        int16_t *__restrict__ stage, uint32_t *__restrict__ flags)
{
    const BoxXfer b = boxes[blockIdx.y];
    int4 *dst_s = reinterpret_cast<int4 *>(stage + (int64_t)blockIdx.y * 2 * kChunkVox);
    int4 *dst_w = dst_s + kChunkUnits;
    bool any = false;
    for (int32_t u = blockIdx.x * kBlock + threadIdx.x; u < kChunkUnits; u += gridDim.x * kBlock) {
        const int64_t slot = chunk_row_slot(b, u, nx, ny, nz);
        int4 *ps = reinterpret_cast<int4 *>(sdf + slot);
        int4 *pw = reinterpret_cast<int4 *>(w + slot);
        const int4 vs = *ps, vw = *pw;
        dst_s[u] = vs;
        dst_w[u] = vw;
        *ps = make_int4(0, 0, 0, 0);
        *pw = make_int4(0, 0, 0, 0);
        any |= (vs.x | vs.y | vs.z | vs.w | vw.x | vw.y | vw.z | vw.w) != 0;
    }
    if (__any(any) && (threadIdx.x & 63u) == 0) atomicOr(&flags[blockIdx.y], 1u);
}

__global__ __launch_bounds__(kBlock) void k_unpack_chunks(const BoxXfer *__restrict__ boxes, int16_t *__restrict__ sdf,
                                                          int16_t *__restrict__ w, int32_t nx, int32_t ny, int32_t nz,
                                                          const int16_t *__restrict__ stage)
{
    const BoxXfer b = boxes[blockIdx.y];
    const int4 *src_s = reinterpret_cast<const int4 *>(stage + (int64_t)blockIdx.y * 2 * kChunkVox);
    const int4 *src_w = src_s + kChunkUnits;
    for (int32_t u = blockIdx.x * kBlock + threadIdx.x; u < kChunkUnits; u += gridDim.x * kBlock) {
        const int64_t slot = chunk_row_slot(b, u, nx, ny, nz);
        *reinterpret_cast<int4 *>(sdf + slot) = src_s[u];
        *reinterpret_cast<int4 *>(w + slot) = src_w[u];
    }
}

uint32_t grid_x(int64_t max_box_vox)
{
    int64_t blocks = (max_box_vox + kBlock - 1) / kBlock;
    if (blocks > 1024) blocks = 1024;
    if (blocks < 1) blocks = 1;
    return (uint32_t)blocks;
}

}  // namespace

hipError_t launch_pack_boxes(const BoxXfer *boxes_dev, int32_t nboxes, int64_t max_box_vox, int16_t *sdf,
                             int16_t *w, const int32_t dims[3], int16_t *stage_sdf, int16_t *stage_w, bool clear,
                             hipStream_t stream)
{
    if (nboxes <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pack, dim3(grid_x(max_box_vox), (uint32_t)nboxes), dim3(kBlock), 0, stream, boxes_dev, sdf,
                       w, dims[0], dims[1], dims[2], stage_sdf, stage_w, clear ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_pack_chunks(const BoxXfer *chunks_dev, int32_t nchunks, int16_t *sdf, int16_t *w,
                              const int32_t dims[3], int16_t *stage, uint32_t *flags, hipStream_t stream)
{
    if (nchunks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pack_chunks, dim3(32, (uint32_t)nchunks), dim3(kBlock), 0, stream, chunks_dev, sdf, w,
                       dims[0], dims[1], dims[2], stage, flags);
    return hipGetLastError();
}

hipError_t launch_unpack_chunks(const BoxXfer *chunks_dev, int32_t nchunks, int16_t *sdf, int16_t *w,
                                const int32_t dims[3], const int16_t *stage, hipStream_t stream)
{
    if (nchunks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_unpack_chunks, dim3(32, (uint32_t)nchunks), dim3(kBlock), 0, stream, chunks_dev, sdf, w,
                       dims[0], dims[1], dims[2], stage);
    return hipGetLastError();
}

hipError_t launch_unpack_boxes(const BoxXfer *boxes_dev, int32_t nboxes, int64_t max_box_vox, int16_t *sdf,
                               int16_t *w, const int32_t dims[3], const int16_t *stage_sdf,
                               const int16_t *stage_w, hipStream_t stream)
{
    if (nboxes <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_unpack, dim3(grid_x(max_box_vox), (uint32_t)nboxes), dim3(kBlock), 0, stream, boxes_dev,
                       sdf, w, dims[0], dims[1], dims[2], stage_sdf, stage_w);
    return hipGetLastError();
}

}  // namespace tsdf
