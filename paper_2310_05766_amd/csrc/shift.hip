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
