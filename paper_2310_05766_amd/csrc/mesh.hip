// Surface extraction for inspection: the zero level set of the resident
// window in a box, by marching tetrahedra (each cube of 8 observed voxel
// centres cut into the 6 tetrahedra around its 0-7 diagonal; one or two
// triangles per tetrahedron with a sign change; edge points at
// t = s_a / (s_a - s_b) in float64). Two passes give a deterministic order,
// cube by cube (x, then y, then z): a count per cube summed per block, and,
// after an exclusive scan of the block sums on the host, an emit pass that
// places each cube's triangles by a block-level scan of the counts.
#include "internal.hpp"

namespace tsdf {

namespace {

constexpr int kMeshBlock = 256;

__constant__ int8_t kTet[6][4] = {{0, 1, 3, 7}, {0, 3, 2, 7}, {0, 2, 6, 7}, {0, 6, 4, 7}, {0, 4, 5, 7}, {0, 5, 1, 7}};

__device__ __forceinline__ void edge_point(const int64_t g[3], int a, int b, const int32_t s[8], double vs, float *p)
{
    const double t = (double)s[a] / ((double)s[a] - (double)s[b]);
    for (int k = 0; k < 3; ++k) {
        const double ga = (double)(g[k] + ((a >> k) & 1)) + 0.5;
        const double gb = (double)(g[k] + ((b >> k) & 1)) + 0.5;
        p[k] = (float)((ga + t * (gb - ga)) * vs);
    }
}

// Triangles of cube c (0 if it is not fully observed); written to out when
// out is not null.
__device__ int cube_triangles(const MeshArgs &A, int64_t c, float *out)
{
    const int64_t cz = c % A.n[2], cxy = c / A.n[2];
    const int64_t g[3] = {A.lo[0] + cxy / A.n[1], A.lo[1] + cxy % A.n[1], A.lo[2] + cz};
    int32_t s[8];
    for (int k = 0; k < 8; ++k) {
        int64_t sl = 0;
        for (int a = 0; a < 3; ++a) {
            int64_t v = (g[a] + ((k >> a) & 1)) % A.dims[a];
            v += v < 0 ? A.dims[a] : 0;
            sl = sl * A.dims[a] + v;
        }
        if (A.w[sl] <= 0) return 0;
        s[k] = A.sdf[sl];
    }
    int n = 0;
    for (int t = 0; t < 6; ++t) {
        int v[4], in[4], nin = 0;
        for (int k = 0; k < 4; ++k) {
            v[k] = kTet[t][k];
            in[k] = s[v[k]] < 0;
            nin += in[k];
        }
        if (nin == 0 || nin == 4) continue;
        if (nin == 1 || nin == 3) {
            // the lone vertex: inside when one is inside, outside when three are
            int lone = 0;
            for (int k = 0; k < 4; ++k)
                if (in[k] == (nin == 1)) lone = k;
            if (out) {
                int e = 0;
                for (int k = 0; k < 4; ++k)
                    if (k != lone) edge_point(g, v[lone], v[k], s, A.vs, out + 9 * n + 3 * e++);
            }
            n += 1;
        } else {
            int i0 = -1, i1 = -1, o0 = -1, o1 = -1;
            for (int k = 0; k < 4; ++k) {
                if (in[k]) {
                    if (i0 < 0) i0 = k;
                    else i1 = k;
                } else {
                    if (o0 < 0) o0 = k;
                    else o1 = k;
                }
            }
            if (out) {
                // the quad i0o0, i0o1, i1o1, i1o0 as triangles (0 1 2), (0 2 3)
                float q[4][3];
                edge_point(g, v[i0], v[o0], s, A.vs, q[0]);
                edge_point(g, v[i0], v[o1], s, A.vs, q[1]);
                edge_point(g, v[i1], v[o1], s, A.vs, q[2]);
                edge_point(g, v[i1], v[o0], s, A.vs, q[3]);
                const int order[6] = {0, 1, 2, 0, 2, 3};
                for (int k = 0; k < 6; ++k)
                    for (int a = 0; a < 3; ++a) out[9 * n + 3 * k + a] = q[order[k]][a];
            }
            n += 2;
        }
    }
    return n;
}

__global__ __launch_bounds__(kMeshBlock) void k_mesh_count(MeshArgs A, uint32_t *block_tris)
{
    __shared__ uint32_t s_sum;
    if (threadIdx.x == 0) s_sum = 0;
    __syncthreads();
    const int64_t c = (int64_t)blockIdx.x * kMeshBlock + threadIdx.x;
    const int n = c < A.ncubes ? cube_triangles(A, c, nullptr) : 0;
    if (n) atomicAdd(&s_sum, (uint32_t)n);
    __syncthreads();
    if (threadIdx.x == 0) block_tris[blockIdx.x] = s_sum;
}

__global__ __launch_bounds__(kMeshBlock) void k_mesh_emit(MeshArgs A, const uint64_t *block_base, float *out)
{
    __shared__ uint32_t s_scan[kMeshBlock];
    const int64_t c = (int64_t)blockIdx.x * kMeshBlock + threadIdx.x;
    const int n = c < A.ncubes ? cube_triangles(A, c, nullptr) : 0;
    s_scan[threadIdx.x] = (uint32_t)n;
    __syncthreads();
    // inclusive scan (Hillis-Steele) of the block's counts
    for (int off = 1; off < kMeshBlock; off <<= 1) {
        const uint32_t add = threadIdx.x >= (uint32_t)off ? s_scan[threadIdx.x - off] : 0u;
        __syncthreads();
        s_scan[threadIdx.x] += add;
        __syncthreads();
    }
    if (n) cube_triangles(A, c, out + 9 * (block_base[blockIdx.x] + s_scan[threadIdx.x] - (uint32_t)n));
}

}  // namespace

hipError_t launch_mesh_count(const MeshArgs &A, uint32_t *block_tris, hipStream_t stream)
{
    const int64_t blocks = (A.ncubes + kMeshBlock - 1) / kMeshBlock;
    if (blocks > 0) hipLaunchKernelGGL(k_mesh_count, dim3((uint32_t)blocks), dim3(kMeshBlock), 0, stream, A, block_tris);
    return hipGetLastError();
}

hipError_t launch_mesh_emit(const MeshArgs &A, const uint64_t *block_base, float *out, hipStream_t stream)
{
    const int64_t blocks = (A.ncubes + kMeshBlock - 1) / kMeshBlock;
    if (blocks > 0)
        hipLaunchKernelGGL(k_mesh_emit, dim3((uint32_t)blocks), dim3(kMeshBlock), 0, stream, A, block_base, out);
    return hipGetLastError();
}

int64_t mesh_blocks(int64_t ncubes) { return (ncubes + kMeshBlock - 1) / kMeshBlock; }

}  // namespace tsdf
