// Point-to-TSDF registration (the paper's stated next step; HATSDF, which
// FeatSense's mapping comes from, localises directly in the TSDF): damped
// Gauss-Newton on sum phi(R p + t)^2, phi the map's signed distance in
// metres, trilinear between the 8 voxel centres around the point (all
// resident, observed, not truncated, else the point is left out), with the
// left update R' = exp([theta]x) R, t' = exp([theta]x) t + rho and the
// Jacobian row J = (grad phi, w x grad phi).
//
// The device computes the normal equations: one thread per point, a fixed
// butterfly over each wave, the waves of a block in order, one row of 29
// partial sums per block (H upper triangle, J^T r, sum r^2, points used);
// the host adds the rows in block order, so the sums do not depend on
// scheduling, and solves the 6 x 6 system.
#include "internal.hpp"

namespace tsdf {

namespace {

constexpr int kRegBlock = 256;

// phi (metres), its gradient (per metre) and the world point of point p;
// false when the point is left out.
__device__ __forceinline__ bool reg_point(const RegArgs &A, float px, float py, float pz, double &phi,
                                          double grad[3], double w[3])
{
    if (!isfinite(px) || !isfinite(py) || !isfinite(pz)) return false;
    const double x = px, y = py, z = pz;
    int64_t i0[3];
    double f[3];
    for (int a = 0; a < 3; ++a) {
        w[a] = __fma_rn(A.M[4 * a + 0], x, __fma_rn(A.M[4 * a + 1], y, __fma_rn(A.M[4 * a + 2], z, A.M[4 * a + 3])));
        const double u = w[a] / A.vs - 0.5;  // voxel g's centre is at u = g
        if (!(fabs(u) < 1073741824.0)) return false;
        const double fl = floor(u);
        i0[a] = (int64_t)fl;
        f[a] = u - fl;
    }
    double c[8];
    for (int k = 0; k < 8; ++k) {
        int64_t sl = 0;
        for (int a = 0; a < 3; ++a) {
            const int64_t g = i0[a] + ((k >> a) & 1);
            if (g < A.origin[a] || g >= (int64_t)A.origin[a] + A.dims[a]) return false;
            int64_t v = g % A.dims[a];
            v += v < 0 ? A.dims[a] : 0;
            sl = sl * A.dims[a] + v;
        }
        if (A.w[sl] <= 0) return false;
        const int32_t sq = A.sdf[sl];
        if (sq <= -A.tau || sq >= A.tau) return false;
        c[k] = (double)sq * A.vs / 1024.0;
    }
    // trilinear value and its derivatives along x, y, z (per voxel)
    const double c00 = c[0] + f[0] * (c[1] - c[0]), c10 = c[2] + f[0] * (c[3] - c[2]);
    const double c01 = c[4] + f[0] * (c[5] - c[4]), c11 = c[6] + f[0] * (c[7] - c[6]);
    const double c0 = c00 + f[1] * (c10 - c00), c1 = c01 + f[1] * (c11 - c01);
    phi = c0 + f[2] * (c1 - c0);
    const double dx0 = (c[1] - c[0]) + f[1] * ((c[3] - c[2]) - (c[1] - c[0]));
    const double dx1 = (c[5] - c[4]) + f[1] * ((c[7] - c[6]) - (c[5] - c[4]));
    grad[0] = (dx0 + f[2] * (dx1 - dx0)) / A.vs;
    grad[1] = ((c10 - c00) + f[2] * ((c11 - c01) - (c10 - c00))) / A.vs;
    grad[2] = (c1 - c0) / A.vs;
    return true;
}

__global__ __launch_bounds__(kRegBlock) void k_reg_sums(RegArgs A, double *partials)
{
    __shared__ double s_w[kRegBlock / 64][kRegSums];
    double v[kRegSums];
    for (int k = 0; k < kRegSums; ++k) v[k] = 0.0;
    const int64_t i = (int64_t)blockIdx.x * kRegBlock + threadIdx.x;
    double phi, g[3], w[3];
    if (i < A.n && reg_point(A, A.xyz[3 * i], A.xyz[3 * i + 1], A.xyz[3 * i + 2], phi, g, w)) {
        const double J[6] = {g[0], g[1], g[2], w[1] * g[2] - w[2] * g[1], w[2] * g[0] - w[0] * g[2],
                             w[0] * g[1] - w[1] * g[0]};
        int k = 0;
        for (int a = 0; a < 6; ++a)
            for (int b = a; b < 6; ++b) v[k++] = J[a] * J[b];
        for (int a = 0; a < 6; ++a) v[21 + a] = J[a] * phi;
        v[27] = phi * phi;
        v[28] = 1.0;
    }
    // fixed butterfly over the wave
    for (int k = 0; k < kRegSums; ++k)
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off);
    const int wave = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0)
        for (int k = 0; k < kRegSums; ++k) s_w[wave][k] = v[k];
    __syncthreads();
    if (threadIdx.x < kRegSums) {
        double s = 0.0;
        for (int q = 0; q < kRegBlock / 64; ++q) s += s_w[q][threadIdx.x];
        partials[(int64_t)blockIdx.x * kRegSums + threadIdx.x] = s;
    }
}

}  // namespace

int64_t reg_blocks(int64_t n) { return (n + kRegBlock - 1) / kRegBlock; }

hipError_t launch_reg_sums(const RegArgs &A, double *partials, hipStream_t stream)
{
    const int64_t blocks = reg_blocks(A.n);
    if (blocks > 0) hipLaunchKernelGGL(k_reg_sums, dim3((uint32_t)blocks), dim3(kRegBlock), 0, stream, A, partials);
    return hipGetLastError();
}

}  // namespace tsdf
