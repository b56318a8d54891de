// Host build of the device free-space walk (csrc/ray.hpp: LongWalk,
// FreeWalk) against the oracle (oracle/tsdf_oracle.c), for free-space
// carving: for random rays longer than tau, from short ones to ones across
// the whole fixed-point range, with face, edge and corner ties and flat axes,
// the free segment [o, S] walked inside a box must visit exactly the
// oracle's voxels of that segment that lie in the box, in order, each with
// the oracle's key. Boxes are random, and they are also the slabs the
// carving scan uses: a window cut into slabs of 8 voxels along the segment's
// longest axis, whose walks must together give the segment's voxels in the
// window. The test driver defines RAY_HPP (a copy of ray.hpp whose one
// inline-asm minimum is replaced by a compare) and links the oracle.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>
#define __device__
#define __forceinline__ inline
#define __fma_rn(a, b, c) std::fma((a), (b), (c))
#define __dmul_rn(a, b) ((a) * (b))
#define __builtin_amdgcn_rcp(x) (1.0 / (x))
#define __builtin_amdgcn_rsq(x) (1.0 / std::sqrt(x))
using std::fabs;
using std::floor;
using std::fmin;
using std::isfinite;
using std::rint;
using std::sqrt;
#include RAY_HPP

extern "C" {
int or_band(const int64_t q[3], const int64_t o[3], int64_t tau_u, int64_t D[3], uint64_t *r_out, int64_t S[3],
            int64_t E[3]);
int64_t or_voxel_sdf(const int64_t q[3], const int64_t D[3], uint64_t r, const int64_t g[3], int64_t tau_u);
uint64_t or_key(int64_t s, uint64_t i);
int or_segment_voxels(const int64_t S[3], const int64_t E[3], int64_t *out, int max);
}

// voxels and keys of the device walk of [o, S] inside [lo, hi)
static std::vector<int64_t> walk_box(const tsdf::Ray &R, const tsdf::RayParams &P, const int32_t lo[3],
                                     const int32_t hi[3], uint32_t i, size_t cap)
{
    std::vector<int64_t> got;
    tsdf::FreeWalk F;
    if (tsdf::free_walk_init(R, P, lo, hi, F)) {
        do {
            if (got.size() >= cap) break;
            for (int a = 0; a < 3; ++a) got.push_back(F.W.g[a]);
            got.push_back((int64_t)tsdf::free_walk_key(F, R, P.tau, i));
        } while (tsdf::free_walk_next(F));
    }
    return got;
}

int main(int argc, char **argv)
{
    std::mt19937_64 rng(argc > 1 ? strtoull(argv[1], nullptr, 10) : 5);
    const int iters = argc > 2 ? atoi(argv[2]) : 3000;
    long bad = 0, cases = 0, visits = 0;
    std::vector<int64_t> buf;
    for (int it = 0; it < iters; ++it) {
        const int mode = it % 6;
        int32_t tau = std::uniform_int_distribution<int>(1, 32767)(rng);
        if (it % 3 == 0) tau = 5120;
        int32_t q[3], o[3];
        for (int a = 0; a < 3; ++a) {
            const int64_t span = mode == 0 ? 20000 : mode == 1 ? 300000 : mode == 2 ? 2000000 : mode == 3 ? 2048 : mode == 4 ? 40 : 60000;
            o[a] = (int32_t)std::uniform_int_distribution<int64_t>(-span, span)(rng);
            q[a] = (int32_t)std::uniform_int_distribution<int64_t>(-span, span)(rng);
            if (mode == 4) {  // on faces, edges and corners
                o[a] *= 512;
                q[a] *= 512;
            }
            if (mode == 5 && a == (it / 6) % 3) q[a] = o[a];  // a flat axis
        }
        if (it % 97 == 0)  // near the fixed-point limits
            for (int a = 0; a < 3; ++a) {
                o[a] = (int32_t)std::uniform_int_distribution<int64_t>(-(1 << 30) + 1, -(1 << 29))(rng);
                q[a] = (int32_t)std::uniform_int_distribution<int64_t>(1 << 29, (1 << 30) - 1)(rng);
                if (rng() & 1) std::swap(o[a], q[a]);
            }
        tsdf::RayParams P{};
        P.tau = tau;
        for (int a = 0; a < 3; ++a) P.o[a] = o[a];
        tsdf::Ray R;
        if (!tsdf::make_ray(q, P, R) || !(R.r > (double)tau)) continue;
        int64_t oo[3] = {o[0], o[1], o[2]}, qq[3] = {q[0], q[1], q[2]}, D[3], S[3], E[3];
        uint64_t r;
        or_band(qq, oo, tau, D, &r, S, E);
        bool same = (uint64_t)R.r == r;
        for (int a = 0; a < 3; ++a) same = same && S[a] == R.S[a];
        if (!same) {
            if (bad < 5) printf("band mismatch at ray %d\n", it);
            ++bad;
            continue;
        }
        // the oracle's free segment, keyed, only for segments it can list here
        int64_t need = 8;
        for (int a = 0; a < 3; ++a) need += std::llabs(S[a] - oo[a]) / 1024 + 2;
        if (need > 4000000) continue;
        if ((int64_t)buf.size() < 3 * need) buf.resize(3 * need);
        const int nv = or_segment_voxels(oo, S, buf.data(), (int)need);
        if (nv <= 0) continue;
        const uint32_t i = (uint32_t)it;
        auto want_in = [&](const int32_t lo[3], const int32_t hi[3]) {
            std::vector<int64_t> w;
            for (int k = 0; k < nv; ++k) {
                bool in = true;
                for (int a = 0; a < 3; ++a) in = in && buf[3 * k + a] >= lo[a] && buf[3 * k + a] < hi[a];
                if (!in) continue;
                for (int a = 0; a < 3; ++a) w.push_back(buf[3 * k + a]);
                w.push_back((int64_t)or_key(or_voxel_sdf(qq, D, r, &buf[3 * k], tau), i));
            }
            return w;
        };
        // a window around a voxel of the segment, random boxes inside it
        const int pick = std::uniform_int_distribution<int>(0, nv - 1)(rng);
        int32_t wlo[3], whi[3];
        for (int a = 0; a < 3; ++a) {
            const int32_t ext = std::uniform_int_distribution<int>(1, 300)(rng);
            wlo[a] = (int32_t)buf[3 * pick + a] - std::uniform_int_distribution<int>(0, ext)(rng);
            whi[a] = wlo[a] + ext;
        }
        for (int b = 0; b < 2; ++b) {
            int32_t lo[3], hi[3];
            for (int a = 0; a < 3; ++a) {
                lo[a] = std::uniform_int_distribution<int32_t>(wlo[a], whi[a] - 1)(rng);
                hi[a] = std::uniform_int_distribution<int32_t>(lo[a] + 1, whi[a])(rng);
            }
            const std::vector<int64_t> want = want_in(lo, hi);
            ++cases;
            visits += (long)want.size() / 4;
            if (walk_box(R, P, lo, hi, i, want.size() + 40) != want) {
                if (bad < 5) printf("box mismatch at ray %d mode %d\n", it, mode);
                ++bad;
            }
        }
        // the window cut into slabs of 8 voxels along the longest axis
        int da = 0;
        int64_t best = -1;
        for (int a = 0; a < 3; ++a) {
            const int64_t L = std::llabs((int64_t)R.S[a] - o[a]);
            if (L > best) {
                best = L;
                da = a;
            }
        }
        const std::vector<int64_t> want = want_in(wlo, whi);
        std::vector<int64_t> joined;
        const int32_t g0 = o[da] >> 10, g1 = R.S[da] >> 10;
        const int32_t gmin = std::max(std::min(g0, g1), wlo[da]), gmax = std::min(std::max(g0, g1), whi[da] - 1);
        std::vector<std::vector<int64_t>> parts;
        for (int32_t k = gmin >> 3; gmin <= gmax && k * 8 <= gmax; ++k) {
            int32_t lo[3] = {wlo[0], wlo[1], wlo[2]}, hi[3] = {whi[0], whi[1], whi[2]};
            lo[da] = std::max(lo[da], k * 8);
            hi[da] = std::min(hi[da], k * 8 + 8);
            if (lo[da] < hi[da]) parts.push_back(walk_box(R, P, lo, hi, i, want.size() + 40));
        }
        // slabs are visited in the walk's direction along da
        if (g1 < g0) std::reverse(parts.begin(), parts.end());
        for (const auto &p : parts) joined.insert(joined.end(), p.begin(), p.end());
        ++cases;
        visits += (long)want.size() / 4;
        if (joined != want) {
            if (bad < 5) printf("slab mismatch at ray %d mode %d\n", it, mode);
            ++bad;
        }
    }
    printf("cases %ld visits %ld mismatches %ld\n", cases, visits, bad);
    return bad != 0 || visits == 0;
}
