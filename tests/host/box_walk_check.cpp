// Host build of the device walk (csrc/ray.hpp) checked for the tile pass's
// resume: for random rays and random tilings of random windows, the binning
// side walks the band on the tile grid and takes, at each tile the ray
// enters, the voxel walk's crossing counts up to the entering event; the tile
// side rebuilds the voxel walk, advances it by those counts, sets it down in
// the tile's box (clipped to the window) and runs the box walk. The voxels it
// visits, in order, with their box index and distance numerator n, must be
// exactly the voxels of the plain voxel walk that lie in that box, and every
// such voxel must be reached from some tile. The walk on the tile grid must
// visit no more cells than band_tiles_bound allows (the entry buffer is sized
// by it), also for rays built to be long on the grid: near the sensor (r <=
// tau, S = o) and along the cube's diagonals. The test driver defines
// RAY_HPP (a copy of ray.hpp whose one inline-asm minimum is replaced by a
// compare).
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
using namespace tsdf;

struct Vox {
    int32_t g[3];
    double n;
};

int main(int argc, char **argv)
{
    std::mt19937_64 rng(argc > 1 ? strtoull(argv[1], nullptr, 10) : 11);
    const int iters = argc > 2 ? atoi(argv[2]) : 20000;
    long bad = 0, tiles = 0, visits = 0, rays = 0, resumes = 0, direct = 0;
    int32_t max_count = 0, max_cells = 0, cells_at_bound = 0;
    // cells of the band walk on a grid of 2^lt voxels against the bound
    auto check_cells = [&](const Ray &R, int32_t tau, const int32_t lt[3], const int32_t org[3]) {
        const int32_t lc[3] = {10 + lt[0], 10 + lt[1], 10 + lt[2]};
        const int32_t base[3] = {1024 * org[0], 1024 * org[1], 1024 * org[2]};
        Walk T;
        walk_init_cells(R, T, lc, base);
        double t_ev = -1.0;
        int typ = 0;
        int32_t n = 1;
        while (walk_next_event(T, t_ev, typ) && n < 1000) ++n;
        const int32_t bound = band_tiles_bound(tau, lt);
        max_cells = std::max(max_cells, n);
        cells_at_bound += n == bound ? 1 : 0;
        if (n > bound) {
            if (bad < 5) printf("band walk visits %d cells, bound %d (tau %d, lt %d %d %d)\n", n, bound, tau, lt[0], lt[1], lt[2]);
            ++bad;
        }
    };
    for (int it = 0; it < iters; ++it) {
        RayParams P{};
        const int64_t lim = 1ll << std::uniform_int_distribution<int>(0, 24)(rng);
        int32_t q[3];
        for (int a = 0; a < 3; ++a) {
            const int64_t o = std::uniform_int_distribution<int64_t>(-(1ll << 24), 1ll << 24)(rng);
            int64_t d = std::uniform_int_distribution<int64_t>(-lim, lim)(rng);
            if (it % 4 == 0 && a == it % 3) d = 0;  // flat axes
            P.o[a] = (int32_t)o;
            q[a] = (int32_t)(o + d);
        }
        P.tau = std::uniform_int_distribution<int>(1, it % 5 == 0 ? 32767 : 12000)(rng);
        Ray R;
        if (!make_ray(q, P, R)) continue;
        ++rays;
        // the plain voxel walk
        std::vector<Vox> all;
        Walk W;
        walk_init(R, W);
        do all.push_back({{W.g[0], W.g[1], W.g[2]}, W.n});
        while (walk_next(W) && all.size() < 100000);
        // a window around the point, tiles of 2^lt voxels per axis
        int32_t lt[3], org[3], dims[3], nt[3];
        for (int a = 0; a < 3; ++a) {
            lt[a] = std::uniform_int_distribution<int>(1, 4)(rng);
            dims[a] = std::uniform_int_distribution<int>(1, 80)(rng);
            org[a] = (q[a] >> 10) - std::uniform_int_distribution<int>(0, dims[a])(rng);
            nt[a] = (dims[a] + (1 << lt[a]) - 1) >> lt[a];
        }
        const int32_t sh[3] = {lt[1] + lt[2], lt[2], 0};
        check_cells(R, P.tau, lt, org);
        const int32_t lc[3] = {10 + lt[0], 10 + lt[1], 10 + lt[2]};
        const int32_t base[3] = {1024 * org[0], 1024 * org[1], 1024 * org[2]};
        // binning side: the tile walk and the crossing counts at each entry
        Walk T, Wv;
        walk_init_cells(R, T, lc, base);
        walk_init(R, Wv);
        double t_in = -1.0;
        int typ_in = 0;
        std::vector<char> reached(all.size(), 0);
        do {
            bool in = true;
            for (int a = 0; a < 3; ++a) in = in && T.g[a] >= 0 && T.g[a] < nt[a];
            if (in) {
                ++tiles;
                int32_t c[3] = {0, 0, 0};
                if (t_in >= 0.0)
                    for (int a = 0; a < 3; ++a)
                        c[a] = (int32_t)crossings_upto(Wv.T[a], Wv.dT[a], Wv.step[a] > 0 ? 0 : 1, t_in, typ_in);
                // through the binning's packings: 8 bits per axis, then 7
                // bits per axis beside a 10-bit slot, and back
                {
                    uint32_t c8 = 0;
                    for (int a = 0; a < 3; ++a) {
                        if (c[a] < 0 || c[a] > 127) ++bad;  // outside the packed range
                        c8 |= (uint32_t)c[a] << (8 * a);
                    }
                    const uint32_t word = 1023u | counts_8to7(c8) << 10;
                    const uint32_t back = counts_7to8(word >> 10);
                    for (int a = 0; a < 3; ++a) {
                        if ((int32_t)((back >> (8 * a)) & 0xffu) != c[a]) ++bad;
                        max_count = std::max(max_count, c[a]);
                    }
                }
                // tile side
                int32_t blo[3], bhi[3];
                for (int a = 0; a < 3; ++a) {
                    blo[a] = org[a] + (T.g[a] << lt[a]);
                    bhi[a] = org[a] + std::min((T.g[a] + 1) << lt[a], dims[a]);
                }
                std::vector<Vox> want;
                std::vector<size_t> idx;
                for (size_t k = 0; k < all.size(); ++k) {
                    bool ib = true;
                    for (int a = 0; a < 3; ++a) ib = ib && all[k].g[a] >= blo[a] && all[k].g[a] < bhi[a];
                    if (ib) {
                        want.push_back(all[k]);
                        idx.push_back(k);
                    }
                }
                Walk X;
                walk_init(R, X);
                walk_advance(X, c);
                {
                    bool in_box = true;
                    for (int a = 0; a < 3; ++a) in_box = in_box && X.g[a] >= blo[a] && X.g[a] < bhi[a];
                    direct += in_box ? 1 : 0;
                }
                std::vector<std::pair<int32_t, double>> got;
                // the tile pass's direct resume from the entry record must
                // give exactly the state of the general steps
                BoxWalk Vd;
                Ray Rd;
                const int32_t offd[3] = {R.E[0] - R.q[0], R.E[1] - R.q[1], R.E[2] - R.q[2]};
                const bool okd = box_walk_resume(R.q, offd, (uint32_t)R.r, c, P.o, P.tau, blo, bhi, sh, 0u, Rd, Vd);
                ++resumes;
                if (walk_enter_box(X, blo, bhi)) {
                    BoxWalk V;
                    box_walk_from(X, blo, bhi, sh, 0u, V);
                    bool same = okd && Vd.lim == V.lim && Vd.n == V.n && Vd.lv == V.lv;
                    for (int a = 0; a < 3; ++a)
                        same = same && Vd.T[a] == V.T[a] && Vd.dT[a] == V.dT[a] && Vd.dn[a] == V.dn[a] &&
                               Vd.dlv[a] == V.dlv[a] && Rd.S[a] == R.S[a] && Rd.E[a] == R.E[a] && Rd.D[a] == R.D[a];
                    same = same && Rd.r == R.r && Rd.r2 == R.r2;
                    if (!same) {
                        if (bad < 5) printf("direct resume differs: ray %d tile (%d %d %d)\n", it, T.g[0], T.g[1], T.g[2]);
                        ++bad;
                    }
                    do got.push_back({V.lv, V.n});
                    while (box_walk_next(V) && got.size() < 100000);
                } else if (okd) {
                    if (bad < 5) printf("direct resume enters a box the walk misses: ray %d\n", it);
                    ++bad;
                }
                bool ok = got.size() == want.size();
                for (size_t k = 0; ok && k < got.size(); ++k) {
                    int32_t lv = 0;
                    for (int a = 0; a < 3; ++a) lv += (want[k].g[a] - blo[a]) << sh[a];
                    ok = got[k].first == lv && got[k].second == want[k].n;
                }
                if (!ok) {
                    if (bad < 5)
                        printf("mismatch: ray %d tile (%d %d %d) lt (%d %d %d): %zu voxels, want %zu\n", it, T.g[0],
                               T.g[1], T.g[2], lt[0], lt[1], lt[2], got.size(), want.size());
                    ++bad;
                }
                for (size_t k : idx) reached[k] = 1;
                visits += (long)got.size();
            }
        } while (walk_next_event(T, t_in, typ_in));
        // every voxel of the walk inside the window belongs to a visited tile
        for (size_t k = 0; k < all.size(); ++k) {
            bool iw = true;
            for (int a = 0; a < 3; ++a) iw = iw && all[k].g[a] >= org[a] && all[k].g[a] < org[a] + dims[a];
            if (iw && !reached[k]) {
                if (bad < 5) printf("voxel of ray %d in the window reached by no tile\n", it);
                ++bad;
            }
        }
    }
    // rays long on the tile grid: short D (r <= tau, the band from the
    // sensor), directions near the cube's diagonals, the largest tau, the
    // smallest tiles, and random sub-tile offsets of the point and the sensor
    for (int it = 0; it < iters; ++it) {
        RayParams P{};
        P.tau = it % 3 == 0 ? 32767 : std::uniform_int_distribution<int>(1, 32767)(rng);
        const int64_t len = it % 2 ? std::uniform_int_distribution<int64_t>(1, 4)(rng)
                                   : std::uniform_int_distribution<int64_t>(1, 3 * (int64_t)P.tau)(rng);
        int32_t q[3], lt[3], org[3];
        for (int a = 0; a < 3; ++a) {
            P.o[a] = std::uniform_int_distribution<int32_t>(-(1 << 20), 1 << 20)(rng);
            const int64_t sgn = rng() & 1 ? 1 : -1;
            q[a] = (int32_t)(P.o[a] + sgn * (len + std::uniform_int_distribution<int64_t>(-2, 2)(rng)));
            lt[a] = it % 4 == 0 ? 2 : std::uniform_int_distribution<int>(2, 6)(rng);
            org[a] = std::uniform_int_distribution<int32_t>(-5000, 5000)(rng);
        }
        Ray R;
        if (!make_ray(q, P, R)) continue;
        ++rays;
        check_cells(R, P.tau, lt, org);
    }
    printf("rays %ld tiles %ld resumes %ld (direct %ld) visits %ld largest crossing count %d largest band walk %d "
           "cells (%d at the bound) mismatches %ld\n",
           rays, tiles, resumes, direct, visits, max_count, max_cells, cells_at_bound, bad);
    return bad != 0 || visits == 0;
}
