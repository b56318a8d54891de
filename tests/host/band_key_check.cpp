// Host build of the device ray arithmetic (csrc/ray.hpp) checked against
// exact integer rounding: the ray itself (r, and S, E from the band offsets
// rdiv(tau D, r)), and for the voxels of band walks of random rays the tile
// pass's band_key (Newton-refined reciprocal, a half-unit bias, no cap) and
// pack_key(voxel_sdf(...)) must both equal
//   pack_key(sign(n) min(floor((2|n| + r) / 2r), tau), i),  n = (q - c) . D,
// computed in 128-bit integers. Rays with tiny components make r small, so
// exact ties (2|n| + r divisible by 2r) are frequent. The hardware
// reciprocal estimate is replaced by 1/d scaled by (1 + p), p running over
// errors up to 2^-14, which the Newton steps absorb. The interpolation's
// float64 forms are checked the same way (and the tile pass's tile_key,
// which carries s's sign in bit 0): band_len against rdiv((c - o) .
// D, r) at every band voxel of rays with r < 2^30, and fill_offset against
// rdiv(h v_a, nv) for random and tiny (tie-prone) vectors v. The test
// driver defines RAY_HPP (a copy of ray.hpp whose one inline-asm minimum is
// replaced by a compare).
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>
#define __device__
#define __forceinline__ inline
#define __fma_rn(a, b, c) std::fma((a), (b), (c))
#define __dmul_rn(a, b) ((a) * (b))
static double g_pert = 0.0, g_rsq_pert = 0.0;
#define __builtin_amdgcn_rcp(x) ((1.0 / (x)) * (1.0 + g_pert))
#define __builtin_amdgcn_rsq(x) ((1.0 / std::sqrt(x)) * (1.0 + g_rsq_pert))
using std::fabs;
using std::floor;
using std::fmin;
using std::isfinite;
using std::rint;
using std::sqrt;
#include RAY_HPP
using namespace tsdf;

int main(int argc, char **argv)
{
    std::mt19937_64 rng(argc > 1 ? strtoull(argv[1], nullptr, 10) : 7);
    const int iters = argc > 2 ? atoi(argv[2]) : 20000;
    const double perts[] = {0.0, 0x1p-20, -0x1p-20, 0x1p-14, -0x1p-14, 0x1p-30, -0x1p-45};
    const double rsq_perts[] = {0.0, 0x1p-18, -0x1p-18, 0x1p-22, -0x1p-22};
    long bad = 0, vox = 0, ties = 0, rays = 0, lens_checked = 0;
    for (int it = 0; it < iters; ++it) {
        g_pert = perts[it % 7];
        g_rsq_pert = rsq_perts[it % 5];
        RayParams P{};
        const int64_t lim = 1ll << std::uniform_int_distribution<int>(0, 31)(rng);
        int32_t q[3];
        for (int a = 0; a < 3; ++a) {
            const int64_t o = std::uniform_int_distribution<int64_t>(-(1ll << 29), 1ll << 29)(rng);
            int64_t d = std::uniform_int_distribution<int64_t>(-lim, lim)(rng);
            if (it % 5 == 0 && a > 0) d = std::uniform_int_distribution<int64_t>(-2, 2)(rng);
            const int64_t p = o + d;  // the fixed point keeps |q| < 2^30
            P.o[a] = (int32_t)o;
            q[a] = (int32_t)(p > -(1ll << 30) && p < (1ll << 30) ? p : o);
        }
        P.tau = it % 3 == 0 ? 32767 : std::uniform_int_distribution<int>(1, 32767)(rng);
        Ray R;
        if (!make_ray(q, P, R)) continue;
        ++rays;
        // the ray itself against exact integers: r = floor(sqrt(|D|^2)),
        // off = rdiv(tau D, r), E = q + off, S = q - off (S = o for r <= tau)
        {
            unsigned __int128 dd = 0;
            __int128 D[3];
            for (int a = 0; a < 3; ++a) {
                D[a] = (__int128)q[a] - P.o[a];
                dd += (unsigned __int128)(D[a] * D[a]);
            }
            unsigned __int128 rr = (unsigned __int128)std::sqrt((long double)dd);
            while (rr * rr > dd) --rr;
            while ((rr + 1) * (rr + 1) <= dd) ++rr;
            bool ok = (double)(uint64_t)rr == R.r;
            for (int a = 0; a < 3 && ok; ++a) {
                const __int128 num = (__int128)P.tau * D[a];
                const __int128 an = num < 0 ? -num : num;
                __int128 off = (2 * an + (__int128)rr) / (2 * (__int128)rr);
                if (num < 0) off = -off;
                ok = R.E[a] == q[a] + (int64_t)off &&
                     R.S[a] == ((__int128)rr <= P.tau ? (int64_t)P.o[a] : q[a] - (int64_t)off);
            }
            if (!ok) {
                if (bad < 5) printf("ray mismatch: |D|^2 = %.17g r = %.17g\n", (double)dd, R.r);
                ++bad;
            }
        }
        const uint32_t i = (uint32_t)rng();
        Walk W;
        walk_init(R, W);
        const bool lens = R.r < 1073741824.0;  // band_len's range: r < 2^30
        __int128 dd2 = 0;
        for (int a = 0; a < 3; ++a) dd2 += (__int128)((int64_t)q[a] - P.o[a]) * ((int64_t)q[a] - P.o[a]);
        const double tt = (double)(dd2 - (__int128)(uint64_t)R.r * (__int128)(uint64_t)R.r);
        do {
            if (lens) {
                // (c - o) . D and its rounded quotient by r, when positive
                __int128 N = 0;
                for (int a = 0; a < 3; ++a)
                    N += (__int128)(1024 * (int64_t)W.g[a] + 512 - P.o[a]) * ((int64_t)q[a] - P.o[a]);
                const __int128 rr = (__int128)(uint64_t)R.r;
                const double got = band_len(W.n, tt, R);
                const bool ok = N > 0 ? got == (double)((2 * N + rr) / (2 * rr)) : got <= 0.0;
                if (!ok) {
                    if (bad < 5) printf("band_len: r=%.17g got %.17g\n", R.r, got);
                    ++bad;
                }
                ++lens_checked;
            }
            __int128 n = 0;
            for (int a = 0; a < 3; ++a)
                n += (__int128)((int64_t)q[a] - (1024 * (int64_t)W.g[a] + 512)) * ((int64_t)q[a] - P.o[a]);
            const __int128 an = n < 0 ? -n : n;
            const __int128 r = (__int128)(uint64_t)R.r;
            const __int128 num = 2 * an + r, den = 2 * r;
            const __int128 k = num / den;
            ties += num % den == 0;
            int32_t s = (int32_t)(k < P.tau ? k : P.tau);
            if (n < 0) s = -s;
            const uint64_t want = pack_key(s, i);
            const bool ok_band = (double)n == W.n && band_key(W.n, R.r + 0.5, R.inv_r2, (double)P.tau, i >> 16, i << 16) == want;
            // the tile pass's key: the same |s| and i above bit 16, s's sign in bit 0
            const uint64_t tk = tile_key(W.n, R.r + 0.5, R.inv_r2, (double)P.tau, i >> 16, i << 16);
            const bool ok_tile = (tk >> 16) == (want >> 16) && (tk & 0xfffeu) == 0 && tile_key_sdf(tk) == s;
            const bool ok_sdf = pack_key(voxel_sdf(W.n, R, P.tau), i) == want;
            if (!ok_band || !ok_sdf || !ok_tile) {
                if (bad < 5)
                    printf("mismatch: r=%llu tau=%d n=%.17g perturbation %g\n", (unsigned long long)(uint64_t)R.r,
                           P.tau, (double)n, g_pert);
                ++bad;
            }
            ++vox;
        } while (walk_next(W));
    }
    // fill offsets e_a = rdiv(h v_a, nv), nv = isqrt(v . v)
    long fills = 0, fill_ties = 0;
    for (int it = 0; it < iters; ++it) {
        int64_t v[3];
        const int64_t lim = it % 3 == 0 ? 4 : (int64_t)1 << std::uniform_int_distribution<int>(1, 30)(rng);
        for (int a = 0; a < 3; ++a) v[a] = std::uniform_int_distribution<int64_t>(-lim, lim)(rng);
        unsigned __int128 vv = 0;
        for (int a = 0; a < 3; ++a) vv += (unsigned __int128)((__int128)v[a] * v[a]);
        if (vv == 0) continue;
        unsigned __int128 nv = (unsigned __int128)std::sqrt((long double)vv);
        while (nv * nv > vv) --nv;
        while ((nv + 1) * (nv + 1) <= vv) ++nv;
        const double nvd = (double)(uint64_t)nv;
        const double inv_2nv = 1.0 / (2.0 * nvd);
        for (int k = 0; k < 8; ++k) {
            const int64_t h = k == 0 ? 65535 : (k == 1 ? 0 : std::uniform_int_distribution<int64_t>(1, 65535)(rng));
            for (int a = 0; a < 3; ++a) {
                const __int128 num = (__int128)h * v[a];
                const __int128 an = num < 0 ? -num : num;
                const __int128 d = (__int128)(uint64_t)nv;
                __int128 want = (2 * an + d) / (2 * d);
                fill_ties += (2 * an + d) % (2 * d) == 0;
                if (num < 0) want = -want;
                const int32_t got = fill_offset((double)h * (double)v[a], nvd + 0.5, inv_2nv);
                if ((__int128)got != want) {
                    if (bad < 5) printf("fill_offset: h %lld v %lld nv %.17g\n", (long long)h, (long long)v[a], nvd);
                    ++bad;
                }
                ++fills;
            }
        }
    }
    printf("rays %ld voxels %ld ties %ld band lengths %ld fill offsets %ld (ties %ld) mismatches %ld\n", rays, vox,
           ties, lens_checked, fills, fill_ties, bad);
    return bad != 0 || ties == 0 || fill_ties == 0 || lens_checked == 0;
}
