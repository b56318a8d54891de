// Host build of the merge's exact division (csrc/ray.hpp) checked against
// exact integer rounding: rdiv_small gives rdiv(n, d) = sign(n) floor((2|n|
// + d) / 2d) for every divisor d in [1, 255] (Eq. (1) with weights below
// 255) and sampled divisors up to 32768, over numerators that cover every
// residue class near zero, every tie and near-tie k d / 2 +- 1 across the
// range, the extremes +-32768 d and random values, with the hardware
// reciprocal modelled as exact and as off by up to 2^-18 either way (its
// error is far below 2^-20; the Newton step squares it). The
// test driver defines RAY_HPP (a copy of ray.hpp whose one inline-asm
// minimum is replaced by a compare).
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>
#define __device__
#define __forceinline__ inline
#define __fma_rn(a, b, c) std::fma((a), (b), (c))
#define __dmul_rn(a, b) ((a) * (b))
static double g_pert = 0.0;
#define __builtin_amdgcn_rcp(x) ((1.0 / (x)) * (1.0 + g_pert))
#define __builtin_amdgcn_rsq(x) (1.0 / std::sqrt(x))
using std::fabs;
using std::floor;
using std::fmin;
using std::isfinite;
using std::rint;
using std::sqrt;
#include RAY_HPP
using namespace tsdf;

static int64_t exact(int64_t n, int64_t d)
{
    const int64_t a = 2 * (n < 0 ? -n : n) + d;
    const int64_t k = a / (2 * d);
    return n < 0 ? -k : k;
}

int main(int argc, char **argv)
{
    std::mt19937_64 rng(argc > 1 ? strtoull(argv[1], nullptr, 10) : 5);
    const double perts[7] = {0.0,  std::ldexp(1.0, -18), -std::ldexp(1.0, -18), std::ldexp(1.0, -20),
                             -std::ldexp(1.0, -20), std::ldexp(1.0, -23), -std::ldexp(1.0, -23)};
    long checks = 0, bad = 0;
    for (double p : perts) {
        g_pert = p;
        for (int32_t di = 1; di <= 255 + 64; ++di) {
            // every divisor up to 255, then 64 spread up to 32768
            const int32_t d = di <= 255 ? di : 255 + (int32_t)(((int64_t)(di - 255) * (32768 - 255)) / 64);
            auto check = [&](int64_t n) {
                if (n > 32768LL * d || n < -32768LL * d) return;  // rdiv_small's range: |n| <= 2^15 d
                const int64_t want = exact(n, d);
                const int32_t got = rdiv_small((int32_t)n, d);
                ++checks;
                if (got != want) {
                    if (bad < 8)
                        printf("n %lld d %d: %d, want %lld (pert %g)\n", (long long)n, d, got, (long long)want, p);
                    ++bad;
                }
            };
            for (int64_t n = -4096; n <= 4096; ++n) check(n);
            // ties and near-ties: 2n = k d + 2e, across the range
            for (int64_t k = -65536; k <= 65536; k += (k > -512 && k < 512) ? 1 : 7) {
                for (int e = -1; e <= 1; ++e) {
                    if ((k * d) % 2 == 0) check(k * d / 2 + e);
                    else check((k * d - 1) / 2 + e);
                }
            }
            for (int e = -2; e <= 2; ++e) {
                check(32768LL * d + e);
                check(-32768LL * d + e);
            }
            std::uniform_int_distribution<int64_t> U(-32768LL * d, 32768LL * d);
            for (int j = 0; j < 2000; ++j) check(U(rng));
        }
    }
    printf("checks %ld mismatches %ld\n", checks, bad);
    return bad != 0 || checks == 0;
}
