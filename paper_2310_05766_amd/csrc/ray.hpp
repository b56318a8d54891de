// Per-ray device arithmetic of the TSDF path (FeatSense, arXiv 2310.05766,
// Sec. VI): world transform and fixed-point rounding of a scan point, the
// truncation band around it, the exact voxel walk across the band, and the
// signed distance each walked voxel receives; further down, the long walk of
// free-space carving, whose ranges are stated with it.
//
// Every integer the band walk and the distance need stays below 2^53 in
// magnitude, so it is carried in float64 registers, where adds, multiplies
// and compares of such integers are exact and run at full rate on CDNA
// (a 64-bit integer add costs two VALU ops, a float64 add one).
//   |q|, |o| < 2^30          fixed-point positions
//   |D| < 2^31               ray vector q - o
//   |L_a| <= 3 tau + 2 < 2^17 band segment extent per axis
//   Lambda = prod |L_a| < 2^51, crossing times scaled by Lambda < 2^52
//   |(q - c) . D| < 2^51     distance numerator
// Only |D|^2 (up to 3 * 2^62) needs 64-bit integers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tsdf {

constexpr uint64_t kEmptyKey = ~0ull;
constexpr double kQLimit = 1073741824.0;  // 2^30

// What every ray of one scan shares.
struct RayParams {
    double M[12];        // rows 0..2 of world_T_sensor, row-major
    double scale;        // 1024 / voxel_size
    int32_t o[3];        // sensor position, fixed point
    int32_t tau;         // truncation, fixed point
};

// q = round-half-even(fma-chain(M, p) * scale); false for a non-finite point
// or |q_a| >= 2^30. The chain is fixed: fma(M0, x, fma(M1, y, fma(M2, z, M3))).
__device__ __forceinline__ bool quantise(float px, float py, float pz, const RayParams &P, int32_t q[3])
{
    if (!isfinite(px) || !isfinite(py) || !isfinite(pz)) return false;
    const double x = px, y = py, z = pz;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double w = __fma_rn(P.M[4 * a + 0], x, __fma_rn(P.M[4 * a + 1], y, __fma_rn(P.M[4 * a + 2], z, P.M[4 * a + 3])));
        double r = rint(__dmul_rn(w, P.scale));
        if (!(fabs(r) < kQLimit)) return false;
        q[a] = (int32_t)r;
    }
    return true;
}

// floor(sqrt(n)) for n < 3 * 2^62 (|D|^2 of a ray): float64 estimate, then
// one exact integer correction each way (the estimate is within one of the
// answer; (r + 1)^2 < 2^64 for r < 2^32).
__device__ __forceinline__ uint64_t isqrt_u64(uint64_t n)
{
    uint64_t r = (uint64_t)sqrt((double)n);
    r -= r * r > n ? 1u : 0u;
    r += (r + 1) * (r + 1) <= n ? 1u : 0u;
    return r;
}

// Approximate 1/d (v_rcp_f64; relative error far below 2^-20). Quotients
// below either correct its estimate exactly afterwards or refine the
// reciprocal by Newton steps first, as their error bounds require.
__device__ __forceinline__ double approx_rcp(double d) { return __builtin_amdgcn_rcp(d); }

// 1 / d to within a few units of 2^-53: the hardware estimate (relative
// error far below 2^-20) and two Newton steps, each of which squares the
// error and adds one rounding.
__device__ __forceinline__ double refined_rcp(double d)
{
    double y = approx_rcp(d);
    double e = __fma_rn(-d, y, 1.0);
    y = __fma_rn(y, e, y);
    e = __fma_rn(-d, y, 1.0);
    return __fma_rn(y, e, y);
}

// floor(sqrt(n)) for 0 < n < 3 * 2^62 (|D|^2 of a ray, so the root is below
// 2^31.8): sqrt(n) estimated as n / sqrt(n) from the hardware reciprocal
// square root (relative error far below 2^-20) with one Newton step, which
// leaves a relative error near 2^-40, an absolute one far below 1; then one
// exact correction each way in 64-bit integers ((r + 1)^2 < 2^64 here).
__device__ __forceinline__ uint32_t isqrt_ray(uint64_t n)
{
    const double x = (double)n;
    const double y = __builtin_amdgcn_rsq(x);
    double s = x * y;
    s = __fma_rn(0.5 * y, __fma_rn(-s, s, x), s);
    uint32_t r = (uint32_t)fmin(fmax(s, 0.0), 4294967295.0);
    r -= (uint64_t)r * r > n ? 1u : 0u;
    r += (uint64_t)(r + 1u) * (r + 1u) <= n ? 1u : 0u;
    return r;
}

// min(a, b) of two doubles that are never NaN, as one v_min_f64. fmin must
// first quiet signalling NaNs, one v_max_f64 x, x per operand the compiler
// cannot trace to an arithmetic result (loop-carried times, invariants), and
// the walk loops would pay for that on every step.
__device__ __forceinline__ double min_nonan(double a, double b)
{
    double r;
    asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// rdiv(n, d) for 1 <= d <= 2^15 and |n| <= 2^15 d (Eq. (1): n = g w + v,
// d = w + 1 with |g|, |v| <= tau < 2^15), with no correction step and no
// branch on the sign. x = (2|n| + d) / 2d is a multiple of 1 / 2d, so y =
// x + 1 / 4d, the quotient of the numerator plus a half, has the floor of x
// and lies at least 1 / 4d >= 2^-17 from every integer. y <= 2^15 + 1 and
// the reciprocal of 2d after one Newton step is off by about the square of
// the estimate's error (far below 2^-20), so the product is off by far less
// than 2^-17. Taken with the sign of n, (2n + sign(n) (d + 1/2)) / 2d =
// sign(n) y, and truncation towards zero gives sign(n) floor(x). The
// numerator is exact (below 2^33, in halves).
__device__ __forceinline__ int32_t rdiv_small(int32_t n, int32_t d)
{
    const double dd = 2.0 * (double)d;
    double y = approx_rcp(dd);
    y = __fma_rn(y, __fma_rn(-dd, y, 1.0), y);
    const double nn = (double)n;
    return (int32_t)(__fma_rn(2.0, nn, copysign((double)d + 0.5, nn)) * y);
}

// One ray: the scan point, its band [S, E] along the ray, and what the
// distance of each walked voxel needs.
struct Ray {
    int32_t q[3];
    double D[3];
    double r, r2, inv_r2;  // r = isqrt(|D|^2), r2 = 2r, inv_r2 = 1/(2r)
    int32_t S[3], E[3];
};

// D = q - o, r = isqrt(|D|^2); off = rdiv(tau D, r); E = q + off;
// S = q - off, or S = o when r <= tau. false for D = 0. The division takes
// no correction step: x = (2|tau D_a| + r) / 2r < 2 tau + 1 < 2^16 is a
// multiple of 1 / 2r, so with half a unit more on the numerator (exact,
// below 2^48) the quotient keeps the floor of x and lies at least 1 / 4r >
// 2^-33.8 from every integer, while its estimate from inv_r2 =
// refined_rcp(2r) is off by under 2^-35.
__device__ __forceinline__ bool make_ray(const int32_t q[3], const RayParams &P, Ray &R)
{
    uint64_t dd = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int32_t Di = q[a] - P.o[a];  // |q|, |o| < 2^30: fits
        dd += (uint64_t)((int64_t)Di * Di);
        R.q[a] = q[a];
        R.D[a] = (double)Di;
    }
    if (dd == 0) return false;
    const uint32_t r = isqrt_ray(dd);
    R.r = (double)r;
    R.r2 = 2.0 * R.r;
    R.inv_r2 = refined_rcp(R.r2);
    const double tau = (double)P.tau, rh = R.r + 0.5;
    const bool near = (double)r <= tau;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int32_t k = (int32_t)floor(__fma_rn(2.0, fabs(tau * R.D[a]), rh) * R.inv_r2);
        const int32_t oi = R.D[a] < 0 ? -k : k;
        R.E[a] = q[a] + oi;
        R.S[a] = near ? P.o[a] : q[a] - oi;
    }
    return true;
}

// Most cells of 2^lt[a] voxels (tiles) that the walk of one band segment
// [S, E] visits, for any ray of truncation tau. With |off_a - tau D_a / r|
// <= 1/2 and r <= |D| < r + 1, |E - S| < 2 tau + 4 in both cases of
// make_ray: 2|off| < 2 tau (1 + 1/r) + sqrt(3) when r > tau, and |D + off| <
// (r + 1)(1 + tau / r) + 1 <= 2 tau + 3 when S = o (1 <= r <= tau). So
// sum_a |L_a| < sqrt(3) (2 tau + 4) < 1774 (2 tau + 4) / 1024. The walk steps
// at most floor(|L_a| / c_a) + 1 times on axis a (cells of c_a fixed-point
// units) and visits one cell more than it takes events.
inline int32_t band_tiles_bound(int32_t tau, const int32_t lt[3])
{
    const int64_t len = (1774 * (2 * (int64_t)tau + 4) + 1023) / 1024;  // > sum_a |L_a|
    const int32_t lmin = lt[0] < lt[1] ? (lt[0] < lt[2] ? lt[0] : lt[2]) : (lt[1] < lt[2] ? lt[1] : lt[2]);
    return 4 + (int32_t)(len >> (10 + lmin));
}

// Signed distance of the voxel whose centre gives numerator n = (q - c) . D:
// clamp(rdiv(n, r), -tau, tau). The quotient floor((2|n| + r) / 2r) is
// capped at tau + 1, so its estimate from the reciprocal is within one and a
// single correction each way makes it exact (compare-and-select, no loop).
__device__ __forceinline__ int32_t voxel_sdf(double n, const Ray &R, int32_t tau)
{
    const double a = 2.0 * fabs(n) + R.r;
    const double cap = (double)tau + 1.0;
    double k = min_nonan(floor(a * R.inv_r2), cap);
    k -= k * R.r2 > a ? 1.0 : 0.0;
    k += (k < cap && __fma_rn(k, R.r2, R.r2) <= a) ? 1.0 : 0.0;
    const int32_t s = (int32_t)min_nonan(k, (double)tau);
    return n < 0 ? -s : s;
}

// key = |s| << 48 | i << 16 | (uint16)s: the smallest key of a voxel is its
// candidate with the smallest |s|, ties to the lowest point index.
__device__ __forceinline__ uint64_t pack_key(int32_t s, uint32_t i)
{
    uint32_t as = (uint32_t)(s < 0 ? -s : s);
    return ((uint64_t)as << 48) | ((uint64_t)i << 16) | (uint64_t)(uint16_t)(int16_t)s;
}

// pack_key(voxel_sdf(n, R, tau), i) for a voxel of the band walk, with
// rh = r + 1/2, inv_r2 = refined_rcp(2r), taud = tau, ihi = i >> 16 and
// ilo = i << 16. Such a voxel lies within one voxel diagonal of [S, E], so
// |q - c| <= tau (1 + 1/r) + 888 (S = o when r <= tau) and x = (2|n| + r) /
// 2r < 2^17.1. x is a multiple of 1 / 2r, so y = x + 1 / 4r = (2|n| + rh) /
// 2r has the floor of x and lies at least 1 / 4r > 2^-33.8 (r < 2^31.8) from
// every integer; its estimate (2|n| + rh) * inv_r2 is off by under 2^-34.8,
// so the estimate's floor is floor(x) with no correction. The numerator is
// exact (below 2^51, in halves). No cap is needed: x is far below 2^53 / 2r.
__device__ __forceinline__ uint64_t band_key(double n, double rh, double inv_r2, double taud, uint32_t ihi,
                                            uint32_t ilo)
{
    const double k = floor(__fma_rn(2.0, fabs(n), rh) * inv_r2);
    const uint32_t as = (uint32_t)min_nonan(k, taud);
    const uint32_t lo = ilo | (n < 0 ? (0x10000u - as) & 0xffffu : as);
    return (uint64_t)(as << 16 | ihi) << 32 | lo;
}

// The tile pass's key of a band walk voxel, ordered like band_key: |s| << 48
// | i << 16 | sign, with the sign of s (that of n) in bit 0 instead of s's
// low 16 bits. A point meets a voxel once per scan, so keys of equal |s|
// and i never meet and the low bits decide nothing; the sign is n's sign
// bit (n is an integer-valued double; -0 only with |s| = 0).
__device__ __forceinline__ uint64_t tile_key(double n, double rh, double inv_r2, double taud, uint32_t ihi,
                                             uint32_t ilo)
{
    const double k = floor(__fma_rn(2.0, fabs(n), rh) * inv_r2);
    const uint32_t as = (uint32_t)min_nonan(k, taud);
    uint64_t nb;
    __builtin_memcpy(&nb, &n, sizeof(nb));  // n's bits (a register move)
    const uint32_t lo = ilo | (uint32_t)(nb >> 63);
    return (uint64_t)(as << 16 | ihi) << 32 | lo;
}

// s of a tile_key: |s| with the sign of bit 0.
__device__ __forceinline__ int32_t tile_key_sdf(uint64_t key)
{
    const int32_t as = (int32_t)(key >> 48);
    return (key & 1u) ? -as : as;
}

// Vertical interpolation (Sec. VI, Eq. (3)/(4)) of a band voxel c, in
// float64 with no 64-bit integer product or correction step.
//
// len = rdiv((c - o) . D, r) when it is positive (otherwise a value <= 0,
// which takes no fill), from n = (q - c) . D and t = |D|^2 - r^2 (0 <= t <=
// 2r), for r < 2^30: (c - o) . D = r^2 + t - n, and for a positive numerator
// the rounding is floor(x + 1/2), so len = r + floor((2 (t - n) + r) / 2r).
// That quotient is a multiple of 1 / 2r and below 2^17.2 in magnitude (|q -
// c| < 2 tau + 2^11 < 2^16.1 and |D| < 2r), and the numerator with half a
// unit more is exact (below 2^48); its estimate from inv_r2 =
// refined_rcp(2r) is off by under 2^-33.5 and keeps the floor, which lies at
// least 1 / 4r > 2^-32 away.
__device__ __forceinline__ double band_len(double n, double t, const Ray &R)
{
    return R.r + floor(__fma_rn(2.0, t - n, R.r + 0.5) * R.inv_r2);
}

// e_a = rdiv(h v_a, |int|) for 0 <= h <= 65535 and |v_a| <= nv = |int| <
// 2^31 (so |e_a| <= h): hv = h v_a is exact (below 2^47), nvh = nv + 1/2 and
// inv_2nv the correctly rounded 1 / 2nv. The quotient with half a unit more
// on the numerator lies at least 1 / 4nv > 2^-33 from every integer, and its
// estimate (below 2^16) is off by under 2^-36.
__device__ __forceinline__ int32_t fill_offset(double hv, double nvh, double inv_2nv)
{
    const int32_t k = (int32_t)floor(__fma_rn(2.0, fabs(hv), nvh) * inv_2nv);
    return hv < 0 ? -k : k;
}

// Exact walk over the cells { floor((P(t) - base) / cell) : t in [0, 1] },
// P(t) = S + t (E - S), with cell = 2^lc per axis in fixed point (lc = 10:
// voxels; 10 + log2(tile edge): tiles). Axis crossings are ordered by their
// time t = dist / |L_a|, compared after scaling every time by Lambda =
// product of the non-zero |L_a| (integers, exact in float64). At equal
// times, crossings on increasing axes (which take effect at t: a point on a
// face belongs to the upper cell) come before crossings on decreasing axes
// (which take effect just after t). Increasing crossings are taken for
// t <= 1, decreasing ones for t < 1.
struct Walk {
    int32_t g[3];
    int32_t step[3];
    double T[3], dT[3];
    double lam;
    double n;       // (q - c(g)) . D for the current voxel (voxel walks)
    double dn[3];   // change of n per +1 step on each axis: -1024 D_a
};

__device__ __forceinline__ void walk_init_cells(const Ray &R, Walk &W, const int32_t lc[3], const int32_t base[3])
{
    double L[3], absL[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        L[a] = (double)(R.E[a] - R.S[a]);
        absL[a] = fabs(L[a]);
        W.g[a] = (int32_t)(((int64_t)R.S[a] - base[a]) >> lc[a]);  // arithmetic shift: floor division
        W.step[a] = L[a] > 0 ? 1 : (L[a] < 0 ? -1 : 0);
    }
    const double f0 = absL[0] > 0 ? absL[0] : 1.0;
    const double f1 = absL[1] > 0 ? absL[1] : 1.0;
    const double f2 = absL[2] > 0 ? absL[2] : 1.0;
    W.lam = f0 * f1 * f2;
    const double other[3] = {f1 * f2, f0 * f2, f0 * f1};
    double n = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double cell = (double)(1 << lc[a]);
        const double lo = (double)base[a] + cell * (double)W.g[a];
        // distance from S to the cell's face ahead (selects, no branches)
        const double x = (double)R.S[a] - lo;
        const double ahead = W.step[a] > 0 ? cell - x : x;
        W.T[a] = W.step[a] != 0 ? ahead * other[a] : INFINITY;
        W.dT[a] = cell * other[a];
        n += ((double)R.q[a] - (lo + 512.0)) * R.D[a];
        W.dn[a] = -1024.0 * R.D[a];
    }
    W.n = n;
}

// The voxel walk (cells of one voxel, global coordinates).
__device__ __forceinline__ void walk_init(const Ray &R, Walk &W)
{
    const int32_t lc[3] = {10, 10, 10}, base[3] = {0, 0, 0};
    walk_init_cells(R, W, lc, base);
}

// Advance to the next cell; false when the segment ends.
__device__ __forceinline__ bool walk_next(Walk &W)
{
    const double tm = min_nonan(W.T[0], min_nonan(W.T[1], W.T[2]));
    const bool e0 = W.T[0] == tm, e1 = W.T[1] == tm, e2 = W.T[2] == tm;
    const bool any_up = (e0 && W.step[0] > 0) || (e1 && W.step[1] > 0) || (e2 && W.step[2] > 0);
    const int dir = any_up ? 1 : -1;
    if (any_up ? (tm > W.lam) : (tm >= W.lam)) return false;
    if (e0 && W.step[0] == dir) { W.g[0] += dir; W.T[0] += W.dT[0]; W.n += dir * W.dn[0]; }
    if (e1 && W.step[1] == dir) { W.g[1] += dir; W.T[1] += W.dT[1]; W.n += dir * W.dn[1]; }
    if (e2 && W.step[2] == dir) { W.g[2] += dir; W.T[2] += W.dT[2]; W.n += dir * W.dn[2]; }
    return true;
}

// walk_next that also reports the event it took: its time and its type
// (0: increasing crossings, 1: decreasing ones).
__device__ __forceinline__ bool walk_next_event(Walk &W, double &t_ev, int &typ)
{
    const double tm = min_nonan(W.T[0], min_nonan(W.T[1], W.T[2]));
    const bool e0 = W.T[0] == tm, e1 = W.T[1] == tm, e2 = W.T[2] == tm;
    const bool any_up = (e0 && W.step[0] > 0) || (e1 && W.step[1] > 0) || (e2 && W.step[2] > 0);
    const int dir = any_up ? 1 : -1;
    if (any_up ? (tm > W.lam) : (tm >= W.lam)) return false;
    if (e0 && W.step[0] == dir) { W.g[0] += dir; W.T[0] += W.dT[0]; W.n += dir * W.dn[0]; }
    if (e1 && W.step[1] == dir) { W.g[1] += dir; W.T[1] += W.dT[1]; W.n += dir * W.dn[1]; }
    if (e2 && W.step[2] == dir) { W.g[2] += dir; W.T[2] += W.dT[2]; W.n += dir * W.dn[2]; }
    t_ev = tm;
    typ = any_up ? 0 : 1;
    return true;
}

// Crossings of one axis, at times T0 + k dT (k = 0, 1, ...) and of type typ
// (0: increasing, 1: decreasing), that come at or before the event (Ts, ts)
// in the walk's order (time, then increasing before decreasing). The event
// lies within the segment (Ts <= lam), so the count is at most
// |L_a| / cell + 1 < 2^7 and the reciprocal's estimate is within one of it.
__device__ __forceinline__ double crossings_upto(double T0, double dT, int typ, double Ts, int ts)
{
    if (!(T0 <= Ts)) return 0.0;  // also for an axis that never crosses (T0 = inf)
    const double span = Ts - T0;   // exact: both are integers < 2^53
    double k = floor(span * approx_rcp(dT));
    k -= k * dT > span ? 1.0 : 0.0;             // exact: every term is an integer < 2^53
    k += (k + 1.0) * dT <= span ? 1.0 : 0.0;
    double c = k + 1.0;
    if (k * dT == span && typ > ts) c -= 1.0;
    return c;
}

// Crossing counts of the three axes (each below 2^7: a band segment spans at
// most (3 tau + 2) / 1024 + 1 < 98 voxel faces per axis) in two packings:
// 8 bits per axis (the entry record) and 7 bits per axis (21 bits, beside a
// 10-bit slot in one 32-bit word).
__device__ __forceinline__ uint32_t counts_8to7(uint32_t c)
{
    return (c & 0x7fu) | ((c >> 8) & 0x7fu) << 7 | ((c >> 16) & 0x7fu) << 14;
}
__device__ __forceinline__ uint32_t counts_7to8(uint32_t c)
{
    return (c & 0x7fu) | ((c >> 7) & 0x7fu) << 8 | ((c >> 14) & 0x7fu) << 16;
}

// Apply c[a] crossings on each axis to a freshly initialised voxel walk (the
// state right after the event whose crossing counts they are).
__device__ __forceinline__ void walk_advance(Walk &W, const int32_t c[3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double k = (double)c[a];
        W.g[a] += W.step[a] * c[a];
        W.T[a] += k * W.dT[a];
        W.n += (double)W.step[a] * k * W.dn[a];
    }
}

// Move a freshly initialised voxel walk to its first voxel inside the box
// [lo, hi) (global voxel coordinates): the state after every event up to the
// one at which the last axis enters the box's range. false when no voxel of
// the walk lies in the box. Coordinates are monotone along a walk, so the
// voxels inside the box form one run that starts here.
__device__ __forceinline__ bool walk_enter_box(Walk &W, const int32_t lo[3], const int32_t hi[3])
{
    double Te = -1.0;
    int te = 0;
    bool inside = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int32_t g0 = W.g[a];
        if (g0 >= lo[a] && g0 < hi[a]) continue;
        inside = false;
        double k;
        int typ;
        if (W.step[a] > 0 && g0 < lo[a]) {
            k = (double)(lo[a] - g0);
            typ = 0;
        } else if (W.step[a] < 0 && g0 >= hi[a]) {
            k = (double)(g0 - hi[a] + 1);
            typ = 1;
        } else {
            return false;  // outside and not moving towards the box
        }
        const double T = W.T[a] + (k - 1.0) * W.dT[a];
        if (T > Te || (T == Te && typ > te)) {
            Te = T;
            te = typ;
        }
    }
    if (inside) return true;
    if (te == 0 ? (Te > W.lam) : (Te >= W.lam)) return false;  // after the segment's end
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (W.step[a] == 0) continue;
        const double c = crossings_upto(W.T[a], W.dT[a], W.step[a] > 0 ? 0 : 1, Te, te);
        W.g[a] += W.step[a] * (int32_t)c;
        W.T[a] += c * W.dT[a];
        W.n += (double)W.step[a] * c * W.dn[a];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
        if (W.g[a] < lo[a] || W.g[a] >= hi[a]) return false;
    return true;
}

// The voxel walk restricted to one box, as the tile pass runs it. Event
// times are re-encoded as T' = 2 T + (1 on a decreasing axis): an increasing
// crossing then sorts before a decreasing one at the same time, crossings of
// one kind at one time stay equal (they step together), and "increasing
// taken for T <= lam, decreasing for T < lam" becomes T' <= 2 lam for both
// (T integer). Leaving the box is one more event per axis, so the whole
// stopping rule is one bound: T' <= lim, lim = min(2 lam, first exit - 1).
// The walk carries the LDS byte address of the voxel's key (a buffer in z
// fastest layout) instead of its coordinates. Magnitudes: T' < 2^53 (T < 2^52, and a box
// exit lies at most 64 crossings past the current time).
struct BoxWalk {
    double T[3], dT[3];
    double lim;
    double n, dn[3];
    int32_t lv, dlv[3];
};

// From a voxel walk that walk_enter_box has placed inside [lo, hi); sh[a] is
// the byte shift of axis a in a key buffer at LDS address base.
__device__ __forceinline__ void box_walk_from(const Walk &W, const int32_t lo[3], const int32_t hi[3],
                                              const int32_t sh[3], uint32_t base, BoxWalk &V)
{
    double first_exit = INFINITY;
    V.lv = (int32_t)base;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        V.lv += (W.g[a] - lo[a]) << sh[a];
        if (W.step[a] == 0) {
            V.T[a] = INFINITY;
            V.dT[a] = 0.0;
            V.dn[a] = 0.0;
            V.dlv[a] = 0;
            continue;
        }
        const bool up = W.step[a] > 0;
        V.T[a] = 2.0 * W.T[a] + (up ? 0.0 : 1.0);
        V.dT[a] = 2.0 * W.dT[a];
        V.dn[a] = up ? W.dn[a] : -W.dn[a];
        V.dlv[a] = up ? (1 << sh[a]) : -(1 << sh[a]);
        // crossings until the walk leaves the box on this axis (at least one)
        const int32_t k = up ? hi[a] - W.g[a] : W.g[a] - lo[a] + 1;
        first_exit = min_nonan(first_exit, V.T[a] + (double)(k - 1) * V.dT[a]);  // never NaN
    }
    V.lim = min_nonan(2.0 * W.lam, first_exit - 1.0);
    V.n = W.n;
}

// The box walk of one tile entry, straight from what the entry record holds:
// the point q, the band offsets off = E - q, r = isqrt(|D|^2) and the voxel
// crossings c[a] taken up to the event that entered the tile. Sets R (the
// ray as make_ray gives it, with inv_r2 = refined_rcp(2r) as band_key
// wants) and V, the state that walk_init, walk_advance(c), walk_enter_box
// and box_walk_from give, with the resumed voxel walk formed directly
// (crossing times and distance numerator at c crossings) instead of by a
// walk from S; walk_enter_box only moves it where the tile is clipped by the
// window's edge. false when no voxel of the walk lies in the box [lo, hi).
// Integer ranges: |q|, |o| < 2^30, so D and the voxel offsets q - c fit
// int32 (|q - c| stays within a voxel diagonal of the band, below 2^17);
// the products below are exact in float64 (< 2^52).
__device__ __forceinline__ bool box_walk_resume(const int32_t q[3], const int32_t off[3], uint32_t r,
                                                const int32_t c[3], const int32_t o[3], int32_t tau,
                                                const int32_t lo[3], const int32_t hi[3], const int32_t sh[3],
                                                uint32_t base, Ray &R, BoxWalk &V)
{
    R.r = (double)r;
    R.r2 = 2.0 * R.r;
    R.inv_r2 = refined_rcp(R.r2);
    const bool near = R.r <= (double)tau;
    Walk W;
    double f[3];
    bool inside = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        R.q[a] = q[a];
        R.D[a] = (double)(q[a] - o[a]);
        R.E[a] = q[a] + off[a];
        R.S[a] = near ? o[a] : q[a] - off[a];
        const int32_t L = R.E[a] - R.S[a];
        W.step[a] = L > 0 ? 1 : (L < 0 ? -1 : 0);
        f[a] = L != 0 ? (double)(L < 0 ? -L : L) : 1.0;
        W.g[a] = (R.S[a] >> 10) + W.step[a] * c[a];  // arithmetic shift: floor division
        inside = inside && W.g[a] >= lo[a] && W.g[a] < hi[a];
    }
    const double other[3] = {f[1] * f[2], f[0] * f[2], f[0] * f[1]};
    W.lam = f[0] * f[1] * f[2];
    double n = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        n += (double)(q[a] - 1024 * W.g[a] - 512) * R.D[a];
        // distance from S to the first face ahead, then c[a] whole cells
        const int32_t g0 = R.S[a] >> 10;
        const int32_t ahead = W.step[a] > 0 ? 1024 * (g0 + 1) - R.S[a] : R.S[a] - 1024 * g0;
        W.T[a] = W.step[a] != 0 ? (double)(ahead + 1024 * c[a]) * other[a] : INFINITY;
        W.dT[a] = 1024.0 * other[a];
        W.dn[a] = -1024.0 * R.D[a];
    }
    W.n = n;
    if (!inside && !walk_enter_box(W, lo, hi)) return false;
    box_walk_from(W, lo, hi, sh, base, V);
    return true;
}

// Advance to the next voxel of the box; false when the walk leaves the box
// or the segment ends (the state then holds a step past the end, never used:
// stepping without a branch costs less than testing first).
__device__ __forceinline__ bool box_walk_next(BoxWalk &V)
{
    const double tm = min_nonan(V.T[0], min_nonan(V.T[1], V.T[2]));
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        // x + (0 or 1) dx as one fma: exact (the sums are integers below
        // 2^53, and an axis that never crosses has dT = dn = 0)
        const bool e = V.T[a] == tm;
        const double ef = e ? 1.0 : 0.0;
        V.T[a] = __fma_rn(ef, V.dT[a], V.T[a]);
        V.n = __fma_rn(ef, V.dn[a], V.n);
        V.lv += e ? V.dlv[a] : 0;
    }
    return tm <= V.lim;
}

// ---------------------------------------------------------------------------
// Long walk: the exact voxel set of a segment [A, B] of any length the fixed
// point allows (|L_a| = |B_a - A_a| < 2^31), clipped to a box of voxels
// [lo, hi). Free-space carving walks the ray from the sensor with it, a
// segment far too long for the products of the band walk above.
//
// With T_a the next crossing time of axis a scaled by |L_a| (an integer at
// most |L_a| + 1024), two axes are ordered by
//   C_ab = 2 (T_a |L_b| - T_b |L_a|) + (dec_a - dec_b),
// dec = 1 on a decreasing axis: C_ab <= 0 when a's crossing comes first or
// at the same time and of the same type (both step), C_ab >= 0 the other way
// round, so the walk's order (time, then increasing before decreasing) needs
// no division. While both axes still cross, their next crossings lie within
// one cell time (1024 / |L|) of the current time, so |C_ab| <= 2048
// max(|L_a|, |L_b|) + 1 < 2^43, and a step of axis a adds the exact integer
// 2048 |L_b|: exact in float64. Setting the walk down inside the box takes
// 64-bit integer products below 2^62.2.
// ---------------------------------------------------------------------------
struct LongWalk {
    int32_t g[3];
    int32_t step[3];
    int32_t rem[3];   // crossings still ahead on each axis (to the segment's end, or to leaving the box)
    int32_t xit;      // bit a: the last of axis a's rem crossings leaves the box
    double C01, C02, C12;
    double K[3];      // 2048 |L_a|
};

// floor(a / b) for 0 <= a < 2^63, 0 < b < 2^42: a float64 estimate, then one
// exact correction each way (the quotient is below 2^22, so the estimate is
// within one of it).
__device__ __forceinline__ int64_t floor_div_i64(int64_t a, int64_t b)
{
    int64_t k = (int64_t)((double)a / (double)b);
    k -= k * b > a ? 1 : 0;
    k += (k + 1) * b <= a ? 1 : 0;
    return k;
}

// Set the walk down on the first voxel of [A, B] inside [lo, hi), with c[a]
// the crossings taken on each axis to get there; false when no voxel of the
// segment lies in the box. Coordinates are monotone along the walk, so the
// voxels inside the box form one run: it starts after the event at which the
// last axis enters the box's range (every crossing at or before that event in
// the walk's order is taken) and ends at the first event that leaves it.
__device__ __forceinline__ bool long_walk_init(const int32_t A[3], const int32_t B[3], const int32_t lo[3],
                                               const int32_t hi[3], LongWalk &W, int32_t c[3])
{
    int64_t absL[3], T0[3];
    int32_t g0[3], N[3], kin[3], X[3];
    bool dec[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int64_t L = (int64_t)B[a] - A[a];
        absL[a] = L < 0 ? -L : L;
        dec[a] = L < 0;
        g0[a] = A[a] >> 10;  // arithmetic shift: floor division
        const int32_t gB = B[a] >> 10;
        W.step[a] = L > 0 ? 1 : (L < 0 ? -1 : 0);
        N[a] = gB > g0[a] ? gB - g0[a] : g0[a] - gB;
        // scaled time of the first crossing: the distance to the next face
        T0[a] = L >= 0 ? (int64_t)(g0[a] + 1) * 1024 - A[a] : (int64_t)A[a] - (int64_t)g0[a] * 1024;
        // crossing counts at which this axis is inside [lo, hi): kin <= k < X
        if (L > 0) {
            kin[a] = lo[a] - g0[a] > 0 ? lo[a] - g0[a] : 0;
            X[a] = hi[a] - g0[a];
        } else if (L < 0) {
            kin[a] = g0[a] - (hi[a] - 1) > 0 ? g0[a] - (hi[a] - 1) : 0;
            X[a] = g0[a] - lo[a] + 1;
        } else {
            if (g0[a] < lo[a] || g0[a] >= hi[a]) return false;
            kin[a] = 0;
            X[a] = 0x7fffffff;
        }
        if (X[a] <= 0 || kin[a] > N[a]) return false;
    }
    // the entry event: the latest of the axes' entering crossings
    int e = -1;
    int64_t Te = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (kin[a] == 0) continue;
        const int64_t Ta = T0[a] + 1024 * (int64_t)(kin[a] - 1);
        if (e >= 0) {
            const int64_t d = Ta * absL[e] - Te * absL[a];
            if (d < 0 || (d == 0 && !(dec[a] && !dec[e]))) continue;  // not after the current latest
        }
        e = a;
        Te = Ta;
    }
    int64_t T[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        int64_t k = 0;
        if (e == b) {
            k = kin[b];
        } else if (e >= 0 && N[b] > 0) {
            // crossings j of b with T0_b + 1024 j scaled by |L_e| at or before
            // Te scaled by |L_b|: 1024 j |L_e| <= num (< num if b decreases
            // and the entry crossing increases: b's crossing comes after it)
            const int64_t num = Te * absL[b] - T0[b] * absL[e];
            const int64_t den = 1024 * absL[e];
            if (!(dec[b] && !dec[e]))
                k = num < 0 ? 0 : floor_div_i64(num, den) + 1;
            else
                k = num <= 0 ? 0 : floor_div_i64(num - 1, den) + 1;
            k = k < N[b] ? k : N[b];
        }
        if (k >= X[b]) return false;  // left the box before it entered on another axis
        c[b] = (int32_t)k;
        W.g[b] = g0[b] + W.step[b] * (int32_t)k;
        W.rem[b] = (N[b] < X[b] ? N[b] : X[b]) - (int32_t)k;
        T[b] = T0[b] + 1024 * k;
        W.K[b] = 2048.0 * (double)absL[b];
    }
    W.xit = (X[0] <= N[0] ? 1 : 0) | (X[1] <= N[1] ? 2 : 0) | (X[2] <= N[2] ? 4 : 0);
    // int64 differences below 2^62.2 (live pairs: below 2^42)
    W.C01 = 2.0 * (double)(T[0] * absL[1] - T[1] * absL[0]) + (double)((int)dec[0] - (int)dec[1]);
    W.C02 = 2.0 * (double)(T[0] * absL[2] - T[2] * absL[0]) + (double)((int)dec[0] - (int)dec[2]);
    W.C12 = 2.0 * (double)(T[1] * absL[2] - T[2] * absL[1]) + (double)((int)dec[1] - (int)dec[2]);
    return true;
}

// Next voxel: the axes that step (bit a for axis a), 0 when the segment ends
// or the walk leaves the box.
__device__ __forceinline__ int long_walk_next(LongWalk &W)
{
    const bool l0 = W.rem[0] > 0, l1 = W.rem[1] > 0, l2 = W.rem[2] > 0;
    const bool s0 = l0 && (!l1 || W.C01 <= 0.0) && (!l2 || W.C02 <= 0.0);
    const bool s1 = l1 && (!l0 || W.C01 >= 0.0) && (!l2 || W.C12 <= 0.0);
    const bool s2 = l2 && (!l0 || W.C02 >= 0.0) && (!l1 || W.C12 >= 0.0);
    const int m = (s0 ? 1 : 0) | (s1 ? 2 : 0) | (s2 ? 4 : 0);
    int last = (W.rem[0] == 1 ? 1 : 0) | (W.rem[1] == 1 ? 2 : 0) | (W.rem[2] == 1 ? 4 : 0);
    if (m & last & W.xit) return 0;  // this event leaves the box
    W.g[0] += s0 ? W.step[0] : 0;
    W.g[1] += s1 ? W.step[1] : 0;
    W.g[2] += s2 ? W.step[2] : 0;
    W.rem[0] -= s0 ? 1 : 0;
    W.rem[1] -= s1 ? 1 : 0;
    W.rem[2] -= s2 ? 1 : 0;
    W.C01 += (s0 ? W.K[1] : 0.0) - (s1 ? W.K[0] : 0.0);
    W.C02 += (s0 ? W.K[2] : 0.0) - (s2 ? W.K[0] : 0.0);
    W.C12 += (s1 ? W.K[2] : 0.0) - (s2 ? W.K[1] : 0.0);
    return m;
}

// The free-space segment [o, S] of a ray longer than tau (free-space
// carving), clipped to the box [lo, hi), walked voxel by voxel with the key
// each voxel receives. The distance numerator n = (q - c) . D falls by
// 1024 |D_a| at every step on axis a (each axis moves the way D points), from
// up to about 3 * 2^62 near the sensor to above -2^42 at S. It is carried
// modulo 2^64 as u = n - H + 2^50, H = tau r - floor(r / 2) the smallest n
// whose distance rounds to tau or more: u never wraps, u >= 2^50 means s =
// +tau without any division, and below that n = u - 2^50 + H is exact in
// float64 (|n| < 2^47).
struct FreeWalk {
    LongWalk W;
    uint64_t u, du[3];
    double Hd;
};
constexpr uint64_t kFreeBias = 1ull << 50;

// false when no voxel of the segment lies in the box.
__device__ __forceinline__ bool free_walk_init(const Ray &R, const RayParams &P, const int32_t lo[3],
                                               const int32_t hi[3], FreeWalk &F)
{
    int32_t c[3];
    if (!long_walk_init(P.o, R.S, lo, hi, F.W, c)) return false;
    const int64_t r = (int64_t)R.r;
    const int64_t H = (int64_t)P.tau * r - (r >> 1);
    F.u = kFreeBias - (uint64_t)H;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int64_t Da = (int64_t)R.D[a];
        F.u += (uint64_t)(((int64_t)R.q[a] - 1024 * (int64_t)F.W.g[a] - 512) * Da);
        F.du[a] = (uint64_t)(1024 * (Da < 0 ? -Da : Da));
    }
    F.Hd = (double)H;
    return true;
}

// Key of the current voxel for point i.
__device__ __forceinline__ uint64_t free_walk_key(const FreeWalk &F, const Ray &R, int32_t tau, uint32_t i)
{
    const int32_t s = F.u >= kFreeBias ? tau : voxel_sdf((double)(int64_t)(F.u - kFreeBias) + F.Hd, R, tau);
    return pack_key(s, i);
}

// Next voxel; false when the segment ends or leaves the box.
__device__ __forceinline__ bool free_walk_next(FreeWalk &F)
{
    const int m = long_walk_next(F.W);
    F.u -= ((m & 1) ? F.du[0] : 0) + ((m & 2) ? F.du[1] : 0) + ((m & 4) ? F.du[2] : 0);
    return m != 0;
}

}  // namespace tsdf
