"""Brute-force references for tiny inputs, in exact rational arithmetic.

These are independent of the oracle's algorithms: the voxel set of a segment
is found by testing every voxel of a small box for a non-empty parameter
interval (instead of walking events), the per-scan volume by a min over all
rays for every voxel, and the float64 transform by exact-rational emulation
of each fused multiply-add.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def fma_exact(a: float, b: float, c: float) -> float:
    """Correctly rounded a*b + c (one rounding), via exact rationals."""
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def quantise(p, M, scale):
    """Fixed-point world coordinates of a float32 point, or None if dropped."""
    x, y, z = (float(np.float32(v)) for v in p)
    if not all(np.isfinite([x, y, z])):
        return None
    q = []
    for a in range(3):
        w = fma_exact(M[a][0], x, fma_exact(M[a][1], y, fma_exact(M[a][2], z, M[a][3])))
        v = round(w * scale)  # Python rounds half to even
        if abs(v) >= 2 ** 30:
            return None
        q.append(int(v))
    return q


def round_half_away(fr: Fraction) -> int:
    """Nearest integer to a rational, ties away from zero."""
    a = abs(fr)
    k = int(a + Fraction(1, 2))  # floor(|x| + 1/2)
    return k if fr >= 0 else -k


def segment_voxels_brute(S, E, lo, hi):
    """Every voxel g in the box [lo, hi) that the closed segment S->E touches:
    exists t in [0,1] with 1024 g_a <= S_a + t L_a < 1024 (g_a + 1) for all a."""
    L = [E[a] - S[a] for a in range(3)]
    out = []
    for gx in range(lo[0], hi[0]):
        for gy in range(lo[1], hi[1]):
            for gz in range(lo[2], hi[2]):
                g = (gx, gy, gz)
                # interval bounds as (value, closed)
                lo_b, hi_b = (Fraction(0), True), (Fraction(1), True)
                empty = False
                for a in range(3):
                    b0, b1 = 1024 * g[a] - S[a], 1024 * (g[a] + 1) - S[a]  # need b0 <= t L < b1
                    if L[a] == 0:
                        if not (b0 <= 0 < b1):
                            empty = True
                        continue
                    if L[a] > 0:
                        cand_lo = (Fraction(b0, L[a]), True)
                        cand_hi = (Fraction(b1, L[a]), False)
                    else:
                        cand_lo = (Fraction(b1, L[a]), False)
                        cand_hi = (Fraction(b0, L[a]), True)
                    if cand_lo[0] > lo_b[0] or (cand_lo[0] == lo_b[0] and not cand_lo[1]):
                        lo_b = cand_lo
                    if cand_hi[0] < hi_b[0] or (cand_hi[0] == hi_b[0] and not cand_hi[1]):
                        hi_b = cand_hi
                if empty:
                    continue
                if lo_b[0] < hi_b[0] or (lo_b[0] == hi_b[0] and lo_b[1] and hi_b[1]):
                    out.append(g)
    return out


def isqrt_floor(n: int) -> int:
    """floor(sqrt(n)) by bisection on exact integers."""
    lo, hi = 0, 1
    while hi * hi <= n:
        hi *= 2
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if mid * mid <= n:
            lo = mid
        else:
            hi = mid
    return lo


def volume_brute(xyz, M, scale, tau_u, origin, dims, carve=False):
    """Per-scan candidate volume over a small window by brute force.

    For every voxel of the window and every ray, the ray contributes if its
    band segment touches the voxel (exact interval test); the voxel keeps the
    candidate with the smallest |s|, ties to the lowest point index. With
    carve, a ray longer than tau also reaches the voxels of the segment from
    the sensor to the start of its band. Returns a dict g -> (|s|, i, s)."""
    o = [round(M[a][3] * scale) for a in range(3)]
    lo = tuple(origin)
    hi = tuple(origin[a] + dims[a] for a in range(3))
    best = {}
    for i, p in enumerate(xyz):
        q = quantise(p, M, scale)
        if q is None:
            continue
        D = [q[a] - o[a] for a in range(3)]
        dd = sum(d * d for d in D)
        if dd == 0:
            continue
        r = isqrt_floor(dd)
        off = [round_half_away(Fraction(tau_u * D[a], r)) for a in range(3)]
        E = [q[a] + off[a] for a in range(3)]
        S = list(o) if r <= tau_u else [q[a] - off[a] for a in range(3)]
        touched = set(segment_voxels_brute(S, E, lo, hi))
        if carve and r > tau_u:
            touched |= set(segment_voxels_brute(o, S, lo, hi))
        for g in touched:
            c = [1024 * g[a] + 512 for a in range(3)]
            dot = sum((q[a] - c[a]) * D[a] for a in range(3))
            s = max(-tau_u, min(tau_u, round_half_away(Fraction(dot, r))))
            cand = (abs(s), i, s)
            if g not in best or cand < best[g]:
                best[g] = cand
    return best
