/*
 * TSDF oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded CPU implementation of the TSDF-mapping path
 * of FeatSense (Gaal et al., arXiv 2310.05766, Sec. VI "TSDF Map Generation").
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load it. It shares no code, header or constant with the GPU library.
 *
 * Build: gcc -O2 -ffp-contract=off -std=c11 -shared -fPIC (no fast-math), so
 * every floating-point operation below is exactly the IEEE operation written.
 *
 * What is computed (paper Sec. VI, readings of the paper's gaps are listed
 * with each function):
 *   1. each scan point is transformed to the world frame in float64 and
 *      rounded to global fixed point, 1/1024 of a voxel;
 *   2. the ray from the sensor position p to the point x is traversed across
 *      the truncation band around x (Sec. VI: voxels are filled while
 *      traversing the ray from p to x); as options, also from p to the start
 *      of the band (free-space carving, the traversal read literally), or
 *      with the vertical fill between scan lines (Sec. VI, Eq. (3), Eq. (4));
 *   3. per scan, each voxel keeps the smallest distance over all rays that
 *      reach it (Sec. VI: the per-scan volume V takes the smallest distance
 *      of all rays for each voxel);
 *   4. the per-scan volume is averaged into the global volume G with the
 *      weighted running average of Eq. (1) and the capped weight of Eq. (2);
 *   5. the local map is a window over G that shifts after a movement
 *      threshold; voxels leaving it are written to a store and voxels
 *      entering it are loaded back (Sec. I, HATSDF's local-map shift, and the
 *      ring-buffer swapping of Kintinuous cited in Sec. II).
 *
 * Parity pins for every function live in tests/ (closed forms, brute force,
 * invariants); nothing here is checked against itself.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOMEM (-2)

#define KEY_EMPTY UINT64_MAX
#define CHUNK 64

/* ------------------------------------------------------------------ */
/* integer helpers                                                     */
/* ------------------------------------------------------------------ */

/* Rounded division n/d for d > 0, to nearest, ties away from zero. Used for
 * every division of the method (the paper leaves rounding unspecified). */
int64_t or_rdiv(int64_t n, int64_t d)
{
    int64_t a = n < 0 ? -n : n;
    int64_t q = (2 * a + d) / (2 * d);
    return n < 0 ? -q : q;
}

/* floor(sqrt(n)), exact for every 64-bit n: bit-by-bit square root. */
uint64_t or_isqrt(uint64_t n)
{
    uint64_t res = 0;
    uint64_t bit = (uint64_t)1 << 62;
    while (bit > n) bit >>= 2;
    while (bit != 0) {
        if (n >= res + bit) {
            n -= res + bit;
            res = (res >> 1) + bit;
        } else {
            res >>= 1;
        }
        bit >>= 2;
    }
    return res;
}

/* floor(a / b) for b > 0 */
static int64_t floor_div(int64_t a, int64_t b)
{
    int64_t q = a / b;
    if ((a % b != 0) && (a < 0)) q -= 1;
    return q;
}

static int64_t floor_mod(int64_t a, int64_t b) { return a - floor_div(a, b) * b; }

static __int128 floor_div128(__int128 a, __int128 b)
{
    __int128 q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0))) q -= 1;
    return q;
}

/* ------------------------------------------------------------------ */
/* step 1: world transform and quantisation                            */
/* ------------------------------------------------------------------ */

/* Point (x,y,z) in the sensor frame -> world coordinate row a of the row-major
 * 4x4 world_T_sensor M, as one fixed chain of fused multiply-adds:
 *   w_a = fma(M[a][0], x, fma(M[a][1], y, fma(M[a][2], z, M[a][3]))).
 * Then q_a = round-half-even(w_a * scale), scale = 1024 / voxel_size.
 * Returns 1 if the point is kept: finite coordinates and |q_a| < 2^30. */
int or_quantise_point(const float p[3], const double M[16], double scale, int64_t q[3])
{
    if (!isfinite(p[0]) || !isfinite(p[1]) || !isfinite(p[2])) return 0;
    double x = (double)p[0], y = (double)p[1], z = (double)p[2];
    for (int a = 0; a < 3; ++a) {
        double w = fma(M[4 * a + 0], x, fma(M[4 * a + 1], y, fma(M[4 * a + 2], z, M[4 * a + 3])));
        double r = nearbyint(w * scale);
        if (!(fabs(r) < 1073741824.0)) return 0;
        q[a] = (int64_t)r;
    }
    return 1;
}

/* Sensor position: o_a = round-half-even(M[a][3] * scale). Returns 0 when the
 * position is not representable (|o_a| >= 2^30 or non-finite). */
int or_quantise_origin(const double M[16], double scale, int64_t o[3])
{
    for (int a = 0; a < 3; ++a) {
        double r = nearbyint(M[4 * a + 3] * scale);
        if (!(fabs(r) < 1073741824.0)) return 0;
        o[a] = (int64_t)r;
    }
    return 1;
}

/* ------------------------------------------------------------------ */
/* step 2: the band around the scan point                               */
/* ------------------------------------------------------------------ */

/* D = q - o, r = isqrt(|D|^2), off = rdiv(tau*D, r), E = q + off and
 * S = q - off, or S = o when the point is within tau of the sensor.
 * Returns 0 for D = 0 (no ray). */
int or_band(const int64_t q[3], const int64_t o[3], int64_t tau_u,
            int64_t D[3], uint64_t *r_out, int64_t S[3], int64_t E[3])
{
    uint64_t dd = 0;
    for (int a = 0; a < 3; ++a) {
        D[a] = q[a] - o[a];
        dd += (uint64_t)(D[a] * D[a]);
    }
    if (dd == 0) return 0;
    uint64_t r = or_isqrt(dd);
    for (int a = 0; a < 3; ++a) {
        int64_t off = or_rdiv(tau_u * D[a], (int64_t)r);
        E[a] = q[a] + off;
        S[a] = ((int64_t)r <= tau_u) ? o[a] : q[a] - off;
    }
    *r_out = r;
    return 1;
}

/* ------------------------------------------------------------------ */
/* step 3: the set of voxels the closed segment [S, E] touches          */
/* ------------------------------------------------------------------ */

typedef struct { int64_t num, den; } frac; /* den > 0 */

static int frac_cmp(const void *pa, const void *pb)
{
    const frac *a = (const frac *)pa, *b = (const frac *)pb;
    __int128 l = (__int128)a->num * b->den, r = (__int128)b->num * a->den;
    return (l > r) - (l < r);
}

/* Voxel of P(t) = S + t (E - S) at rational t = num/den (den > 0), under
 * half-open ownership [k*1024, (k+1)*1024). */
static void voxel_at(const int64_t S[3], const int64_t L[3], __int128 num, __int128 den, int64_t g[3])
{
    for (int a = 0; a < 3; ++a)
        g[a] = (int64_t)floor_div128((__int128)S[a] * den + num * L[a], den * 1024);
}

/* Writes every voxel of { floor(P(t)/1024) : t in [0,1] } to out (as xyz
 * triples, in increasing t) and returns how many there are, or -1 if more
 * than max. The set is evaluated by its definition: P(t)/1024 changes voxel
 * only at times where a coordinate reaches a multiple of 1024, so the set is
 * the voxels at t = 0, t = 1, at every such time, and at one time strictly
 * inside each interval between consecutive such times. */
int or_segment_voxels(const int64_t S[3], const int64_t E[3], int64_t *out, int max)
{
    int64_t L[3] = {E[0] - S[0], E[1] - S[1], E[2] - S[2]};
    /* event times: all t in [0,1] where S_a + t L_a is a multiple of 1024 */
    int cap = 8;
    for (int a = 0; a < 3; ++a) cap += (int)((L[a] < 0 ? -L[a] : L[a]) / 1024) + 2;
    frac *ev = (frac *)malloc(sizeof(frac) * (size_t)cap);
    if (!ev) return -1;
    int ne = 0;
    ev[ne++] = (frac){0, 1};
    ev[ne++] = (frac){1, 1};
    for (int a = 0; a < 3; ++a) {
        if (L[a] == 0) continue;
        int64_t lo = S[a] < E[a] ? S[a] : E[a];
        int64_t hi = S[a] < E[a] ? E[a] : S[a];
        int64_t k0 = floor_div(lo + 1023, 1024); /* smallest multiple >= lo */
        for (int64_t k = k0; k * 1024 <= hi; ++k) {
            int64_t num = k * 1024 - S[a];
            int64_t den = L[a];
            if (den < 0) { num = -num; den = -den; }
            ev[ne++] = (frac){num, den};
        }
    }
    qsort(ev, (size_t)ne, sizeof(frac), frac_cmp);

    int n = 0;
    int64_t g[3], prev[3] = {0, 0, 0};
    int have = 0;
    for (int i = 0; i < ne; ++i) {
        /* the event time itself */
        for (int pass = 0; pass < 2; ++pass) {
            __int128 num, den;
            if (pass == 0) {
                num = ev[i].num;
                den = ev[i].den;
            } else {
                if (i + 1 >= ne) break;
                if (frac_cmp(&ev[i], &ev[i + 1]) == 0) continue;
                /* midpoint of (ev[i], ev[i+1]) */
                num = (__int128)ev[i].num * ev[i + 1].den + (__int128)ev[i + 1].num * ev[i].den;
                den = (__int128)2 * ev[i].den * ev[i + 1].den;
            }
            voxel_at(S, L, num, den, g);
            if (have && g[0] == prev[0] && g[1] == prev[1] && g[2] == prev[2]) continue;
            if (n >= max) { free(ev); return -1; }
            out[3 * n + 0] = g[0];
            out[3 * n + 1] = g[1];
            out[3 * n + 2] = g[2];
            prev[0] = g[0]; prev[1] = g[1]; prev[2] = g[2];
            have = 1;
            ++n;
        }
    }
    free(ev);
    return n;
}

/* ------------------------------------------------------------------ */
/* step 4: the signed distance a voxel receives, and its candidate key  */
/* ------------------------------------------------------------------ */

/* s = clamp(rdiv((q - c) . D, r), -tau, +tau) with c the voxel centre in
 * fixed point (c = 1024 g + 512): the voxel centre projected onto the ray
 * and measured from the scan point, positive on the sensor side. The dot
 * product is formed in 128 bits: for a voxel near the sensor of a long ray
 * (free-space carving) it reaches about 3 * 2^62. */
int64_t or_voxel_sdf(const int64_t q[3], const int64_t D[3], uint64_t r, const int64_t g[3], int64_t tau_u)
{
    __int128 dot = 0;
    for (int a = 0; a < 3; ++a) dot += (__int128)(q[a] - (1024 * g[a] + 512)) * D[a];
    /* rdiv in 128 bits: sign(dot) floor((2 |dot| + r) / 2r) */
    const __int128 mag = dot < 0 ? -dot : dot;
    const __int128 k = (2 * mag + (__int128)r) / (2 * (__int128)r);
    __int128 s = dot < 0 ? -k : k;
    if (s > tau_u) s = tau_u;
    if (s < -tau_u) s = -tau_u;
    return (int64_t)s;
}

/* key = |s| << 48 | i << 16 | (uint16)s. The smallest key of a voxel is the
 * candidate with the smallest |s|, ties to the lowest point index. */
uint64_t or_key(int64_t s, uint64_t i)
{
    uint64_t as = (uint64_t)(s < 0 ? -s : s);
    return (as << 48) | ((i & 0xffffffffULL) << 16) | (uint64_t)(uint16_t)(int16_t)s;
}

/* ------------------------------------------------------------------ */
/* vertical interpolation between scan lines (Sec. VI, Eq. (3), Eq. (4)) */
/* ------------------------------------------------------------------ */

/* Eq. (3): delta_z = tan(rad(vfov / hlines)), vfov in degrees (reading: the
 * angle between neighbouring scan lines, converted to radians), as a fixed-
 * point integer in 1/2^20 units; 0 for an invalid sensor description or an
 * angle of 45 degrees or more (delta_z >= 1). */
int64_t or_interp_delta(double vfov_deg, int32_t hlines)
{
    if (!(vfov_deg > 0.0) || !isfinite(vfov_deg) || hlines < 1) return 0;
    const double angle_deg = vfov_deg / (double)hlines; /* between neighbouring lines */
    if (!(angle_deg < 45.0)) return 0;
    return (int64_t)llrint(tan(angle_deg * (M_PI / 180.0)) * 1048576.0);
}

/* The sensor's up vector (its z axis in the world frame, column 2 of the
 * pose's rotation) in 1/1024 units, rounded half to even. */
void or_up_vector(const double M[16], int64_t U[3])
{
    for (int a = 0; a < 3; ++a) U[a] = (int64_t)llrint(M[4 * a + 2] * 1024.0);
}

/* out = a x b, component k = a[k+1] b[k+2] - a[k+2] b[k+1] (indices mod 3) */
static void cross3(const int64_t a[3], const int64_t b[3], int64_t out[3])
{
    for (int k = 0; k < 3; ++k) {
        const int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
        out[k] = a[k1] * b[k2] - a[k2] * b[k1];
    }
}

/* The fill offset e of one band voxel g of a ray (q, D, r): the paper fills
 * the voxels along the interpolation vector int = d x (d x up), scaled to
 * h = delta_z * len (Eq. (4)), above and below the ray. Readings, all in
 * exact integers:
 *   d  = rdiv(1024 D, r)                 (the ray direction, |d| ~ 1024)
 *   int = d x (d x U)                    (U: up vector in 1/1024 units)
 *   len = rdiv((c - o) . D, r)           (distance of the voxel centre c
 *                                          along the ray, fixed point)
 *   h  = min(rdiv(dq len, 2^20), 65535) if len > 0, else 0
 *   e  = rdiv(h int, |int|), |int| = isqrt(int . int); e = 0 if |int| = 0
 * The fill height is capped at 64 voxels (65535 in 1/1024 units), and rays
 * of r >= 2^30 get no fill (e = 0). The filled voxels are the floor-set of
 * the closed segment [c - e, c + e]. */
void or_fill_offset(const int64_t q[3], const int64_t o[3], const int64_t D[3], uint64_t r, const int64_t U[3],
                    const int64_t g[3], int64_t dq, int64_t e[3])
{
    e[0] = e[1] = e[2] = 0;
    if (dq <= 0 || r == 0 || r >= ((uint64_t)1 << 30)) return;
    const int64_t rr = (int64_t)r;
    int64_t d[3], w[3], v[3];
    for (int a = 0; a < 3; ++a) d[a] = or_rdiv(1024 * D[a], rr);
    cross3(d, U, w); /* d x up */
    cross3(d, w, v); /* d x (d x up) */
    const int64_t nv = (int64_t)or_isqrt((uint64_t)(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]));
    if (nv == 0) return;
    int64_t proj = 0; /* (c - o) . D */
    for (int a = 0; a < 3; ++a) proj += (1024 * g[a] + 512 - o[a]) * D[a];
    const int64_t len = or_rdiv(proj, rr);
    if (len <= 0) return;
    int64_t h = or_rdiv(dq * len, (int64_t)1 << 20);
    if (h > 65535) h = 65535;
    for (int a = 0; a < 3; ++a) e[a] = or_rdiv(h * v[a], nv);
}

/* ------------------------------------------------------------------ */
/* map: window over the global volume G, plus the store of what left it */
/* ------------------------------------------------------------------ */

typedef struct {
    int64_t key[3];
    int16_t *sdf, *w; /* CHUNK^3 each, [x][y][z] z fastest */
} chunk_t;

typedef struct omap_s {
    int32_t dims[3];
    int32_t origin[3];
    double voxel_size, scale;
    int64_t tau_u, w_max;
    int64_t interp_dq; /* vertical interpolation: delta_z in 1/2^20 units, 0 = off */
    int carve;         /* free-space carving: every ray is walked from the sensor */
    int64_t nvox;
    int16_t *sdf, *w; /* resident window, slot = floor_mod(g, dims) */
    uint64_t *K;      /* per-scan volume V as candidate keys, EMPTY = none */
    int64_t *touched; /* slots whose key left EMPTY during the current scan */
    int64_t ntouched;
    /* store: open-addressing hash of chunks keyed by floor_div(g, CHUNK) */
    chunk_t *tab;
    int64_t tab_cap, tab_n;
    int64_t last_hit; /* index of the last chunk found, or -1 */
} omap;

static chunk_t *store_find_slow(struct omap_s *m, const int64_t k[3], int create);

static int64_t slot_of(const omap *m, const int64_t g[3])
{
    int64_t sx = floor_mod(g[0], m->dims[0]);
    int64_t sy = floor_mod(g[1], m->dims[1]);
    int64_t sz = floor_mod(g[2], m->dims[2]);
    return (sx * m->dims[1] + sy) * m->dims[2] + sz;
}

static int in_window(const int32_t origin[3], const int32_t dims[3], const int64_t g[3])
{
    for (int a = 0; a < 3; ++a)
        if (g[a] < origin[a] || g[a] >= (int64_t)origin[a] + dims[a]) return 0;
    return 1;
}

/* Bucket of a chunk key: the spatial hash of Teschner et al. (2003,
 * "Optimized Spatial Hashing for Collision Detection of Deformable Objects"):
 * the xor of the coordinates times three large primes. It only places chunks
 * in the open-addressing table; no voxel value depends on it. */
static uint64_t hash3(const int64_t k[3])
{
    return ((uint64_t)k[0] * 73856093u) ^ ((uint64_t)k[1] * 19349663u) ^ ((uint64_t)k[2] * 83492791u);
}

static chunk_t *store_find(omap *m, const int64_t k[3], int create)
{
    if (m->last_hit >= 0) {
        chunk_t *c = &m->tab[m->last_hit];
        if (c->key[0] == k[0] && c->key[1] == k[1] && c->key[2] == k[2]) return c;
    }
    chunk_t *c = store_find_slow(m, k, create);
    m->last_hit = c ? (int64_t)(c - m->tab) : -1;
    return c;
}

static chunk_t *store_find_slow(omap *m, const int64_t k[3], int create)
{
    if (create && (m->tab_n + 1) * 2 > m->tab_cap) {
        int64_t ncap = m->tab_cap ? m->tab_cap * 2 : 1024;
        chunk_t *nt = (chunk_t *)calloc((size_t)ncap, sizeof(chunk_t));
        if (!nt) return NULL;
        for (int64_t i = 0; i < m->tab_cap; ++i) {
            if (!m->tab[i].sdf) continue;
            uint64_t h = hash3(m->tab[i].key) & (uint64_t)(ncap - 1);
            while (nt[h].sdf) h = (h + 1) & (uint64_t)(ncap - 1);
            nt[h] = m->tab[i];
        }
        free(m->tab);
        m->tab = nt;
        m->tab_cap = ncap;
    }
    if (m->tab_cap == 0) return NULL;
    uint64_t h = hash3(k) & (uint64_t)(m->tab_cap - 1);
    while (m->tab[h].sdf) {
        if (m->tab[h].key[0] == k[0] && m->tab[h].key[1] == k[1] && m->tab[h].key[2] == k[2]) return &m->tab[h];
        h = (h + 1) & (uint64_t)(m->tab_cap - 1);
    }
    if (!create) return NULL;
    chunk_t *c = &m->tab[h];
    c->sdf = (int16_t *)calloc(CHUNK * CHUNK * CHUNK, sizeof(int16_t));
    c->w = (int16_t *)calloc(CHUNK * CHUNK * CHUNK, sizeof(int16_t));
    if (!c->sdf || !c->w) return NULL;
    c->key[0] = k[0]; c->key[1] = k[1]; c->key[2] = k[2];
    m->tab_n++;
    return c;
}

static int64_t chunk_index(const int64_t g[3])
{
    return (floor_mod(g[0], CHUNK) * CHUNK + floor_mod(g[1], CHUNK)) * CHUNK + floor_mod(g[2], CHUNK);
}

static void chunk_key(const int64_t g[3], int64_t k[3])
{
    for (int a = 0; a < 3; ++a) k[a] = floor_div(g[a], CHUNK);
}

/* store[g] = (sdf, w) */
static int store_put(omap *m, const int64_t g[3], int16_t sdf, int16_t w)
{
    int64_t k[3];
    chunk_key(g, k);
    chunk_t *c = store_find(m, k, sdf != 0 || w != 0);
    if (!c) return (sdf == 0 && w == 0) ? OR_OK : OR_ENOMEM;
    int64_t i = chunk_index(g);
    c->sdf[i] = sdf;
    c->w[i] = w;
    return OR_OK;
}

/* (sdf, w) = store.pop(g, (0, 0)); a popped voxel reads (0, 0) afterwards */
static void store_pop(omap *m, const int64_t g[3], int16_t *sdf, int16_t *w, int pop)
{
    int64_t k[3];
    chunk_key(g, k);
    chunk_t *c = store_find(m, k, 0);
    if (!c) { *sdf = 0; *w = 0; return; }
    int64_t i = chunk_index(g);
    *sdf = c->sdf[i];
    *w = c->w[i];
    if (pop) { c->sdf[i] = 0; c->w[i] = 0; }
}

omap *or_map_create(const int32_t dims[3], const int32_t origin[3], double voxel_size,
                    int32_t tau_u, int32_t w_max)
{
    for (int a = 0; a < 3; ++a)
        if (dims[a] < 1) return NULL;
    if (!(voxel_size > 0) || tau_u < 1 || tau_u > 32767 || w_max < 1 || w_max > 32767) return NULL;
    omap *m = (omap *)calloc(1, sizeof(omap));
    if (!m) return NULL;
    memcpy(m->dims, dims, sizeof(m->dims));
    memcpy(m->origin, origin, sizeof(m->origin));
    m->voxel_size = voxel_size;
    m->scale = 1024.0 / voxel_size;
    m->tau_u = tau_u;
    m->w_max = w_max;
    m->nvox = (int64_t)dims[0] * dims[1] * dims[2];
    m->last_hit = -1;
    m->sdf = (int16_t *)calloc((size_t)m->nvox, sizeof(int16_t));
    m->w = (int16_t *)calloc((size_t)m->nvox, sizeof(int16_t));
    m->K = (uint64_t *)malloc((size_t)m->nvox * sizeof(uint64_t));
    m->touched = (int64_t *)malloc((size_t)m->nvox * sizeof(int64_t));
    if (!m->sdf || !m->w || !m->K || !m->touched) {
        free(m->sdf); free(m->w); free(m->K); free(m->touched); free(m);
        return NULL;
    }
    for (int64_t i = 0; i < m->nvox; ++i) m->K[i] = KEY_EMPTY;
    return m;
}

void or_map_destroy(omap *m)
{
    if (!m) return;
    for (int64_t i = 0; i < m->tab_cap; ++i) {
        free(m->tab[i].sdf);
        free(m->tab[i].w);
    }
    free(m->tab);
    free(m->sdf); free(m->w); free(m->K); free(m->touched);
    free(m);
}

/* Per-scan volume V (candidates only, no merge): for every point i with a
 * ray, for every voxel g of its band segment inside the window,
 * K[g] = min(K[g], key(s, i)). stats: points_valid, visits. */
static int build_volume(omap *m, const float *xyz, int64_t n, const double M[16], const int64_t *order,
                        int64_t *valid, int64_t *visits)
{
    int64_t o[3];
    if (!or_quantise_origin(M, m->scale, o)) return OR_EINVAL;
    int64_t cap = 4096;
    int64_t *vox = (int64_t *)malloc(sizeof(int64_t) * 3 * (size_t)cap);
    if (!vox) return OR_ENOMEM;
    const int64_t fcap = 4096; /* a fill segment spans at most 2 * 64 voxels per axis */
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * 3 * (size_t)fcap);
    if (!fill) { free(vox); return OR_ENOMEM; }
    int64_t U[3];
    or_up_vector(M, U);
    *valid = 0;
    *visits = 0;
    for (int64_t k = 0; k < n; ++k) {
        /* point i keeps its index (its row) whatever order the points are
         * taken in: the per-voxel minimum of Sec. VI does not depend on it */
        const int64_t i = order ? order[k] : k;
        int64_t q[3], D[3], S[3], E[3];
        uint64_t r;
        if (!or_quantise_point(&xyz[3 * i], M, m->scale, q)) continue;
        if (!or_band(q, o, m->tau_u, D, &r, S, E)) continue;
        (*valid)++;
        /* the band [S, E]; with free-space carving (rays longer than tau)
         * first the free-space segment [o, S] from the sensor to the start
         * of the band, whose voxels receive this ray's distance the same way
         * (the ray traversed from p towards the point). Visits count both
         * segments, so the voxel where they meet counts twice. */
        const int nseg = (m->carve && (int64_t)r > m->tau_u) ? 2 : 1;
        for (int sg = 0; sg < nseg; ++sg) {
            const int64_t *A0 = (nseg == 2 && sg == 0) ? o : S;
            const int64_t *A1 = (nseg == 2 && sg == 0) ? S : E;
            /* a segment touches at most 1 + sum_a (|L_a| / 1024 + 1) voxels */
            int64_t need = 4;
            for (int a = 0; a < 3; ++a) need += (A1[a] > A0[a] ? A1[a] - A0[a] : A0[a] - A1[a]) / 1024 + 1;
            if (need > cap) {
                if (need > ((int64_t)1 << 30)) { free(vox); free(fill); return OR_ENOMEM; }
                int64_t *nvx = (int64_t *)realloc(vox, sizeof(int64_t) * 3 * (size_t)need);
                if (!nvx) { free(vox); free(fill); return OR_ENOMEM; }
                vox = nvx;
                cap = need;
            }
            int nv = or_segment_voxels(A0, A1, vox, (int)cap);
            if (nv < 0) { free(vox); free(fill); return OR_ENOMEM; }
            for (int k = 0; k < nv; ++k) {
                int64_t *g = &vox[3 * k];
                int64_t s = or_voxel_sdf(q, D, r, g, m->tau_u);
                uint64_t key = or_key(s, (uint64_t)i);
                /* the voxels this band voxel gives its value to: itself, or with
                 * vertical interpolation the floor-set of [c - e, c + e] (a band
                 * voxel outside the window may still fill voxels inside it) */
                int nf = 1;
                const int64_t *fv = g;
                if (m->interp_dq > 0) {
                    int64_t e[3], A[3], Bv[3];
                    or_fill_offset(q, o, D, r, U, g, m->interp_dq, e);
                    for (int a = 0; a < 3; ++a) {
                        A[a] = 1024 * g[a] + 512 - e[a];
                        Bv[a] = 1024 * g[a] + 512 + e[a];
                    }
                    nf = or_segment_voxels(A, Bv, fill, (int)fcap);
                    if (nf < 0) { free(vox); free(fill); return OR_ENOMEM; }
                    fv = fill;
                }
                for (int f = 0; f < nf; ++f) {
                    const int64_t *gf = &fv[3 * f];
                    if (!in_window(m->origin, m->dims, gf)) continue;
                    (*visits)++;
                    int64_t sl = slot_of(m, gf);
                    if (m->K[sl] == KEY_EMPTY) m->touched[m->ntouched++] = sl;
                    if (key < m->K[sl]) m->K[sl] = key;
                }
            }
        }
    }
    free(vox);
    free(fill);
    return OR_OK;
}

/* Eq. (1) and Eq. (2) with v.weight = 1 per scan:
 *   g.value  = rdiv(g.value * g.weight + v.value, g.weight + 1)
 *   g.weight = min(w_max, g.weight + 1)
 * applied to every voxel that V holds a value for; V is then emptied.
 * (Each voxel's update is independent of the others, so visiting the
 * touched voxels in any order gives the same map.) */
static int64_t merge_volume(omap *m)
{
    int64_t U = 0;
    for (int64_t t = 0; t < m->ntouched; ++t) {
        int64_t sl = m->touched[t];
        uint64_t key = m->K[sl];
        int64_t v = (int64_t)(int16_t)(uint16_t)(key & 0xffff);
        int64_t gw = m->w[sl];
        int64_t gv = m->sdf[sl];
        m->sdf[sl] = (int16_t)or_rdiv(gv * gw + v, gw + 1);
        m->w[sl] = (int16_t)(gw + 1 < m->w_max ? gw + 1 : m->w_max);
        m->K[sl] = KEY_EMPTY;
        ++U;
    }
    m->ntouched = 0;
    return U;
}

/* Vertical interpolation for the following scans: dq = delta_z in 1/2^20
 * units (or_interp_delta), 0 to turn it off. */
int or_set_interpolation(omap *m, int64_t dq)
{
    if (!m || dq < 0 || dq >= ((int64_t)1 << 20)) return OR_EINVAL;
    if (dq > 0 && m->carve) return OR_EINVAL; /* not together with carving */
    m->interp_dq = dq;
    return OR_OK;
}

/* Free-space carving for the following scans (on = 1; Sec. VI, the ray
 * traversed from the sensor position p to the point x): each ray longer than
 * tau also walks the segment [o, S] from the sensor position to the start
 * of its band, so the voxels in front of the surface receive their (mostly
 * truncated, +tau) distance as well; the band is unchanged. Not together
 * with vertical interpolation. */
int or_set_carving(omap *m, int on)
{
    if (!m || (on != 0 && on != 1)) return OR_EINVAL;
    if (on && m->interp_dq > 0) return OR_EINVAL;
    m->carve = on;
    return OR_OK;
}

/* stats[4] = points_in, points_valid, visits, voxels_updated */
int or_integrate(omap *m, const float *xyz, int64_t n, const double M[16], int64_t *stats)
{
    if (!m || n < 0 || (n > 0 && !xyz) || !M) return OR_EINVAL;
    if (n > 0xffffffffLL) return OR_EINVAL;
    for (int k = 0; k < 12; ++k)
        if (!isfinite(M[k])) return OR_EINVAL;
    int64_t o[3];
    if (!or_quantise_origin(M, m->scale, o)) return OR_EINVAL;
    int64_t valid = 0, visits = 0;
    int rc = build_volume(m, xyz, n, M, NULL, &valid, &visits);
    if (rc != OR_OK) return rc;
    int64_t U = merge_volume(m);
    if (stats) {
        stats[0] = n;
        stats[1] = valid;
        stats[2] = visits;
        stats[3] = U;
    }
    return OR_OK;
}

/* The per-scan volume V alone, as keys over the window in slot order
 * (EMPTY where no ray reached), without touching the map. order (nullable):
 * a permutation of 0..n-1, the order in which the points are taken; each
 * point keeps its row as its index. */
int or_volume(omap *m, const float *xyz, int64_t n, const double M[16], const int64_t *order, uint64_t *keys_out)
{
    if (!m || n < 0 || !M || !keys_out) return OR_EINVAL;
    if (order) {
        /* a permutation: every row exactly once */
        unsigned char *seen = (unsigned char *)calloc((size_t)(n > 0 ? n : 1), 1);
        if (!seen) return OR_ENOMEM;
        for (int64_t k = 0; k < n; ++k) {
            if (order[k] < 0 || order[k] >= n || seen[order[k]]) { free(seen); return OR_EINVAL; }
            seen[order[k]] = 1;
        }
        free(seen);
    }
    int64_t valid, visits;
    int rc = build_volume(m, xyz, n, M, order, &valid, &visits);
    if (rc != OR_OK) return rc;
    memcpy(keys_out, m->K, (size_t)m->nvox * sizeof(uint64_t));
    for (int64_t t = 0; t < m->ntouched; ++t) m->K[m->touched[t]] = KEY_EMPTY;
    m->ntouched = 0;
    return OR_OK;
}

/* Move the window to new_origin. Every voxel leaving the window is written
 * to the store and its slot cleared; every voxel entering it is taken from
 * the store, or (0, 0) if the store has none. Slot addressing floor_mod(g, n)
 * means a voxel that stays never moves. */
int or_shift(omap *m, const int32_t new_origin[3])
{
    if (!m || !new_origin) return OR_EINVAL;
    /* changed[a][s]: the voxel held by slot coordinate s on axis a differs
     * between the two windows. A slot whose three coordinates are all
     * unchanged holds the same voxel before and after, so it is skipped. */
    uint8_t *changed[3];
    int64_t *zlist = (int64_t *)malloc(sizeof(int64_t) * (size_t)m->dims[2]);
    int64_t nz_changed = 0;
    for (int a = 0; a < 3; ++a) {
        changed[a] = (uint8_t *)malloc((size_t)m->dims[a]);
        for (int64_t v = 0; v < m->dims[a]; ++v)
            changed[a][v] = (m->origin[a] + floor_mod(v - m->origin[a], m->dims[a])) !=
                            (new_origin[a] + floor_mod(v - new_origin[a], m->dims[a]));
    }
    for (int64_t v = 0; v < m->dims[2]; ++v)
        if (changed[2][v]) zlist[nz_changed++] = v;
    int rc = OR_OK;
    for (int64_t sx = 0; sx < m->dims[0] && rc == OR_OK; ++sx)
        for (int64_t sy = 0; sy < m->dims[1] && rc == OR_OK; ++sy) {
            const int all_z = changed[0][sx] || changed[1][sy];
            const int64_t count = all_z ? m->dims[2] : nz_changed;
            for (int64_t iz = 0; iz < count; ++iz) {
                const int64_t sz = all_z ? iz : zlist[iz];
                int64_t s[3] = {sx, sy, sz};
                int64_t g_old[3], g_new[3];
                for (int a = 0; a < 3; ++a) {
                    /* the unique g = s (mod n) inside [origin, origin + n) */
                    g_old[a] = m->origin[a] + floor_mod(s[a] - m->origin[a], m->dims[a]);
                    g_new[a] = new_origin[a] + floor_mod(s[a] - new_origin[a], m->dims[a]);
                }
                if (g_old[0] == g_new[0] && g_old[1] == g_new[1] && g_old[2] == g_new[2]) continue;
                int64_t sl = (sx * m->dims[1] + sy) * m->dims[2] + sz;
                if (store_put(m, g_old, m->sdf[sl], m->w[sl]) != OR_OK) { rc = OR_ENOMEM; break; }
                store_pop(m, g_new, &m->sdf[sl], &m->w[sl], 1);
            }
        }
    for (int a = 0; a < 3; ++a) free(changed[a]);
    free(zlist);
    if (rc != OR_OK) return rc;
    memcpy(m->origin, new_origin, sizeof(m->origin));
    return OR_OK;
}

/* Global box [lo, hi) in C order [x][y][z]: resident value, else stored
 * value, else (0, 0). */
int or_readback(omap *m, const int32_t lo[3], const int32_t hi[3], int16_t *sdf, int16_t *w)
{
    if (!m || !lo || !hi || !sdf || !w) return OR_EINVAL;
    for (int a = 0; a < 3; ++a)
        if (hi[a] < lo[a]) return OR_EINVAL;
    int64_t ny = hi[1] - lo[1], nz = hi[2] - lo[2];
    for (int64_t x = lo[0]; x < hi[0]; ++x)
        for (int64_t y = lo[1]; y < hi[1]; ++y)
            for (int64_t z = lo[2]; z < hi[2]; ++z) {
                int64_t g[3] = {x, y, z};
                int64_t o = ((x - lo[0]) * ny + (y - lo[1])) * nz + (z - lo[2]);
                if (in_window(m->origin, m->dims, g)) {
                    int64_t sl = slot_of(m, g);
                    sdf[o] = m->sdf[sl];
                    w[o] = m->w[sl];
                } else {
                    store_pop(m, g, &sdf[o], &w[o], 0);
                }
            }
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* surface extraction for inspection: marching tetrahedra              */
/* ------------------------------------------------------------------ */

/* The zero level set of the resident window inside the box [lo, hi), as
 * triangles (9 floats each: three vertices, x y z in metres, world frame).
 * A cube is the 8 voxel centres g + {0,1}^3 with g and g + 1 in the box, all
 * observed (w > 0). It is cut into the 6 tetrahedra around its diagonal from
 * corner 0 to corner 7 (corner k = (k & 1, k >> 1 & 1, k >> 2 & 1)). In a
 * tetrahedron, a vertex is inside when its sdf is negative; one inside (or
 * one outside) vertex gives one triangle, two give two. An edge from
 * corner a to b crosses at t = s_a / (s_a - s_b), the point
 * (g_a + 1/2 + t (g_b - g_a)) voxel_size, in float64, then rounded to
 * float32. Output order: cubes by x, then y, then z; tetrahedra in the
 * order below; the triangles of a tetrahedron as listed below. Returns the
 * number of triangles (writing at most max_tris), or -1 for a bad box. */
static const int kTets[6][4] = {{0, 1, 3, 7}, {0, 3, 2, 7}, {0, 2, 6, 7}, {0, 6, 4, 7}, {0, 4, 5, 7}, {0, 5, 1, 7}};

static void edge_point(const int64_t g[3], int a, int b, const int64_t s[8], double vs, float *out)
{
    /* s_a - s_b is an exact integer (|s| < 2^15) */
    const double t = (double)s[a] / (double)(s[a] - s[b]);
    for (int k = 0; k < 3; ++k) {
        const int bit_a = (a >> k) & 1, bit_b = (b >> k) & 1;
        /* centre of corner a along axis k, and the edge's direction (-1, 0, 1) */
        const double centre_a = (double)g[k] + (double)bit_a + 0.5;
        const double dir = (double)(bit_b - bit_a);
        out[k] = (float)((centre_a + t * dir) * vs);
    }
}

int64_t or_mesh(omap *m, const int32_t lo[3], const int32_t hi[3], float *out, int64_t max_tris)
{
    if (!m || !lo || !hi) return -1;
    for (int a = 0; a < 3; ++a)
        if (hi[a] < lo[a] || lo[a] < m->origin[a] || hi[a] > (int64_t)m->origin[a] + m->dims[a]) return -1;
    int64_t n = 0;
    for (int64_t x = lo[0]; x + 1 < hi[0]; ++x)
        for (int64_t y = lo[1]; y + 1 < hi[1]; ++y)
            for (int64_t z = lo[2]; z + 1 < hi[2]; ++z) {
                const int64_t g[3] = {x, y, z};
                int64_t s[8];
                int seen = 1;
                for (int k = 0; k < 8 && seen; ++k) {
                    const int64_t c[3] = {x + (k & 1), y + ((k >> 1) & 1), z + ((k >> 2) & 1)};
                    const int64_t sl = slot_of(m, c);
                    if (m->w[sl] <= 0) seen = 0;
                    s[k] = m->sdf[sl];
                }
                if (!seen) continue;
                for (int t = 0; t < 6; ++t) {
                    const int *v = kTets[t];
                    int in[4], nin = 0;
                    for (int k = 0; k < 4; ++k) {
                        in[k] = s[v[k]] < 0;
                        nin += in[k];
                    }
                    if (nin % 4 == 0) continue; /* all inside or all outside: no surface */
                    float tri[2][9];
                    int ntri;
                    if (nin == 1 || nin == 3) {
                        /* the lone vertex: the only inside one (nin == 1) or
                         * the only outside one (nin == 3) */
                        const int lone_is_inside = nin == 1;
                        int lone = 0;
                        for (int k = 0; k < 4; ++k)
                            if (in[k] == lone_is_inside) lone = k;
                        int e = 0;
                        for (int k = 0; k < 4; ++k)
                            if (k != lone) edge_point(g, v[lone], v[k], s, m->voxel_size, &tri[0][3 * e++]);
                        ntri = 1;
                    } else {
                        /* two inside (ins[0] < ins[1]), two outside (outs[0] <
                         * outs[1]): the quad i0o0, i0o1, i1o1, i1o0 as the two
                         * triangles (i0o0, i0o1, i1o1) and (i0o0, i1o1, i1o0) */
                        int ins[2], outs[2], ni = 0, no = 0;
                        for (int k = 0; k < 4; ++k) {
                            if (in[k]) ins[ni++] = k;
                            else outs[no++] = k;
                        }
                        float p00[3], p01[3], p11[3], p10[3];
                        edge_point(g, v[ins[0]], v[outs[0]], s, m->voxel_size, p00);
                        edge_point(g, v[ins[0]], v[outs[1]], s, m->voxel_size, p01);
                        edge_point(g, v[ins[1]], v[outs[1]], s, m->voxel_size, p11);
                        edge_point(g, v[ins[1]], v[outs[0]], s, m->voxel_size, p10);
                        memcpy(&tri[0][0], p00, sizeof p00);
                        memcpy(&tri[0][3], p01, sizeof p01);
                        memcpy(&tri[0][6], p11, sizeof p11);
                        memcpy(&tri[1][0], p00, sizeof p00);
                        memcpy(&tri[1][3], p11, sizeof p11);
                        memcpy(&tri[1][6], p10, sizeof p10);
                        ntri = 2;
                    }
                    for (int k = 0; k < ntri; ++k) {
                        if (out && n < max_tris) memcpy(&out[9 * n], tri[k], 9 * sizeof(float));
                        ++n;
                    }
                }
            }
    return n;
}

/* ------------------------------------------------------------------ */
/* point-to-TSDF registration (the paper's stated next step, Sec. VIII; */
/* HATSDF registers scans directly in the TSDF, Sec. I)                  */
/* ------------------------------------------------------------------ */

/* Readings (the paper names the method, not its algorithm): a scan point p
 * under the pose (R, t) lands at w = R p + t (the fixed fma chain of the
 * integration, in metres). Its residual is the map's signed distance there,
 * phi(w) in metres, trilinear between the 8 voxel centres around w; the
 * point is used only when all 8 are resident, observed (weight > 0) and not
 * truncated (|sdf| < tau). Gauss-Newton on sum phi^2 with a left update
 * w' = R_d w + rho, R_d = exp([theta]x): the Jacobian row is
 * J = (grad phi, w x grad phi). */
int or_reg_point(omap *m, const float p[3], const double M[16], double *phi, double grad[3], double wout[3])
{
    if (!isfinite(p[0]) || !isfinite(p[1]) || !isfinite(p[2])) return 0;
    const double x = (double)p[0], y = (double)p[1], z = (double)p[2];
    double u[3], w[3];
    int64_t i0[3];
    double f[3];
    for (int a = 0; a < 3; ++a) {
        w[a] = fma(M[4 * a + 0], x, fma(M[4 * a + 1], y, fma(M[4 * a + 2], z, M[4 * a + 3])));
        u[a] = w[a] / m->voxel_size - 0.5;  /* voxel g's centre is at u = g */
        if (!(fabs(u[a]) < 1073741824.0)) return 0;
        const double fl = floor(u[a]);
        i0[a] = (int64_t)fl;
        f[a] = u[a] - fl;
    }
    double c[8];
    for (int k = 0; k < 8; ++k) {
        const int64_t g[3] = {i0[0] + (k & 1), i0[1] + ((k >> 1) & 1), i0[2] + ((k >> 2) & 1)};
        if (!in_window(m->origin, m->dims, g)) return 0;
        const int64_t sl = slot_of(m, g);
        if (m->w[sl] <= 0) return 0;
        const int64_t sq = m->sdf[sl];
        if (sq <= -m->tau_u || sq >= m->tau_u) return 0;
        c[k] = (double)sq * m->voxel_size / 1024.0; /* metres */
    }
    /* the trilinear interpolant by its definition: corner k has weight
     * prod_a (f_a if bit a of k is set, else 1 - f_a); its derivative along
     * axis b replaces factor b by +1 or -1 (per voxel, then per metre) */
    double val = 0.0, dval[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < 8; ++k) {
        double fac[3], dfac[3];
        for (int a = 0; a < 3; ++a) {
            const int bit = (k >> a) & 1;
            fac[a] = bit ? f[a] : 1.0 - f[a];
            dfac[a] = bit ? 1.0 : -1.0;
        }
        val += c[k] * (fac[0] * fac[1] * fac[2]);
        dval[0] += c[k] * (dfac[0] * fac[1] * fac[2]);
        dval[1] += c[k] * (fac[0] * dfac[1] * fac[2]);
        dval[2] += c[k] * (fac[0] * fac[1] * dfac[2]);
    }
    *phi = val;
    for (int a = 0; a < 3; ++a) grad[a] = dval[a] / m->voxel_size;
    for (int a = 0; a < 3; ++a) wout[a] = w[a];
    return 1;
}

/* Normal equations at a pose: sums[0..20] = H (upper triangle, row-major),
 * sums[21..26] = J^T r, sums[27] = sum r^2, sums[28] = points used. */
int or_reg_sums(omap *m, const float *xyz, int64_t n, const double M[16], double sums[29])
{
    if (!m || n < 0 || (n > 0 && !xyz) || !M || !sums) return OR_EINVAL;
    for (int k = 0; k < 29; ++k) sums[k] = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double phi, gr[3], w[3];
        if (!or_reg_point(m, &xyz[3 * i], M, &phi, gr, w)) continue;
        const double J[6] = {gr[0], gr[1], gr[2], w[1] * gr[2] - w[2] * gr[1], w[2] * gr[0] - w[0] * gr[2],
                             w[0] * gr[1] - w[1] * gr[0]};
        int k = 0;
        for (int a = 0; a < 6; ++a)
            for (int b = a; b < 6; ++b) sums[k++] += J[a] * J[b];
        for (int a = 0; a < 6; ++a) sums[21 + a] += J[a] * phi;
        sums[27] += phi * phi;
        sums[28] += 1.0;
    }
    return OR_OK;
}

/* One damped Gauss-Newton step from the sums: (H + lambda I) d = -J^T r by
 * Cholesky, then R' = exp([theta]x) R, t' = exp([theta]x) t + rho for
 * d = (rho, theta). Returns 0 when the system is not positive definite. */
int or_reg_step(const double sums[29], double lambda, const double M[16], double Mout[16], double d[6])
{
    double A[6][6], b[6];
    int k = 0;
    for (int a = 0; a < 6; ++a)
        for (int c = a; c < 6; ++c) A[a][c] = A[c][a] = sums[k++];
    for (int a = 0; a < 6; ++a) {
        A[a][a] += lambda;
        b[a] = -sums[21 + a];
    }
    double L[6][6] = {{0}};
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j <= i; ++j) {
            double acc = A[i][j];
            for (int q = 0; q < j; ++q) acc -= L[i][q] * L[j][q];
            if (i == j) {
                if (!(acc > 0.0)) return 0;
                L[i][i] = sqrt(acc);
            } else {
                L[i][j] = acc / L[j][j];
            }
        }
    double yv[6];
    for (int i = 0; i < 6; ++i) {
        double acc = b[i];
        for (int q = 0; q < i; ++q) acc -= L[i][q] * yv[q];
        yv[i] = acc / L[i][i];
    }
    for (int back = 0; back < 6; ++back) { /* rows 5, 4, ..., 0 */
        const int i = 5 - back;
        double acc = yv[i];
        for (int q = i + 1; q < 6; ++q) acc -= L[q][i] * d[q];
        d[i] = acc / L[i][i];
    }
    const double th[3] = {d[3], d[4], d[5]};
    const double an = sqrt(th[0] * th[0] + th[1] * th[1] + th[2] * th[2]);
    const double K[3][3] = {{0, -th[2], th[1]}, {th[2], 0, -th[0]}, {-th[1], th[0], 0}};
    double Rd[3][3];
    const double s1 = an > 1e-12 ? sin(an) / an : 1.0;
    const double s2 = an > 1e-12 ? (1.0 - cos(an)) / (an * an) : 0.5;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double kk = 0.0;
            for (int q = 0; q < 3; ++q) kk += K[i][q] * K[q][j];
            Rd[i][j] = (i == j ? 1.0 : 0.0) + s1 * K[i][j] + s2 * kk;
        }
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) {
            double acc = 0.0;
            for (int q = 0; q < 3; ++q) acc += Rd[i][q] * M[4 * q + j];
            Mout[4 * i + j] = acc;
        }
        double acc = d[i];
        for (int q = 0; q < 3; ++q) acc += Rd[i][q] * M[4 * q + 3];
        Mout[4 * i + 3] = acc;
    }
    Mout[12] = 0.0; Mout[13] = 0.0; Mout[14] = 0.0; Mout[15] = 1.0;
    return 1;
}

/* iterations damped Gauss-Newton steps from M0; info = {points used at the
 * last pose, cost at the last pose, norm of the last step, steps taken}. */
int or_register(omap *m, const float *xyz, int64_t n, const double M0[16], int32_t iterations, double lambda,
                double Mout[16], double info[4])
{
    if (!m || !M0 || !Mout || iterations < 0 || !(lambda >= 0.0)) return OR_EINVAL;
    double M[16], sums[29], d[6] = {0};
    memcpy(M, M0, sizeof(M));
    int32_t it = 0;
    double step = 0.0;
    for (; it < iterations; ++it) {
        or_reg_sums(m, xyz, n, M, sums);
        if (sums[28] < 6.0) break;
        double Mn[16];
        if (!or_reg_step(sums, lambda, M, Mn, d)) break;
        memcpy(M, Mn, sizeof(M));
        double ss = 0.0;
        for (int a = 0; a < 6; ++a) ss += d[a] * d[a];
        step = sqrt(ss);
    }
    or_reg_sums(m, xyz, n, M, sums);
    memcpy(Mout, M, sizeof(M));
    if (info) {
        info[0] = sums[28];
        info[1] = sums[27];
        info[2] = step;
        info[3] = it;
    }
    return OR_OK;
}

/* Test helper: write a box of voxels (resident part only). */
int or_set_voxels(omap *m, const int32_t lo[3], const int32_t hi[3], const int16_t *sdf, const int16_t *w)
{
    if (!m || !lo || !hi || !sdf || !w) return OR_EINVAL;
    int64_t ny = hi[1] - lo[1], nz = hi[2] - lo[2];
    for (int64_t x = lo[0]; x < hi[0]; ++x)
        for (int64_t y = lo[1]; y < hi[1]; ++y)
            for (int64_t z = lo[2]; z < hi[2]; ++z) {
                int64_t g[3] = {x, y, z};
                if (!in_window(m->origin, m->dims, g)) continue;
                int64_t o = ((x - lo[0]) * ny + (y - lo[1])) * nz + (z - lo[2]);
                int64_t sl = slot_of(m, g);
                m->sdf[sl] = sdf[o];
                m->w[sl] = w[o];
            }
    return OR_OK;
}

/* The resident window in slot order (the raw device-layout view). */
int or_window(omap *m, int16_t *sdf, int16_t *w, int32_t origin[3])
{
    if (!m) return OR_EINVAL;
    if (sdf) memcpy(sdf, m->sdf, (size_t)m->nvox * sizeof(int16_t));
    if (w) memcpy(w, m->w, (size_t)m->nvox * sizeof(int16_t));
    if (origin) memcpy(origin, m->origin, sizeof(m->origin));
    return OR_OK;
}

int64_t or_store_chunks(omap *m) { return m ? m->tab_n : 0; }

/* Recentre rule of the local map: when the sensor voxel position o (fixed
 * point) is farther than radius_u (fixed point) from the window centre
 * 1024 (origin + dims/2), the window is re-centred on the chunk-grid point
 * nearest the sensor voxel: origin' = chunk * floor((floor(o/1024) +
 * chunk/2) / chunk) - dims/2. Returns 1 and writes origin' if a shift is
 * due, 0 otherwise, -1 for an unrepresentable pose. With force = 1 the
 * origin is always computed (placement of the first window). */
int or_recentre(const int32_t dims[3], const int32_t origin[3], double voxel_size, const double M[16],
                int64_t radius_u, int32_t chunk, int force, int32_t out[3])
{
    int64_t o[3];
    if (!or_quantise_origin(M, 1024.0 / voxel_size, o)) return -1;
    __int128 d2 = 0;
    for (int a = 0; a < 3; ++a) {
        __int128 c = (__int128)1024 * ((int64_t)origin[a] + dims[a] / 2);
        __int128 d = (__int128)o[a] - c;
        d2 += d * d;
    }
    if (!force && d2 <= (__int128)radius_u * radius_u) return 0;
    for (int a = 0; a < 3; ++a) {
        int64_t sv = floor_div(o[a], 1024);
        out[a] = (int32_t)(chunk * floor_div(sv + chunk / 2, chunk) - dims[a] / 2);
    }
    return 1;
}
