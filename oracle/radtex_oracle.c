/*
 * radtex_oracle.c -- plain, slow FP64 CPU oracle for the radiance-bucket lookup
 * of "Radiance Textures for Rasterizing Ray-Traced Data" (Fober, 2023,
 * arXiv 2301.01719).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent reference that the
 * GPU path is checked against.  It shares no code, header, table or constant
 * generator with the HIP library, and only the test-suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it.  Nothing in the product
 * path calls it.
 *
 * Everything is double precision and written as the paper states it, step by
 * step, with no blocking or fusion:
 *
 *   tangent-space incidence   Sec. 2.1: the incidence vector is moved into the
 *                             orthogonal texture space (N_z = 1) by the
 *                             per-fragment frame M = [T;B;N] and normalised
 *   equisolid projection      Eq. (1b) (and the general-normal Eq. (1a))
 *   disc -> square            Eq. (3)
 *   bucket-edge clamp         the Note after Eq. (3): B clamped to
 *                             [1/n - 1, 1 - 1/n]^2
 *   bucket selection          Sec. 2: texture u,v index the bucket matrix
 *   filtered fetch            bilinear inside the bucket (the clamp only has a
 *                             purpose for a filtered fetch)
 *   inverse mappings          Eqs. (2a)-(2c), (4a), (4b)
 *   minification              a mip chain of bucket matrices (2 x 2 bucket
 *                             means) and a trilinear lookup whose level is
 *                             log2 of the UV footprint in buckets
 *   bake                      the reflection vector of every sample centre
 *                             (Eqs. (4a), (4b)) carried to scene coordinates
 *                             by the bucket frame; an analytic environment
 *                             stands in for the ray-traced radiance
 *   shadowing                 Sec. 5 (Shadowing): 1-bit storage, the lookup
 *                             with the light direction in place of the
 *                             incidence, averaged over an area light's
 *                             samples; analytic occluders stand in for the
 *                             ray-traced visibility of the bake
 *   bucket dictionary         the compression of repetitive buckets (Sec. 1,
 *                             Sec. 2) as a codebook, an index map and gains;
 *                             Lloyd's assignment and update steps build it
 *
 * Readings of points the paper leaves open (texel-centre convention, UV wrap,
 * axis orientation, the A = 0 case of Eq. (3), the storage formats) are listed
 * with the design notes of the repository; each is restated where it is used.
 *
 * Parity pins: every function here is checked by the CPU test-suite against
 * closed forms, a second formulation from the paper, brute force, or an
 * independent library routine (see tests/test_oracle_pins.py).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_FMT_F32 0
#define ORC_FMT_BF16 1
#define ORC_FMT_FP8_E4M3 2
#define ORC_FMT_F64 3 /* oracle-only: for finite differences w.r.t. texels */
#define ORC_FMT_BIT1 4 /* one bit per sample, bucket-major words (Sec. 5, Shadowing) */

#define ORC_MODE_NEAREST 0
#define ORC_MODE_BILINEAR 1

static const double SQRT2 = 1.41421356237309504880168872420969808;

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the parallel loops from here on (at least 1). */
void orc_set_num_threads(int k)
{
#ifdef _OPENMP
    omp_set_num_threads(k > 0 ? k : 1);
#else
    (void)k;
#endif
}

/* ------------------------------------------------------------------------ */
/* Storage formats (the quantised storage is an addition to the paper, which  */
/* only says buckets compress well; see the abstract and Sec. 2).             */
/* ------------------------------------------------------------------------ */

/* BF16 is, by definition, the upper 16 bits of an IEEE binary32. */
double orc_bf16_to_f64(uint16_t code)
{
    uint32_t bits = (uint32_t)code << 16;
    float f;
    memcpy(&f, &bits, 4);
    return (double)f;
}

/* OCP 8-bit E4M3 ("FN" variant): 1 sign, 4 exponent (bias 7), 3 mantissa
 * bits; exponent field 0 is subnormal (M * 2^-9); S.1111.111 is NaN; there is
 * no infinity; largest finite magnitude 448. */
double orc_e4m3_to_f64(uint8_t code)
{
    int s = code >> 7;
    int E = (code >> 3) & 15;
    int M = code & 7;
    double v;
    if (E == 15 && M == 7)
        return NAN;
    if (E == 0)
        v = ldexp((double)M, -9);
    else
        v = ldexp(1.0 + M / 8.0, E - 7);
    return s ? -v : v;
}

/* Round-to-nearest-even of a binary32 to BF16, written from the definition:
 * the two BF16 neighbours of x are found, the nearer one is taken, and a tie
 * goes to the one whose code is even. */
uint16_t orc_f32_to_bf16_rne(float x)
{
    uint32_t bits;
    memcpy(&bits, &x, 4);
    if (isnan(x))
        return (uint16_t)((bits >> 16) | 0x0040u); /* quiet NaN, sign kept */
    if (isinf(x))
        return (uint16_t)(bits >> 16);
    uint32_t sign = bits & 0x80000000u;
    uint32_t mag = bits & 0x7FFFFFFFu;
    uint32_t lo_code = mag >> 16;        /* neighbour toward zero */
    uint32_t hi_code = lo_code + 1;      /* neighbour away from zero */
    double ax = fabs((double)x);
    double vlo = fabs(orc_bf16_to_f64((uint16_t)lo_code));
    double vhi;
    if (hi_code == 0x7F80u)
        vhi = ldexp(1.0, 128); /* overflow threshold of round-to-nearest */
    else
        vhi = fabs(orc_bf16_to_f64((uint16_t)hi_code));
    uint32_t pick;
    double dlo = ax - vlo, dhi = vhi - ax;
    if (dlo < dhi)
        pick = lo_code;
    else if (dhi < dlo)
        pick = hi_code;
    else
        pick = (lo_code & 1u) ? hi_code : lo_code;
    return (uint16_t)((sign >> 16) | pick);
}

/* Round-to-nearest-even to E4M3 with saturation to +-448 ("satfinite"),
 * written from the definition: the non-negative finite codes 0x00..0x7E are
 * in increasing order of value, the nearest one to |y| is chosen, ties go to
 * the even code, values above 448 (and infinities) become 448, NaN stays NaN.
 * tab[k] holds the value of code k (0 <= k <= 0x7E); the code just below |y|
 * is found by bisection over that ordered list. */
static uint8_t e4m3_encode_sat(float y, const double *tab)
{
    if (isnan(y))
        return (uint8_t)(signbit(y) ? 0xFF : 0x7F);
    int neg = signbit(y) ? 1 : 0;
    double a = fabs((double)y);
    int best;
    if (a >= 448.0) {
        best = 0x7E;
    } else {
        /* the largest k with v(k) <= a (v(0) = 0 <= a) */
        int lo = 0, hi = 0x7E;
        while (lo < hi) {
            int mid = (lo + hi + 1) / 2;
            if (tab[mid] <= a)
                lo = mid;
            else
                hi = mid - 1;
        }
        int k = lo;
        if (k == 0x7E) {
            best = 0x7E;
        } else {
            double vl = tab[k], vh = tab[k + 1];
            double dl = a - vl, dh = vh - a;
            if (dl < dh)
                best = k;
            else if (dh < dl)
                best = k + 1;
            else
                best = (k & 1) ? k + 1 : k;
        }
    }
    return (uint8_t)((neg << 7) | best);
}

static void e4m3_table(double tab[0x7F])
{
    for (int k = 0; k <= 0x7E; k++)
        tab[k] = orc_e4m3_to_f64((uint8_t)k);
}

uint8_t orc_f32_to_e4m3_sat(float y)
{
    double tab[0x7F];
    e4m3_table(tab);
    return e4m3_encode_sat(y, tab);
}

/* Per-bucket quantiser.  Texture is bucket-major [H][W][n][n][C] float32.
 * fmt == ORC_FMT_BF16: codes_u16 receives RNE BF16 codes, no scale.
 * fmt == ORC_FMT_FP8_E4M3: per bucket b, amax = max |x| (binary32), and if
 * amax is zero or not finite then scale = inv = 1, else inv = 448/amax and
 * scale = amax/448, both rounded to binary32; every value becomes
 * e4m3_sat(x * inv) (product rounded to binary32).  The decision that yields
 * an integer code is therefore taken in binary32 arithmetic, as in the GPU
 * quantiser; the rounding to the code is done from the definition above. */
void orc_quantize(const float *tex, int64_t n_buckets, int64_t bucket_elems, int fmt,
                  void *codes, float *scales)
{
    if (fmt == ORC_FMT_BF16) {
        uint16_t *out = (uint16_t *)codes;
        int64_t total = n_buckets * bucket_elems;
#pragma omp parallel for schedule(static)
        for (int64_t e = 0; e < total; e++)
            out[e] = orc_f32_to_bf16_rne(tex[e]);
        return;
    }
    uint8_t *out = (uint8_t *)codes;
    double tab[0x7F];
    e4m3_table(tab);
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < n_buckets; b++) {
        const float *src = tex + b * bucket_elems;
        float amax = 0.0f;
        for (int64_t e = 0; e < bucket_elems; e++) {
            float a = fabsf(src[e]);
            if (a > amax)
                amax = a;
        }
        volatile float inv, scale; /* force binary32 rounding of each step */
        if (amax == 0.0f || !isfinite(amax)) {
            inv = 1.0f;
            scale = 1.0f;
        } else {
            inv = 448.0f / amax;
            scale = amax / 448.0f;
        }
        for (int64_t e = 0; e < bucket_elems; e++) {
            volatile float y = src[e] * inv;
            out[b * bucket_elems + e] = e4m3_encode_sat(y, tab);
        }
        scales[b] = scale;
    }
}

/* ------------------------------------------------------------------------ */
/* Mapping of the incidence vector to the radiance bucket (Sec. 2.1)         */
/* ------------------------------------------------------------------------ */

/* Eq. (1b): equisolid azimuthal projection in orthogonal texture space
 * (N = e_z).  I is a unit vector from the surface toward the viewer.
 * The projection is singular only for I = -N, where the paper's denominator
 * vanishes; that direction is mapped to A = 0 (a reading; it is measure-zero
 * and lies below the horizon). */
void orc_equisolid_tangent(const double I[3], double A[2])
{
    double D = sqrt(I[0] * I[0] + I[1] * I[1] + (I[2] + 1.0) * (I[2] + 1.0));
    if (D == 0.0) {
        A[0] = A[1] = 0.0;
        return;
    }
    A[0] = SQRT2 * I[0] / D;
    A[1] = SQRT2 * I[1] / D;
}

/* Eq. (1a): the same projection for a general unit normal N.  The double-bar
 * is read as "direction of" (normalisation), so the result is
 * sqrt(2) * (I + N) / |I + N|; its first two components are the projection
 * expressed in the frame of the vectors, its third is sqrt(2) cos(theta/2)
 * when N = e_z. */
void orc_equisolid_general(const double I[3], const double N[3], double out[3])
{
    double s0 = I[0] + N[0], s1 = I[1] + N[1], s2 = I[2] + N[2];
    double len = sqrt(s0 * s0 + s1 * s1 + s2 * s2);
    if (len == 0.0) {
        out[0] = out[1] = out[2] = 0.0;
        return;
    }
    out[0] = SQRT2 * s0 / len;
    out[1] = SQRT2 * s1 / len;
    out[2] = SQRT2 * s2 / len;
}

/* Eq. (3): disc -> square.  B = (|A|_2 / max(|A_x|,|A_y|)) A.  The paper's
 * condition is read as "A is not the zero vector"; B = 0 at A = 0, which is
 * the limit of the map there. */
void orc_square(const double A[2], double B[2])
{
    double rho = sqrt(A[0] * A[0] + A[1] * A[1]);
    double m = fmax(fabs(A[0]), fabs(A[1]));
    if (m == 0.0) {
        B[0] = B[1] = 0.0;
        return;
    }
    B[0] = rho / m * A[0];
    B[1] = rho / m * A[1];
}

/* Eq. (4a): square -> disc, the inverse of Eq. (3). */
void orc_unsquare(const double B[2], double A[2])
{
    double rho = sqrt(B[0] * B[0] + B[1] * B[1]);
    double m = fmax(fabs(B[0]), fabs(B[1]));
    if (rho == 0.0) {
        A[0] = A[1] = 0.0;
        return;
    }
    A[0] = m / rho * B[0];
    A[1] = m / rho * B[1];
}

/* Eq. (2c): inverse equisolid mapping in orthogonal texture space. */
void orc_inverse_equisolid_tangent(const double A[2], double I[3])
{
    double r2 = A[0] * A[0] + A[1] * A[1];
    double w = sqrt(fmax(0.0, 2.0 - r2));
    I[0] = A[0] * w;
    I[1] = A[1] * w;
    I[2] = 1.0 - r2;
}

/* Eqs. (2a)-(2b): inverse mapping for a general normal; A' is the half-vector
 * built from A in the frame where the normal is e_z (Eq. 2a), and the
 * incidence is the normal reflected about A' (Eq. 2b). */
void orc_inverse_equisolid_general(const double A[2], const double N[3], double I[3])
{
    double Ap[3];
    Ap[0] = A[0] * sqrt(0.5);
    Ap[1] = A[1] * sqrt(0.5);
    Ap[2] = sqrt(fmax(0.0, 1.0 - A[0] * A[0] / 2.0 - A[1] * A[1] / 2.0));
    double d = Ap[0] * N[0] + Ap[1] * N[1] + Ap[2] * N[2];
    for (int k = 0; k < 3; k++)
        I[k] = 2.0 * (d * Ap[k] - N[k]) + N[k];
}

/* Eq. (4b): equisolid reflection vector, the incidence mirrored about N. */
void orc_reflection(const double A[2], double R[3])
{
    double r2 = A[0] * A[0] + A[1] * A[1];
    double w = sqrt(fmax(0.0, 2.0 - r2));
    R[0] = -A[0] * w;
    R[1] = -A[1] * w;
    R[2] = 1.0 - r2;
}

/* Bucket-edge clamp (the Note after Eq. (3)) followed by the texel-centre
 * reading: B in [-1,1] spans the bucket's n samples with sample centres at
 * B = (2k+1)/n - 1, so the continuous sample coordinate is
 * s = (B + 1) n/2 - 1/2 and the clamp range [1/n - 1, 1 - 1/n] becomes
 * exactly [0, n-1].  The final min/max only removes rounding residue of the
 * affine map (it is the identity in exact arithmetic).
 * s_unclamped receives the coordinate before the clamp. */
static void texel_coord(const double B[2], int n, double s[2], double s_unclamped[2],
                        int clamped[2])
{
    double lo = 1.0 / n - 1.0, hi = 1.0 - 1.0 / n;
    for (int k = 0; k < 2; k++) {
        double b = B[k];
        s_unclamped[k] = (b + 1.0) * n / 2.0 - 0.5;
        clamped[k] = !(b > lo && b < hi);
        if (b < lo)
            b = lo;
        if (b > hi)
            b = hi;
        double t = (b + 1.0) * n / 2.0 - 0.5;
        if (!(t >= 0.0))
            t = 0.0; /* also maps NaN (undefined input) to the first sample */
        if (t > n - 1)
            t = n - 1;
        s[k] = t;
    }
}

void orc_texel_coord(const double B[2], int n, double s[2])
{
    double su[2];
    int cl[2];
    texel_coord(B, n, s, su, cl);
}

/* Sec. 2.1: the incidence vector in orthogonal texture space.  The frame M
 * has rows T, B, N (row-major, vectors as columns, as in the paper's naming
 * convention), u = M V, and I = u / |u|. */
static int tangent_incidence(const double tbn[9], const double V[3], double u[3], double I[3],
                             double *L)
{
    for (int k = 0; k < 3; k++)
        u[k] = tbn[3 * k + 0] * V[0] + tbn[3 * k + 1] * V[1] + tbn[3 * k + 2] * V[2];
    *L = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    if (!(*L > 0.0) || !isfinite(*L)) {
        I[0] = I[1] = I[2] = NAN;
        return 0;
    }
    for (int k = 0; k < 3; k++)
        I[k] = u[k] / *L;
    return 1;
}

/* The texture coordinate of Sec. 2 selects the bucket: the UV plane is read
 * as repeating (wrap), the bucket column is floor(frac(u) W) and the row
 * floor(frac(v) H) with row 0 first in memory.  A rounding result of W is
 * put in the last column; non-finite coordinates give bucket 0. */
static int bucket_index(double u, int W, double *edge_dist)
{
    double f = u - floor(u);
    if (!isfinite(f)) {
        if (edge_dist)
            *edge_dist = INFINITY;
        return 0;
    }
    double p = f * W;
    int i = (int)floor(p);
    if (i > W - 1)
        i = W - 1;
    if (i < 0)
        i = 0;
    if (edge_dist) {
        double k = floor(p + 0.5);
        *edge_dist = fabs(p - k) / W;
    }
    return i;
}

/* distance (in units of the bucket side) of the unclamped sample coordinate
 * to the nearest cell edge, the clamp bounds included */
static double sample_edge_dist(double su, int n)
{
    double k;
    if (su <= 0.0)
        k = 0.0;
    else if (su >= n - 1)
        k = n - 1;
    else
        k = floor(su + 0.5);
    return fabs(su - k) / n;
}

typedef struct {
    int W, H, n, C, fmt;
    const void *data;
    const float *scales;
    /* bucket dictionary (NULL: none): bucket b reads entry index[b] of data,
     * times gains[b] (NULL: 1) */
    const int32_t *index;
    const float *gains;
} tex_t;

/* Texel (row y, column x, channel c) of bucket (column i, row j).  Storage is
 * bucket-major [H][W][n][n][C]; the decoded value is exact in binary64. */
static double texel(const tex_t *t, int i, int j, int y, int x, int c)
{
    int64_t b = (int64_t)j * t->W + i;
    if (t->index) {
        /* the dictionary form: the decoded bucket is gain(b) times its entry */
        double g = t->gains ? (double)t->gains[b] : 1.0;
        tex_t plain = {t->W, t->H, t->n, t->C, t->fmt, t->data, t->scales, NULL, NULL};
        int64_t k = t->index[b];
        return g * texel(&plain, (int)(k % t->W), (int)(k / t->W), y, x, c);
    }
    int64_t e = ((b * t->n + y) * t->n + x) * t->C + c;
    switch (t->fmt) {
    case ORC_FMT_F32:
        return (double)((const float *)t->data)[e];
    case ORC_FMT_BF16:
        return orc_bf16_to_f64(((const uint16_t *)t->data)[e]);
    case ORC_FMT_FP8_E4M3:
        return orc_e4m3_to_f64(((const uint8_t *)t->data)[e]) * (double)t->scales[b];
    case ORC_FMT_BIT1: {
        /* one channel; sample k = y n + x of bucket b is bit k % 32 of word
         * b wpb + k / 32, wpb = ceil(n n / 32) words per bucket */
        int64_t wpb = ((int64_t)t->n * t->n + 31) / 32;
        int64_t k = (int64_t)y * t->n + x;
        uint32_t w = ((const uint32_t *)t->data)[b * wpb + k / 32];
        return (double)((w >> (k % 32)) & 1u);
    }
    default:
        return ((const double *)t->data)[e];
    }
}

typedef struct {
    double s[2], su[2];
    int clamped[2];
    int x0, y0, x1, y1;
    double fx, fy;
    double A[2], B[2];
    double u[3], I[3], L;
    int valid;
} dirmap_t;

/* All steps from the view vector to the bilinear footprint inside a bucket. */
static void map_direction(const double tbn[9], const double V[3], int n, dirmap_t *d)
{
    d->valid = tangent_incidence(tbn, V, d->u, d->I, &d->L);
    if (d->valid) {
        orc_equisolid_tangent(d->I, d->A);
        orc_square(d->A, d->B);
    } else {
        d->A[0] = d->A[1] = NAN;
        d->B[0] = d->B[1] = NAN;
    }
    texel_coord(d->B, n, d->s, d->su, d->clamped);
    d->x0 = (int)floor(d->s[0]);
    d->y0 = (int)floor(d->s[1]);
    d->fx = d->s[0] - d->x0;
    d->fy = d->s[1] - d->y0;
    d->x1 = d->x0 + 1 < n - 1 ? d->x0 + 1 : n - 1;
    d->y1 = d->y0 + 1 < n - 1 ? d->y0 + 1 : n - 1;
}

/* Bilinear value inside bucket (i,j) at the footprint of d, channel c. */
static double bilerp(const tex_t *t, int i, int j, const dirmap_t *d, int c)
{
    double T00 = texel(t, i, j, d->y0, d->x0, c);
    double T01 = texel(t, i, j, d->y0, d->x1, c);
    double T10 = texel(t, i, j, d->y1, d->x0, c);
    double T11 = texel(t, i, j, d->y1, d->x1, c);
    return (1.0 - d->fy) * ((1.0 - d->fx) * T00 + d->fx * T01) +
           d->fy * ((1.0 - d->fx) * T10 + d->fx * T11);
}

/* Bucket footprint in UV: nearest (one bucket, weight 1) or, in the
 * bilinear-bucket mode, the four buckets around p = frac(u) W - 1/2 with
 * bilinear weights, wrapping across the matrix edges. */
typedef struct {
    int i[4], j[4];
    double w[4];
    int count;
    double a, b;       /* bilinear-bucket fractions */
    int i0, i1, j0, j1;
} bucketfp_t;

static void bucket_footprint(double u, double v, int W, int H, int mode, bucketfp_t *f)
{
    if (mode == ORC_MODE_NEAREST) {
        f->count = 1;
        f->i[0] = bucket_index(u, W, NULL);
        f->j[0] = bucket_index(v, H, NULL);
        f->w[0] = 1.0;
        f->a = f->b = 0.0;
        return;
    }
    double fu = u - floor(u), fv = v - floor(v);
    if (!isfinite(fu))
        fu = 0.0;
    if (!isfinite(fv))
        fv = 0.0;
    double p = fu * W - 0.5, q = fv * H - 0.5;
    double pi0 = floor(p), qj0 = floor(q);
    double a = p - pi0, b = q - qj0;
    int i0 = (int)pi0, j0 = (int)qj0;
    /* wrap */
    i0 = ((i0 % W) + W) % W;
    j0 = ((j0 % H) + H) % H;
    int i1 = (i0 + 1) % W, j1 = (j0 + 1) % H;
    f->count = 4;
    f->i0 = i0; f->i1 = i1; f->j0 = j0; f->j1 = j1;
    f->a = a; f->b = b;
    f->i[0] = i0; f->j[0] = j0; f->w[0] = (1.0 - a) * (1.0 - b);
    f->i[1] = i1; f->j[1] = j0; f->w[1] = a * (1.0 - b);
    f->i[2] = i0; f->j[2] = j1; f->w[2] = (1.0 - a) * b;
    f->i[3] = i1; f->j[3] = j1; f->w[3] = a * b;
}

static void widen_fragment(const float *uv, const float *tbn, const float *view, int64_t f,
                           double U[2], double M[9], double V[3])
{
    U[0] = uv[2 * f];
    U[1] = uv[2 * f + 1];
    for (int k = 0; k < 9; k++)
        M[k] = tbn[9 * f + k];
    for (int k = 0; k < 3; k++)
        V[k] = view[3 * f + k];
}

static void lookup_one(const tex_t *t, const double U[2], const double M[9], const double V[3],
                       int mode, double *out)
{
    dirmap_t d;
    bucketfp_t bf;
    map_direction(M, V, t->n, &d);
    bucket_footprint(U[0], U[1], t->W, t->H, mode, &bf);
    for (int c = 0; c < t->C; c++) {
        double acc = 0.0;
        for (int k = 0; k < bf.count; k++)
            acc += bf.w[k] * bilerp(t, bf.i[k], bf.j[k], &d, c);
        out[c] = acc;
    }
}

/* Forward lookup of N fragments: out[f][c] in binary64. */
void orc_lookup_fwd(int64_t N, const float *uv, const float *tbn, const float *view, int W,
                    int H, int n, int C, int fmt, const void *data, const float *scales,
                    int mode, double *out)
{
    tex_t t = {W, H, n, C, fmt, data, scales};
#pragma omp parallel for schedule(static)
    for (int64_t f = 0; f < N; f++) {
        double U[2], M[9], V[3];
        widen_fragment(uv, tbn, view, f, U, M, V);
        lookup_one(&t, U, M, V, mode, out + f * C);
    }
}

/* Forward lookup of a single fragment given in binary64 (finite differences). */
void orc_lookup_one_f64(const double U[2], const double M[9], const double V[3], int W, int H,
                        int n, int C, int fmt, const void *data, const float *scales, int mode,
                        double *out)
{
    tex_t t = {W, H, n, C, fmt, data, scales};
    lookup_one(&t, U, M, V, mode, out);
}

/* Forward lookup of N fragments given in binary64 (finite differences over
 * many fragments at once): the same lookup as orc_lookup_one_f64 per
 * fragment, U [N][2], M [N][9], V [N][3], out [N][C]. */
void orc_lookup_fwd_f64(int64_t N, const double *U, const double *M, const double *V, int W,
                        int H, int n, int C, int fmt, const void *data, const float *scales,
                        int mode, double *out)
{
    tex_t t = {W, H, n, C, fmt, data, scales};
#pragma omp parallel for schedule(static)
    for (int64_t f = 0; f < N; f++)
        lookup_one(&t, U + 2 * f, M + 9 * f, V + 3 * f, mode, out + f * C);
}

/* Per-fragment indices of the nearest-bucket lookup, for bit-exact checks:
 * idx[f] = (i, j, x0, y0), frac[f] = (fx, fy), and the distances of the
 * unrounded quantities to the points where a result changes discontinuously
 * or is not differentiable: edge[f] = (bucket distance in units of the matrix
 * side, sample distance in units of the bucket side with the clamp bounds
 * included, distance | |A_x| - |A_y| | to the diagonal where Eq. (3) switches
 * between its two branches). */
void orc_indices(int64_t N, const float *uv, const float *tbn, const float *view, int W, int H,
                 int n, int32_t *idx, double *frac, double *edge)
{
#pragma omp parallel for schedule(static)
    for (int64_t f = 0; f < N; f++) {
        double U[2], M[9], V[3], du, dv;
        widen_fragment(uv, tbn, view, f, U, M, V);
        dirmap_t d;
        map_direction(M, V, n, &d);
        idx[4 * f + 0] = bucket_index(U[0], W, &du);
        idx[4 * f + 1] = bucket_index(U[1], H, &dv);
        idx[4 * f + 2] = d.x0;
        idx[4 * f + 3] = d.y0;
        frac[2 * f + 0] = d.fx;
        frac[2 * f + 1] = d.fy;
        if (edge) {
            double sd = fmin(sample_edge_dist(d.su[0], n), sample_edge_dist(d.su[1], n));
            if (!d.valid)
                sd = INFINITY;
            edge[3 * f + 0] = fmin(du, dv);
            edge[3 * f + 1] = sd;
            edge[3 * f + 2] = d.valid ? fabs(fabs(d.A[0]) - fabs(d.A[1])) : INFINITY;
        }
    }
}

/* Intermediate values of the mapping for one direction, in binary64:
 * out = (A_x, A_y, B_x, B_y, s_x, s_y). */
void orc_map_one(const double M[9], const double V[3], int n, double out[6])
{
    dirmap_t d;
    map_direction(M, V, n, &d);
    out[0] = d.A[0];
    out[1] = d.A[1];
    out[2] = d.B[0];
    out[3] = d.B[1];
    out[4] = d.s[0];
    out[5] = d.s[1];
}

/* ------------------------------------------------------------------------ */
/* Backward (an addition to the paper: analytic derivatives of the lookup)   */
/* ------------------------------------------------------------------------ */

/* dB/dA of Eq. (3), as a 2x2 matrix J[r][c] = dB_r/dA_c.  On the branch
 * |A_x| >= |A_y| the map is B = (rho sgn(A_x), rho A_y/|A_x|); the other
 * branch is its mirror image.  At A = 0 the limit along the axes (identity)
 * is used. */
static void square_jacobian(const double A[2], double J[2][2])
{
    double ax = A[0], ay = A[1];
    double rho = sqrt(ax * ax + ay * ay);
    if (rho == 0.0) {
        J[0][0] = 1.0; J[0][1] = 0.0; J[1][0] = 0.0; J[1][1] = 1.0;
        return;
    }
    if (fabs(ax) >= fabs(ay)) {
        double sx = ax >= 0 ? 1.0 : -1.0;
        J[0][0] = fabs(ax) / rho;
        J[0][1] = sx * ay / rho;
        J[1][0] = -sx * ay * ay * ay / (rho * ax * ax);
        J[1][1] = (ay * ay + rho * rho) / (rho * fabs(ax));
    } else {
        double sy = ay >= 0 ? 1.0 : -1.0;
        J[1][1] = fabs(ay) / rho;
        J[1][0] = sy * ax / rho;
        J[0][1] = -sy * ax * ax * ax / (rho * ay * ay);
        J[0][0] = (ax * ax + rho * rho) / (rho * fabs(ay));
    }
}

/* dA/dI of Eq. (1b) taken literally (I free in R^3), J[r][c] = dA_r/dI_c. */
static void equisolid_jacobian(const double I[3], double J[2][3])
{
    double D2 = I[0] * I[0] + I[1] * I[1] + (I[2] + 1.0) * (I[2] + 1.0);
    double D = sqrt(D2);
    if (D == 0.0) {
        memset(J, 0, sizeof(double) * 6);
        return;
    }
    double D3 = D2 * D;
    double dD[3] = {I[0], I[1], I[2] + 1.0}; /* times 1/D: dD/dI */
    for (int r = 0; r < 2; r++)
        for (int c = 0; c < 3; c++)
            J[r][c] = SQRT2 * ((r == c ? 1.0 / D : 0.0) - I[r] * dD[c] / D3);
}

/* Gradient of the loss w.r.t. the view vector of one fragment, given
 * dL/ds (per axis) accumulated over all buckets of the footprint:
 * dL/dB = (n/2) dL/ds on unclamped axes (0 on clamped axes),
 * dL/dA = J3^T dL/dB, dL/dI = J1^T dL/dA, dL/du = (1/L)(P) dL/dI with
 * P = 1 - I I^T (normalisation), dL/dV = M^T dL/du. */
static void view_gradient(const double M[9], const dirmap_t *d, int n, const double gs[2],
                          int absolute, double gV[3])
{
    gV[0] = gV[1] = gV[2] = 0.0;
    if (!d->valid)
        return;
    double gB[2];
    for (int k = 0; k < 2; k++)
        gB[k] = d->clamped[k] ? 0.0 : gs[k] * n / 2.0;
    double J3[2][2], J1[2][3], I[3] = {d->I[0], d->I[1], d->I[2]}, Mx[9];
    square_jacobian(d->A, J3);
    equisolid_jacobian(d->I, J1);
    memcpy(Mx, M, sizeof(Mx));
    if (absolute) { /* every factor by its magnitude: the scale of the rounding */
        for (int r = 0; r < 2; r++) {
            for (int c = 0; c < 2; c++)
                J3[r][c] = fabs(J3[r][c]);
            for (int c = 0; c < 3; c++)
                J1[r][c] = fabs(J1[r][c]);
        }
        for (int k = 0; k < 3; k++)
            I[k] = fabs(I[k]);
        for (int k = 0; k < 9; k++)
            Mx[k] = fabs(Mx[k]);
    }
    double gA[2] = {J3[0][0] * gB[0] + J3[1][0] * gB[1], J3[0][1] * gB[0] + J3[1][1] * gB[1]};
    double gI[3];
    for (int c = 0; c < 3; c++)
        gI[c] = J1[0][c] * gA[0] + J1[1][c] * gA[1];
    double dot = gI[0] * I[0] + gI[1] * I[1] + gI[2] * I[2];
    double gu[3];
    for (int c = 0; c < 3; c++)
        gu[c] = absolute ? (gI[c] + I[c] * dot) / d->L : (gI[c] - I[c] * dot) / d->L;
    for (int m = 0; m < 3; m++)
        gV[m] = Mx[0 * 3 + m] * gu[0] + Mx[1 * 3 + m] * gu[1] + Mx[2 * 3 + m] * gu[2];
}

/* dL/ds of one fragment (per axis, summed over the buckets of its footprint
 * with their weights) and, per footprint bucket, sum_c g_c times the bucket's
 * bilinear value, at the in-bucket fractions of d (gf: the upstream gradient
 * in binary64). */
static void footprint_slopes(const tex_t *t, const bucketfp_t *bf, const dirmap_t *d,
                             const double gf[4], double gs[2], double Lb[4])
{
    gs[0] = gs[1] = 0.0;
    Lb[0] = Lb[1] = Lb[2] = Lb[3] = 0.0;
    for (int k = 0; k < bf->count; k++) {
        int i = bf->i[k], j = bf->j[k];
        for (int c = 0; c < t->C; c++) {
            double T00 = texel(t, i, j, d->y0, d->x0, c);
            double T01 = texel(t, i, j, d->y0, d->x1, c);
            double T10 = texel(t, i, j, d->y1, d->x0, c);
            double T11 = texel(t, i, j, d->y1, d->x1, c);
            double dsx = (1.0 - d->fy) * (T01 - T00) + d->fy * (T11 - T10);
            double dsy = (1.0 - d->fx) * (T10 - T00) + d->fx * (T11 - T01);
            gs[0] += bf->w[k] * gf[c] * dsx;
            gs[1] += bf->w[k] * gf[c] * dsy;
            Lb[k] += gf[c] * bilerp(t, i, j, d, c);
        }
    }
}

/* dL/d(u, v) of one fragment from its buckets' values Lb: zero in nearest
 * mode (piecewise constant in u, v) and for non-finite coordinates; in the
 * bilinear-bucket mode the derivative of sum_k w_k(a, b) L_k with
 * a = frac(u) W - 1/2, b = frac(v) H - 1/2. */
static void uv_gradient(const bucketfp_t *bf, const double Lb[4], const double U[2], int W,
                        int H, int mode, double guv[2])
{
    if (mode == ORC_MODE_NEAREST || !isfinite(U[0] - floor(U[0])) ||
        !isfinite(U[1] - floor(U[1]))) {
        guv[0] = guv[1] = 0.0;
        return;
    }
    double a = bf->a, b = bf->b;
    guv[0] = W * ((1.0 - b) * (Lb[1] - Lb[0]) + b * (Lb[3] - Lb[2]));
    guv[1] = H * ((1.0 - a) * (Lb[2] - Lb[0]) + a * (Lb[3] - Lb[1]));
}

/* Backward of N fragments with upstream gradient g[N][C] (binary32).
 *   grad_tex   dL/d(texel) accumulated in fragment order, binary64, over the
 *              bucket window [bi0, bi0+bw) x [bj0, bj0+bh) only (laid out
 *              [bh][bw][n][n][C]); NULL skips it.  abs_tex receives the sum of
 *              |weight * g| per element (the scale of the error criterion) and
 *              absg_tex the sum of |g| over the taps that include the element
 *              (the scale of the rounding of the weights themselves); either
 *              may be NULL.
 *   grad_view  dL/dV [N][3]; grad_uv dL/d(u,v) [N][2] (zero in nearest mode
 *              away from bucket edges, where the lookup is piecewise constant
 *              in u,v).  Either may be NULL.
 *   scale_view, scale_uv  the same chain rule evaluated with the magnitude of
 *              every factor and term (the scale against which a binary32
 *              evaluation's rounding error is measured); either may be NULL.
 * Taps that coincide (x1 = x0 at the clamp bound) each receive their own
 * weight, so the texel gets the sum. */
/* The body of the backward for one texture; wf (may be NULL: all 1) scales
 * fragment f's upstream gradient by wf[f] (the level weight of a trilinear
 * lookup). */
static void lookup_bwd_core(int64_t N, const float *uv, const float *tbn, const float *view,
                            const float *g, const double *wf, const tex_t *tp, int mode,
                            double *grad_tex, double *abs_tex, double *absg_tex, int bi0,
                            int bj0, int bw, int bh, double *grad_view, double *grad_uv,
                            double *scale_view, double *scale_uv)
{
    const tex_t t = *tp;
    const int W = t.W, H = t.H, n = t.n, C = t.C;
    if (grad_view || grad_uv || scale_view || scale_uv) {
#pragma omp parallel for schedule(static)
        for (int64_t f = 0; f < N; f++) {
            double U[2], M[9], V[3];
            widen_fragment(uv, tbn, view, f, U, M, V);
            dirmap_t d;
            bucketfp_t bf;
            map_direction(M, V, n, &d);
            bucket_footprint(U[0], U[1], W, H, mode, &bf);
            double gf[4];
            for (int c = 0; c < C; c++)
                gf[c] = (wf ? wf[f] : 1.0) * (double)g[f * C + c];
            double gs[2], gsa[2] = {0.0, 0.0};
            double Lb[4]; /* sum_c g_c * bilerp per footprint bucket */
            double La[4] = {0, 0, 0, 0}; /* the same with magnitudes */
            footprint_slopes(&t, &bf, &d, gf, gs, Lb);
            for (int k = 0; k < bf.count; k++) {
                int i = bf.i[k], j = bf.j[k];
                for (int c = 0; c < C; c++) {
                    double T00 = texel(&t, i, j, d.y0, d.x0, c);
                    double T01 = texel(&t, i, j, d.y0, d.x1, c);
                    double T10 = texel(&t, i, j, d.y1, d.x0, c);
                    double T11 = texel(&t, i, j, d.y1, d.x1, c);
                    double ag = fabs(bf.w[k] * gf[c]);
                    gsa[0] += ag * ((1.0 - d.fy) * fabs(T01 - T00) + d.fy * fabs(T11 - T10));
                    gsa[1] += ag * ((1.0 - d.fx) * fabs(T10 - T00) + d.fx * fabs(T11 - T01));
                    La[k] += fabs(gf[c]) *
                             ((1.0 - d.fy) * ((1.0 - d.fx) * fabs(T00) + d.fx * fabs(T01)) +
                              d.fy * ((1.0 - d.fx) * fabs(T10) + d.fx * fabs(T11)));
                }
            }
            if (grad_view)
                view_gradient(M, &d, n, gs, 0, grad_view + 3 * f);
            if (scale_view)
                view_gradient(M, &d, n, gsa, 1, scale_view + 3 * f);
            if (scale_uv) {
                if (mode == ORC_MODE_NEAREST) {
                    scale_uv[2 * f] = scale_uv[2 * f + 1] = 0.0;
                } else {
                    double a = bf.a, b = bf.b;
                    scale_uv[2 * f + 0] = W * ((1.0 - b) * (La[1] + La[0]) + b * (La[3] + La[2]));
                    scale_uv[2 * f + 1] = H * ((1.0 - a) * (La[2] + La[0]) + a * (La[3] + La[1]));
                }
            }
            if (grad_uv)
                uv_gradient(&bf, Lb, U, W, H, mode, grad_uv + 2 * f);
        }
    }
    if (grad_tex) {
        int64_t win = (int64_t)bw * bh * n * n * C;
        memset(grad_tex, 0, sizeof(double) * win);
        if (abs_tex)
            memset(abs_tex, 0, sizeof(double) * win);
        if (absg_tex)
            memset(absg_tex, 0, sizeof(double) * win);
        for (int64_t f = 0; f < N; f++) { /* fragment order: sequential */
            double U[2], M[9], V[3];
            widen_fragment(uv, tbn, view, f, U, M, V);
            dirmap_t d;
            bucketfp_t bf;
            map_direction(M, V, n, &d);
            bucket_footprint(U[0], U[1], W, H, mode, &bf);
            double gf[4];
            for (int c = 0; c < C; c++)
                gf[c] = (wf ? wf[f] : 1.0) * (double)g[f * C + c];
            double wt[4] = {(1.0 - d.fx) * (1.0 - d.fy), d.fx * (1.0 - d.fy),
                            (1.0 - d.fx) * d.fy, d.fx * d.fy};
            int ty[4] = {d.y0, d.y0, d.y1, d.y1};
            int tx[4] = {d.x0, d.x1, d.x0, d.x1};
            for (int k = 0; k < bf.count; k++) {
                int i = bf.i[k] - bi0, j = bf.j[k] - bj0;
                if (i < 0 || i >= bw || j < 0 || j >= bh)
                    continue;
                for (int tap = 0; tap < 4; tap++) {
                    int64_t base = ((((int64_t)j * bw + i) * n + ty[tap]) * n + tx[tap]) * C;
                    for (int c = 0; c < C; c++) {
                        double contrib = bf.w[k] * wt[tap] * gf[c];
                        grad_tex[base + c] += contrib;
                        if (abs_tex)
                            abs_tex[base + c] += fabs(contrib);
                        if (absg_tex)
                            absg_tex[base + c] += fabs(gf[c]);
                    }
                }
            }
        }
    }
}

void orc_lookup_bwd(int64_t N, const float *uv, const float *tbn, const float *view,
                    const float *g, int W, int H, int n, int C, int fmt, const void *data,
                    const float *scales, int mode, double *grad_tex, double *abs_tex,
                    double *absg_tex, int bi0,
                    int bj0, int bw, int bh, double *grad_view, double *grad_uv,
                    double *scale_view, double *scale_uv)
{
    tex_t t = {W, H, n, C, fmt, data, scales};
    lookup_bwd_core(N, uv, tbn, view, g, NULL, &t, mode, grad_tex, abs_tex, absg_tex, bi0, bj0,
                    bw, bh, grad_view, grad_uv, scale_view, scale_uv);
}

/* How far the view and uv gradients of each fragment move under the rounding
 * that a binary32 evaluation cannot avoid in the quantities its taps are
 * weighted with: the sample coordinate s (the texel coordinate of the clamp
 * Note after Eq. (3)), held to within delta_s, and, in the bilinear-bucket
 * mode, the bucket fractions a, b, held to within delta_w.  The result is the
 * largest |grad(moved) - grad|_2 over the sign patterns of the moves (fx +-
 * delta_s, fy +- delta_s, and a +- delta_w, b +- delta_w), every other factor
 * of the chain held at the fragment's own values.  The moved in-bucket
 * fractions stay on the same taps (the cell's bilinear patch extended past
 * it) and the clamp decisions are those of s.  round_view [N], round_uv [N]
 * (either may be NULL; round_uv is 0 in nearest mode). */
void orc_lookup_bwd_round(int64_t N, const float *uv, const float *tbn, const float *view,
                          const float *g, int W, int H, int n, int C, int fmt, const void *data,
                          const float *scales, int mode, double delta_s, double delta_w,
                          double *round_view, double *round_uv)
{
    tex_t t = {W, H, n, C, fmt, data, scales};
    const int nw = mode == ORC_MODE_NEAREST ? 1 : 4; /* sign patterns of (a, b) */
#pragma omp parallel for schedule(static)
    for (int64_t f = 0; f < N; f++) {
        double U[2], M[9], V[3];
        widen_fragment(uv, tbn, view, f, U, M, V);
        dirmap_t d;
        bucketfp_t bf;
        map_direction(M, V, n, &d);
        bucket_footprint(U[0], U[1], W, H, mode, &bf);
        double gf[4];
        for (int c = 0; c < C; c++)
            gf[c] = (double)g[f * C + c];
        double gs[2], Lb[4], gV[3], guv[2];
        footprint_slopes(&t, &bf, &d, gf, gs, Lb);
        view_gradient(M, &d, n, gs, 0, gV);
        uv_gradient(&bf, Lb, U, W, H, mode, guv);
        double rv = 0.0, ru = 0.0;
        for (int q = 0; q < 4 * nw; q++) {
            const int sx = (q & 1) ? 1 : -1, sy = (q & 2) ? 1 : -1;
            const int sa = (q & 4) ? 1 : -1, sb = (q & 8) ? 1 : -1;
            dirmap_t e = d;
            e.fx = d.fx + sx * delta_s;
            e.fy = d.fy + sy * delta_s;
            bucketfp_t bm = bf;
            if (mode != ORC_MODE_NEAREST) {
                bm.a = bf.a + sa * delta_w;
                bm.b = bf.b + sb * delta_w;
                bm.w[0] = (1.0 - bm.a) * (1.0 - bm.b);
                bm.w[1] = bm.a * (1.0 - bm.b);
                bm.w[2] = (1.0 - bm.a) * bm.b;
                bm.w[3] = bm.a * bm.b;
            }
            double gs2[2], Lb2[4], gV2[3], guv2[2];
            footprint_slopes(&t, &bm, &e, gf, gs2, Lb2);
            view_gradient(M, &e, n, gs2, 0, gV2);
            uv_gradient(&bm, Lb2, U, W, H, mode, guv2);
            double dv = sqrt((gV2[0] - gV[0]) * (gV2[0] - gV[0]) +
                             (gV2[1] - gV[1]) * (gV2[1] - gV[1]) +
                             (gV2[2] - gV[2]) * (gV2[2] - gV[2]));
            double du = sqrt((guv2[0] - guv[0]) * (guv2[0] - guv[0]) +
                             (guv2[1] - guv[1]) * (guv2[1] - guv[1]));
            if (dv > rv)
                rv = dv;
            if (du > ru)
                ru = du;
        }
        if (round_view)
            round_view[f] = rv;
        if (round_uv)
            round_uv[f] = ru;
    }
}

/* ------------------------------------------------------------------------- */
/* The bake: filling a radiance texture from scene radiance (Sec. 2.1, after */
/* Eq. (4b): the reflection vector is what ray-traced data is sampled along). */
/* ------------------------------------------------------------------------- */

/* The centre of sample (x, y) of an n x n bucket in B coordinates, by the
 * texel-centre reading used throughout: B = ((2x+1)/n - 1, (2y+1)/n - 1). */
static void texel_centre(int x, int y, int n, double B[2])
{
    B[0] = (2.0 * x + 1.0) / n - 1.0;
    B[1] = (2.0 * y + 1.0) / n - 1.0;
}

/* Directions of the sample centres of one bucket in orthogonal texture space:
 * inc[(y n + x) 3 + k] the incidence I that the lookup maps onto the sample
 * (Eq. (4a) then Eq. (2c)), refl[...] the reflection vector R of Eq. (4b)
 * (Eq. (4a) then Eq. (4b)).  Either may be NULL. */
void orc_bake_directions(int n, double *inc, double *refl)
{
    for (int y = 0; y < n; y++) {
        for (int x = 0; x < n; x++) {
            double B[2], A[2];
            texel_centre(x, y, n, B);
            orc_unsquare(B, A);
            if (inc)
                orc_inverse_equisolid_tangent(A, inc + 3 * (y * n + x));
            if (refl)
                orc_reflection(A, refl + 3 * (y * n + x));
        }
    }
}

/* The analytic stand-in for ray-traced scene radiance: per channel c,
 *   env_c(d) = ambient_c + sum_k a_{k,c} exp(lambda_k (mu_k . d - 1))
 * for a unit direction d (spherical Gaussian lobes; mu_k is the lobe's axis
 * normalised, lambda_k >= 0 its sharpness).  lobes[k] holds 8 floats: axis
 * x, y, z, sharpness, amplitudes for channels 0..3. */
static double env_eval(const float *lobes, int K, const float *ambient, int c, const double d[3])
{
    double v = ambient[c];
    for (int k = 0; k < K; k++) {
        const float *L = lobes + 8 * k;
        double mx = L[0], my = L[1], mz = L[2];
        double mn = sqrt(mx * mx + my * my + mz * mz);
        double dot = (mx * d[0] + my * d[1] + mz * d[2]) / mn;
        v += (double)L[4 + c] * exp((double)L[3] * (dot - 1.0));
    }
    return v;
}

/* Bake of the buckets in the window [bi0, bi0+bw) x [bj0, bj0+bh) of a W x H
 * matrix: out[(((j - bj0) bw + (i - bi0)) n + y) n + x][c] =
 *   env_c(normalize(M^T R(x, y))),
 * where R is the reflection vector of the sample centre (Eq. (4b)) in the
 * bucket's orthogonal texture space and M = [T;B;N] the bucket's frame
 * (frames [H][W][9], rows T, B, N; NULL: the identity), so M^T R is R in
 * the scene's coordinates. */
void orc_bake_environment(int W, int H, int n, int C, const float *frames, const float *lobes,
                          int K, const float *ambient, int bi0, int bj0, int bw, int bh,
                          double *out)
{
    (void)W;
    (void)H;
    double *R = (double *)malloc(sizeof(double) * 3 * n * n);
    if (!R)
        return;
    orc_bake_directions(n, NULL, R);
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < (int64_t)bw * bh; b++) {
        int i = bi0 + (int)(b % bw), j = bj0 + (int)(b / bw);
        double M[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
        if (frames)
            for (int k = 0; k < 9; k++)
                M[k] = frames[((int64_t)j * W + i) * 9 + k];
        for (int s = 0; s < n * n; s++) {
            const double *r = R + 3 * s;
            double d[3];
            for (int k = 0; k < 3; k++) /* (M^T r)_k = sum_m M[m][k] r_m */
                d[k] = M[0 * 3 + k] * r[0] + M[1 * 3 + k] * r[1] + M[2 * 3 + k] * r[2];
            double len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            for (int k = 0; k < 3; k++)
                d[k] /= len;
            for (int c = 0; c < C; c++)
                out[(b * n * n + s) * C + c] = env_eval(lobes, K, ambient, c, d);
        }
    }
    free(R);
}

/* env_c at one direction (normalised here), for the tests' analytic
 * references. */
void orc_env_eval(const float *lobes, int K, const float *ambient, int C, const double d_in[3],
                  double *out)
{
    double len = sqrt(d_in[0] * d_in[0] + d_in[1] * d_in[1] + d_in[2] * d_in[2]);
    double d[3] = {d_in[0] / len, d_in[1] / len, d_in[2] / len};
    for (int c = 0; c < C; c++)
        out[c] = env_eval(lobes, K, ambient, c, d);
}

/* ------------------------------------------------------------------------- */
/* Minification across the bucket matrix: a mip chain of bucket matrices and */
/* a trilinear lookup whose level follows the fragment's UV footprint.       */
/* ------------------------------------------------------------------------- */

/* Sec. 2: one sample per bucket synthesises an ordinary W x H texture, and
 * the lookup is linear in the buckets (the sample position depends only on
 * the view), so the minified texture of a 2 x 2 block of pixels is the lookup
 * in the texel-wise mean of the 2 x 2 buckets.  Level l+1 from level l:
 * W_{l+1} = max(1, W_l / 2) (W a power of two; a side of 1 is not halved),
 * and bucket (i, j) of level l+1 is the mean of the buckets of level l it
 * covers (4, or 2 once a side is 1).  src [H][W][n][n][C], dst
 * [H'][W'][n][n][C], binary64. */
void orc_build_mip(int W, int H, int n, int C, const double *src, double *dst)
{
    int W2 = W > 1 ? W / 2 : 1, H2 = H > 1 ? H / 2 : 1;
    int sx = W > 1 ? 2 : 1, sy = H > 1 ? 2 : 1;
    int64_t per = (int64_t)n * n * C;
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < (int64_t)W2 * H2; b++) {
        int i = (int)(b % W2), j = (int)(b / W2);
        for (int64_t e = 0; e < per; e++) {
            double acc = 0.0;
            for (int dj = 0; dj < sy; dj++)
                for (int di = 0; di < sx; di++)
                    acc += src[((int64_t)(j * sy + dj) * W + (i * sx + di)) * per + e];
            dst[b * per + e] = acc / (sx * sy);
        }
    }
}

static int level_dim(int D, int l)
{
    int v = D >> l;
    return v > 0 ? v : 1;
}

/* Level of detail of a fragment from its UV screen derivatives duv =
 * (du/dx, dv/dx, du/dy, dv/dy): the footprint of one pixel in buckets of
 * level 0, rho = max(|(du/dx W, dv/dx H)|, |(du/dy W, dv/dy H)|), and
 * lambda = log2 rho, clamped to [0, levels - 1] (0 when rho is 0 or not
 * finite). */
double orc_lod(const double duv[4], int W, int H, int levels)
{
    double ax = duv[0] * W, ay = duv[1] * H, bx = duv[2] * W, by = duv[3] * H;
    double rho = fmax(sqrt(ax * ax + ay * ay), sqrt(bx * bx + by * by));
    if (!(rho > 0.0) || !isfinite(rho))
        return 0.0;
    double lambda = log2(rho);
    if (lambda < 0.0)
        lambda = 0.0;
    if (lambda > levels - 1)
        lambda = levels - 1;
    return lambda;
}

/* Trilinear lookup: levels l0 = floor(lambda) and l0 + 1 weighted 1 - t and
 * t (t = lambda - l0; one level when t = 0 or l0 is the last level), each a
 * lookup as in the forward with the level's W_l x H_l buckets.  chain holds
 * the levels 0..levels-1 back to back in binary64; lod (may be NULL)
 * receives lambda per fragment. */
void orc_lookup_lod(int64_t N, const float *uv, const float *tbn, const float *view,
                    const float *duv, int W, int H, int n, int C, int levels,
                    const double *chain, int mode, double *out, double *lod)
{
    const double **lv = (const double **)malloc(sizeof(double *) * levels);
    if (!lv)
        return;
    int64_t off = 0;
    for (int l = 0; l < levels; l++) {
        lv[l] = chain + off;
        off += (int64_t)level_dim(W, l) * level_dim(H, l) * n * n * C;
    }
#pragma omp parallel for schedule(static)
    for (int64_t f = 0; f < N; f++) {
        double U[2], M[9], V[3], D[4];
        widen_fragment(uv, tbn, view, f, U, M, V);
        for (int k = 0; k < 4; k++)
            D[k] = duv[4 * f + k];
        double lambda = orc_lod(D, W, H, levels);
        if (lod)
            lod[f] = lambda;
        int l0 = (int)floor(lambda);
        double t = lambda - l0;
        if (l0 >= levels - 1) {
            l0 = levels - 1;
            t = 0.0;
        }
        double a[4], b[4];
        tex_t t0 = {level_dim(W, l0), level_dim(H, l0), n, C, ORC_FMT_F64, lv[l0], NULL};
        lookup_one(&t0, U, M, V, mode, a);
        if (t > 0.0) {
            tex_t t1 = {level_dim(W, l0 + 1), level_dim(H, l0 + 1), n, C, ORC_FMT_F64,
                        lv[l0 + 1], NULL};
            lookup_one(&t1, U, M, V, mode, b);
        }
        for (int c = 0; c < C; c++)
            out[f * C + c] = t > 0.0 ? (1.0 - t) * a[c] + t * b[c] : a[c];
    }
    free(lv);
}

/* Backward of the trilinear lookup: with the level weights w_l(f) = 1 - t on
 * l0, t on l0 + 1 and 0 elsewhere (lambda, l0 and t as in orc_lookup_lod;
 * the level of detail is taken as given, not differentiated), the gradient
 * of level l's texels is the plain backward on level l with upstream
 * w_l(f) g(f), and dL/dview, dL/duv are the sums over the levels of theirs.
 * grad_chain (may be NULL) receives every level's dense gradient back to
 * back in the layout of chain, abs_chain / absg_chain (may be NULL) the
 * magnitude sums of orc_lookup_bwd per level; grad_view [N][3], grad_uv
 * [N][2] and their magnitude scales scale_view, scale_uv (summed over the
 * levels) may be NULL. */
void orc_lookup_lod_bwd(int64_t N, const float *uv, const float *tbn, const float *view,
                        const float *duv, const float *g, int W, int H, int n, int C, int levels,
                        const double *chain, int mode, double *grad_chain, double *abs_chain,
                        double *absg_chain, double *grad_view, double *grad_uv,
                        double *scale_view, double *scale_uv)
{
    int64_t M = N > 0 ? N : 1;
    double *wf = (double *)malloc(sizeof(double) * M);
    double *tv = (double *)malloc(sizeof(double) * 3 * M);
    double *tu = (double *)malloc(sizeof(double) * 2 * M);
    double *sv = (double *)malloc(sizeof(double) * 3 * M);
    double *su = (double *)malloc(sizeof(double) * 2 * M);
    if (!wf || !tv || !tu || !sv || !su) {
        free(wf);
        free(tv);
        free(tu);
        free(sv);
        free(su);
        return;
    }
    double *acc[4] = {grad_view, grad_uv, scale_view, scale_uv};
    int64_t len[4] = {3 * N, 2 * N, 3 * N, 2 * N};
    for (int a = 0; a < 4; a++)
        if (acc[a])
            for (int64_t q = 0; q < len[a]; q++)
                acc[a][q] = 0.0;
    int64_t off = 0;
    for (int l = 0; l < levels; l++) {
        const int Wl = level_dim(W, l), Hl = level_dim(H, l);
        for (int64_t f = 0; f < N; f++) {
            double D[4];
            for (int k = 0; k < 4; k++)
                D[k] = duv[4 * f + k];
            double lambda = orc_lod(D, W, H, levels);
            int l0 = (int)floor(lambda);
            double t = lambda - l0;
            if (l0 >= levels - 1) {
                l0 = levels - 1;
                t = 0.0;
            }
            wf[f] = l == l0 ? 1.0 - t : (l == l0 + 1 ? t : 0.0);
        }
        tex_t tl = {Wl, Hl, n, C, ORC_FMT_F64, chain + off, NULL, NULL, NULL};
        lookup_bwd_core(N, uv, tbn, view, g, wf, &tl, mode, grad_chain ? grad_chain + off : NULL,
                        abs_chain ? abs_chain + off : NULL, absg_chain ? absg_chain + off : NULL,
                        0, 0, Wl, Hl, grad_view ? tv : NULL, grad_uv ? tu : NULL,
                        scale_view ? sv : NULL, scale_uv ? su : NULL);
        double *part[4] = {tv, tu, sv, su};
        for (int a = 0; a < 4; a++)
            if (acc[a])
                for (int64_t q = 0; q < len[a]; q++)
                    acc[a][q] += part[a][q];
        off += (int64_t)Wl * Hl * n * n * C;
    }
    free(wf);
    free(tv);
    free(tu);
    free(sv);
    free(su);
}

/* Adjoint of one level of the chain (orc_build_mip): level l+1's bucket
 * (i, j) is the mean of the buckets of level l it covers, so each of those
 * buckets receives the parent's gradient divided by their number.
 * grad_src [H][W][n][n][C] (level l, W and H as in orc_build_mip) is added
 * to; grad_dst is level l+1's gradient. */
void orc_build_mip_adjoint(int W, int H, int n, int C, const double *grad_dst, double *grad_src)
{
    int W2 = W > 1 ? W / 2 : 1, H2 = H > 1 ? H / 2 : 1;
    int fx = W > 1 ? 2 : 1, fy = H > 1 ? 2 : 1;
    int64_t E = (int64_t)n * n * C;
    for (int j = 0; j < H; j++)
        for (int i = 0; i < W; i++) {
            int64_t parent = (int64_t)(j / fy) * W2 + i / fx;
            int64_t child = (int64_t)j * W + i;
            for (int64_t e = 0; e < E; e++)
                grad_src[child * E + e] += grad_dst[parent * E + e] / (fx * fy);
        }
    (void)H2;
}

/* ------------------------------------------------------------------------- */
/* Shadowing (Sec. 5, Shadowing): a 1-bit radiance texture holds the         */
/* occlusion of static geometry, and the lookup takes the direction toward   */
/* the light in place of the incidence vector; several light directions per */
/* fragment, averaged, give an area light's soft shadow.                     */
/* ------------------------------------------------------------------------- */

/* The 1-bit storage: each sample becomes the bit (x >= 1/2), NaN giving 0.
 * Bucket b of nn = n n samples occupies wpb = ceil(nn / 32) words; sample k
 * is bit k % 32 of word b wpb + k / 32 and the bits past nn are zero. */
void orc_pack_bits(const float *tex, int64_t n_buckets, int nn, uint32_t *words)
{
    int64_t wpb = ((int64_t)nn + 31) / 32;
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < n_buckets; b++) {
        for (int64_t w = 0; w < wpb; w++)
            words[b * wpb + w] = 0u;
        for (int k = 0; k < nn; k++)
            if (tex[b * nn + k] >= 0.5f)
                words[b * wpb + k / 32] |= 1u << (k % 32);
    }
}

/* Light lookup: for fragment f and light sample s the direction toward the
 * light is L = vec[s] (kind 0, a directional light: the same for every
 * fragment) or L = vec[s] - pos[f] (kind 1, a point light sampled at the
 * points vec[s]); the lookup of Sec. 2 and 2.1 is taken with L in place of
 * the view vector, and out[f][c] is the mean over the S samples. */
void orc_lookup_light(int64_t N, const float *uv, const float *tbn, const float *pos, int kind,
                      int S, const float *vec, int W, int H, int n, int C, int fmt,
                      const void *data, const float *scales, int mode, double *out)
{
    tex_t t = {W, H, n, C, fmt, data, scales};
#pragma omp parallel for schedule(static)
    for (int64_t f = 0; f < N; f++) {
        double U[2] = {uv[2 * f], uv[2 * f + 1]};
        double M[9];
        for (int k = 0; k < 9; k++)
            M[k] = tbn[9 * f + k];
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int s = 0; s < S; s++) {
            double L[3], v[4];
            for (int k = 0; k < 3; k++)
                L[k] = kind == 0 ? (double)vec[3 * s + k]
                                 : (double)vec[3 * s + k] - (double)pos[3 * f + k];
            lookup_one(&t, U, M, L, mode, v);
            for (int c = 0; c < C; c++)
                acc[c] += v[c];
        }
        for (int c = 0; c < C; c++)
            out[f * C + c] = acc[c] / S;
    }
}

/* Whether the ray o + t d, t > 0, meets the closed ball (c, r): with d a unit
 * vector, t* = d . (c - o) is the ray parameter of the line's point nearest
 * c and h2 = |c - o|^2 - t*^2 its squared distance from c; the ray meets the
 * ball iff o is inside it, or t* > 0 and h2 <= r^2.  *margin receives
 * | sqrt(h2) - r | when t* > 0 (how far the ray is from grazing the sphere),
 * and +inf otherwise. */
static int ray_meets_ball(const double o[3], const double d[3], const double c[3], double r,
                          double *margin)
{
    double oc[3] = {c[0] - o[0], c[1] - o[1], c[2] - o[2]};
    double l2 = oc[0] * oc[0] + oc[1] * oc[1] + oc[2] * oc[2];
    double ts = d[0] * oc[0] + d[1] * oc[1] + d[2] * oc[2];
    *margin = INFINITY;
    if (l2 <= r * r)
        return 1;
    if (ts <= 0.0)
        return 0;
    double h2 = l2 - ts * ts;
    if (h2 < 0.0)
        h2 = 0.0;
    *margin = fabs(sqrt(h2) - r);
    return h2 <= r * r;
}

/* Bake of a 1-bit shadow texture from analytic occluders (balls) standing in
 * for ray-traced visibility: bucket (i, j) sits at the scene point
 * origins[j][i] with frame M = frames[j][i] (rows T, B, N; NULL: identity);
 * sample (x, y) is lit (bit 1) iff the ray from the origin along M^T I(x, y)
 * meets none of the K balls spheres[k] = (centre x, y, z, radius), I(x, y)
 * being the incidence of the sample centre (Eq. (4a) then Eq. (2c)): the
 * direction that the light lookup maps onto that sample.  words as in
 * orc_pack_bits; margin[(j W + i) n n + y n + x] (if not NULL) receives the
 * smallest grazing margin of that sample's ray over the balls. */
void orc_bake_shadow(int W, int H, int n, const float *origins, const float *frames,
                     const float *spheres, int K, uint32_t *words, double *margin)
{
    int nn = n * n;
    int64_t wpb = ((int64_t)nn + 31) / 32;
    double *I = (double *)malloc(sizeof(double) * 3 * nn);
    if (!I)
        return;
    orc_bake_directions(n, I, NULL);
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < (int64_t)W * H; b++) {
        double M[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
        if (frames)
            for (int k = 0; k < 9; k++)
                M[k] = frames[b * 9 + k];
        double o[3] = {origins[b * 3 + 0], origins[b * 3 + 1], origins[b * 3 + 2]};
        for (int64_t w = 0; w < wpb; w++)
            words[b * wpb + w] = 0u;
        for (int s = 0; s < nn; s++) {
            const double *q = I + 3 * s;
            double d[3];
            for (int k = 0; k < 3; k++) /* (M^T q)_k */
                d[k] = M[0 * 3 + k] * q[0] + M[1 * 3 + k] * q[1] + M[2 * 3 + k] * q[2];
            double len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            for (int k = 0; k < 3; k++)
                d[k] /= len;
            int hit = 0;
            double mg = INFINITY;
            for (int k = 0; k < K; k++) {
                double c[3] = {spheres[4 * k], spheres[4 * k + 1], spheres[4 * k + 2]};
                double m1;
                hit |= ray_meets_ball(o, d, c, spheres[4 * k + 3], &m1);
                if (m1 < mg)
                    mg = m1;
            }
            if (!hit)
                words[b * wpb + s / 32] |= 1u << (s % 32);
            if (margin)
                margin[b * nn + s] = mg;
        }
    }
    free(I);
}

/* ------------------------------------------------------------------------- */
/* Bucket dictionary (the "simple compression" of repetitive buckets, Sec. 1 */
/* and Sec. 2): a codebook of K bucket entries, an index map giving each     */
/* bucket its entry, and optionally a gain per bucket.  Decoded bucket b is  */
/* gain(b) * entry(index(b)); the lookup is the lookup of the decoded matrix. */
/* The codebook is built by Lloyd's k-means iteration on the buckets as      */
/* vectors of D = n n C values.                                              */
/* ------------------------------------------------------------------------- */

/* Lookup of N fragments on a dictionary texture: the codebook (K entries of
 * n n C values, format fmt: F32 or BF16 codes) seen as a K x 1 matrix of
 * buckets, index [H W] int32 in [0, K), gains [H W] or NULL. */
void orc_lookup_fwd_dict(int64_t N, const float *uv, const float *tbn, const float *view, int W,
                         int H, int n, int C, int fmt, const void *codebook, int K,
                         const int32_t *index, const float *gains, int mode, double *out)
{
    /* W_entries = K so that entry k is "bucket" (k, 0) of the codebook */
    tex_t t = {W, H, n, C, fmt, codebook, NULL, index, gains};
    (void)K;
#pragma omp parallel for schedule(static)
    for (int64_t f = 0; f < N; f++) {
        double U[2], M[9], V[3];
        widen_fragment(uv, tbn, view, f, U, M, V);
        lookup_one(&t, U, M, V, mode, out + f * C);
    }
}

/* Assignment step: e(b) = argmin_k |x_b - c_k|^2 over the K entries, the
 * squared distance summed in binary64 from the binary32 values; ties go to
 * the smallest k.  dist[b] receives the minimum. */
void orc_vq_assign(int64_t M, int D, const float *X, int K, const float *Cb, int32_t *assign,
                   double *dist)
{
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < M; b++) {
        const float *x = X + b * D;
        double best = INFINITY;
        int bk = 0;
        for (int k = 0; k < K; k++) {
            const float *c = Cb + (int64_t)k * D;
            double d = 0.0;
            for (int i = 0; i < D; i++) {
                double e = (double)x[i] - (double)c[i];
                d += e * e;
            }
            if (d < best) {
                best = d;
                bk = k;
            }
        }
        assign[b] = bk;
        if (dist)
            dist[b] = best;
    }
}

/* Update step: each entry becomes the mean of the vectors assigned to it
 * (summed in binary64 in increasing b); an entry with no vector keeps its
 * previous value.  out [K][D] binary64, counts [K]. */
void orc_vq_update(int64_t M, int D, const float *X, const int32_t *assign, int K,
                   const float *Cb, double *out, int64_t *counts)
{
    for (int64_t q = 0; q < (int64_t)K * D; q++)
        out[q] = 0.0;
    for (int k = 0; k < K; k++)
        counts[k] = 0;
    for (int64_t b = 0; b < M; b++) {
        int k = assign[b];
        counts[k]++;
        for (int i = 0; i < D; i++)
            out[(int64_t)k * D + i] += (double)X[b * D + i];
    }
    for (int k = 0; k < K; k++)
        for (int i = 0; i < D; i++) {
            int64_t q = (int64_t)k * D + i;
            out[q] = counts[k] ? out[q] / (double)counts[k] : (double)Cb[q];
        }
}
