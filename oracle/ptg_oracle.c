/*
 * ptg_oracle.c -- plain FP64 CPU oracle for polynomial gradient-noise fBm.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg load this library.  The product path (the HIP library) never
 * calls it, and this file shares no code, header, table or constant generator with
 * that library: every constant below is typed here from its definition.
 *
 * Source: Thorimbert & Chopard, "Polynomial methods for fast Procedural Terrain
 * Generation" (arXiv:1610.03525).
 *
 *  - Sec. 2.1, eq. (mixedderiv): corner constraints are prescribed values of the
 *    mixed partial derivatives h^d at the 2^D corners of the unit cell.
 *  - Sec. 2.1, eq. (independance): on an edge, h depends on that edge's two corners
 *    only (so neighbouring cells agree on shared edges).
 *  - Sec. 2.2, eq. (polynomial): h is a tensor polynomial with exponents 0..n per axis,
 *    (n+1)^D coefficients; eq. (nconstraints) bounds the constraint count.  Any order
 *    M = 1..6 (n = 2M+1; the Conclusion's arbitrary smoothness): 1D bases from their
 *    closed forms (orc_hermite_monomials), explicit for M <= 3.
 *  - Sec. 3.4: D1M1N3 with h(0)=0, h(1)=1 and zero end slopes is the smoothstep S3;
 *    D3M1N3 is the 3D analogue; second-order constraints (M=2) give smoother cells.
 *  - Sec. 3.2: Perlin's blend (comparison path) with fade S3 (or S5, Sec. 5.1).
 *  - Sec. 4: the fBm octave sum, amplitude ratio (persistence) and frequency ratio
 *    (lacunarity) per octave.
 *  - Sec. 3.3, eq. (zg): the zero-gradient D2M1N3 cell (random corner heights, zero
 *    corner gradients), with the sign of its xy term read from the Sec. 3.1
 *    coefficients (see orc_zg_cell).
 *  - Sec. 3.1 with non-zero heights and Sec. 4's gradient weight w: corner heights and
 *    w-scaled corner gradients in the same tensor Hermite form (see orc_hg_cell).
 *  - Sec. 5.1 (the gradient-norm maps): the height field's analytic gradient, per octave
 *    the cell derivative times the octave frequency (see orc_fbm_2d_grad).
 *
 * Readings taken where the paper is silent (each one is listed in the design notes):
 *  - Cell polynomial: the unique tensor polynomial of degree n = 2M+1 per axis whose
 *    value is 0 at every corner, whose first partial derivatives equal the corner's
 *    gradient, and whose every other mixed derivative h^d with 0 <= d_k <= M is 0.
 *    With these (M+1)^D conditions per corner the system is square.  Its solution
 *    is the tensor Hermite form evaluated below.
 *  - Octaves o = 0..N-1, amplitude p^o, frequency f0*L^o (both by repeated FP64
 *    multiplication), no normalisation of the sum.
 *  - Sample X (int64 world index) sits at the sample centre: u = (X + 1/2) * f_o,
 *    cell = floor(u), local t = u - cell.
 *  - Lattice: a stated 32-bit hash of (node index, octave, seed) built from the
 *    MurmurHash3 32-bit finalizer (fmix32), mapped to a unit gradient (circle angle
 *    in 2D, Archimedes' cylinder map on the sphere in 3D), or for the zero-gradient
 *    model to a node height uniform on [-1, 1) from the same key's top 24 bits.
 *
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -fopenmp -fPIC -shared
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_MAX_OCTAVES 32
#define ORC_MAX_SMOOTH 6               /* smoothness orders M = 1..6: degree n = 2M+1 <= 13 */
#define ORC_MAX_N1 (2 * ORC_MAX_SMOOTH + 2)

static const double ORC_TWO_PI = 6.283185307179586476925286766559;

/* ------------------------------------------------------------------------- */
/* Lattice hash                                                              */
/* ------------------------------------------------------------------------- */

/* MurmurHash3 32-bit finalizer (Appleby): xor-shift / multiply avalanche. */
uint32_t orc_fmix32(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}

/* Absorb one int64 lattice index: its low 32-bit word, then its high word
 * (two's complement), each xor-ed into the state and followed by fmix32. */
static uint32_t orc_absorb_index(uint32_t k, int64_t i)
{
    uint64_t u = (uint64_t)i;
    uint32_t lo = (uint32_t)(u & 0xFFFFFFFFu);
    uint32_t hi = (uint32_t)(u >> 32);
    k = orc_fmix32(k ^ lo);
    k = orc_fmix32(k ^ hi);
    return k;
}

/* Per-(seed, octave) prefix of every key. */
uint32_t orc_prefix(uint32_t seed, int32_t octave)
{
    uint32_t k = orc_fmix32(seed ^ 0x9E3779B9u);
    k = orc_fmix32(k ^ (uint32_t)octave);
    return k;
}

/* 2D key: the y index is absorbed after the prefix, the x index is hashed from its
 * own salt, and the two are combined by one more fmix32. */
uint32_t orc_key2(int64_t ix, int64_t iy, int32_t octave, uint32_t seed)
{
    uint32_t ky = orc_absorb_index(orc_prefix(seed, octave), iy);
    uint32_t kx = orc_absorb_index(0x27D4EB2Fu, ix);
    return orc_fmix32(ky ^ kx);
}

/* 3D key: z, then y, absorbed after the prefix; x as in 2D. */
uint32_t orc_key3(int64_t ix, int64_t iy, int64_t iz, int32_t octave, uint32_t seed)
{
    uint32_t kzy = orc_absorb_index(orc_absorb_index(orc_prefix(seed, octave), iz), iy);
    uint32_t kx = orc_absorb_index(0x27D4EB2Fu, ix);
    return orc_fmix32(kzy ^ kx);
}

/* Second 32-bit word of a 3D node (the azimuth of its gradient). */
uint32_t orc_key3_second(uint32_t key)
{
    return orc_fmix32(key ^ 0x165667B1u);
}

/* 2D unit gradient: angle = 2*pi * (top 24 bits of the key) / 2^24. */
void orc_grad2(uint32_t key, double *g)
{
    double turns = (double)(key >> 8) * (1.0 / 16777216.0);
    double th = ORC_TWO_PI * turns;
    g[0] = cos(th);
    g[1] = sin(th);
}

/* 3D unit gradient, uniform on the sphere (Archimedes: z uniform on [-1,1]):
 * z = 1 - (2m+1)/2^24 with m the top 24 bits of the key, azimuth from the second word. */
void orc_grad3(uint32_t key, double *g)
{
    uint32_t m1 = key >> 8;
    uint32_t m2 = orc_key3_second(key) >> 8;
    double z = 1.0 - (2.0 * (double)m1 + 1.0) * (1.0 / 16777216.0);
    double phi = ORC_TWO_PI * ((double)m2 * (1.0 / 16777216.0));
    double r2 = 1.0 - z * z;
    double r = sqrt(r2 > 0.0 ? r2 : 0.0);
    g[0] = r * cos(phi);
    g[1] = r * sin(phi);
    g[2] = z;
}

/* ------------------------------------------------------------------------- */
/* Coordinate step and octave parameters                                     */
/* ------------------------------------------------------------------------- */

/* Frequencies f_o = f0 * L^o and amplitudes a_o = p^o, by repeated multiplication. */
void orc_octave_params(double f0, double lac, double pers, int32_t n, double *freq, double *amp)
{
    double f = f0, a = 1.0;
    for (int32_t o = 0; o < n; ++o) {
        if (freq) freq[o] = f;
        if (amp) amp[o] = a;
        f = f * lac;
        a = a * pers;
    }
}

/* Sample centre X + 1/2 in lattice units of frequency f: cell index and local fraction. */
void orc_coord(int64_t X, double f, int64_t *cell, double *t)
{
    double u = ((double)X + 0.5) * f;
    double c = floor(u);
    *cell = (int64_t)c;
    *t = u - c;
}

/* ------------------------------------------------------------------------- */
/* 1D Hermite bases on [0,1]                                                 */
/* ------------------------------------------------------------------------- */

/* Binomial coefficient C(n, k) (exact in FP64 for the small n used here). */
static double orc_binom(int n, int k)
{
    if (k < 0 || k > n) return 0.0;
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (double)(n - k + i) / (double)i;
    return r;
}

/* Monomial coefficients of the 1D Hermite bases of any order M (Sec. 2.2 with n = 2M+1:
 * the value and the first M derivatives prescribed at both ends of [0, 1]), from their
 * closed forms (two-point Taylor interpolation):
 *   S(t)     = t^(M+1) sum_{k=0..M} C(M+k, k) (1-t)^k          (value 1 at t = 1, b0[1])
 *   b1[0](t) = t (1-t)^(M+1) sum_{k=0..M-1} C(M+k, k) t^k       (unit slope at t = 0)
 *   b1[1](t) = -b1[0](1 - t),  b0[0] = 1 - S.
 * Each factor (1-t)^p is expanded with binomial coefficients.  bases[k][e] is the
 * coefficient of t^e of b0[0], b0[1], b1[0], b1[1] (k = 0..3). */
static void orc_hermite_monomials(int32_t M, double bases[4][ORC_MAX_N1])
{
    memset(bases, 0, sizeof(double) * 4 * ORC_MAX_N1);
    for (int k = 0; k <= M; ++k)  /* C(M+k,k) t^(M+1) (1-t)^k */
        for (int i = 0; i <= k; ++i)
            bases[1][M + 1 + i] += orc_binom(M + k, k) * orc_binom(k, i) * ((i & 1) ? -1.0 : 1.0);
    for (int e = 0; e < ORC_MAX_N1; ++e) bases[0][e] = (e == 0 ? 1.0 : 0.0) - bases[1][e];
    for (int k = 0; k < M; ++k)  /* C(M+k,k) t^(k+1) (1-t)^(M+1) */
        for (int i = 0; i <= M + 1; ++i)
            bases[2][1 + k + i] += orc_binom(M + k, k) * orc_binom(M + 1, i) * ((i & 1) ? -1.0 : 1.0);
    for (int p = 0; p < ORC_MAX_N1; ++p)  /* -sum_p c_p (1-t)^p */
        if (bases[2][p] != 0.0)
            for (int j = 0; j <= p; ++j) bases[3][j] -= bases[2][p] * orc_binom(p, j) * ((j & 1) ? -1.0 : 1.0);
}

/* Value (d = 0) or first derivative (d = 1) of a monomial expansion by Horner's rule. */
static double orc_horner(const double *c, int n1, int d, double t)
{
    double v = 0.0;
    for (int e = n1 - 1; e >= d; --e) v = v * t + (d ? (double)e * c[e] : c[e]);
    return v;
}

/* The closed forms above evaluated for any order (including M <= 3, whose explicit forms
 * below are the ones the oracle uses; the tests compare the two). */
void orc_hermite_closed(int32_t M, double t, double *b0, double *b1)
{
    double B[4][ORC_MAX_N1];
    if (M < 1 || M > ORC_MAX_SMOOTH) return;
    orc_hermite_monomials(M, B);
    const int n1 = 2 * M + 2;
    b0[0] = orc_horner(B[0], n1, 0, t);
    b0[1] = orc_horner(B[1], n1, 0, t);
    b1[0] = orc_horner(B[2], n1, 0, t);
    b1[1] = orc_horner(B[3], n1, 0, t);
}

/* Value bases b0[c] (1 at corner c, 0 at the other, zero derivatives up to M at both
 * ends) and slope bases b1[c] (zero value, unit first derivative at corner c, zero
 * first derivative at the other end, zero higher derivatives up to M).
 * Cubic (M=1): b0[1] = S3 = 3t^2 - 2t^3 (Sec. 3.2), b1[0] = t(1-t)^2, b1[1] = -t^2(1-t).
 * Quintic (M=2): b0[1] = S5 = 6t^5 - 15t^4 + 10t^3 (Sec. 5.1),
 *   b1[0] = t - 6t^3 + 8t^4 - 3t^5, b1[1] = -4t^3 + 7t^4 - 3t^5.
 * Septic (M=3, derivatives up to 3 constrained, Sec. 2.2 with n = 7):
 *   b0[1] = S7 = 35t^4 - 84t^5 + 70t^6 - 20t^7,
 *   b1[0] = t - 20t^4 + 45t^5 - 36t^6 + 10t^7, b1[1] = -15t^4 + 39t^5 - 34t^6 + 10t^7.
 * M = 4..6: the closed forms of orc_hermite_monomials. */
void orc_basis(int32_t smooth, double t, double *b0, double *b1)
{
    double t2 = t * t, t3 = t2 * t;
    if (smooth >= 4) { /* any higher order: the closed forms of orc_hermite_monomials */
        double B[4][ORC_MAX_N1];
        orc_hermite_monomials(smooth, B);
        const int n1 = 2 * smooth + 2;
        b0[0] = orc_horner(B[0], n1, 0, t);
        b0[1] = orc_horner(B[1], n1, 0, t);
        b1[0] = orc_horner(B[2], n1, 0, t);
        b1[1] = orc_horner(B[3], n1, 0, t);
        return;
    }
    if (smooth == 1) {
        double s = 3.0 * t2 - 2.0 * t3;
        b0[0] = 1.0 - s;
        b0[1] = s;
        b1[0] = t * (1.0 - t) * (1.0 - t);
        b1[1] = -t2 * (1.0 - t);
    } else if (smooth == 2) {
        double t4 = t3 * t, t5 = t4 * t;
        double s = 6.0 * t5 - 15.0 * t4 + 10.0 * t3;
        b0[0] = 1.0 - s;
        b0[1] = s;
        b1[0] = t - 6.0 * t3 + 8.0 * t4 - 3.0 * t5;
        b1[1] = -4.0 * t3 + 7.0 * t4 - 3.0 * t5;
    } else {
        double t4 = t3 * t, t5 = t4 * t, t6 = t5 * t, t7 = t6 * t;
        double s = 35.0 * t4 - 84.0 * t5 + 70.0 * t6 - 20.0 * t7;
        b0[0] = 1.0 - s;
        b0[1] = s;
        b1[0] = t - 20.0 * t4 + 45.0 * t5 - 36.0 * t6 + 10.0 * t7;
        b1[1] = -15.0 * t4 + 39.0 * t5 - 34.0 * t6 + 10.0 * t7;
    }
}

/* Monomial coefficients of the same bases: bases[k][e] is the coefficient of t^e,
 * k = 0: b0[0], 1: b0[1], 2: b1[0], 3: b1[1]; degree n = 2M+1. */
static void orc_basis_monomials(int32_t smooth, double bases[4][ORC_MAX_N1])
{
    memset(bases, 0, sizeof(double) * 4 * ORC_MAX_N1);
    if (smooth >= 4) {
        orc_hermite_monomials(smooth, bases);
    } else if (smooth == 1) {
        /* 1 - 3t^2 + 2t^3 */
        bases[0][0] = 1.0; bases[0][2] = -3.0; bases[0][3] = 2.0;
        /* 3t^2 - 2t^3 */
        bases[1][2] = 3.0; bases[1][3] = -2.0;
        /* t - 2t^2 + t^3 */
        bases[2][1] = 1.0; bases[2][2] = -2.0; bases[2][3] = 1.0;
        /* -t^2 + t^3 */
        bases[3][2] = -1.0; bases[3][3] = 1.0;
    } else if (smooth == 2) {
        /* 1 - 10t^3 + 15t^4 - 6t^5 */
        bases[0][0] = 1.0; bases[0][3] = -10.0; bases[0][4] = 15.0; bases[0][5] = -6.0;
        /* 10t^3 - 15t^4 + 6t^5 */
        bases[1][3] = 10.0; bases[1][4] = -15.0; bases[1][5] = 6.0;
        /* t - 6t^3 + 8t^4 - 3t^5 */
        bases[2][1] = 1.0; bases[2][3] = -6.0; bases[2][4] = 8.0; bases[2][5] = -3.0;
        /* -4t^3 + 7t^4 - 3t^5 */
        bases[3][3] = -4.0; bases[3][4] = 7.0; bases[3][5] = -3.0;
    } else {
        /* 1 - 35t^4 + 84t^5 - 70t^6 + 20t^7 */
        bases[0][0] = 1.0; bases[0][4] = -35.0; bases[0][5] = 84.0; bases[0][6] = -70.0; bases[0][7] = 20.0;
        /* 35t^4 - 84t^5 + 70t^6 - 20t^7 */
        bases[1][4] = 35.0; bases[1][5] = -84.0; bases[1][6] = 70.0; bases[1][7] = -20.0;
        /* t - 20t^4 + 45t^5 - 36t^6 + 10t^7 */
        bases[2][1] = 1.0; bases[2][4] = -20.0; bases[2][5] = 45.0; bases[2][6] = -36.0; bases[2][7] = 10.0;
        /* -15t^4 + 39t^5 - 34t^6 + 10t^7 */
        bases[3][4] = -15.0; bases[3][5] = 39.0; bases[3][6] = -34.0; bases[3][7] = 10.0;
    }
}

/* ------------------------------------------------------------------------- */
/* One cell                                                                  */
/* ------------------------------------------------------------------------- */

/* 2D cell: corners are indexed c = cx + 2*cy, grad[2*c + a] is component a (0 = x,
 * 1 = y) of the gradient at corner c.
 * h = sum_c [ gx_c * b1[cx](tx) * b0[cy](ty) + gy_c * b0[cx](tx) * b1[cy](ty) ]. */
double orc_cell_2d(int32_t smooth, const double *grad, double tx, double ty)
{
    double bx0[2], bx1[2], by0[2], by1[2];
    orc_basis(smooth, tx, bx0, bx1);
    orc_basis(smooth, ty, by0, by1);
    double h = 0.0;
    for (int cy = 0; cy < 2; ++cy)
        for (int cx = 0; cx < 2; ++cx) {
            int c = cx + 2 * cy;
            h += grad[2 * c + 0] * bx1[cx] * by0[cy];
            h += grad[2 * c + 1] * bx0[cx] * by1[cy];
        }
    return h;
}

/* 3D cell: corner c = cx + 2*cy + 4*cz, grad[3*c + a]. */
double orc_cell_3d(int32_t smooth, const double *grad, double tx, double ty, double tz)
{
    double b0[3][2], b1[3][2];
    orc_basis(smooth, tx, b0[0], b1[0]);
    orc_basis(smooth, ty, b0[1], b1[1]);
    orc_basis(smooth, tz, b0[2], b1[2]);
    double h = 0.0;
    for (int cz = 0; cz < 2; ++cz)
        for (int cy = 0; cy < 2; ++cy)
            for (int cx = 0; cx < 2; ++cx) {
                int c = cx + 2 * cy + 4 * cz;
                h += grad[3 * c + 0] * b1[0][cx] * b0[1][cy] * b0[2][cz];
                h += grad[3 * c + 1] * b0[0][cx] * b1[1][cy] * b0[2][cz];
                h += grad[3 * c + 2] * b0[0][cx] * b0[1][cy] * b1[2][cz];
            }
    return h;
}

/* Monomial coefficients c[i*(n+1) + j] of x^i y^j (eq. polynomial, D = 2) obtained by
 * expanding the Hermite form above. */
void orc_coeffs_2d(int32_t smooth, const double *grad, double *c)
{
    double B[4][ORC_MAX_N1];
    orc_basis_monomials(smooth, B);
    int n1 = 2 * smooth + 2;
    memset(c, 0, sizeof(double) * (size_t)(n1 * n1));
    for (int cy = 0; cy < 2; ++cy)
        for (int cx = 0; cx < 2; ++cx) {
            int k = cx + 2 * cy;
            double gx = grad[2 * k + 0], gy = grad[2 * k + 1];
            for (int i = 0; i < n1; ++i)
                for (int j = 0; j < n1; ++j) {
                    /* x-slope basis of corner cx times y-value basis of corner cy */
                    c[i * n1 + j] += gx * B[2 + cx][i] * B[cy][j];
                    c[i * n1 + j] += gy * B[cx][i] * B[2 + cy][j];
                }
        }
}

/* Monomial coefficients c[(i*(n+1) + j)*(n+1) + k] of x^i y^j z^k (D = 3). */
void orc_coeffs_3d(int32_t smooth, const double *grad, double *c)
{
    double B[4][ORC_MAX_N1];
    orc_basis_monomials(smooth, B);
    int n1 = 2 * smooth + 2;
    memset(c, 0, sizeof(double) * (size_t)(n1 * n1 * n1));
    for (int cz = 0; cz < 2; ++cz)
        for (int cy = 0; cy < 2; ++cy)
            for (int cx = 0; cx < 2; ++cx) {
                int q = cx + 2 * cy + 4 * cz;
                double gx = grad[3 * q + 0], gy = grad[3 * q + 1], gz = grad[3 * q + 2];
                for (int i = 0; i < n1; ++i)
                    for (int j = 0; j < n1; ++j)
                        for (int k = 0; k < n1; ++k) {
                            double *dst = &c[(i * n1 + j) * n1 + k];
                            *dst += gx * B[2 + cx][i] * B[cy][j] * B[cz][k];
                            *dst += gy * B[cx][i] * B[2 + cy][j] * B[cz][k];
                            *dst += gz * B[cx][i] * B[cy][j] * B[2 + cz][k];
                        }
            }
}

/* Perlin's polynomial (Sec. 3.2) on one cell, fade S3 (order 3) or S5 (order 5):
 * v_ij = f_ij (x - i) + g_ij (y - j); h0 = v00 + S(x)(v10 - v00);
 * h1 = v01 + S(x)(v11 - v01); h = h0 + S(y)(h1 - h0).  Same corner indexing as above. */
double orc_perlin_cell(int32_t fade_order, const double *grad, double x, double y)
{
    double v[4];
    for (int cy = 0; cy < 2; ++cy)
        for (int cx = 0; cx < 2; ++cx) {
            int c = cx + 2 * cy;
            v[c] = grad[2 * c] * (x - cx) + grad[2 * c + 1] * (y - cy);
        }
    double sx, sy;
    if (fade_order == 5) {
        sx = 6.0 * pow(x, 5) - 15.0 * pow(x, 4) + 10.0 * pow(x, 3);
        sy = 6.0 * pow(y, 5) - 15.0 * pow(y, 4) + 10.0 * pow(y, 3);
    } else {
        sx = 3.0 * x * x - 2.0 * x * x * x;
        sy = 3.0 * y * y - 2.0 * y * y * y;
    }
    double h0 = v[0] + sx * (v[1] - v[0]);
    double h1 = v[2] + sx * (v[3] - v[2]);
    return h0 + sy * (h1 - h0);
}

/* Simplex-lattice gradient noise (the comparison path standing for the paper's OpenSimplex
 * timings, Sec. 5.2; the paper does not define it).  Written from the public mathematical
 * description of 2D simplex noise: the point u is skewed by F2 = (sqrt 3 - 1) / 2 onto the
 * square lattice (i, j) = floor(u + (ux + uy) F2), the cell's lower or upper triangle is
 * chosen by comparing the unskewed offsets, and each of the three corners c (unskewed by
 * G2 = (3 - sqrt 3) / 6) contributes max(0, 1/2 - |d|^2)^4 (g_c . d), d = u minus the
 * corner, with g_c the unit gradient the lattice hash gives the skewed index; the sum is
 * scaled by 70.  PARITY UNPINNED against any outside implementation: the tests pin only
 * its own properties (zero at lattice points, gradient 70 / 16 g there, smoothness). */
static double orc_simplex_corner(int64_t i, int64_t j, int32_t octave, uint32_t seed, double dx, double dy)
{
    const double t = 0.5 - dx * dx - dy * dy;
    if (t <= 0.0) return 0.0;
    double g[2];
    orc_grad2(orc_key2(i, j, octave, seed), g);
    const double t2 = t * t;
    return t2 * t2 * (g[0] * dx + g[1] * dy);
}

double orc_simplex_at(double ux, double uy, int32_t octave, uint32_t seed)
{
    const double F2 = 0.5 * (sqrt(3.0) - 1.0), G2 = (3.0 - sqrt(3.0)) / 6.0;
    const double s = (ux + uy) * F2;
    const double fi = floor(ux + s), fj = floor(uy + s);
    const double t = (fi + fj) * G2;
    const double x0 = ux - (fi - t), y0 = uy - (fj - t);
    const int i1 = x0 > y0 ? 1 : 0, j1 = 1 - i1;
    const int64_t i = (int64_t)fi, j = (int64_t)fj;
    double n = orc_simplex_corner(i, j, octave, seed, x0, y0);
    n += orc_simplex_corner(i + i1, j + j1, octave, seed, x0 - i1 + G2, y0 - j1 + G2);
    n += orc_simplex_corner(i + 1, j + 1, octave, seed, x0 - 1.0 + 2.0 * G2, y0 - 1.0 + 2.0 * G2);
    return 70.0 * n;
}

/* ------------------------------------------------------------------------- */
/* fBm over samples                                                          */
/* ------------------------------------------------------------------------- */

static int orc_check(int32_t smooth, int32_t octaves, double f0, double lac, double pers)
{
    if (smooth < 1 || smooth > ORC_MAX_SMOOTH) return ORC_EINVAL;
    if (octaves < 1 || octaves > ORC_MAX_OCTAVES) return ORC_EINVAL;
    if (!(f0 > 0.0) || !(lac > 0.0) || !(pers > 0.0)) return ORC_EINVAL;
    if (!isfinite(f0) || !isfinite(lac) || !isfinite(pers)) return ORC_EINVAL;
    return ORC_OK;
}

/* H at one 2D sample (X, Y): sum over octaves o of p^o * h_o, in octave order. */
static double orc_sample_2d(int32_t smooth, int32_t octaves, const double *freq, const double *amp,
                            uint32_t seed, int64_t X, int64_t Y)
{
    double H = 0.0;
    for (int32_t o = 0; o < octaves; ++o) {
        int64_t cx, cy;
        double tx, ty, grad[8];
        orc_coord(X, freq[o], &cx, &tx);
        orc_coord(Y, freq[o], &cy, &ty);
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx)
                orc_grad2(orc_key2(cx + dx, cy + dy, o, seed), &grad[2 * (dx + 2 * dy)]);
        H += amp[o] * orc_cell_2d(smooth, grad, tx, ty);
    }
    return H;
}

static double orc_sample_3d(int32_t smooth, int32_t octaves, const double *freq, const double *amp,
                            uint32_t seed, int64_t X, int64_t Y, int64_t Z)
{
    double H = 0.0;
    for (int32_t o = 0; o < octaves; ++o) {
        int64_t cx, cy, cz;
        double tx, ty, tz, grad[24];
        orc_coord(X, freq[o], &cx, &tx);
        orc_coord(Y, freq[o], &cy, &ty);
        orc_coord(Z, freq[o], &cz, &tz);
        for (int dz = 0; dz < 2; ++dz)
            for (int dy = 0; dy < 2; ++dy)
                for (int dx = 0; dx < 2; ++dx)
                    orc_grad3(orc_key3(cx + dx, cy + dy, cz + dz, o, seed),
                              &grad[3 * (dx + 2 * dy + 4 * dz)]);
        H += amp[o] * orc_cell_3d(smooth, grad, tx, ty, tz);
    }
    return H;
}

static void orc_set_threads(int32_t nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

/* Row-major [ny][nx] field; sample (i, j) is world (x0 + i, y0 + j). */
int orc_fbm_2d(int32_t smooth, int32_t octaves, double pers, double lac, double f0, uint32_t seed,
               int64_t x0, int64_t y0, int64_t nx, int64_t ny, double *out, int32_t nthreads)
{
    if (orc_check(smooth, octaves, f0, lac, pers) != ORC_OK || nx < 0 || ny < 0 || !out)
        return ORC_EINVAL;
    double freq[ORC_MAX_OCTAVES], amp[ORC_MAX_OCTAVES];
    orc_octave_params(f0, lac, pers, octaves, freq, amp);
    orc_set_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < ny; ++j)
        for (int64_t i = 0; i < nx; ++i)
            out[j * nx + i] = orc_sample_2d(smooth, octaves, freq, amp, seed, x0 + i, y0 + j);
    return ORC_OK;
}

/* Row-major [nz][ny][nx] volume. */
int orc_fbm_3d(int32_t smooth, int32_t octaves, double pers, double lac, double f0, uint32_t seed,
               int64_t x0, int64_t y0, int64_t z0, int64_t nx, int64_t ny, int64_t nz, double *out,
               int32_t nthreads)
{
    if (orc_check(smooth, octaves, f0, lac, pers) != ORC_OK || nx < 0 || ny < 0 || nz < 0 || !out)
        return ORC_EINVAL;
    double freq[ORC_MAX_OCTAVES], amp[ORC_MAX_OCTAVES];
    orc_octave_params(f0, lac, pers, octaves, freq, amp);
    orc_set_threads(nthreads);
    int64_t lines = ny * nz;
#pragma omp parallel for schedule(static)
    for (int64_t l = 0; l < lines; ++l) {
        int64_t j = l % ny, k = l / ny;
        for (int64_t i = 0; i < nx; ++i)
            out[l * nx + i] = orc_sample_3d(smooth, octaves, freq, amp, seed, x0 + i, y0 + j, z0 + k);
    }
    return ORC_OK;
}

/* The same sum at an explicit list of world samples (for sampled checks of large fields). */
int orc_fbm_points_2d(int32_t smooth, int32_t octaves, double pers, double lac, double f0,
                      uint32_t seed, const int64_t *X, const int64_t *Y, int64_t n, double *out,
                      int32_t nthreads)
{
    if (orc_check(smooth, octaves, f0, lac, pers) != ORC_OK || n < 0 || !X || !Y || !out)
        return ORC_EINVAL;
    double freq[ORC_MAX_OCTAVES], amp[ORC_MAX_OCTAVES];
    orc_octave_params(f0, lac, pers, octaves, freq, amp);
    orc_set_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < n; ++q)
        out[q] = orc_sample_2d(smooth, octaves, freq, amp, seed, X[q], Y[q]);
    return ORC_OK;
}

int orc_fbm_points_3d(int32_t smooth, int32_t octaves, double pers, double lac, double f0,
                      uint32_t seed, const int64_t *X, const int64_t *Y, const int64_t *Z, int64_t n,
                      double *out, int32_t nthreads)
{
    if (orc_check(smooth, octaves, f0, lac, pers) != ORC_OK || n < 0 || !X || !Y || !Z || !out)
        return ORC_EINVAL;
    double freq[ORC_MAX_OCTAVES], amp[ORC_MAX_OCTAVES];
    orc_octave_params(f0, lac, pers, octaves, freq, amp);
    orc_set_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < n; ++q)
        out[q] = orc_sample_3d(smooth, octaves, freq, amp, seed, X[q], Y[q], Z[q]);
    return ORC_OK;
}

/* Perlin fBm (comparison path, Sec. 3.2) over a 2D field with the same lattice, octave
 * and coordinate conventions. */
int orc_perlin_2d(int32_t fade_order, int32_t octaves, double pers, double lac, double f0,
                  uint32_t seed, int64_t x0, int64_t y0, int64_t nx, int64_t ny, double *out,
                  int32_t nthreads)
{
    if ((fade_order != 3 && fade_order != 5) || orc_check(1, octaves, f0, lac, pers) != ORC_OK ||
        nx < 0 || ny < 0 || !out)
        return ORC_EINVAL;
    double freq[ORC_MAX_OCTAVES], amp[ORC_MAX_OCTAVES];
    orc_octave_params(f0, lac, pers, octaves, freq, amp);
    orc_set_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < ny; ++j)
        for (int64_t i = 0; i < nx; ++i) {
            double H = 0.0;
            for (int32_t o = 0; o < octaves; ++o) {
                int64_t cx, cy;
                double tx, ty, grad[8];
                orc_coord(x0 + i, freq[o], &cx, &tx);
                orc_coord(y0 + j, freq[o], &cy, &ty);
                for (int dy = 0; dy < 2; ++dy)
                    for (int dx = 0; dx < 2; ++dx)
                        orc_grad2(orc_key2(cx + dx, cy + dy, o, seed), &grad[2 * (dx + 2 * dy)]);
                H += amp[o] * orc_perlin_cell(fade_order, grad, tx, ty);
            }
            out[j * nx + i] = H;
        }
    return ORC_OK;
}

/* Simplex-lattice fBm (comparison path, parity unpinned): octave o at u = (X + 1/2) f_o. */
int orc_simplex_2d(int32_t octaves, double pers, double lac, double f0, uint32_t seed, int64_t x0, int64_t y0,
                   int64_t nx, int64_t ny, double *out, int32_t nthreads)
{
    if (orc_check(1, octaves, f0, lac, pers) != ORC_OK || nx < 0 || ny < 0 || !out) return ORC_EINVAL;
    double freq[ORC_MAX_OCTAVES], amp[ORC_MAX_OCTAVES];
    orc_octave_params(f0, lac, pers, octaves, freq, amp);
    orc_set_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < ny; ++j)
        for (int64_t i = 0; i < nx; ++i) {
            double H = 0.0;
            for (int32_t o = 0; o < octaves; ++o)
                H += amp[o] * orc_simplex_at(((double)(x0 + i) + 0.5) * freq[o], ((double)(y0 + j) + 0.5) * freq[o],
                                             o, seed);
            out[j * nx + i] = H;
        }
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Zero-gradient D2M1N3 (Sec. 3.3, eq. zg)                                   */
/* ------------------------------------------------------------------------- */

/* Node height of the zero-gradient model: uniform on [-1, 1) from the top 24 bits of
 * the node's key, h = m / 2^23 - 1 (exact in binary). */
double orc_height2(uint32_t key)
{
    return (double)(key >> 8) / 8388608.0 - 1.0;
}

/* D2M1N3 with all corner gradients zero (Sec. 3.3): with the corner heights
 * h = {h00, h10, h01, h11}, dx = h10 - h00, dy = h01 - h00, A = h11 + h00 - h10 - h01
 * and the smoothstep S3(t) = 3t^2 - 2t^3,
 *   h(x, y) = h00 + S3(x) dx + S3(y) dy + A (S3(x) y + S3(y) x - x y).
 * The paper prints the last term as +xy; the Sec. 3.1 coefficients with f = g = 0
 * (c11 = -A, c21 = c12 = 3A, c31 = c13 = -2A) give -xy, which is also what makes
 * h(1, 1) = h11.  That corrected form is the one evaluated here. */
double orc_zg_cell(const double *h, double x, double y)
{
    double sx = x * x * (3.0 - 2.0 * x), sy = y * y * (3.0 - 2.0 * y);
    double dx = h[1] - h[0], dy = h[2] - h[0], A = h[3] + h[0] - h[1] - h[2];
    return h[0] + sx * dx + sy * dy + A * (sx * y + sy * x - x * y);
}

static double orc_zg_sample(int32_t octaves, const double *freq, const double *amp, uint32_t seed, int64_t X,
                            int64_t Y)
{
    double H = 0.0;
    for (int32_t o = 0; o < octaves; ++o) {
        int64_t cx, cy;
        double tx, ty, h[4];
        orc_coord(X, freq[o], &cx, &tx);
        orc_coord(Y, freq[o], &cy, &ty);
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) h[dx + 2 * dy] = orc_height2(orc_key2(cx + dx, cy + dy, o, seed));
        H += amp[o] * orc_zg_cell(h, tx, ty);
    }
    return H;
}

/* Zero-gradient fBm over a row-major [ny][nx] field (same lattice, octave and
 * coordinate conventions as orc_fbm_2d). */
int orc_zg_fbm_2d(int32_t octaves, double pers, double lac, double f0, uint32_t seed, int64_t x0, int64_t y0,
                  int64_t nx, int64_t ny, double *out, int32_t nthreads)
{
    if (orc_check(1, octaves, f0, lac, pers) != ORC_OK || nx < 0 || ny < 0 || !out) return ORC_EINVAL;
    double freq[ORC_MAX_OCTAVES], amp[ORC_MAX_OCTAVES];
    orc_octave_params(f0, lac, pers, octaves, freq, amp);
    orc_set_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < ny; ++j)
        for (int64_t i = 0; i < nx; ++i) out[j * nx + i] = orc_zg_sample(octaves, freq, amp, seed, x0 + i, y0 + j);
    return ORC_OK;
}

int orc_zg_fbm_points_2d(int32_t octaves, double pers, double lac, double f0, uint32_t seed, const int64_t *X,
                         const int64_t *Y, int64_t n, double *out, int32_t nthreads)
{
    if (orc_check(1, octaves, f0, lac, pers) != ORC_OK || n < 0 || !X || !Y || !out) return ORC_EINVAL;
    double freq[ORC_MAX_OCTAVES], amp[ORC_MAX_OCTAVES];
    orc_octave_params(f0, lac, pers, octaves, freq, amp);
    orc_set_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < n; ++q) out[q] = orc_zg_sample(octaves, freq, amp, seed, X[q], Y[q]);
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Heights and weighted gradients (Sec. 3.1 with non-zero heights, Sec. 4 w) */
/* ------------------------------------------------------------------------- */

/* Node height of the height-and-gradient model: uniform on [-1, 1) from the top 24 bits
 * of the node's second word (the gradient takes the first word's top bits, so the two
 * are independent). */
double orc_height2_second(uint32_t key)
{
    return orc_height2(orc_key3_second(key));
}

/* Tensor Hermite cell with corner heights h[c] and corner gradients w * grad[2c..2c+1]
 * (c = cx + 2 cy; mixed derivatives zero): h(x, y) = sum_c h_c B0_cx(x) B0_cy(y) plus
 * w times the zero-height cell of orc_cell_2d. */
double orc_hg_cell(int32_t smooth, const double *h, const double *grad, double w, double tx, double ty)
{
    double bx0[2], bx1[2], by0[2], by1[2];
    orc_basis(smooth, tx, bx0, bx1);
    orc_basis(smooth, ty, by0, by1);
    double v = 0.0;
    for (int cy = 0; cy < 2; ++cy)
        for (int cx = 0; cx < 2; ++cx) v += h[cx + 2 * cy] * bx0[cx] * by0[cy];
    return v + w * orc_cell_2d(smooth, grad, tx, ty);
}

static double orc_hg_sample(int32_t smooth, int32_t octaves, const double *freq, const double *amp, double w,
                            uint32_t seed, int64_t X, int64_t Y)
{
    double H = 0.0;
    for (int32_t o = 0; o < octaves; ++o) {
        int64_t cx, cy;
        double tx, ty, h[4], grad[8];
        orc_coord(X, freq[o], &cx, &tx);
        orc_coord(Y, freq[o], &cy, &ty);
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                uint32_t key = orc_key2(cx + dx, cy + dy, o, seed);
                h[dx + 2 * dy] = orc_height2_second(key);
                orc_grad2(key, &grad[2 * (dx + 2 * dy)]);
            }
        H += amp[o] * orc_hg_cell(smooth, h, grad, w, tx, ty);
    }
    return H;
}

/* Height-and-gradient fBm over a row-major [ny][nx] field; w = gradient weight. */
int orc_hg_fbm_2d(int32_t smooth, int32_t octaves, double pers, double lac, double f0, double w, uint32_t seed,
                  int64_t x0, int64_t y0, int64_t nx, int64_t ny, double *out, int32_t nthreads)
{
    if (orc_check(smooth, octaves, f0, lac, pers) != ORC_OK || !isfinite(w) || nx < 0 || ny < 0 || !out)
        return ORC_EINVAL;
    double freq[ORC_MAX_OCTAVES], amp[ORC_MAX_OCTAVES];
    orc_octave_params(f0, lac, pers, octaves, freq, amp);
    orc_set_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < ny; ++j)
        for (int64_t i = 0; i < nx; ++i)
            out[j * nx + i] = orc_hg_sample(smooth, octaves, freq, amp, w, seed, x0 + i, y0 + j);
    return ORC_OK;
}

int orc_hg_fbm_points_2d(int32_t smooth, int32_t octaves, double pers, double lac, double f0, double w,
                         uint32_t seed, const int64_t *X, const int64_t *Y, int64_t n, double *out, int32_t nthreads)
{
    if (orc_check(smooth, octaves, f0, lac, pers) != ORC_OK || !isfinite(w) || n < 0 || !X || !Y || !out)
        return ORC_EINVAL;
    double freq[ORC_MAX_OCTAVES], amp[ORC_MAX_OCTAVES];
    orc_octave_params(f0, lac, pers, octaves, freq, amp);
    orc_set_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < n; ++q) out[q] = orc_hg_sample(smooth, octaves, freq, amp, w, seed, X[q], Y[q]);
    return ORC_OK;
}

/* 3D (D3M1N3 / D3M2N5 with node heights, Sec. 3.4 with Sec. 3.1's heights and Sec. 4's
 * w).  The 3D gradient takes the first word's top bits (polar coordinate) and the second
 * word's (azimuth), so the node height comes from a third word: the second-word map
 * applied once more to the second word. */
double orc_height3(uint32_t key)
{
    return orc_height2(orc_key3_second(orc_key3_second(key)));
}

/* 3D tensor Hermite cell with corner heights h[c] and corner gradients w * grad[3c..3c+2]
 * (c = cx + 2 cy + 4 cz; every other mixed derivative zero): the trilinear-in-B0 height
 * term sum_c h_c B0_cx(x) B0_cy(y) B0_cz(z) plus w times the zero-height cell. */
double orc_hg_cell_3d(int32_t smooth, const double *h, const double *grad, double w, double tx, double ty,
                      double tz)
{
    double b0[3][2], b1[3][2];
    orc_basis(smooth, tx, b0[0], b1[0]);
    orc_basis(smooth, ty, b0[1], b1[1]);
    orc_basis(smooth, tz, b0[2], b1[2]);
    double v = 0.0;
    for (int cz = 0; cz < 2; ++cz)
        for (int cy = 0; cy < 2; ++cy)
            for (int cx = 0; cx < 2; ++cx) v += h[cx + 2 * cy + 4 * cz] * b0[0][cx] * b0[1][cy] * b0[2][cz];
    return v + w * orc_cell_3d(smooth, grad, tx, ty, tz);
}

static double orc_hg_sample_3d(int32_t smooth, int32_t octaves, const double *freq, const double *amp, double w,
                               uint32_t seed, int64_t X, int64_t Y, int64_t Z)
{
    double H = 0.0;
    for (int32_t o = 0; o < octaves; ++o) {
        int64_t cx, cy, cz;
        double tx, ty, tz, h[8], grad[24];
        orc_coord(X, freq[o], &cx, &tx);
        orc_coord(Y, freq[o], &cy, &ty);
        orc_coord(Z, freq[o], &cz, &tz);
        for (int dz = 0; dz < 2; ++dz)
            for (int dy = 0; dy < 2; ++dy)
                for (int dx = 0; dx < 2; ++dx) {
                    const int c = dx + 2 * dy + 4 * dz;
                    const uint32_t key = orc_key3(cx + dx, cy + dy, cz + dz, o, seed);
                    h[c] = orc_height3(key);
                    orc_grad3(key, &grad[3 * c]);
                }
        H += amp[o] * orc_hg_cell_3d(smooth, h, grad, w, tx, ty, tz);
    }
    return H;
}

/* Height-and-gradient fBm over a dense [nz][ny][nx] volume; w = gradient weight. */
int orc_hg_fbm_3d(int32_t smooth, int32_t octaves, double pers, double lac, double f0, double w, uint32_t seed,
                  int64_t x0, int64_t y0, int64_t z0, int64_t nx, int64_t ny, int64_t nz, double *out,
                  int32_t nthreads)
{
    if (orc_check(smooth, octaves, f0, lac, pers) != ORC_OK || !isfinite(w) || nx < 0 || ny < 0 || nz < 0 || !out)
        return ORC_EINVAL;
    double freq[ORC_MAX_OCTAVES], amp[ORC_MAX_OCTAVES];
    orc_octave_params(f0, lac, pers, octaves, freq, amp);
    orc_set_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i)
                out[(k * ny + j) * nx + i] = orc_hg_sample_3d(smooth, octaves, freq, amp, w, seed, x0 + i, y0 + j,
                                                               z0 + k);
    return ORC_OK;
}

int orc_hg_fbm_points_3d(int32_t smooth, int32_t octaves, double pers, double lac, double f0, double w,
                         uint32_t seed, const int64_t *X, const int64_t *Y, const int64_t *Z, int64_t n, double *out,
                         int32_t nthreads)
{
    if (orc_check(smooth, octaves, f0, lac, pers) != ORC_OK || !isfinite(w) || n < 0 || !X || !Y || !Z || !out)
        return ORC_EINVAL;
    double freq[ORC_MAX_OCTAVES], amp[ORC_MAX_OCTAVES];
    orc_octave_params(f0, lac, pers, octaves, freq, amp);
    orc_set_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < n; ++q)
        out[q] = orc_hg_sample_3d(smooth, octaves, freq, amp, w, seed, X[q], Y[q], Z[q]);
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Analytic gradient of the height field (the gradient maps of Sec. 5.1)     */
/* ------------------------------------------------------------------------- */

/* Derivatives d/dt of the 1D bases of orc_basis. */
void orc_basis_deriv(int32_t smooth, double t, double *db0, double *db1)
{
    double t2 = t * t, t3 = t2 * t;
    double ds;
    if (smooth >= 4) {
        double B[4][ORC_MAX_N1];
        orc_hermite_monomials(smooth, B);
        const int n1 = 2 * smooth + 2;
        db0[0] = orc_horner(B[0], n1, 1, t);
        db0[1] = orc_horner(B[1], n1, 1, t);
        db1[0] = orc_horner(B[2], n1, 1, t);
        db1[1] = orc_horner(B[3], n1, 1, t);
        return;
    }
    if (smooth == 1) {
        ds = 6.0 * t - 6.0 * t2;
        db1[0] = 1.0 - 4.0 * t + 3.0 * t2;
        db1[1] = -2.0 * t + 3.0 * t2;
    } else if (smooth == 2) {
        double t4 = t3 * t;
        ds = 30.0 * t2 - 60.0 * t3 + 30.0 * t4;
        db1[0] = 1.0 - 18.0 * t2 + 32.0 * t3 - 15.0 * t4;
        db1[1] = -12.0 * t2 + 28.0 * t3 - 15.0 * t4;
    } else {
        double t4 = t3 * t, t5 = t4 * t, t6 = t5 * t;
        ds = 140.0 * t3 - 420.0 * t4 + 420.0 * t5 - 140.0 * t6;
        db1[0] = 1.0 - 80.0 * t3 + 225.0 * t4 - 216.0 * t5 + 70.0 * t6;
        db1[1] = -60.0 * t3 + 195.0 * t4 - 204.0 * t5 + 70.0 * t6;
    }
    db0[0] = -ds;
    db0[1] = ds;
}

/* Value and its derivatives in the cell coordinates (d/dtx, d/dty) of one cell of model
 * 0 (gradient), 1 (zero-gradient, smooth = 1) or 2 (heights and w-weighted gradients);
 * h[4] heights (models 1, 2), grad[8] gradients (models 0, 2). */
void orc_cell_2d_grad(int32_t model, int32_t smooth, const double *h, const double *grad, double w, double tx,
                      double ty, double *out)
{
    if (model == 1) {
        double sx = tx * tx * (3.0 - 2.0 * tx), sy = ty * ty * (3.0 - 2.0 * ty);
        double dsx = 6.0 * tx * (1.0 - tx), dsy = 6.0 * ty * (1.0 - ty);
        double dx = h[1] - h[0], dy = h[2] - h[0], A = h[3] + h[0] - h[1] - h[2];
        out[0] = orc_zg_cell(h, tx, ty);
        out[1] = dsx * dx + A * (dsx * ty + sy - ty);
        out[2] = dsy * dy + A * (sx + dsy * tx - tx);
        return;
    }
    double bx0[2], bx1[2], by0[2], by1[2], dbx0[2], dbx1[2], dby0[2], dby1[2];
    orc_basis(smooth, tx, bx0, bx1);
    orc_basis(smooth, ty, by0, by1);
    orc_basis_deriv(smooth, tx, dbx0, dbx1);
    orc_basis_deriv(smooth, ty, dby0, dby1);
    double v = 0.0, vx = 0.0, vy = 0.0;
    double gw = (model == 2) ? w : 1.0;
    for (int cy = 0; cy < 2; ++cy)
        for (int cx = 0; cx < 2; ++cx) {
            int c = cx + 2 * cy;
            double gx = gw * grad[2 * c], gy = gw * grad[2 * c + 1];
            v += gx * bx1[cx] * by0[cy] + gy * bx0[cx] * by1[cy];
            vx += gx * dbx1[cx] * by0[cy] + gy * dbx0[cx] * by1[cy];
            vy += gx * bx1[cx] * dby0[cy] + gy * bx0[cx] * dby1[cy];
            if (model == 2) {
                v += h[c] * bx0[cx] * by0[cy];
                vx += h[c] * dbx0[cx] * by0[cy];
                vy += h[c] * bx0[cx] * dby0[cy];
            }
        }
    out[0] = v;
    out[1] = vx;
    out[2] = vy;
}

/* H and its world-space gradient (dH/dX, dH/dY = sum_o a_o f_o dh_o/dt) over a row-major
 * [ny][nx] field, for any of the three models. */
int orc_fbm_2d_grad(int32_t model, int32_t smooth, int32_t octaves, double pers, double lac, double f0, double w,
                    uint32_t seed, int64_t x0, int64_t y0, int64_t nx, int64_t ny, double *out_h, double *out_dx,
                    double *out_dy, int32_t nthreads)
{
    if (orc_check(smooth, octaves, f0, lac, pers) != ORC_OK || model < 0 || model > 2 || (model == 1 && smooth != 1) ||
        !isfinite(w) || nx < 0 || ny < 0 || !out_h || !out_dx || !out_dy)
        return ORC_EINVAL;
    double freq[ORC_MAX_OCTAVES], amp[ORC_MAX_OCTAVES];
    orc_octave_params(f0, lac, pers, octaves, freq, amp);
    orc_set_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < ny; ++j)
        for (int64_t i = 0; i < nx; ++i) {
            double H = 0.0, HX = 0.0, HY = 0.0;
            for (int32_t o = 0; o < octaves; ++o) {
                int64_t cx, cy;
                double tx, ty, h[4], grad[8], v[3];
                orc_coord(x0 + i, freq[o], &cx, &tx);
                orc_coord(y0 + j, freq[o], &cy, &ty);
                for (int dy = 0; dy < 2; ++dy)
                    for (int dx = 0; dx < 2; ++dx) {
                        uint32_t key = orc_key2(cx + dx, cy + dy, o, seed);
                        int c = dx + 2 * dy;
                        h[c] = (model == 1) ? orc_height2(key) : orc_height2_second(key);
                        orc_grad2(key, &grad[2 * c]);
                    }
                orc_cell_2d_grad(model, smooth, h, grad, w, tx, ty, v);
                H += amp[o] * v[0];
                HX += amp[o] * freq[o] * v[1];
                HY += amp[o] * freq[o] * v[2];
            }
            out_h[j * nx + i] = H;
            out_dx[j * nx + i] = HX;
            out_dy[j * nx + i] = HY;
        }
    return ORC_OK;
}

/* Number of OpenMP threads a parallel region would use (reported with timings). */
int32_t orc_max_threads(void)
{
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}
