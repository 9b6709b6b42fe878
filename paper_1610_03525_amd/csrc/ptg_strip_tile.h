// ptg_strip_tile.h -- K3 for 2D dyadic octave ladders (base frequency 2^-k, lacunarity 2),
// plain FP32 form on the vector ALUs: the per-strip device code, shared by the dense
// kernel (ptg_fbm_strip.hip) and the persistent serving kernel (ptg_serve.hip).
//
// With f_o = 2^-s the sample-centre fraction is exact: t = (2 (X mod 2^s) + 1) / 2^(s+1).
// One wave owns a world-aligned strip of kStripW x kStripH (64 x 64) samples, lane = column,
// and walks strips with a grid stride; the waves of a workgroup never synchronise after the
// prologue.
//
// Cell polynomial (Sec. 2, Sec. 3.4), fixed column x: the 1D Hermite form in y
//   h(y) = E0 + (E1 - E0) S(t) + Q0 b10(t) + Q1 b11(t),
//   E_cy = gx(cx, cy) b10(tx) + gx(cx+1, cy) b11(tx),  Q_cy = gy(cx, cy) + S(tx) (gy(cx+1, cy) - gy(cx, cy)).
// Octaves are summed in three ways:
//  * period >= 64: a lane's column meets one cell of the octave over the whole strip, so
//    each such octave's column form is re-expanded in the strip's centred row coordinate
//    v = (2 r - 63) / 128 (t - 1/2 = tau + sigma v, sigma = 64 / P) and all of them are added
//    into ONE polynomial of degree 2M+1 per lane;
//  * periods 32 and 16 (and 8 for cubic cells): the same, once per half / quarter /
//    period-8 cell, after the fused polynomial is re-centred there (a piece is never
//    evaluated away from its own cell: FP32 error of a quintic piece expanded about the
//    strip centre would reach 4e-5 of the total amplitude); rows are evaluated in pairs
//    symmetric about the segment centre from the polynomial's even and odd parts;
//  * the finer periods: each node row is collapsed along x once (adjacent cells share it)
//    and evaluated per row with the row bases as constants (the row's position inside its
//    cell is fixed by the unrolled row loop); which of these periods occur is a template
//    parameter (the finest shift LO), so the row loop carries no per-row tests.
// x-weights of the periods <= 64 depend on the lane only and are formed once per wave; the
// octave amplitude is folded into them.  Octaves accumulate in FP32; each sample is stored
// once.
//
// Per strip the wave first hashes its own footprint nodes into a private LDS block (K1
// logic: one key per node column and row, one fmix32 per node, unit gradients); the work
// lists that map lanes to nodes are the same for every strip and are built once per
// workgroup.  Periods 2 and 1 are streamed instead: each row segment hashes its own node
// rows of those octaves into a block one segment high (a whole strip's 65 x 65 nodes at
// period 1 would fill the LDS with one or two waves per CU).
#pragma once

#include <hip/hip_fp16.h>

#include "ptg_device.h"
#include "ptg_launch.h"

namespace ptg {

template <typename T>
__device__ __forceinline__ T st_out(float v);
template <>
__device__ __forceinline__ float st_out<float>(float v)
{
    return v;
}
template <>
__device__ __forceinline__ __half st_out<__half>(float v)
{
    return __float2half_rn(v);
}

struct XB {  // 1D bases of a column fraction: S, b10, b11
    float s, b10, b11;
};

template <int M>
__device__ __forceinline__ XB xbases(float t)
{
    XB r;
    Basis<M>::eval(t, r.s, r.b10, r.b11);
    return r;
}

// A lane's x-weights of one octave with the octave amplitude folded in: the value term of a
// node row is gx0 e0 + gx1 e1 (e = amp b1), its y-slope term gy0 q0 + gy1 q1 (q = amp b0).
// Height-and-gradient model (MD = 2): the gradient weights carry w, and the node heights'
// value term is h0 v0 + h1 v1 (v = amp b0).
struct XA {
    float q0, q1, e0, e1, v0, v1;
};

// DX = true: the weights' derivatives d/dt (a node row's E and Q are linear in the lane's
// weights, so the same row machinery then sums d/dt of every cell; the caller folds 1/P into
// amp for d/dX in samples).
template <int M, int MD = 0, bool DX = false>
__device__ __forceinline__ XA xweights(float t, float amp, float gw = 1.0f)
{
    XB b;
    float tt = t, one = 1.0f;  // t and 1 - t, or their derivatives 1 and 0
    if (DX) {
        BasisD<M>::eval(t, b.s, b.b10, b.b11);
        tt = 1.0f;
        one = 0.0f;
    } else {
        b = xbases<M>(t);
    }
    if (MD == 1)  // zero-gradient model: the nodes hold heights (E = h0 + S D, Q = (S - t) D)
        return XA{amp * (tt - b.s), amp * (b.s - tt), amp * (one - b.s), amp * b.s, 0.0f, 0.0f};
    if (MD == 2) {
        const float aw = amp * gw;
        return XA{aw * (one - b.s), aw * b.s, aw * b.b10, aw * b.b11, amp * (one - b.s), amp * b.s};
    }
    return XA{amp * (one - b.s), amp * b.s, amp * b.b10, amp * b.b11, 0.0f, 0.0f};
}

// Row bases at the fraction (j + 1/2) / P: constant once the row loop is unrolled.
template <int M>
__host__ __device__ constexpr XB row_bases(int j, int P)
{
    const float t = (float)(2 * j + 1) / (float)(2 * P);
    const float t2 = t * t;
    const float u = 1.0f - t;
    if (M == 1) return XB{t2 * (3.0f - 2.0f * t), t * u * u, -t2 * u};
    const float t3 = t2 * t;
    if (M == 3) {
        const float t4 = t2 * t2;
        return XB{t4 * (35.0f + t * (-84.0f + t * (70.0f - 20.0f * t))),
                  t + t4 * (-20.0f + t * (45.0f + t * (-36.0f + 10.0f * t))),
                  t4 * (-15.0f + t * (39.0f + t * (-34.0f + 10.0f * t)))};
    }
    return XB{t3 * (10.0f + t * (-15.0f + 6.0f * t)), t + t3 * (-6.0f + t * (8.0f - 3.0f * t)),
              t3 * (-4.0f + t * (7.0f - 3.0f * t))};
}

// Derivatives d/dt of the row bases at the fraction (j + 1/2) / P, times 1/P (d/dY in
// samples).
template <int M>
__host__ __device__ constexpr XB row_dbases(int j, int P)
{
    const float t = (float)(2 * j + 1) / (float)(2 * P), ip = 1.0f / (float)P;
    const float t2 = t * t;
    if (M == 1) return XB{6.0f * t * (1.0f - t) * ip, (1.0f + t * (-4.0f + 3.0f * t)) * ip, t * (-2.0f + 3.0f * t) * ip};
    if (M == 3) {
        const float t3 = t2 * t;
        return XB{t3 * (140.0f + t * (-420.0f + t * (420.0f - 140.0f * t))) * ip,
                  (1.0f + t3 * (-80.0f + t * (225.0f + t * (-216.0f + 70.0f * t)))) * ip,
                  t3 * (-60.0f + t * (195.0f + t * (-204.0f + 70.0f * t))) * ip};
    }
    return XB{t2 * (30.0f + t * (-60.0f + 30.0f * t)) * ip, (1.0f + t2 * (-18.0f + t * (32.0f - 15.0f * t))) * ip,
              t2 * (-12.0f + t * (28.0f - 15.0f * t)) * ip};
}

// Septic cells: powers of u = t - 1/2 of S and b10 (exact binary fractions; b11(u) = -b10(-u),
// S(u) - 1/2 is odd):
//   S   = 1/2 + 35/16 u - 35/4 u^3 + 21 u^5 - 20 u^7
//   b10 = 11/64 - 19/32 u - 15/16 u^2 + 35/8 u^3 + 5/4 u^4 - 21/2 u^5 - u^6 + 10 u^7
__host__ __device__ constexpr float septic_s(int e)
{
    return e == 1 ? 2.1875f : e == 3 ? -8.75f : e == 5 ? 21.0f : e == 7 ? -20.0f : 0.0f;
}
__host__ __device__ constexpr float septic_b10(int e)
{
    return e == 0 ? 0.171875f : e == 1 ? -0.59375f : e == 2 ? -0.9375f : e == 3 ? 4.375f : e == 4 ? 1.25f
         : e == 5 ? -10.5f : e == 6 ? -1.0f : 10.0f;
}

struct CF {  // column form of one cell at one column
    float E0, dE, Q0, Q1;
};

// nb -> node (cx, cy) of the cell; (cx, cy + 1) follows, column cx + 1 is nny further.
// Zero-gradient model (MD = 1, Sec. 3.3): the cell is E0 + dE S(t) + dQ (t - S(t)) and
// t - S(t) = b10(t) + b11(t), i.e. the gradient form with Q0 = Q1 = dQ.
template <int MD = 0>
__device__ __forceinline__ CF column_form(const float2 *nb, int nny, const XA &xa, const float *hb = nullptr)
{
    const float2 n00 = nb[0], n01 = nb[1], n10 = nb[nny], n11 = nb[nny + 1];
    CF c;
    c.E0 = n00.x * xa.e0 + n10.x * xa.e1;
    float E1 = n01.x * xa.e0 + n11.x * xa.e1;
    if (MD == 2) {  // heights (hb: the node heights at the same offsets)
        c.E0 += hb[0] * xa.v0 + hb[nny] * xa.v1;
        E1 += hb[1] * xa.v0 + hb[nny + 1] * xa.v1;
    }
    c.dE = E1 - c.E0;
    c.Q0 = n00.y * xa.q0 + n10.y * xa.q1;
    c.Q1 = n01.y * xa.q0 + n11.y * xa.q1;
    if (MD == 1) c.Q0 = c.Q1 = c.Q1 - c.Q0;
    return c;
}

// c(v) -> c(d + w) as a polynomial in w (repeated synthetic division).
template <int M>
__device__ __forceinline__ void taylor_shift(float (&c)[2 * M + 2], float d)
{
    constexpr int D = 2 * M + 1;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = D - 1; j >= i; --j) c[j] += d * c[j + 1];
}

// Add the column form, as a polynomial in v with t - 1/2 = tau + sigma v, to C.
// Powers of u = t - 1/2 of the bases (exact binary fractions):
//   cubic:   S = 1/2 + 3/2 u - 2 u^3,  b10 = 1/8 - 1/4 u - 1/2 u^2 + u^3,  b11 = -1/8 - 1/4 u + 1/2 u^2 + u^3
//   quintic: S = 1/2 + 15/8 u - 5 u^3 + 6 u^5,
//            b10 = 5/32 - 7/16 u - 3/4 u^2 + 5/2 u^3 + 1/2 u^4 - 3 u^5,
//            b11 = -5/32 - 7/16 u + 3/4 u^2 + 5/2 u^3 - 1/2 u^4 - 3 u^5
template <int M, bool SHIFT = true>
__device__ __forceinline__ void add_mapped(float (&C)[2 * M + 2], const CF &c, float tau, float sigma)
{
    constexpr int D = 2 * M + 1;
    const float Dq = c.Q0 - c.Q1, Sq = c.Q0 + c.Q1;
    float m[D + 1];
    if (M == 1) {
        m[0] = c.E0 + 0.5f * c.dE + 0.125f * Dq;
        m[1] = 1.5f * c.dE - 0.25f * Sq;
        m[2] = -0.5f * Dq;
        m[3] = Sq - 2.0f * c.dE;
    } else if (M == 2) {
        m[0] = c.E0 + 0.5f * c.dE + 0.15625f * Dq;
        m[1] = 1.875f * c.dE - 0.4375f * Sq;
        m[2] = -0.75f * Dq;
        m[3] = 2.5f * Sq - 5.0f * c.dE;
        m[4] = 0.5f * Dq;
        m[D] = 6.0f * c.dE - 3.0f * Sq;
    } else {  // septic: odd powers from dE and Sq, even powers from Dq (b11(u) = -b10(-u))
        m[0] = c.E0 + 0.5f * c.dE + septic_b10(0) * Dq;
#pragma unroll
        for (int e = 1; e <= D; ++e)
            m[e] = (e & 1) ? septic_s(e) * c.dE + septic_b10(e) * Sq : septic_b10(e) * Dq;
    }
    // Taylor shift to u = tau (repeated synthetic division), then scale u - tau = sigma v
    if (SHIFT) {
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int j = D - 1; j >= i; --j) m[j] += tau * m[j + 1];
    }
    float sp = 1.0f;  // sigma is a power of two: exact powers
#pragma unroll
    for (int b = 0; b <= D; ++b) {
        C[b] += m[b] * sp;
        sp *= sigma;
    }
}

// An octave of fixed period P <= 64: the lane's node column (strips are 64-aligned, so the
// column index is lane >> s and a column holds 64 / P + 1 node rows) and its x-bases.
struct Fixed {
    const float2 *col;
    XA xa;
    const float *hcol;  // the column's node heights (height-and-gradient model)
};

// A node's LDS entry: its unit gradient, or for the zero-gradient model its height in both
// components (the node-row collapse then reads the height for E and for Q).
template <int MD>
__device__ __forceinline__ float2 node_value(uint32_t key)
{
    if (MD == 1) {
        const float h = height2(key);
        return make_float2(h, h);
    }
    return grad2(key);
}

// A streamed octave (period P <= 2): its block (column-major, R / P + 1 rows) and the
// offsets of its column and row keys in the wave's key block.
struct Streamed {
    float2 *blk;
    int kx, ky;
    float *hblk;  // node heights (height-and-gradient model)
};

struct RowCtx {
    Fixed f32, f16, f8, f4, f2, f1;
    int64_t pitch;
    const uint32_t *keys;
    Streamed s2, s1;
};

// Wave-private LDS written by some lanes and read by others: order the accesses (the LDS
// serves one wave's requests in order; the fences keep the compiler from moving them).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Hash node rows [j0, j0 + NROWS) of a streamed octave (period P, strip-relative rows) into
// rows [l0, l0 + NROWS) of its block (R / P + 1 rows): the same keys and gradients as the
// per-strip hashing.
template <int P, int R, int NROWS, int MD = 0>
__device__ __forceinline__ void stream_rows(const uint32_t *keys, const Streamed &st, int j0, int l0, int lane)
{
    constexpr int NB = R / P + 1, NNX = kStripW / P + 1, N = NNX * NROWS;
    for (int q = lane; q < N; q += 64) {  // column-major: consecutive lanes, consecutive rows
        const int i = q / NROWS, jj = q - i * NROWS;
        const uint32_t key = key_combine(keys[st.ky + j0 + jj], keys[st.kx + i]);
        st.blk[i * NB + l0 + jj] = node_value<MD>(key);
        if (MD == 2) st.hblk[i * NB + l0 + jj] = height2_second(key);
    }
}

// Both streamed octaves at once (periods 2 and 1): NR2 node rows of period 2 from row j2
// and NR1 of period 1 from row j1, into rows [l0, ...) of their blocks, as one list of nodes
// -- period 1's first, then period 2's -- so that the lanes period 1 leaves idle in its last
// iteration take period 2's first nodes (the same nodes, keys and values as two
// stream_rows calls).
template <int R, int NR2, int NR1, int MD = 0>
__device__ __forceinline__ void stream_rows_21(const uint32_t *keys, const Streamed &s2, const Streamed &s1, int j2,
                                               int j1, int l0, int lane)
{
    constexpr int NB2 = R / 2 + 1, NB1 = R + 1;
    constexpr int N2 = (kStripW / 2 + 1) * NR2, N1 = (kStripW + 1) * NR1, FULL = N1 / 64;
    static_assert((NR1 & (NR1 - 1)) == 0 && (NR2 * 2 == NR1 || NR2 == NR1), "row counts");
    // iterations wholly inside period 1
#pragma unroll
    for (int it = 0; it < FULL; ++it) {
        const int q = 64 * it + lane, i = q / NR1, jj = q - i * NR1;
        const uint32_t key = key_combine(keys[s1.ky + j1 + jj], keys[s1.kx + i]);
        s1.blk[i * NB1 + l0 + jj] = node_value<MD>(key);
        if (MD == 2) s1.hblk[i * NB1 + l0 + jj] = height2_second(key);
    }
    // one iteration with period 1's last nodes and period 2's first: each lane picks its
    // octave's keys and block (selected as values)
    {
        const int q = 64 * FULL + lane;
        const bool in1 = q < N1;
        const int qq = in1 ? q : q - N1;
        const int i = in1 ? qq / NR1 : qq / NR2, jj = qq - i * (in1 ? NR1 : NR2);
        float2 *const b1 = s1.blk, *const b2 = s2.blk;
        float *const h1 = s1.hblk, *const h2 = s2.hblk;
        const int ky1 = s1.ky + j1, ky2 = s2.ky + j2, kx1 = s1.kx, kx2 = s2.kx;
        if (q < N1 + N2) {
            const uint32_t key = key_combine(keys[(in1 ? ky1 : ky2) + jj], keys[(in1 ? kx1 : kx2) + i]);
            const int at = i * (in1 ? NB1 : NB2) + l0 + jj;
            (in1 ? b1 : b2)[at] = node_value<MD>(key);
            if (MD == 2) (in1 ? h1 : h2)[at] = height2_second(key);
        }
    }
    // the rest of period 2
    for (int q = 64 * (FULL + 1) - N1 + lane; q < N2; q += 64) {
        const int i = q / NR2, jj = q - i * NR2;
        const uint32_t key = key_combine(keys[s2.ky + j2 + jj], keys[s2.kx + i]);
        s2.blk[i * NB2 + l0 + jj] = node_value<MD>(key);
        if (MD == 2) s2.hblk[i * NB2 + l0 + jj] = height2_second(key);
    }
}

// A node row collapsed along x at the lane's column: value term E and y-slope term Q.  The
// cell between node rows lo and hi has the column form E0 = lo.E, dE = hi.E - lo.E,
// Q0 = lo.Q, Q1 = hi.Q, and adjacent cells share their common node row.
struct NR {
    float E, Q;
};

template <int NNY, int MD = 0>
__device__ __forceinline__ NR node_row(const Fixed &f, int j)
{
    const float2 a = f.col[j], b = f.col[j + NNY];
    NR r{a.x * f.xa.e0 + b.x * f.xa.e1, a.y * f.xa.q0 + b.y * f.xa.q1};
    if (MD == 2) r.E += f.hcol[j] * f.xa.v0 + f.hcol[j + NNY] * f.xa.v1;
    return r;
}

// Add the cell between node rows lo and hi, as a polynomial in the segment coordinate w
// (t - 1/2 = SIG w: the cell is centred on the segment), to C.  The constants are the
// centred power coefficients of the bases listed at add_mapped, times SIG^b.
template <int M, int SIG, int MD = 0>
__device__ __forceinline__ void add_piece(float (&C)[2 * M + 2], const NR &lo, const NR &hi)
{
    constexpr float s1 = (float)SIG, s2 = s1 * s1, s3 = s2 * s1, s4 = s3 * s1, s5 = s4 * s1;
    const float dE = hi.E - lo.E, Sq = lo.Q + hi.Q, Dq = lo.Q - hi.Q;
    C[0] += lo.E;
    C[0] = __builtin_fmaf(dE, 0.5f, C[0]);
    if (MD == 1) {  // zero-gradient model (M = 1): Q0 = Q1 = dQ, so Dq = 0 and Sq = 2 dQ
        const float dQ = hi.Q - lo.Q;
        C[1] = __builtin_fmaf(dE, 1.5f * s1, C[1]);
        C[1] = __builtin_fmaf(dQ, -0.5f * s1, C[1]);
        C[3] = __builtin_fmaf(dQ, 2.0f * s3, C[3]);
        C[3] = __builtin_fmaf(dE, -2.0f * s3, C[3]);
    } else if (M == 1) {
        C[0] = __builtin_fmaf(Dq, 0.125f, C[0]);
        C[1] = __builtin_fmaf(dE, 1.5f * s1, C[1]);
        C[1] = __builtin_fmaf(Sq, -0.25f * s1, C[1]);
        C[2] = __builtin_fmaf(Dq, -0.5f * s2, C[2]);
        C[3] = __builtin_fmaf(Sq, s3, C[3]);
        C[3] = __builtin_fmaf(dE, -2.0f * s3, C[3]);
    } else if (M == 2) {
        C[0] = __builtin_fmaf(Dq, 0.15625f, C[0]);
        C[1] = __builtin_fmaf(dE, 1.875f * s1, C[1]);
        C[1] = __builtin_fmaf(Sq, -0.4375f * s1, C[1]);
        C[2] = __builtin_fmaf(Dq, -0.75f * s2, C[2]);
        C[3] = __builtin_fmaf(Sq, 2.5f * s3, C[3]);
        C[3] = __builtin_fmaf(dE, -5.0f * s3, C[3]);
        C[4] = __builtin_fmaf(Dq, 0.5f * s4, C[4]);
        C[5] = __builtin_fmaf(dE, 6.0f * s5, C[5]);
        C[5] = __builtin_fmaf(Sq, -3.0f * s5, C[5]);
    } else {  // septic
        C[0] = __builtin_fmaf(Dq, septic_b10(0), C[0]);
        float sp = 1.0f;
#pragma unroll
        for (int e = 1; e <= 2 * M + 1; ++e) {
            sp *= s1;  // SIG^e (exact)
            if (e & 1) {
                C[e] = __builtin_fmaf(dE, septic_s(e) * sp, C[e]);
                C[e] = __builtin_fmaf(Sq, septic_b10(e) * sp, C[e]);
            } else {
                C[e] = __builtin_fmaf(Dq, septic_b10(e) * sp, C[e]);
            }
        }
    }
}

// val += dE S + Q0 b10 + Q1 b11 at one row (E0 is in the constant term), as an FMA chain.
template <int MD = 0>
__device__ __forceinline__ float add_direct(float val, const NR &lo, const NR &hi, const XB &rb)
{
    val = __builtin_fmaf(hi.E - lo.E, rb.s, val);
    if (MD == 1) return __builtin_fmaf(hi.Q - lo.Q, rb.b10 + rb.b11, val);  // zero-gradient: t - S(t)
    val = __builtin_fmaf(lo.Q, rb.b10, val);
    return __builtin_fmaf(hi.Q, rb.b11, val);
}

// Node rows [r0 / P, (r0 + R) / P] of a direct octave over a segment; the first one is
// carried from the previous segment and the last one is carried to the next.
template <int P, int R, int MD = 0>
struct SegRows {
    NR n[R / P + 1];
    __device__ __forceinline__ void load(const Fixed &f, int r0, NR &carry)
    {
        n[0] = carry;
#pragma unroll
        for (int j = 1; j <= R / P; ++j) n[j] = node_row<64 / P + 1, MD>(f, r0 / P + j);
        carry = n[R / P];
    }
    // streamed octave: the segment's rows are rows 1 .. R / P of its block
    __device__ __forceinline__ void load_streamed(const Fixed &f, NR &carry)
    {
        n[0] = carry;
#pragma unroll
        for (int j = 1; j <= R / P; ++j) n[j] = node_row<R / P + 1, MD>(f, j);
        carry = n[R / P];
    }
};

// The R rows [r0, r0 + R) of a strip, given the polynomial Cs of everything coarser than the
// direct octaves, centred on the segment (row k at w = (2 k - R + 1) / 128).  Rows are taken
// in pairs symmetric about the centre, w and -w, from the even and odd parts of Cs; the
// direct octaves' E0 terms go into each row's constant term, the rest is 3 FMA per octave.
// G selects what is written: 0 and 1 the rows' values (G = 1: the strip machinery run on the
// x-weights' derivatives) to rp; 2 their d/dY to rp; 3 both, the values to rp and d/dY to
// rp2.  d/dY (w = (Y - centre) / 64): the derivative of Cs, and the direct octaves' row-basis
// derivatives (their E0 terms are constant along y).
template <int M, typename OutT, int R, bool D8, bool D4, bool D2, bool D1, bool FULL, int MD = 0, int G = 0>
__device__ __forceinline__ void segment_rows(const RowCtx &x, const float (&Cs)[2 * M + 2], int r0, NR (&carry)[4],
                                             OutT *rp, OutT *rp2, int lane, int rlo, int rhi, bool lane_ok)
{
    constexpr int D = 2 * M + 1;
    constexpr bool WV = G != 2, WD = G >= 2;  // values, derivatives
    float Pd[D];  // d/dY of the segment polynomial, degree D - 1 (WD)
#pragma unroll
    for (int b = 0; b < D; ++b) Pd[b] = WD ? (float)(b + 1) * (1.0f / 64.0f) * Cs[b + 1] : 0.0f;
    SegRows<8, R, MD> s8;
    SegRows<4, R, MD> s4;
    SegRows<2, R, MD> s2;
    SegRows<1, R, MD> s1;
    if (D8) s8.load(x.f8, r0, carry[0]);
    if (D4) s4.load(x.f4, r0, carry[1]);
    if (D2 || D1) {  // streamed periods: hash this segment's node rows first
        wave_lds_sync();  // the previous segment has read its rows
        if (D2 && D1) {
            stream_rows_21<R, R / 2, R, MD>(x.keys, x.s2, x.s1, r0 / 2 + 1, r0 + 1, 1, lane);
        } else {
            if (D2) stream_rows<2, R, R / 2, MD>(x.keys, x.s2, r0 / 2 + 1, 1, lane);
            if (D1) stream_rows<1, R, R, MD>(x.keys, x.s1, r0 + 1, 1, lane);
        }
        wave_lds_sync();
    }
    if (D2) s2.load_streamed(x.f2, carry[2]);
    if (D1) s1.load_streamed(x.f1, carry[3]);
    // row pointers walk outwards from the centre pair (uniform, one add each per pair)
    OutT *pa = rp + (int64_t)(r0 + R / 2 - 1) * x.pitch, *pb = pa + x.pitch;
    OutT *qa = (G == 3 ? rp2 : rp) + (int64_t)(r0 + R / 2 - 1) * x.pitch, *qb = qa + x.pitch;
#pragma unroll
    for (int p = 0; p < R / 2; ++p) {
        const int rb = R / 2 + p;
        const float w = (float)(2 * rb - R + 1) * (1.0f / 128.0f);
        const float w2 = w * w;
        // odd part in w^2 (C1, C3, ...) and the even part beyond C0 (C2, C4, ...)
        float odd = 0.0f, even2 = 0.0f, oddd = 0.0f, even2d = 0.0f;
        if (WV) {
            odd = Cs[D];
#pragma unroll
            for (int e = D - 2; e >= 1; e -= 2) odd = __builtin_fmaf(odd, w2, Cs[e]);
            even2 = Cs[D - 1];
#pragma unroll
            for (int e = D - 3; e >= 2; e -= 2) even2 = __builtin_fmaf(even2, w2, Cs[e]);
        }
        if (WD) {  // degree D - 1 = 2M: odd part P1, P3, ..., P(D-2); even part P2, ..., P(D-1)
            oddd = Pd[D - 2];
#pragma unroll
            for (int e = D - 4; e >= 1; e -= 2) oddd = __builtin_fmaf(oddd, w2, Pd[e]);
            even2d = Pd[D - 1];
#pragma unroll
            for (int e = D - 3; e >= 2; e -= 2) even2d = __builtin_fmaf(even2d, w2, Pd[e]);
        }
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const int k = side ? rb : R / 2 - 1 - p;  // row in the segment
            const int row = r0 + k;                   // row in the strip
            const bool keep = FULL || (row >= rlo && row < rhi && lane_ok);
            if (WV) {
                float c0 = Cs[0];
                if (D8) c0 += s8.n[k / 8].E;
                if (D4) c0 += s4.n[k / 4].E;
                if (D2) c0 += s2.n[k / 2].E;
                if (D1) c0 += s1.n[k].E;
                float val = __builtin_fmaf(even2, w2, c0);
                val = __builtin_fmaf(side ? w : -w, odd, val);
                if (D8) val = add_direct<MD>(val, s8.n[k / 8], s8.n[k / 8 + 1], row_bases<M>(row & 7, 8));
                if (D4) val = add_direct<MD>(val, s4.n[k / 4], s4.n[k / 4 + 1], row_bases<M>(row & 3, 4));
                if (D2) val = add_direct<MD>(val, s2.n[k / 2], s2.n[k / 2 + 1], row_bases<M>(row & 1, 2));
                if (D1) val = add_direct<MD>(val, s1.n[k], s1.n[k + 1], row_bases<M>(0, 1));
                OutT *const rrow = side ? pb : pa;
                if (keep) rrow[lane] = st_out<OutT>(val);
            }
            if (WD) {
                float val = __builtin_fmaf(even2d, w2, Pd[0]);
                val = __builtin_fmaf(side ? w : -w, oddd, val);
                if (D8) val = add_direct<MD>(val, s8.n[k / 8], s8.n[k / 8 + 1], row_dbases<M>(row & 7, 8));
                if (D4) val = add_direct<MD>(val, s4.n[k / 4], s4.n[k / 4 + 1], row_dbases<M>(row & 3, 4));
                if (D2) val = add_direct<MD>(val, s2.n[k / 2], s2.n[k / 2 + 1], row_dbases<M>(row & 1, 2));
                if (D1) val = add_direct<MD>(val, s1.n[k], s1.n[k + 1], row_dbases<M>(0, 1));
                OutT *const rrow = side ? qb : qa;
                if (keep) rrow[lane] = st_out<OutT>(val);
            }
        }
        pa -= x.pitch;
        pb += x.pitch;
        qa -= x.pitch;
        qb += x.pitch;
        // keep each pair's stores next to its arithmetic: without this the scheduler hoists
        // most of a strip's row arithmetic ahead of the first store and then issues the
        // stores in one burst, with the values held in registers
        __builtin_amdgcn_sched_barrier(0);
    }
}

// The rows of a strip.  The fused polynomial C (in the strip coordinate v) is re-centred
// on each half strip, where the period-32 piece is added (t - 1/2 = 2 w), and again on each
// quarter, where the period-16 piece is added (t - 1/2 = 4 w).  For cubic cells the same is
// done once more per period-8 cell (t - 1/2 = 8 w), where re-centring (6 FMA) and the piece
// cost less than evaluating the octave on its own at every row; for quintic cells (15 FMA
// per re-centring) period 8 stays a direct octave.  No piece is evaluated away from its own
// cell.  FULL = every sample of the strip is stored.
template <int M, typename OutT, int LO, bool FULL, int MD = 0, int G = 0>
__device__ __forceinline__ void strip_rows(const RowCtx &x, const float (&C)[2 * M + 2], OutT *rp, OutT *rp2, int lane,
                                           int rlo, int rhi, bool lane_ok)
{
    constexpr int D1 = 2 * M + 2;
    constexpr bool H32 = LO <= 5, H16 = LO <= 4, H8 = LO <= 3, H4 = LO <= 2, H2 = LO <= 1, H1 = LO == 0;
    constexpr bool PIECE8 = H8 && M == 1;
    constexpr int R = (M == 1 && H8) ? 8 : 16;  // row segment (streamed block height)
    NR carry[4];  // bottom node rows of the next segment: periods 8, 4, 2, 1
    if (H8) carry[0] = node_row<9, MD>(x.f8, 0);
    if (H4) carry[1] = node_row<17, MD>(x.f4, 0);
    if (H2 || H1) {  // streamed periods: node row 0 of the strip into block row 0
        wave_lds_sync();  // the previous strip has read its blocks
        if (H2 && H1) {
            stream_rows_21<R, 1, 1, MD>(x.keys, x.s2, x.s1, 0, 0, 0, lane);
        } else {
            if (H2) stream_rows<2, R, 1, MD>(x.keys, x.s2, 0, 0, lane);
            if (H1) stream_rows<1, R, 1, MD>(x.keys, x.s1, 0, 0, lane);
        }
        wave_lds_sync();
    }
    if (H2) carry[2] = node_row<R / 2 + 1, MD>(x.f2, 0);
    if (H1) carry[3] = node_row<R + 1, MD>(x.f1, 0);
    NR n32[3], n16lo;
    if (H32) {
#pragma unroll
        for (int j = 0; j < 3; ++j) n32[j] = node_row<3, MD>(x.f32, j);
    }
    if (H16) n16lo = node_row<5, MD>(x.f16, 0);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        float Ch[D1];
#pragma unroll
        for (int b = 0; b < D1; ++b) Ch[b] = C[b];
        taylor_shift<M>(Ch, (float)(2 * h - 1) * 0.25f);  // half centre v = -1/4, +1/4
        if (H32) add_piece<M, 2, MD>(Ch, n32[h], n32[h + 1]);
#pragma unroll
        for (int qh = 0; qh < 2; ++qh) {
            const int q = 2 * h + qh;
            float Cq[D1];
#pragma unroll
            for (int b = 0; b < D1; ++b) Cq[b] = Ch[b];
            taylor_shift<M>(Cq, (float)(2 * qh - 1) * 0.125f);  // quarter centre, from the half's
            if (H16) {
                const NR hi = node_row<5, MD>(x.f16, q + 1);
                add_piece<M, 4, MD>(Cq, n16lo, hi);
                n16lo = hi;
            }
            if (PIECE8) {
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    float Ce[D1];
#pragma unroll
                    for (int b = 0; b < D1; ++b) Ce[b] = Cq[b];
                    taylor_shift<M>(Ce, (float)(2 * e - 1) * 0.0625f);  // period-8 cell centre
                    const NR lo = carry[0], hi = node_row<9, MD>(x.f8, 2 * q + e + 1);
                    add_piece<M, 8, MD>(Ce, lo, hi);
                    carry[0] = hi;
                    segment_rows<M, OutT, 8, false, H4, H2, H1, FULL, MD, G>(x, Ce, 16 * q + 8 * e, carry, rp, rp2,
                                                                              lane, rlo, rhi, lane_ok);
                }
            } else {
                segment_rows<M, OutT, 16, H8, H4, H2, H1, FULL, MD, G>(x, Cq, 16 * q, carry, rp, rp2, lane, rlo,
                                                                        rhi, lane_ok);
            }
        }
    }
}

}  // namespace ptg

#include "ptg_strip_mx.h"

namespace ptg {

// Per-octave constants a workgroup stages in LDS once (the strip code reads them from there).
struct StripShared {
    uint32_t pre_key[kMaxOctaves];
    int shift[kMaxOctaves], noff[kMaxOctaves], nbr[kMaxOctaves];
    float amp[kMaxOctaves], inv2p[kMaxOctaves];
    float gw;  // gradient weight (height-and-gradient model)
};

// Once per workgroup (every thread, a barrier after it): the work lists that map lanes to
// keys and nodes (the same for every strip of a field) and the per-octave constants.
__device__ __forceinline__ void strip_prologue(const Fbm2dStripArgs &a, StripShared &sh, uint32_t *wl_key,
                                               uint32_t *wl_node, int tid, int nthreads)
{
    const int N = a.octaves;
    for (int o = 0; o < N; ++o) {
        const int nnx = a.nnx[o], nny = a.nny[o], kx = a.kxoff[o], ky = a.kyoff[o], no = a.noff[o];
        for (int i = tid; i < nnx + nny; i += nthreads) {
            if (i < nnx)
                wl_key[kx + i] = ((uint32_t)o << 24) | (uint32_t)i;
            else
                wl_key[ky + i - nnx] = ((uint32_t)o << 24) | (uint32_t)(i - nnx);
        }
        if (no >= a.nodes_hashed) continue;  // streamed: hashed per row segment
        for (int q = tid; q < nnx * nny; q += nthreads) {  // byte offsets of the node's two keys
            const int i = q / nny, j = q - i * nny;          // column-major
            wl_node[no + q] = ((uint32_t)(ky + j) << 18) | ((uint32_t)(kx + i) << 2);
        }
    }
    if (tid < N) {
        sh.pre_key[tid] = key_prefix(a.seed, tid);
        sh.shift[tid] = a.shift[tid];
        sh.noff[tid] = a.noff[tid];
        sh.nbr[tid] = a.nbr[tid];
        if (tid == 0) sh.gw = a.gw;
        sh.amp[tid] = a.amp[tid];
        sh.inv2p[tid] = a.inv2p[tid];
    }
}

// One wave's strips of a field: the lane's x-weights of the fixed-period octaves (formed
// once) and the strip column whose keys its LDS block holds.  G selects the output: 0 the
// field H, 1 dH/dX (the x-weights' derivatives), 2 dH/dY (the rows' derivatives), both in
// world units per sample; 4 all three (H to a.out, dH/dX to a.out_dx, dH/dY to a.out_dy)
// from one hashing of each strip: the rows' values and d/dY in one pass, then the same
// strip with the derivative x-weights.
template <int M, typename OutT, int LO, int MD = 0, int PREC = 0, int G = 0>
struct StripWave {
    static_assert(PREC == 0 || G == 0, "the precision form writes the field only");
    static constexpr int D1 = 2 * M + 2;
    static constexpr bool H32 = LO <= 5, H16 = LO <= 4, H8 = LO <= 3, H4 = LO <= 2, H2 = LO <= 1, H1 = LO == 0;
    float2 *nodes;
    float *heights;  // height-and-gradient model: a height per node after the gradients
    uint32_t *keys;
    int lane;
    Fixed f64;
    RowCtx rc0;
    // the column keys stay valid while the wave's strips share a strip column (the stride
    // over strips is often a multiple of the strips per row)
    int64_t keyed_bsx = -1;
    MxConst<PREC ? PREC : 1> mc;  // precision form (PREC 1 / 2): the MFMA's row operands

    // An octave's node column and the lane's x-weights (DX: their derivatives, times 1/P).
    template <bool DX>
    __device__ __forceinline__ Fixed fixed(const StripShared &sh, int o) const
    {
        Fixed f{nodes, XA{0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f}, heights};
        if (o >= 0) {
            const int s = sh.shift[o];
            f.col = nodes + sh.noff[o] + (lane >> s) * sh.nbr[o];
            f.hcol = heights + sh.noff[o] + (lane >> s) * sh.nbr[o];
            const float inv2p = sh.inv2p[o];
            f.xa = xweights<M, MD, DX>((float)(2 * (lane & ((1 << s) - 1)) + 1) * inv2p,
                                       DX ? sh.amp[o] * (2.0f * inv2p) : sh.amp[o], sh.gw);
        }
        return f;
    }

    __device__ __forceinline__ Streamed streamed(const StripShared &sh, const Fbm2dStripArgs &a, int o) const
    {
        return o >= 0 ? Streamed{nodes + sh.noff[o], a.kxoff[o], a.kyoff[o], heights + sh.noff[o]}
                      : Streamed{nodes, 0, 0, heights};
    }

    __device__ __forceinline__ StripWave(const Fbm2dStripArgs &a, const StripShared &sh, float2 *nodes_, int lane_)
        : nodes(nodes_), heights(reinterpret_cast<float *>(nodes_ + a.nodes_total)),
          keys(reinterpret_cast<uint32_t *>(nodes_ + a.nodes_total) + (MD == 2 ? a.nodes_total : 0)), lane(lane_)
    {
        f64 = fixed<G == 1>(sh, a.o64);
        if constexpr (PREC > 0) mc.init(a.basis, lane);
        rc0 = ctx<G == 1>(a, sh);
    }

    template <bool DX>
    __device__ __forceinline__ RowCtx ctx(const Fbm2dStripArgs &a, const StripShared &sh) const
    {
        return RowCtx{fixed<DX>(sh, H32 ? a.o32 : -1), fixed<DX>(sh, H16 ? a.o16 : -1), fixed<DX>(sh, H8 ? a.o8 : -1),
                      fixed<DX>(sh, H4 ? a.o4 : -1),   fixed<DX>(sh, H2 ? a.o2 : -1),   fixed<DX>(sh, H1 ? a.o1 : -1),
                      a.pitch,
                      keys,
                      streamed(sh, a, H2 ? a.o2 : -1),
                      streamed(sh, a, H1 ? a.o1 : -1)};
    }

    // The polynomial in v of the octaves of period >= 64 at the lane's column (DX: with the
    // x-weights' derivatives; fx is the period-64 octave's column with those weights).
    template <bool DX>
    __device__ __forceinline__ void coarse(const Fbm2dStripArgs &a, const Fixed &fx, int64_t X0, int64_t Y0,
                                           float (&C)[D1]) const
    {
#pragma unroll
        for (int b = 0; b < D1; ++b) C[b] = 0.0f;
        for (int o = 0; o < a.n_generic; ++o) {  // period >= 128: the strip is inside one cell
            // per-octave values from the arguments: uniform (scalar) in the dense kernel
            const int s = a.shift[o];
            const uint32_t mask = (1u << s) - 1u;
            const float inv2p = a.inv2p[o];
            const XA xa = xweights<M, MD, DX>((float)(2u * (((uint32_t)X0 & mask) + (uint32_t)lane) + 1u) * inv2p,
                                              DX ? a.amp[o] * (2.0f * inv2p) : a.amp[o], a.gw);
            const CF c = column_form<MD>(nodes + a.noff[o], 2, xa, heights + a.noff[o]);
            const float invp = 2.0f * inv2p;
            const float tau = (float)(((uint32_t)Y0 & mask) + (uint32_t)(kStripH / 2)) * invp - 0.5f;
            add_mapped<M>(C, c, tau, (float)kStripH * invp);
        }
        if (a.o64 >= 0) add_piece<M, 1, MD>(C, node_row<2, MD>(fx, 0), node_row<2, MD>(fx, 1));  // t - 1/2 = v
    }

    // Strip st of the field: hash its footprint, sum its coarse octaves, write its rows.
    __device__ __forceinline__ void run(const Fbm2dStripArgs &a, const StripShared &sh, const uint32_t *wl_key,
                                        const uint32_t *wl_node, int64_t st)
    {
        const int nodes_hashed = a.nodes_hashed, keys_total = a.keys_total, keys_col = a.keys_col;
        const int64_t bsy = st / a.strips_x, bsx = st - bsy * a.strips_x;
        const int64_t X0 = a.sx_base + bsx * kStripW, Y0 = a.sy_base + bsy * kStripH;

        // ---- hashing: column keys (x salt), row keys (octave prefix), then node gradients
        // (unit vectors: the amplitude is in the lanes' x-weights) -------------------------
        if (bsx != keyed_bsx) {
            for (int q = lane; q < keys_col; q += 64) {
                const uint32_t it = wl_key[q];
                keys[q] = key_xline((X0 >> sh.shift[it >> 24]) + (int64_t)(it & 0xFFFFFF));
            }
            keyed_bsx = bsx;
        }
        for (int q = keys_col + lane; q < keys_total; q += 64) {
            const uint32_t it = wl_key[q];
            const int o = it >> 24;
            keys[q] = absorb_index(sh.pre_key[o], (Y0 >> sh.shift[o]) + (int64_t)(it & 0xFFFFFF));
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const char *key_bytes = reinterpret_cast<const char *>(keys);
        for (int q = lane; q < nodes_hashed; q += 64) {
            const uint32_t it = wl_node[q];
            const uint32_t krow = *reinterpret_cast<const uint32_t *>(key_bytes + (it >> 16));
            const uint32_t kcol = *reinterpret_cast<const uint32_t *>(key_bytes + (it & 0xFFFFu));
            const uint32_t key = key_combine(krow, kcol);
            nodes[q] = node_value<MD>(key);
            if (MD == 2) heights[q] = height2_second(key);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

        // ---- octaves of period >= 64: one polynomial in v per lane ------------------------
        float C[D1];
        coarse<G == 1>(a, f64, X0, Y0, C);

        // ---- rows: one store per row of the wave; interior strips take the unmasked path --
        const int64_t xe = a.x0 + a.nx, ye = a.y0 + a.ny;
        const int rlo = (int)max<int64_t>(0, min<int64_t>(kStripH, a.y0 - Y0));
        const int rhi = (int)max<int64_t>(0, min<int64_t>(kStripH, ye - Y0));
        const int clo = (int)max<int64_t>(0, min<int64_t>(kStripW, a.x0 - X0));
        const int chi = (int)max<int64_t>(0, min<int64_t>(kStripW, xe - X0));
        const int64_t at = (Y0 - a.y0) * a.pitch + (X0 - a.x0);
        OutT *row0 = reinterpret_cast<OutT *>(a.out) + at;
        if constexpr (PREC > 0) {  // cubic cells, gradient model
            if (rlo == 0 && rhi == kStripH && clo == 0 && chi == kStripW)
                strip_rows_mx<OutT, LO, PREC, true>(rc0, C, row0, lane, 0, kStripH, false, mc);
            else
                strip_rows_mx<OutT, LO, PREC, false>(rc0, C, row0, lane, rlo, rhi, lane >= clo && lane < chi, mc);
        } else if constexpr (G == 4) {
            // the values and d/dY in one pass; then d/dX: the same rows with the x-weights'
            // derivatives (formed here per strip, not held across strips)
            OutT *rowy = reinterpret_cast<OutT *>(a.out_dy) + at, *rowx = reinterpret_cast<OutT *>(a.out_dx) + at;
            float Cx[D1];
            if (rlo == 0 && rhi == kStripH && clo == 0 && chi == kStripW) {
                strip_rows<M, OutT, LO, true, MD, 3>(rc0, C, row0, rowy, lane, 0, kStripH, false);
                coarse<true>(a, fixed<true>(sh, a.o64), X0, Y0, Cx);
                strip_rows<M, OutT, LO, true, MD, 1>(ctx<true>(a, sh), Cx, rowx, nullptr, lane, 0, kStripH, false);
            } else {
                const bool lane_ok = lane >= clo && lane < chi;
                strip_rows<M, OutT, LO, false, MD, 3>(rc0, C, row0, rowy, lane, rlo, rhi, lane_ok);
                coarse<true>(a, fixed<true>(sh, a.o64), X0, Y0, Cx);
                strip_rows<M, OutT, LO, false, MD, 1>(ctx<true>(a, sh), Cx, rowx, nullptr, lane, rlo, rhi, lane_ok);
            }
        } else if (rlo == 0 && rhi == kStripH && clo == 0 && chi == kStripW) {
            strip_rows<M, OutT, LO, true, MD, G>(rc0, C, row0, nullptr, lane, 0, kStripH, false);
        } else {
            strip_rows<M, OutT, LO, false, MD, G>(rc0, C, row0, nullptr, lane, rlo, rhi, lane >= clo && lane < chi);
        }
        __builtin_amdgcn_wave_barrier();  // the next strip rewrites this wave's keys and nodes
    }
};

// A dense field's kernel body (one wave per 64 x 64 strip, a grid-stride walk over the
// field's strips): lds is the dynamic LDS block, sh the workgroup's per-octave constants.
template <int M, typename OutT, int LO, int MD, int PREC, int G>
__device__ __forceinline__ void strip_field(const Fbm2dStripArgs &a, uint32_t *lds, StripShared &sh)
{
    const int tid = threadIdx.x, lane = tid & 63, nthreads = blockDim.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wpg = nthreads >> 6;  // waves per workgroup
    // LDS: [wl_key | wl_node] shared, then per wave [nodes (float2) | keys (u32)]
    uint32_t *wl_key = lds;
    uint32_t *wl_node = wl_key + a.keys_total;
    const int shared_words = strip_shared_words(a.nodes_hashed, a.keys_total);
    const int wave_words = strip_wave_words(a.nodes_total, a.keys_total, MD == 2);
    float2 *nodes = reinterpret_cast<float2 *>(lds + shared_words + wave * wave_words);

    strip_prologue(a, sh, wl_key, wl_node, tid, nthreads);
    __syncthreads();
    StripWave<M, OutT, LO, MD, PREC, G> w(a, sh, nodes, lane);
    const int64_t nwaves = (int64_t)gridDim.x * wpg;
    for (int64_t st = (int64_t)blockIdx.x * wpg + wave; st < a.strips; st += nwaves) w.run(a, sh, wl_key, wl_node, st);
}

}  // namespace ptg
