// ptg_strip_mx.h -- the FP16 / BF16 precision form of the 2D strip kernel (C1 cells): the
// coarse and middle octaves of every 4 rows x 64 columns of a strip are evaluated as one
// v_mfma_f32_16x16x32_{f16,bf16} with FP32 accumulation (the Vandermonde contraction
// V(y) . (C V(x)^T) of Sec. 2.2, eq. polynomial, with the x side already contracted per
// column), the finest octaves and every constant term in FP32 on the vector ALUs.
//
// Layout.  The wave's lane is the strip column, as in the plain strip code.  The MFMA's B
// operand (K = 32 x 16 columns) takes 8 consecutive K values from each lane: lane
// 16 g + n gives B[8 g .. 8 g + 7][n], its own column's 8 coefficients.  With an A operand
// that is block diagonal -- A[4 g + i][8 g' + j] = W_i[j] when g = g', else 0 -- the result
// D[4 g + i][n] = sum_j W_i[j] B[8 g + j][n] is row i of column 16 g + n, and the MFMA's
// result layout (lane 16 g + n holds D[4 g + i][n], i = 0..3) hands every lane its own
// column's four rows.  A depends only on the row's place inside the strip, so each wave
// forms it once.
//
// The 8 K values of a column for the 4 rows of block b of quarter q (rows 16 q + 4 b + i):
//   [0..2] the octaves of period >= 16, summed as one cubic per column and quarter (the
//          strip code's fused polynomial, re-centred per half and quarter), powers 1..3;
//   [3..5] the period-8 cell that holds the block: its three non-constant terms;
//   [6, 7] the period-4 cell (= the block): two terms; its third term is one FP32 FMA.
// Bases of those terms (ptg_params.basis):
//   monomial: powers of the cell's own corner coordinate t (the fused cubic in powers of
//             the quarter's corner coordinate);
//   centred:  powers of t - 1/2 (the fused cubic about the quarter's centre);
//   hermite:  the cells' 1D Hermite bases S, b10, b11 (the fused cubic centred).
// The constant terms (the fused cubic's, and each cell's value at its first node row)
// stay in FP32: they go into the accumulator with the finer octaves (periods 2 and 1, the
// strip code's direct rows), so FP16 / BF16 rounding touches only terms that vanish at a
// node row or the quarter's centre.
#pragma once

#include "ptg.h"

// included by ptg_strip_tile.h after the row code it builds on
namespace ptg {

typedef float mx_f4 __attribute__((ext_vector_type(4)));
typedef _Float16 mx_h8 __attribute__((ext_vector_type(8)));
typedef short mx_s8 __attribute__((ext_vector_type(8)));
typedef __bf16 mx_b8 __attribute__((ext_vector_type(8)));

// Operand element of the precision form: PREC 1 = FP16, 2 = BF16 (round to nearest even).
template <int PREC>
struct MxOp;

template <>
struct MxOp<1> {
    typedef mx_h8 vec;
    __device__ __forceinline__ static _Float16 cvt(float v) { return (_Float16)v; }
    __device__ __forceinline__ static mx_f4 mma(const vec &a, const vec &b, const mx_f4 &c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};

template <>
struct MxOp<2> {
    typedef mx_s8 vec;
    __device__ __forceinline__ static short cvt(float v)
    {
        uint32_t u = __builtin_bit_cast(uint32_t, v);
        u += 0x7FFFu + ((u >> 16) & 1u);
        return (short)(u >> 16);
    }
    __device__ __forceinline__ static mx_f4 mma(const vec &a, const vec &b, const mx_f4 &c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(mx_b8, a), __builtin_bit_cast(mx_b8, b), c,
                                                       0, 0, 0);
    }
};

// The three non-constant basis functions of a cell coordinate t (C1 cells) per basis.
__host__ __device__ inline void mx_cell_basis(int basis, float t, float &f1, float &f2, float &f3)
{
    if (basis == PTG_BASIS_MONOMIAL) {
        f1 = t;
        f2 = t * t;
        f3 = t * t * t;
    } else if (basis == PTG_BASIS_CENTRED) {
        const float s = t - 0.5f;
        f1 = s;
        f2 = s * s;
        f3 = s * s * s;
    } else {  // Hermite: S, b10, b11
        const float u = 1.0f - t;
        f1 = t * t * (3.0f - 2.0f * t);
        f2 = t * u * u;
        f3 = -t * t * u;
    }
}

// Coefficients of a cell between node rows lo and hi in a basis: k0 (constant, FP32), k1..k3.
struct MxK {
    float k0, k1, k2, k3;
};

__device__ __forceinline__ MxK mx_cell_coeffs(int basis, const NR &lo, const NR &hi)
{
    const float dE = hi.E - lo.E, Q0 = lo.Q, Q1 = hi.Q;
    if (basis == PTG_BASIS_MONOMIAL)  // E0 + Q0 t + (3 dE - 2 Q0 - Q1) t^2 + (Q0 + Q1 - 2 dE) t^3
        return MxK{lo.E, Q0, __builtin_fmaf(3.0f, dE, -2.0f * Q0 - Q1), __builtin_fmaf(-2.0f, dE, Q0 + Q1)};
    if (basis == PTG_BASIS_CENTRED) {  // the same cubic in powers of s = t - 1/2
        const float Sq = Q0 + Q1, Dq = Q0 - Q1;
        return MxK{__builtin_fmaf(0.125f, Dq, __builtin_fmaf(0.5f, dE, lo.E)), __builtin_fmaf(1.5f, dE, -0.25f * Sq),
                   -0.5f * Dq, __builtin_fmaf(-2.0f, dE, Sq)};
    }
    return MxK{lo.E, dE, Q0, Q1};
}

// Per-wave constants: the A operand of each of a quarter's four row blocks (zeros off the
// block diagonal) and the period-4 cell's third basis function at the four rows (FP32).
template <int PREC>
struct MxConst {
    typename MxOp<PREC>::vec A[4];
    float b3[4];
    int basis;

    __device__ __forceinline__ void init(int basis_, int lane)
    {
        basis = basis_;
        const int m = lane & 15, i = m & 3;
        const bool on = (lane >> 4) == (m >> 2);
#pragma unroll
        for (int r = 0; r < 4; ++r) {  // every lane adds the third term for all four rows
            float u1, u2;
            mx_cell_basis(basis, (float)(2 * r + 1) * 0.125f, u1, u2, b3[r]);
        }
        float p4f1, p4f2, p4f3;
        mx_cell_basis(basis, (float)(2 * i + 1) * 0.125f, p4f1, p4f2, p4f3);
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int k = 4 * b + i;  // the row of A this lane holds, inside the quarter
            // fused cubic: powers of the quarter's corner coordinate (monomial) or of its
            // centred coordinate w = (2k - 15) / 128
            const float z = (basis == PTG_BASIS_MONOMIAL) ? (float)(2 * k + 1) * (1.0f / 128.0f)
                                                          : (float)(2 * k - 15) * (1.0f / 128.0f);
            float p8f1, p8f2, p8f3;
            mx_cell_basis(basis, (float)(2 * (4 * (b & 1) + i) + 1) * 0.0625f, p8f1, p8f2, p8f3);
            const float w[8] = {z, z * z, z * z * z, p8f1, p8f2, p8f3, p4f1, p4f2};
#pragma unroll
            for (int j = 0; j < 8; ++j) A[b][j] = MxOp<PREC>::cvt(on ? w[j] : 0.0f);
        }
    }
};

// The rows of a strip in the precision form (cubic cells): the same hashing, fused coarse
// polynomial and node rows as strip_rows, row blocks of 4 evaluated by one MFMA each.
// Streamed periods (2, 1) are hashed per 8-row half quarter.
template <typename OutT, int LO, int PREC, bool FULL>
__device__ __forceinline__ void strip_rows_mx(const RowCtx &x, const float (&C)[4], OutT *rp, int lane, int rlo,
                                              int rhi, bool lane_ok, const MxConst<PREC> &mc)
{
    typedef MxOp<PREC> Op;
    constexpr bool H32 = LO <= 5, H16 = LO <= 4, H8 = LO <= 3, H4 = LO <= 2, H2 = LO <= 1, H1 = LO == 0;
    // streamed periods: node rows hashed per half quarter (8 rows, as in the plain C1 form),
    // which keeps a wave's blocks small enough for three workgroups of four waves per CU
    constexpr int RS = 8;
    const int basis = mc.basis;
    NR c8, c4, c2, c1;  // node row carried into the next quarter (or block)
    if (H8) c8 = node_row<9>(x.f8, 0);
    if (H4) c4 = node_row<17>(x.f4, 0);
    if (H2 || H1) {
        wave_lds_sync();  // the previous strip has read its blocks
        if (H2 && H1) {
            stream_rows_21<RS, 1, 1>(x.keys, x.s2, x.s1, 0, 0, 0, lane);
        } else {
            if (H2) stream_rows<2, RS, 1>(x.keys, x.s2, 0, 0, lane);
            if (H1) stream_rows<1, RS, 1>(x.keys, x.s1, 0, 0, lane);
        }
        wave_lds_sync();
    }
    if (H2) c2 = node_row<RS / 2 + 1>(x.f2, 0);
    if (H1) c1 = node_row<RS + 1>(x.f1, 0);
    NR n32[3], n16lo;
    if (H32) {
#pragma unroll
        for (int j = 0; j < 3; ++j) n32[j] = node_row<3>(x.f32, j);
    }
    if (H16) n16lo = node_row<5>(x.f16, 0);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        float Ch[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) Ch[b] = C[b];
        taylor_shift<1>(Ch, (float)(2 * h - 1) * 0.25f);
        if (H32) add_piece<1, 2>(Ch, n32[h], n32[h + 1]);
#pragma unroll
        for (int qh = 0; qh < 2; ++qh) {
            const int q = 2 * h + qh;
            float Cq[4];
#pragma unroll
            for (int b = 0; b < 4; ++b) Cq[b] = Ch[b];
            taylor_shift<1>(Cq, (float)(2 * qh - 1) * 0.125f);  // centred on the quarter
            if (H16) {
                const NR hi = node_row<5>(x.f16, q + 1);
                add_piece<1, 4>(Cq, n16lo, hi);
                n16lo = hi;
            }
            if (basis == PTG_BASIS_MONOMIAL) taylor_shift<1>(Cq, -0.125f);  // about the quarter's first row edge
            typename Op::vec B;
            B[0] = Op::cvt(Cq[1]);
            B[1] = Op::cvt(Cq[2]);
            B[2] = Op::cvt(Cq[3]);
            float k80 = 0.0f;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                if ((H2 || H1) && (b & 1) == 0) {  // streamed periods: this half quarter's node rows
                    const int r8 = 8 * (2 * q + (b >> 1));  // its first row in the strip
                    wave_lds_sync();
                    if (H2 && H1) {
                        stream_rows_21<RS, RS / 2, RS>(x.keys, x.s2, x.s1, r8 / 2 + 1, r8 + 1, 1, lane);
                    } else {
                        if (H2) stream_rows<2, RS, RS / 2>(x.keys, x.s2, r8 / 2 + 1, 1, lane);
                        if (H1) stream_rows<1, RS, RS>(x.keys, x.s1, r8 + 1, 1, lane);
                    }
                    wave_lds_sync();
                }
                if (H8 && (b & 1) == 0) {  // the period-8 cell of blocks b, b + 1
                    const NR hi = node_row<9>(x.f8, 2 * q + (b >> 1) + 1);
                    const MxK k8 = mx_cell_coeffs(basis, c8, hi);
                    c8 = hi;
                    k80 = k8.k0;
                    B[3] = Op::cvt(k8.k1);
                    B[4] = Op::cvt(k8.k2);
                    B[5] = Op::cvt(k8.k3);
                } else if (!H8 && b == 0) {
                    B[3] = B[4] = B[5] = Op::cvt(0.0f);
                }
                float c0 = Cq[0] + k80, k43 = 0.0f;
                if (H4) {
                    const NR hi = node_row<17>(x.f4, 4 * q + b + 1);
                    const MxK k4 = mx_cell_coeffs(basis, c4, hi);
                    c4 = hi;
                    c0 += k4.k0;
                    k43 = k4.k3;
                    B[6] = Op::cvt(k4.k1);
                    B[7] = Op::cvt(k4.k2);
                } else if (b == 0) {
                    B[6] = B[7] = Op::cvt(0.0f);
                }
                // the block's node rows of the streamed periods (rows of the half quarter's block)
                NR s2[3], s1[5];
                if (H2) {
                    s2[0] = c2;
#pragma unroll
                    for (int j = 1; j <= 2; ++j) s2[j] = node_row<RS / 2 + 1>(x.f2, 2 * (b & 1) + j);
                    c2 = s2[2];
                }
                if (H1) {
                    s1[0] = c1;
#pragma unroll
                    for (int j = 1; j <= 4; ++j) s1[j] = node_row<RS + 1>(x.f1, 4 * (b & 1) + j);
                    c1 = s1[4];
                }
                mx_f4 acc;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int row = 16 * q + 4 * b + i;
                    float v = c0;
                    if (H4) v = __builtin_fmaf(k43, mc.b3[i], v);
                    if (H2) {
                        v += s2[i / 2].E;
                        v = add_direct(v, s2[i / 2], s2[i / 2 + 1], row_bases<1>(row & 1, 2));
                    }
                    if (H1) {
                        v += s1[i].E;
                        v = add_direct(v, s1[i], s1[i + 1], row_bases<1>(0, 1));
                    }
                    acc[i] = v;
                }
                acc = Op::mma(mc.A[b], B, acc);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int row = 16 * q + 4 * b + i;
                    if (FULL || (row >= rlo && row < rhi && lane_ok))
                        rp[(int64_t)row * x.pitch + lane] = st_out<OutT>(acc[i]);
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
}

}  // namespace ptg
