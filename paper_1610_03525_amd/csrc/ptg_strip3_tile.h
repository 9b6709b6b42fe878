// ptg_strip3_tile.h -- K3 for 3D dyadic octave ladders (base frequency 2^-k, lacunarity 2),
// plain FP32 form on the vector ALUs: the per-block device code, shared by the dense kernel
// (ptg_fbm3d_strip.hip) and the persistent serving kernel (ptg_serve.hip).
//
// One wave owns a world-aligned block of k3BlockX x k3BlockY x k3BlockZ (64 x 8 x 16)
// samples, lane = x column, and walks its 16 slices in z.  Cell polynomial (Sec. 2, Sec. 3.4;
// the 3D tensor Hermite form, value h and gradient g at the corners):
//   h = sum_c [h_c B0(x) B0(y) B0(z) + gx_c B1(x) B0(y) B0(z) + gy_c B0 B1 B0 + gz_c B0 B0 B1],
// with h_c = 0 for the gradient model.  For the lane's column each (y, z) node pair of a cell
// collapses along x to three numbers (value E, y-slope Qy, z-slope Qz; "corner"), a slice
// collapses two z-corners to the 1D Hermite form in y (value V, slope W per y node), and a
// row adds V0 + (V1 - V0) S(ty) + W0 b10(ty) + W1 b11(ty).
//
// Octaves are handled in two classes:
//  * coarse (period >= 16): the block lies inside one cell in y and z.  The lane's four
//    corners are expanded, per octave and block, into a polynomial in the block's centred
//    coordinates (v_y, v_z) (degree 2M+1 in each; Sec. 2.2 eq. polynomial), and every
//    coarse octave is added into ONE such polynomial per lane.  Per slice it is contracted
//    in z (Horner), and the rows are evaluated in pairs +-v_y from its even and odd parts.
//    Every expansion point (the block centre) lies inside the octave's own cell.
//  * fine (periods 8, 4, 2): z-planes of nodes are hashed as the walk enters a new z cell
//    (two plane slots per octave in the wave's LDS block; gradient model: period 2 two
//    planes ahead at every period-4 cell, in four slots); the lane's corners of the two
//    planes of the current z cell stay in registers; per slice each y node gives V, W and
//    each row 4 operations, with compile-time row and slice bases.  Period 8 is one cell in
//    y over the block: its slice cell is added to the coarse polynomial instead.
// Octaves accumulate in FP32; each sample is stored once.
//
// Coarse nodes are hashed per block from a work list (built once per workgroup); column
// keys are kept while a wave's blocks share their x range.
#pragma once

#include <hip/hip_fp16.h>

#include "ptg_device.h"
#include "ptg_launch.h"

namespace ptg {

template <typename T>
__device__ __forceinline__ T s3_out(float v);
template <>
__device__ __forceinline__ float s3_out<float>(float v)
{
    return v;
}
template <>
__device__ __forceinline__ __half s3_out<__half>(float v)
{
    return __float2half_rn(v);
}

struct B3 {  // S, b10, b11 at one fraction
    float s, b10, b11;
};

template <int M>
__device__ __forceinline__ B3 b3_eval(float t)
{
    B3 r;
    Basis<M>::eval(t, r.s, r.b10, r.b11);
    return r;
}

// Bases at the fraction (j + 1/2) / P (constant once the loops are unrolled).
template <int M>
__host__ __device__ constexpr B3 b3_const(int j, int P)
{
    const float t = (float)(2 * j + 1) / (float)(2 * P);
    const float t2 = t * t;
    const float u = 1.0f - t;
    if (M == 1) return B3{t2 * (3.0f - 2.0f * t), t * u * u, -t2 * u};
    const float t3 = t2 * t;
    return B3{t3 * (10.0f + t * (-15.0f + 6.0f * t)), t + t3 * (-6.0f + t * (8.0f - 3.0f * t)),
              t3 * (-4.0f + t * (7.0f - 3.0f * t))};
}

// Powers of u = t - 1/2 of the bases (exact binary fractions), e = 0 .. 2M+1:
//   cubic:   S = 1/2 + 3/2 u - 2 u^3,  b10 = 1/8 - 1/4 u - 1/2 u^2 + u^3,  b11 = -1/8 - 1/4 u + 1/2 u^2 + u^3
//   quintic: S = 1/2 + 15/8 u - 5 u^3 + 6 u^5,
//            b10 = 5/32 - 7/16 u - 3/4 u^2 + 5/2 u^3 + 1/2 u^4 - 3 u^5,
//            b11 = -5/32 - 7/16 u + 3/4 u^2 + 5/2 u^3 - 1/2 u^4 - 3 u^5
template <int M>
__device__ __forceinline__ float centred_pow(int which, int e)
{
    if (M == 1) {
        constexpr float c[3][4] = {{0.5f, 1.5f, 0.0f, -2.0f}, {0.125f, -0.25f, -0.5f, 1.0f}, {-0.125f, -0.25f, 0.5f, 1.0f}};
        return c[which][e];
    }
    constexpr float c[3][6] = {{0.5f, 1.875f, 0.0f, -5.0f, 0.0f, 6.0f},
                               {0.15625f, -0.4375f, -0.75f, 2.5f, 0.5f, -3.0f},
                               {-0.15625f, -0.4375f, 0.75f, 2.5f, -0.5f, -3.0f}};
    return c[which][e];
}

// The three bases of an octave as polynomials in a block coordinate v, where the cell
// coordinate is t - 1/2 = tau + sigma v (tau, sigma uniform: the block's place in its cell).
template <int M>
struct BlockBasis {
    float p[3][2 * M + 2];  // S, b10, b11; coefficient of v^e
};

template <int M>
__device__ __forceinline__ void block_basis(BlockBasis<M> &B, float tau, float sigma)
{
    constexpr int D = 2 * M + 1;
#pragma unroll
    for (int w = 0; w < 3; ++w) {
        float *c = B.p[w];
#pragma unroll
        for (int e = 0; e <= D; ++e) c[e] = centred_pow<M>(w, e);
#pragma unroll
        for (int i = 0; i < D; ++i)  // Taylor shift to u = tau (repeated synthetic division)
#pragma unroll
            for (int j = D - 1; j >= i; --j) c[j] = __builtin_fmaf(tau, c[j + 1], c[j]);
        float sp = sigma;  // sigma is a power of two: exact powers
#pragma unroll
        for (int e = 1; e <= D; ++e) {
            c[e] *= sp;
            sp *= sigma;
        }
    }
}

// A lane's corner: a (y, z) node pair of its cell collapsed along x.
struct XC3 {
    float E, Qy, Qz;
};

// Per-octave constants a workgroup stages in LDS once.
struct Strip3Shared {
    uint32_t pre_key[kMaxOctaves];
    int shift[kMaxOctaves], coff[kMaxOctaves], kxoff[kMaxOctaves], ytoff[kMaxOctaves], ztoff[kMaxOctaves];
    float amp[kMaxOctaves], inv2p[kMaxOctaves];
    float gw;
};

// Once per workgroup (every thread, a barrier after it): the work lists of the keys and
// coarse nodes hashed per block, and the per-octave constants.
//   wl_key[q], q < keys_col: column key (o << 24 | i);  then 4 row keys per coarse octave
//   (o << 24 | 1 << 23 | 2 k + j).  wl_node[q], q < coarse_nodes: node q = coff + 4 i + 2 k + j
//   of octave o: (o << 28 | row key index << 14 | column key index).
//   Then, for each fine octave, its plane list at wl_node[fwl[f] + q], q = i * nny + j:
//   (j << 16 | column key index).
//   The basis table: for a coarse octave of period P <= k3TabMaxP, its three bases as
//   polynomials in the block coordinate (block_basis) for each of the P / k3BlockY block
//   positions in y (from ytoff) and the P / k3BlockZ positions in z (from ztoff).
template <int M>
__device__ __forceinline__ void strip3_prologue(const Fbm3dStripArgs &a, Strip3Shared &sh, float4 *tab4,
                                                uint32_t *wl_key, uint32_t *wl_node, int tid, int nthreads)
{
    const int N = a.octaves;
    constexpr int E = 3 * (2 * M + 2);
    float *tab = reinterpret_cast<float *>(tab4);
    for (int o = 0; o < a.n_coarse; ++o) {
        if (a.ytoff[o] < 0) continue;
        const int P = 1 << a.shift[o], ny = P / k3BlockY, n = ny + P / k3BlockZ;
        const float invp = 2.0f * a.inv2p[o];
        for (int e = tid; e < n; e += nthreads) {
            const bool y = e < ny;
            const int pos = y ? e : e - ny, blk = y ? k3BlockY : k3BlockZ;
            BlockBasis<M> B;
            block_basis<M>(B, (float)(pos * blk + blk / 2) * invp - 0.5f, (float)blk * invp);
            float *dst = tab + (y ? a.ytoff[o] : a.ztoff[o]) + pos * E;
#pragma unroll
            for (int w = 0; w < 3; ++w)
#pragma unroll
                for (int k = 0; k < 2 * M + 2; ++k) dst[w * (2 * M + 2) + k] = B.p[w][k];
        }
    }
    const int fo[3] = {a.o8, a.o4, a.o2};
    for (int f = 0; f < 3; ++f) {
        if (fo[f] < 0) continue;
        const int P = 8 >> f, nny = k3BlockY / P + 1, n = (k3BlockX / P + 1) * nny, kx = a.kxoff[fo[f]];
        for (int q = tid; q < n; q += nthreads) {
            const int i = q / nny, j = q - i * nny;
            wl_node[a.fwl[f] + q] = ((uint32_t)j << 16) | (uint32_t)(kx + i);
        }
    }
    for (int o = 0; o < N; ++o) {
        const int nnx = a.nnx[o], kx = a.kxoff[o];
        for (int i = tid; i < nnx; i += nthreads) wl_key[kx + i] = ((uint32_t)o << 24) | (uint32_t)i;
        if (o < a.n_coarse) {
            const int rk = a.keys_col + 4 * o;
            if (tid < 4) wl_key[rk + tid] = ((uint32_t)o << 24) | (1u << 23) | (uint32_t)tid;
            for (int q = tid; q < 4 * nnx; q += nthreads) {
                const int i = q >> 2, kj = q & 3;
                wl_node[a.coff[o] + q] = ((uint32_t)o << 28) | ((uint32_t)(rk + kj) << 14) | (uint32_t)(kx + i);
            }
        }
    }
    if (tid < N) {
        sh.pre_key[tid] = key_prefix(a.seed, tid);
        sh.shift[tid] = a.shift[tid];
        sh.coff[tid] = a.coff[tid];
        sh.kxoff[tid] = a.kxoff[tid];
        sh.ytoff[tid] = a.ytoff[tid];
        sh.ztoff[tid] = a.ztoff[tid];
        sh.amp[tid] = a.amp[tid];
        sh.inv2p[tid] = a.inv2p[tid];
        if (tid == 0) sh.gw = a.gw;
    }
}

__device__ __forceinline__ void wave_sync3()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One wave's blocks of a volume.  MD = 0: gradient model; MD = 2: node heights and
// w-weighted gradients (the height comes from the key's third word).
// AHEAD: the period-2 planes two at a time (four plane slots for period 2 in the node block;
// the plan sizes the block to match: the dense kernel takes it for both models, a serving
// workgroup, whose LDS is smaller, for the gradient model only).
template <int M, typename OutT, int LO, int MD = 0, bool AHEAD = MD == 0>
struct Strip3Wave {
    static constexpr int BX = k3BlockX, BY = k3BlockY, BZ = k3BlockZ, D1 = 2 * M + 2;
    static constexpr bool H8 = LO <= 3, H4 = LO <= 2, H2 = LO <= 1;
    static_assert(BY == 8 && BZ == 16, "the fine-octave classes assume 8-row, 16-slice blocks");

    // AHEAD: the period-2 planes are hashed two at a time, at every other z cell of period 2,
    // together with the period-4 (and period-8) plane due at the same slice, so the three
    // octaves' nodes share wave iterations; period 2 then keeps four plane slots.
    static constexpr bool AH = H2 && AHEAD;

    // A fine octave of period P: its node planes (SLOTS slots of NNX x NNY nodes, column-major;
    // plane iz in slot iz mod SLOTS), the lane's x-bases and node column, and its corners of
    // the current z cell.
    template <int P>
    struct Fine {
        static constexpr int NNX = BX / P + 1, NNY = BY / P + 1, PLANE = NNX * NNY;
        static constexpr int SLOTS = P == 2 && AHEAD ? 4 : 2;
        int o = -1, s = 0, poff = 0, kx = 0, rk = 0;
        float sc = 0.0f, amp = 0.0f;
        B3 xb{0.0f, 0.0f, 0.0f};
        int col = 0;  // first node of the lane's column in a plane
        XC3 lo[NNY], hi[NNY];
    };

    float *gx, *gy, *gz, *hh;
    uint32_t *keys;
    int lane;
    int64_t keyed_x0 = INT64_MIN;  // column keys are valid for this block x origin
    Fine<8> f8;
    Fine<4> f4;
    Fine<2> f2;

    template <int P>
    __device__ __forceinline__ void fine_init(Fine<P> &f, const Fbm3dStripArgs &a, const Strip3Shared &sh, int o)
    {
        if (o < 0) return;
        f.o = o;
        f.s = sh.shift[o];
        f.poff = a.poff[o];
        f.kx = sh.kxoff[o];
        f.rk = a.keys_col + 4 * a.n_coarse + (P == 8 ? 0 : P == 4 ? kRk4 : kRk2);
        f.amp = sh.amp[o];
        f.sc = MD == 2 ? sh.amp[o] * sh.gw : sh.amp[o];
        f.xb = b3_eval<M>((float)(2 * (lane & (P - 1)) + 1) * (1.0f / (float)(2 * P)));
        f.col = (lane / P) * Fine<P>::NNY;
    }

    __device__ __forceinline__ Strip3Wave(const Fbm3dStripArgs &a, const Strip3Shared &sh, float *gx_, int lane_)
        : gx(gx_), gy(gx_ + a.nodes_total), gz(gx_ + 2 * a.nodes_total), hh(gx_ + 3 * a.nodes_total),
          keys(reinterpret_cast<uint32_t *>(gx_ + (MD == 2 ? 4 : 3) * a.nodes_total)), lane(lane_)
    {
        if (H8) fine_init(f8, a, sh, a.o8);
        if (H4) fine_init(f4, a, sh, a.o4);
        if (H2) fine_init(f2, a, sh, a.o2);
    }

    // Node q of the wave's block from its key: unit gradient times sc; MD = 2: height times amp.
    __device__ __forceinline__ void put_node(int q, uint32_t key, float sc, float amp)
    {
        const uint32_t second = key3_second(key);
        const float3 g = grad3_of(key, second);
        gx[q] = g.x * sc;
        gy[q] = g.y * sc;
        gz[q] = g.z * sc;
        if (MD == 2) hh[q] = height3_of_second(second) * amp;
    }

    // Corner of nodes a (column i) and a + nstride (column i + 1).
    __device__ __forceinline__ XC3 corner(int a, int nstride, const B3 &xb) const
    {
        const int b = a + nstride;
        XC3 c{gx[a] * xb.b10 + gx[b] * xb.b11, gy[a] + xb.s * (gy[b] - gy[a]), gz[a] + xb.s * (gz[b] - gz[a])};
        if (MD == 2) c.E += hh[a] + xb.s * (hh[b] - hh[a]);
        return c;
    }

    // Row keys of every fine octave's node planes of the block (planes Z0 / P .. Z0 / P +
    // BZ / P, NNY rows each), one list: period 8 from 0, period 4 from kRk4, period 2 from kRk2.
    static constexpr int kRk4 = (BZ / 8 + 1) * (BY / 8 + 1), kRk2 = kRk4 + (BZ / 4 + 1) * (BY / 4 + 1),
                         kRkAll = kRk2 + (BZ / 2 + 1) * (BY / 2 + 1);
    __device__ __forceinline__ void fine_rowkeys(const Strip3Shared &sh, int rk0, int64_t Y0, int64_t Z0, int o8,
                                                 int o4, int o2)
    {
        for (int q = lane; q < kRkAll; q += 64) {
            const bool p8 = q < kRk4, p4 = !p8 && q < kRk2;
            const int o = p8 ? o8 : p4 ? o4 : o2;
            if (o < 0) continue;
            const int nny = p8 ? BY / 8 + 1 : p4 ? BY / 4 + 1 : BY / 2 + 1, s = p8 ? 3 : p4 ? 2 : 1;
            const int r = q - (p8 ? 0 : p4 ? kRk4 : kRk2), pl = r / nny, j = r - pl * nny;
            keys[rk0 + q] = absorb_index(absorb_index(sh.pre_key[o], (Z0 >> s) + pl), (Y0 >> s) + j);
        }
    }

    // Nodes of planes iz0 .. iz0 + np - 1 (np = 1, 2, 3) into their slots, from the octave's
    // plane list.
    // (ib = iz0 - Z0 / P: the plane's index in the block's row-key list)
    template <int P>
    __device__ __forceinline__ void fine_nodes(const Fine<P> &f, const uint32_t *wl, int64_t iz0, int ib, int np)
    {
        constexpr int NNY = Fine<P>::NNY, PLANE = Fine<P>::PLANE, SM = Fine<P>::SLOTS - 1;
        for (int q = lane; q < np * PLANE; q += 64) {
            const int pl = q >= 2 * PLANE ? 2 : q >= PLANE ? 1 : 0, rem = q - pl * PLANE;
            const uint32_t it = wl[rem];
            const uint32_t key = key_combine(keys[f.rk + (ib + pl) * NNY + (int)(it >> 16)], keys[it & 0xFFFF]);
            put_node(f.poff + (int)((iz0 + pl) & SM) * PLANE + rem, key, f.sc, f.amp);
        }
    }

    // AHEAD, a slice that starts a z cell of period 4 (q = Z - Z0): the period-2
    // planes Z / 2 + 1 and Z / 2 + 2, the period-4 plane Z / 4 + 1 and, at the start of a
    // period-8 cell, the period-8 plane Z / 8 + 1, as one list of nodes over the wave's lanes.
    template <int Q>
    __device__ __forceinline__ void fine_nodes_merged(const Fbm3dStripArgs &a, const uint32_t *wl_node, int64_t Z,
                                                      int q)
    {
        constexpr int P2 = Fine<2>::PLANE, P4 = Fine<4>::PLANE, P8 = Fine<8>::PLANE;
        constexpr int N2 = 2 * P2, N4 = N2 + P4, N = N4 + (Q == 0 ? P8 : 0), FULL = N2 / 64;
        static_assert(64 * FULL >= P2, "the mixed iterations hold the second period-2 plane only");
        const int64_t c2 = (Z >> 1) + 1, c4 = (Z >> 2) + 1, c8 = (Z >> 3) + 1;
        const int ib2 = q / 2 + 1;
        // iterations wholly inside the two period-2 planes
#pragma unroll
        for (int i = 0; i < FULL; ++i) {
            const int t = 64 * i + lane;
            const int pl = t >= P2 ? 1 : 0, rem = t - pl * P2;
            const uint32_t it = wl_node[a.fwl[2] + rem];
            const uint32_t key =
                key_combine(keys[f2.rk + (ib2 + pl) * Fine<2>::NNY + (int)(it >> 16)], keys[it & 0xFFFF]);
            put_node(f2.poff + (int)((c2 + pl) & 3) * P2 + rem, key, f2.sc, f2.amp);
        }
        // the rest: the second period-2 plane's last nodes, then period 4, then period 8; each
        // lane picks its octave's work list, row keys, slot and scale (selected as values: a
        // selection among the members themselves would place the octave records in scratch)
        const int wl2 = a.fwl[2] - P2, wl4 = a.fwl[1] - N2, wl8 = a.fwl[0] - N4;
        const int kr2 = f2.rk + (ib2 + 1) * Fine<2>::NNY, kr4 = f4.rk + (q / 4 + 1) * Fine<4>::NNY,
                  kr8 = f8.rk + (q / 8 + 1) * Fine<8>::NNY;
        const int d2 = f2.poff + (int)((c2 + 1) & 3) * P2 - P2, d4 = f4.poff + (int)(c4 & 1) * P4 - N2,
                  d8 = f8.poff + (int)(c8 & 1) * P8 - N4;
        const float s2 = f2.sc, s4 = f4.sc, s8 = f8.sc, a2 = f2.amp, a4 = f4.amp, a8 = f8.amp;
        for (int t = 64 * FULL + lane; t < N; t += 64) {
            const bool in2 = t < N2, in4 = t < N4;
            const int wl = in2 ? wl2 : in4 ? wl4 : wl8;    // + t: the node's work-list entry
            const int krow = in2 ? kr2 : in4 ? kr4 : kr8;  // its plane's row keys
            const int dst = in2 ? d2 : in4 ? d4 : d8;      // + t: its place in the slot
            const float sc = in2 ? s2 : in4 ? s4 : s8, amp = in2 ? a2 : in4 ? a4 : a8;
            const uint32_t it = wl_node[wl + t];
            const uint32_t key = key_combine(keys[krow + (int)(it >> 16)], keys[it & 0xFFFF]);
            put_node(dst + t, key, sc, amp);
        }
    }

    // The lane's corners of plane iz (its slot).
    template <int P>
    __device__ __forceinline__ void fine_corners(const Fine<P> &f, int64_t iz, XC3 (&c)[Fine<P>::NNY]) const
    {
        constexpr int NNY = Fine<P>::NNY, PLANE = Fine<P>::PLANE, SM = Fine<P>::SLOTS - 1;
        const int base = f.poff + (int)(iz & SM) * PLANE + f.col;
#pragma unroll
        for (int j = 0; j < NNY; ++j) c[j] = corner(base + j, NNY, f.xb);
    }

    // Slice ZQ of a z cell of period P: V and W per y node, then the rows.
    template <int P, int ZQ>
    __device__ __forceinline__ void fine_rows(const Fine<P> &f, float (&t)[BY]) const
    {
        constexpr int NNY = Fine<P>::NNY;
        constexpr B3 zb = b3_const<M>(ZQ, P);
        float V[NNY], W[NNY];
#pragma unroll
        for (int j = 0; j < NNY; ++j) {
            const XC3 &l = f.lo[j], &h = f.hi[j];
            V[j] = __builtin_fmaf(h.Qz, zb.b11, __builtin_fmaf(l.Qz, zb.b10, __builtin_fmaf(zb.s, h.E - l.E, l.E)));
            W[j] = __builtin_fmaf(zb.s, h.Qy - l.Qy, l.Qy);
        }
#pragma unroll
        for (int c = 0; c < BY / P; ++c) {
            const float dV = V[c + 1] - V[c];
#pragma unroll
            for (int rr = 0; rr < P; ++rr) {
                const B3 yb = b3_const<M>(rr, P);
                float v = t[c * P + rr] + V[c];
                v = __builtin_fmaf(dV, yb.s, v);
                v = __builtin_fmaf(W[c], yb.b10, v);
                t[c * P + rr] = __builtin_fmaf(W[c + 1], yb.b11, v);
            }
        }
    }

    // Add coarse octave o (period >= 16) of the block to the fused polynomial Cb[e_y][e_z].
    __device__ __forceinline__ void coarse_add(float (&Cb)[D1][D1], const Strip3Shared &sh, const float *tab, int o,
                                               int64_t X0, int64_t Y0, int64_t Z0) const
    {
        const int s = sh.shift[o];
        const uint32_t mask = (1u << s) - 1u;
        const float inv2p = sh.inv2p[o], invp = 2.0f * inv2p;
        const uint32_t xl = ((uint32_t)X0 & mask) + (uint32_t)lane;
        const B3 xb = b3_eval<M>((float)(2u * (xl & mask) + 1u) * inv2p);
        const int a0 = sh.coff[o] + 4 * (int)(xl >> s);
        XC3 c00 = corner(a0, 4, xb), c10 = corner(a0 + 1, 4, xb), c01 = corner(a0 + 2, 4, xb),
            c11 = corner(a0 + 3, 4, xb);  // c[j][k]: y node j, z node k
        BlockBasis<M> yb, zb;
        const int yt = sh.ytoff[o];
        if (yt >= 0) {  // uniform: the octave's table (periods <= k3TabMaxP)
            const float *ye = tab + yt + (int)(((uint32_t)Y0 & mask) / BY) * (3 * D1);
            const float *ze = tab + sh.ztoff[o] + (int)(((uint32_t)Z0 & mask) / BZ) * (3 * D1);
#pragma unroll
            for (int w = 0; w < 3; ++w)
#pragma unroll
                for (int k = 0; k < D1; ++k) {
                    yb.p[w][k] = ye[w * D1 + k];
                    zb.p[w][k] = ze[w * D1 + k];
                }
        } else {
            block_basis<M>(yb, (float)(((uint32_t)Y0 & mask) + (uint32_t)(BY / 2)) * invp - 0.5f, (float)BY * invp);
            block_basis<M>(zb, (float)(((uint32_t)Z0 & mask) + (uint32_t)(BZ / 2)) * invp - 0.5f, (float)BZ * invp);
        }
        // h = Y0(v_y) + Sz(v_z) (Y1 - Y0)(v_y) + b10z(v_z) Y2(v_y) + b11z(v_z) Y3(v_y)
        const float dE0 = c10.E - c00.E, dE1 = c11.E - c01.E, dQ0 = c10.Qz - c00.Qz, dQ1 = c11.Qz - c01.Qz;
#pragma unroll
        for (int e = 0; e < D1; ++e) {
            float y0 = __builtin_fmaf(c10.Qy, yb.p[2][e], __builtin_fmaf(c00.Qy, yb.p[1][e], dE0 * yb.p[0][e]));
            float y1 = __builtin_fmaf(c11.Qy, yb.p[2][e], __builtin_fmaf(c01.Qy, yb.p[1][e], dE1 * yb.p[0][e]));
            float y2 = dQ0 * yb.p[0][e], y3 = dQ1 * yb.p[0][e];
            if (e == 0) {
                y0 += c00.E;
                y1 += c01.E;
                y2 += c00.Qz;
                y3 += c01.Qz;
            }
            const float d = y1 - y0;
            Cb[e][0] += y0;
#pragma unroll
            for (int ez = 0; ez < D1; ++ez)
                Cb[e][ez] = __builtin_fmaf(y3, zb.p[2][ez], __builtin_fmaf(y2, zb.p[1][ez], __builtin_fmaf(d, zb.p[0][ez], Cb[e][ez])));
        }
    }

    // Block blk of the volume (blocks are numbered z fastest: a column of blocks in z is a
    // run of consecutive indices).  carry: this wave's previous block was the one below it
    // in z, whose last node planes of the fine octaves (and the lane's corners of them) are
    // the first of this block -- they are kept instead of hashed again.
    __device__ __forceinline__ void run(const Fbm3dStripArgs &a, const Strip3Shared &sh, const float4 *tab4,
                                        const uint32_t *wl_key, const uint32_t *wl_node, int64_t blk,
                                        bool carry = false)
    {
        const int64_t col = blk / a.blocks_z, bz = blk - col * a.blocks_z;
        const int64_t by = col / a.blocks_x, bx = col - by * a.blocks_x;
        const int64_t X0 = a.bx_base + bx * BX, Y0 = a.by_base + by * BY, Z0 = a.bz_base + bz * BZ;
        const int keys_col = a.keys_col, nrk = keys_col + 4 * a.n_coarse;

        // ---- keys: column keys (while the x origin is unchanged they stay), the coarse
        // octaves' row keys, the fine octaves' row keys of their first two planes ----------
        if (X0 != keyed_x0) {
            for (int q = lane; q < keys_col; q += 64) {
                const uint32_t it = wl_key[q];
                keys[q] = key_xline((X0 >> sh.shift[it >> 24]) + (int64_t)(it & 0xFFFF));
            }
            keyed_x0 = X0;
        }
        for (int q = keys_col + lane; q < nrk; q += 64) {
            const uint32_t it = wl_key[q];
            const int o = it >> 24, s = sh.shift[o];
            const int j = it & 1, k = (it >> 1) & 1;
            keys[q] = absorb_index(absorb_index(sh.pre_key[o], (Z0 >> s) + k), (Y0 >> s) + j);
        }
        if (H8) fine_rowkeys(sh, nrk, Y0, Z0, f8.o, H4 ? f4.o : -1, H2 ? f2.o : -1);
        wave_sync3();
        for (int q = lane; q < a.coarse_nodes; q += 64) {
            const uint32_t it = wl_node[q];
            const int o = it >> 28;
            const uint32_t key = key_combine(keys[(it >> 14) & 0x3FFF], keys[it & 0x3FFF]);
            put_node(q, key, MD == 2 ? sh.amp[o] * sh.gw : sh.amp[o], sh.amp[o]);
        }
        if (!carry) {
            if (H8) fine_nodes(f8, wl_node + a.fwl[0], Z0 >> 3, 0, 2);
            if (H4) fine_nodes(f4, wl_node + a.fwl[1], Z0 >> 2, 0, 2);
            if (H2) fine_nodes(f2, wl_node + a.fwl[2], Z0 >> 1, 0, AH ? 3 : 2);
        }
        wave_sync3();

        // ---- coarse octaves: one polynomial in (v_y, v_z) per lane ----------------------
        float Cb[D1][D1];
#pragma unroll
        for (int e = 0; e < D1; ++e)
#pragma unroll
            for (int ez = 0; ez < D1; ++ez) Cb[e][ez] = 0.0f;
        const float *tab = reinterpret_cast<const float *>(tab4);
        for (int o = 0; o < a.n_coarse; ++o) coarse_add(Cb, sh, tab, o, X0, Y0, Z0);

        // ---- fine octaves: the corners of their first z cell (carried: the first slice
        // advances from the previous block's last cell) -------------------------------------
        if (!carry && H8) {
            fine_corners(f8, Z0 >> 3, f8.lo);
            fine_corners(f8, (Z0 >> 3) + 1, f8.hi);
        }
        if (!carry && H4) {
            fine_corners(f4, Z0 >> 2, f4.lo);
            fine_corners(f4, (Z0 >> 2) + 1, f4.hi);
        }
        if (!carry && H2) {
            fine_corners(f2, Z0 >> 1, f2.lo);
            fine_corners(f2, (Z0 >> 1) + 1, f2.hi);
        }

        // ---- slices ---------------------------------------------------------------------
        const int64_t xe = a.x0 + a.nx, ye = a.y0 + a.ny, ze = a.z0 + a.nz;
        const bool full_xy = X0 >= a.x0 && X0 + BX <= xe && Y0 >= a.y0 && Y0 + BY <= ye;
        const bool lane_ok = X0 + lane >= a.x0 && X0 + lane < xe;
        const int qlo = (int)max<int64_t>(0, a.z0 - Z0), qhi = (int)min<int64_t>(BZ, ze - Z0);  // stored slices
        // slice 0's first row of the block in the output (uniform)
        OutT *const base = reinterpret_cast<OutT *>(a.out) + (((Z0 - a.z0) * a.ny + (Y0 - a.y0)) * a.nx + (X0 - a.x0));
#pragma unroll 1
        for (int g = 0; g < BZ / 8; ++g) {
            slice<0>(a, sh, wl_node, Cb, g, carry, Y0, Z0, ye, qlo, qhi, full_xy, lane_ok, base);
            slice<1>(a, sh, wl_node, Cb, g, carry, Y0, Z0, ye, qlo, qhi, full_xy, lane_ok, base);
            slice<2>(a, sh, wl_node, Cb, g, carry, Y0, Z0, ye, qlo, qhi, full_xy, lane_ok, base);
            slice<3>(a, sh, wl_node, Cb, g, carry, Y0, Z0, ye, qlo, qhi, full_xy, lane_ok, base);
            slice<4>(a, sh, wl_node, Cb, g, carry, Y0, Z0, ye, qlo, qhi, full_xy, lane_ok, base);
            slice<5>(a, sh, wl_node, Cb, g, carry, Y0, Z0, ye, qlo, qhi, full_xy, lane_ok, base);
            slice<6>(a, sh, wl_node, Cb, g, carry, Y0, Z0, ye, qlo, qhi, full_xy, lane_ok, base);
            slice<7>(a, sh, wl_node, Cb, g, carry, Y0, Z0, ye, qlo, qhi, full_xy, lane_ok, base);
        }
        __builtin_amdgcn_wave_barrier();  // the next block rewrites this wave's keys and nodes
    }

    // Slice 8 g + Q of the block.
    template <int Q>
    __device__ __forceinline__ void slice(const Fbm3dStripArgs &a, const Strip3Shared &sh, const uint32_t *wl_node,
                                          const float (&Cb)[D1][D1], int g, bool carry, int64_t Y0, int64_t Z0,
                                          int64_t ye, int qlo, int qhi, bool full_xy, bool lane_ok, OutT *base)
    {
        const int q = 8 * g + Q;
        const int64_t Z = Z0 + q;
        // a new z cell of the fine octaves whose period divides q: its upper plane
        constexpr bool A8 = H8 && Q == 0, A4 = H4 && Q % 4 == 0, A2 = H2 && Q % 2 == 0;
        // period-2 planes are hashed here (with AH: at every other period-2 cell, two planes)
        constexpr bool N2 = A2 && (!AH || Q % 4 == 0);
        if ((A8 || A4 || A2) && (Q > 0 || g > 0 || carry)) {
            if (A8 || A4 || N2) {
                wave_sync3();  // every lane has read the slots that are rewritten
                if (AH && N2) {
                    fine_nodes_merged<Q>(a, wl_node, Z, q);
                } else {
                    if (A8) fine_nodes(f8, wl_node + a.fwl[0], (Z >> 3) + 1, q / 8 + 1, 1);
                    if (A4) fine_nodes(f4, wl_node + a.fwl[1], (Z >> 2) + 1, q / 4 + 1, 1);
                    if (N2) fine_nodes(f2, wl_node + a.fwl[2], (Z >> 1) + 1, q / 2 + 1, 1);
                }
                wave_sync3();
            }
            if (A8) {
#pragma unroll
                for (int j = 0; j < Fine<8>::NNY; ++j) f8.lo[j] = f8.hi[j];
                fine_corners(f8, (Z >> 3) + 1, f8.hi);
            }
            if (A4) {
#pragma unroll
                for (int j = 0; j < Fine<4>::NNY; ++j) f4.lo[j] = f4.hi[j];
                fine_corners(f4, (Z >> 2) + 1, f4.hi);
            }
            if (A2) {
#pragma unroll
                for (int j = 0; j < Fine<2>::NNY; ++j) f2.lo[j] = f2.hi[j];
                fine_corners(f2, (Z >> 1) + 1, f2.hi);
            }
        }
        // coarse: contract in z, then the rows in pairs +-v_y about the block centre
        const float vz = (float)(2 * q - (BZ - 1)) * (1.0f / (float)(2 * BZ));
        float C[D1];
#pragma unroll
        for (int e = 0; e < D1; ++e) {
            float c = Cb[e][D1 - 1];
#pragma unroll
            for (int ez = D1 - 2; ez >= 0; --ez) c = __builtin_fmaf(c, vz, Cb[e][ez]);
            C[e] = c;
        }
        // period 8: the block is one cell in y, centred on it (t - 1/2 = v_y), so its slice
        // cell joins the polynomial through the bases' centred powers
        if (H8) {
            constexpr B3 zb = b3_const<M>(Q % 8, 8);
            const XC3 &l0 = f8.lo[0], &h0 = f8.hi[0], &l1 = f8.lo[1], &h1 = f8.hi[1];
            const float V0 = __builtin_fmaf(h0.Qz, zb.b11, __builtin_fmaf(l0.Qz, zb.b10, __builtin_fmaf(zb.s, h0.E - l0.E, l0.E)));
            const float V1 = __builtin_fmaf(h1.Qz, zb.b11, __builtin_fmaf(l1.Qz, zb.b10, __builtin_fmaf(zb.s, h1.E - l1.E, l1.E)));
            const float W0 = __builtin_fmaf(zb.s, h0.Qy - l0.Qy, l0.Qy), W1 = __builtin_fmaf(zb.s, h1.Qy - l1.Qy, l1.Qy);
            const float dV = V1 - V0;
            C[0] += V0;
#pragma unroll
            for (int e = 0; e < D1; ++e) {
                const float cs = centred_pow<M>(0, e), c10 = centred_pow<M>(1, e), c11 = centred_pow<M>(2, e);
                float c = C[e];
                if (cs != 0.0f) c = __builtin_fmaf(dV, cs, c);
                c = __builtin_fmaf(W0, c10, c);
                C[e] = __builtin_fmaf(W1, c11, c);
            }
        }
        float t[BY];
#pragma unroll
        for (int p = 0; p < BY / 2; ++p) {
            const float w = (float)(2 * p + 1) * (1.0f / (float)(2 * BY));
            const float w2 = w * w;
            float even = C[D1 - 2], odd = C[D1 - 1];
#pragma unroll
            for (int e = D1 - 4; e >= 0; e -= 2) {
                even = __builtin_fmaf(even, w2, C[e]);
                odd = __builtin_fmaf(odd, w2, C[e + 1]);
            }
            t[BY / 2 + p] = __builtin_fmaf(w, odd, even);
            t[BY / 2 - 1 - p] = __builtin_fmaf(-w, odd, even);
        }
        if (H4) fine_rows<4, Q % 4>(f4, t);
        if (H2) fine_rows<2, Q % 2>(f2, t);
        // stores: a uniform row pointer per row plus the lane's 32-bit column offset
        if (q >= qlo && q < qhi) {
            OutT *row = base + (int64_t)q * a.ny * a.nx;
            if (full_xy) {
#pragma unroll
                for (int r = 0; r < BY; ++r) {
                    row[(uint32_t)lane] = s3_out<OutT>(t[r]);
                    row += a.nx;
                }
            } else {
#pragma unroll
                for (int r = 0; r < BY; ++r) {
                    if (Y0 + r >= a.y0 && Y0 + r < ye && lane_ok) row[(uint32_t)lane] = s3_out<OutT>(t[r]);
                    row += a.nx;
                }
            }
        }
        // keep each slice's work together: without this the scheduler interleaves the unrolled
        // slices and holds several slices' values in registers at once
        __builtin_amdgcn_sched_barrier(0);
    }
};

}  // namespace ptg
