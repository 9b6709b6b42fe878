// ptg_strip3_tile.h -- K3 for 3D dyadic octave ladders (base frequency 2^-k, lacunarity 2),
// plain FP32 form on the vector ALUs: the per-block device code, shared by the dense kernel
// (ptg_fbm3d_strip.hip) and the persistent serving kernel (ptg_serve.hip).
//
// One wave owns a world-aligned block of k3BlockX x k3BlockY x k3BlockZ samples (lane = x
// column) and walks blocks with a grid stride; after the prologue the waves of a workgroup
// never synchronise.  Per block the wave hashes its footprint nodes into a private LDS
// block (K1 logic: one key per node column and per (z, y) node row, one fmix32 per node,
// amplitude folded in).
//
// Cell polynomial (Sec. 2, Sec. 3.4; 3D tensor Hermite form, value 0 and gradient g at the
// corners): h = sum_c [gx b1_cx(x) b0_cy(y) b0_cz(z) + gy b0_cx b1_cy b0_cz + gz b0_cx b0_cy b1_cz].
// For the lane's column x and one z slice it collapses to the 1D Hermite form in y
//   x:  Ex(cy,cz) = gx(0,cy,cz) b10(tx) + gx(1,cy,cz) b11(tx),  Qy, Qz = lerp_x(gy), lerp_x(gz);
//   z:  V(cy) = lerp_z(Ex(cy,.)) + Qz(cy,0) b10(tz) + Qz(cy,1) b11(tz),  W(cy) = lerp_z(Qy(cy,.));
//   y:  h(y) = V0 + (V1 - V0) S(ty) + W0 b10(ty) + W1 b11(ty),
// so each row of a slice adds 4 operations per octave.  Octaves of period >= 8 cover the
// block with one cell (runtime loop, bases from an LDS table or evaluated); periods 4, 2, 1
// are template classes whose row and slice bases are compile-time constants.
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

// Bases at world index W of an octave of period 2^s: from the table, or evaluated.
template <int M>
__device__ __forceinline__ B3 b3_at(const float4 *tab, int toff, int64_t W, uint32_t mask, float inv2p)
{
    if (toff >= 0) {
        const float4 e = tab[toff + (int)((uint32_t)W & mask)];
        return B3{e.y, e.z, e.w};
    }
    return b3_eval<M>((float)(2u * ((uint32_t)W & mask) + 1u) * inv2p);
}

struct Y1 {  // 1D Hermite form in y of one cell at one column and slice
    float E0, dE, W0, W1;
};

// Node row j of a block at one column and slice, collapsed along x and z: the value-in-y
// term V(j) and the slope-in-y term W(j).  Cell c of the row uses rows c and c + 1:
// E0 = V(c), dE = V(c+1) - V(c), W0 = W(c), W1 = W(c+1).
struct VW {
    float V, W;
};

__device__ __forceinline__ VW row_vw(const float *gx, const float *gy, const float *gz, int na, int sx, const B3 &xb,
                                     const B3 &zb)
{
    float Ex[2], Qy[2], Qz[2];
#pragma unroll
    for (int dk = 0; dk < 2; ++dk) {
        const int a = na + dk, b = a + sx;
        Ex[dk] = gx[a] * xb.b10 + gx[b] * xb.b11;
        Qy[dk] = gy[a] + xb.s * (gy[b] - gy[a]);
        Qz[dk] = gz[a] + xb.s * (gz[b] - gz[a]);
    }
    return VW{Ex[0] + zb.s * (Ex[1] - Ex[0]) + Qz[0] * zb.b10 + Qz[1] * zb.b11, Qy[0] + zb.s * (Qy[1] - Qy[0])};
}

__device__ __forceinline__ Y1 cell_y1(const VW &lo, const VW &hi) { return Y1{lo.V, hi.V - lo.V, lo.W, hi.W}; }

// One node (y, z) of a block collapsed along x at the lane's column (value term E, slope
// terms Qy, Qz); two of them on consecutive z nodes give the row's V and W at a slice.
struct XC {
    float E, Qy, Qz;
};

__device__ __forceinline__ XC col_x(const float *gx, const float *gy, const float *gz, int na, int sx, const B3 &xb)
{
    const int b = na + sx;
    return XC{gx[na] * xb.b10 + gx[b] * xb.b11, gy[na] + xb.s * (gy[b] - gy[na]), gz[na] + xb.s * (gz[b] - gz[na])};
}

__device__ __forceinline__ VW z_vw(const XC &lo, const XC &hi, const B3 &zb)
{
    return VW{lo.E + zb.s * (hi.E - lo.E) + lo.Qz * zb.b10 + hi.Qz * zb.b11, lo.Qy + zb.s * (hi.Qy - lo.Qy)};
}

__device__ __forceinline__ float y1_at(const Y1 &f, const B3 &yb)
{
    return f.E0 + f.dE * yb.s + f.W0 * yb.b10 + f.W1 * yb.b11;
}


// Per-octave constants a workgroup stages in LDS once.
struct Strip3Shared {
    uint32_t pre_key[kMaxOctaves];
    int shift[kMaxOctaves], noff[kMaxOctaves], nny[kMaxOctaves], nnz[kMaxOctaves], toff[kMaxOctaves];
    float amp[kMaxOctaves], inv2p[kMaxOctaves];
};

// Once per workgroup (every thread, a barrier after it): the basis table of the periods
// <= 64, the key and node work lists (the same for every block) and the per-octave constants.
template <int M>
__device__ __forceinline__ void strip3_prologue(const Fbm3dStripArgs &a, Strip3Shared &sh, float4 *tab,
                                                uint32_t *wl_key, uint32_t *wl_node, int tid, int nthreads)
{
    const int N = a.octaves;
    for (int o = 0; o < N; ++o) {
        const int nnx = a.nnx[o], nny = a.nny[o], nnz = a.nnz[o], kx = a.kxoff[o], kzy = a.kzyoff[o];
        const int no = a.noff[o], to = a.toff[o];
        if (to >= 0) {
            const int P = 1 << a.shift[o];
            for (int r = tid; r < P; r += nthreads) {
                float S, b10, b11;
                Basis<M>::eval((float)(2 * r + 1) * a.inv2p[o], S, b10, b11);
                tab[to + r] = make_float4(1.0f - S, S, b10, b11);
            }
        }
        for (int i = tid; i < nnx + nny * nnz; i += nthreads)
            wl_key[kx + i] = ((uint32_t)o << 24) | (i < nnx ? (uint32_t)i : ((1u << 23) | (uint32_t)(i - nnx)));
        const int plane = nny * nnz;
        for (int q = tid; q < nnx * plane; q += nthreads) {
            const int i = q / plane, rem = q - i * plane;
            const int j = rem / nnz, k = rem - j * nnz;  // node (i, j, k) at noff + (i * nny + j) * nnz + k
            wl_node[no + q] = ((uint32_t)o << 28) | ((uint32_t)(kzy + k * nny + j) << 14) | (uint32_t)(kx + i);
        }
    }
    if (tid < N) {
        sh.pre_key[tid] = key_prefix(a.seed, tid);
        sh.shift[tid] = a.shift[tid];
        sh.noff[tid] = a.noff[tid];
        sh.nny[tid] = a.nny[tid];
        sh.nnz[tid] = a.nnz[tid];
        sh.toff[tid] = a.toff[tid];
        sh.amp[tid] = a.amp[tid];
        sh.inv2p[tid] = a.inv2p[tid];
    }
}

// One wave's blocks of a volume: the lane's x-bases of the fixed periods 4, 2, 1 (formed
// once) and its private node block.
template <int M, typename OutT, int LO>
struct Strip3Wave {
    static constexpr int BX = k3BlockX, BY = k3BlockY, BZ = k3BlockZ;
    static constexpr bool H4 = LO <= 2, H2 = LO <= 1, H1 = LO == 0;
    struct Fine {
        int noff, nny, nnz;
        B3 xb;
    };
    float *gx, *gy, *gz;
    uint32_t *keys;
    int lane;
    Fine f4, f2, f1;

    __device__ __forceinline__ Fine fine(const Strip3Shared &sh, int o) const
    {
        Fine f{0, 2, 2, B3{0.0f, 0.0f, 0.0f}};
        if (o >= 0) {
            const int s = sh.shift[o];
            f.noff = sh.noff[o];
            f.nny = sh.nny[o];
            f.nnz = sh.nnz[o];
            f.xb = b3_eval<M>((float)(2 * (lane & ((1 << s) - 1)) + 1) * sh.inv2p[o]);
        }
        return f;
    }

    __device__ __forceinline__ Strip3Wave(const Fbm3dStripArgs &a, const Strip3Shared &sh, float *gx_, int lane_)
        : gx(gx_), gy(gx_ + a.nodes_total), gz(gx_ + 2 * a.nodes_total),
          keys(reinterpret_cast<uint32_t *>(gx_ + 3 * a.nodes_total)), lane(lane_)
    {
        f4 = fine(sh, H4 ? a.o4 : -1);
        f2 = fine(sh, H2 ? a.o2 : -1);
        f1 = fine(sh, H1 ? a.o1 : -1);
    }

    // Block blk of the volume: hash its footprint, then every octave and the stores.
    __device__ __forceinline__ void run(const Fbm3dStripArgs &a, const Strip3Shared &sh, const float4 *tab,
                                        const uint32_t *wl_key, const uint32_t *wl_node, int64_t blk)
    {
        const int nodes_total = a.nodes_total, keys_total = a.keys_total;
        const int n_coarse = a.n_coarse;
        const int64_t xe = a.x0 + a.nx, ye = a.y0 + a.ny, ze = a.z0 + a.nz;
        const int64_t bplane = (int64_t)a.blocks_x * a.blocks_y;
        OutT *out = reinterpret_cast<OutT *>(a.out);
        const int64_t bz = blk / bplane, rem = blk - bz * bplane;
        const int64_t by = rem / a.blocks_x, bx = rem - by * a.blocks_x;
        const int64_t X0 = a.bx_base + bx * BX, Y0 = a.by_base + by * BY, Z0 = a.bz_base + bz * BZ;

        // ---- hashing: column keys and (z, y) row keys, then node gradients ---------------
        for (int q = lane; q < keys_total; q += 64) {
            const uint32_t it = wl_key[q];
            const int o = it >> 24;
            const int s = sh.shift[o];
            const int idx = it & 0x7FFFFF;
            uint32_t key;
            if (it & (1u << 23)) {
                const int nny = sh.nny[o], k = idx / nny, j = idx - k * nny;
                key = absorb_index(absorb_index(sh.pre_key[o], (Z0 >> s) + k), (Y0 >> s) + j);
            } else {
                key = key_xline((X0 >> s) + idx);
            }
            keys[q] = key;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (int q = lane; q < nodes_total; q += 64) {
            const uint32_t it = wl_node[q];
            const float amp = sh.amp[it >> 28];
            const float3 g = grad3(key_combine(keys[(it >> 14) & 0x3FFF], keys[it & 0x3FFF]));
            gx[q] = g.x * amp;
            gy[q] = g.y * amp;
            gz[q] = g.z * amp;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

        const int64_t X = X0 + lane;
        const bool lane_ok = X >= a.x0 && X < xe;
        // ---- periods >= 8: one cell over the block; its nodes and bases are read once ------
        float acc[BZ][BY], e0[BZ];  // per row: the dE / W terms; per slice: the cells' E0 terms
#pragma unroll
        for (int zz = 0; zz < BZ; ++zz) {
            e0[zz] = 0.0f;
#pragma unroll
            for (int r = 0; r < BY; ++r) acc[zz][r] = 0.0f;
        }
        for (int o = 0; o < n_coarse; ++o) {
            // per-octave values from the arguments: uniform (scalar) in the dense kernel
            const int s = a.shift[o];
            const uint32_t mask = (1u << s) - 1u;
            const float inv2p = a.inv2p[o];
            const int to = a.toff[o];
            const B3 xb = b3_at<M>(tab, to, X, mask, inv2p);
            const int nny = a.nny[o], nnz = a.nnz[o];
            const int cxl = (int)((((uint32_t)X0 & mask) + (uint32_t)lane) >> s);
            const int n0 = a.noff[o] + cxl * nny * nnz, sx = nny * nnz;
            float ex[2][2], qy[2][2], qz[2][2];  // x-collapsed corners (y node, z node)
#pragma unroll
            for (int dj = 0; dj < 2; ++dj)
#pragma unroll
                for (int dk = 0; dk < 2; ++dk) {
                    const int na = n0 + dj * nnz + dk, nb = na + sx;
                    ex[dj][dk] = gx[na] * xb.b10 + gx[nb] * xb.b11;
                    qy[dj][dk] = gy[na] + xb.s * (gy[nb] - gy[na]);
                    qz[dj][dk] = gz[na] + xb.s * (gz[nb] - gz[na]);
                }
            B3 yb[BY];
#pragma unroll
            for (int r = 0; r < BY; ++r) yb[r] = b3_at<M>(tab, to, Y0 + r, mask, inv2p);
#pragma unroll
            for (int zz = 0; zz < BZ; ++zz) {
                const B3 zb = b3_at<M>(tab, to, Z0 + zz, mask, inv2p);
                VW vw[2];
#pragma unroll
                for (int dj = 0; dj < 2; ++dj)
                    vw[dj] = VW{ex[dj][0] + zb.s * (ex[dj][1] - ex[dj][0]) + qz[dj][0] * zb.b10 + qz[dj][1] * zb.b11,
                                qy[dj][0] + zb.s * (qy[dj][1] - qy[dj][0])};
                const Y1 f = cell_y1(vw[0], vw[1]);
                e0[zz] += f.E0;  // the same at every row of the slice
#pragma unroll
                for (int r = 0; r < BY; ++r) {
                    float v = __builtin_fmaf(f.dE, yb[r].s, acc[zz][r]);
                    v = __builtin_fmaf(f.W0, yb[r].b10, v);
                    acc[zz][r] = __builtin_fmaf(f.W1, yb[r].b11, v);
                }
            }
        }
#pragma unroll
        for (int zz = 0; zz < BZ; ++zz)
#pragma unroll
            for (int r = 0; r < BY; ++r) acc[zz][r] += e0[zz];

        // ---- periods 4, 2, 1 and the stores, slice by slice.  Period 4 has one cell in z
        // over the block: its nodes are collapsed along x once.  Slices go in pairs that share
        // one period-2 cell in z (a rolled loop over the pairs keeps the fine cells' node loads
        // from being hoisted for every slice at once) ------------------------------------------
        XC x4[BY / 4 + 1][2];
        if (H4) {
            const int n0 = f4.noff + (lane >> 2) * f4.nny * f4.nnz;
#pragma unroll
            for (int j = 0; j <= BY / 4; ++j)
#pragma unroll
                for (int dk = 0; dk < 2; ++dk) x4[j][dk] = col_x(gx, gy, gz, n0 + j * f4.nnz + dk, f4.nny * f4.nnz, f4.xb);
        }
#pragma unroll 1
        for (int pz = 0; pz < BZ / 2; ++pz) {
            XC x2[BY / 2 + 1][2];
            if (H2) {  // period 2: node rows 0..4, z nodes pz and pz + 1
                const int n0 = f2.noff + (lane >> 1) * f2.nny * f2.nnz + pz;
#pragma unroll
                for (int j = 0; j <= BY / 2; ++j)
#pragma unroll
                    for (int dk = 0; dk < 2; ++dk)
                        x2[j][dk] = col_x(gx, gy, gz, n0 + j * f2.nnz + dk, f2.nny * f2.nnz, f2.xb);
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int zz = 2 * pz + h;
                const int64_t Z = Z0 + zz;
                float t[BY];
                B3 zb4;
                switch (zz) {  // uniform: the slice's coarse sum (no indexed registers) and period-4 z-bases
                case 0:
#pragma unroll
                    for (int r = 0; r < BY; ++r) t[r] = acc[0][r];
                    zb4 = b3_const<M>(0, 4);
                    break;
                case 1:
#pragma unroll
                    for (int r = 0; r < BY; ++r) t[r] = acc[1][r];
                    zb4 = b3_const<M>(1, 4);
                    break;
                case 2:
#pragma unroll
                    for (int r = 0; r < BY; ++r) t[r] = acc[2][r];
                    zb4 = b3_const<M>(2, 4);
                    break;
                default:
#pragma unroll
                    for (int r = 0; r < BY; ++r) t[r] = acc[BZ - 1][r];
                    zb4 = b3_const<M>(3, 4);
                    break;
                }
                if (H4) {  // period 4: two cells in y (node rows 0..2)
                    VW vw[BY / 4 + 1];
#pragma unroll
                    for (int j = 0; j <= BY / 4; ++j) vw[j] = z_vw(x4[j][0], x4[j][1], zb4);
#pragma unroll
                    for (int c = 0; c < BY / 4; ++c) {
                        const Y1 f = cell_y1(vw[c], vw[c + 1]);
#pragma unroll
                        for (int r = 0; r < 4; ++r) t[4 * c + r] += y1_at(f, b3_const<M>(r, 4));
                    }
                }
                if (H2) {
                    const B3 zb = b3_const<M>(h, 2);
                    VW vw[BY / 2 + 1];
#pragma unroll
                    for (int j = 0; j <= BY / 2; ++j) vw[j] = z_vw(x2[j][0], x2[j][1], zb);
#pragma unroll
                    for (int c = 0; c < BY / 2; ++c) {
                        const Y1 f = cell_y1(vw[c], vw[c + 1]);
#pragma unroll
                        for (int r = 0; r < 2; ++r) t[2 * c + r] += y1_at(f, b3_const<M>(r, 2));
                    }
                }
                if (H1) {  // period 1: node rows 0..8
                    const B3 zb = b3_const<M>(0, 1);
                    const int n0 = f1.noff + lane * f1.nny * f1.nnz + zz;
                    VW prev = row_vw(gx, gy, gz, n0, f1.nny * f1.nnz, f1.xb, zb);
#pragma unroll
                    for (int c = 0; c < BY; ++c) {
                        const VW next = row_vw(gx, gy, gz, n0 + (c + 1) * f1.nnz, f1.nny * f1.nnz, f1.xb, zb);
                        t[c] += y1_at(cell_y1(prev, next), b3_const<M>(0, 1));
                        prev = next;
                    }
                }
                if (Z >= a.z0 && Z < ze && lane_ok) {
                    OutT *slice = out + ((Z - a.z0) * a.ny + (Y0 - a.y0)) * a.nx + (X - a.x0);
#pragma unroll
                    for (int r = 0; r < BY; ++r) {
                        const int64_t Y = Y0 + r;
                        if (Y >= a.y0 && Y < ye) slice[(int64_t)r * a.nx] = s3_out<OutT>(t[r]);
                    }
                }
            }
        }
        __builtin_amdgcn_wave_barrier();  // the next block rewrites this wave's keys and nodes
    }
};

}  // namespace ptg
