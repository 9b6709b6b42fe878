// ptg_fbm_dyadic.hip -- K3 for dyadic octave ladders (base frequency 2^-k, lacunarity 2),
// with the per-cell evaluation on the FP32 matrix cores.
//
// With f_o = 2^-s (s = k - o) the sample-centre coordinate step is exact integer
// arithmetic: cell = X >> s and t = (2 (X mod 2^s) + 1) / 2^(s+1).  Tiles are aligned to
// the world grid (kDyTileX x kDyTileY samples), so a cell of period P >= 16 never straddles
// a 16 x 16 sub-tile and a cell of period 4 or 8 never straddles a 4 x 4 block.
//
// Cell polynomial (Sec. 2; 2D tensor Hermite form, value 0 and gradient g at the corners):
//   h(x, y) = sum_k A_k(y) B_k(x),   B = (b0_0, b0_1, b1_0, b1_1)(x)       (column bases)
//   A = (G_0, G_1, F_0, F_1)(y),     G_cx(y) = gy(cx,0) b1_0(y) + gy(cx,1) b1_1(y)
//                                    F_cx(y) = gx(cx,0) b0_0(y) + gx(cx,1) b0_1(y)
// i.e. the contraction V(y) C V(x)^T written in the Hermite basis, K = 4 per octave.
//  * P >= 16: one v_mfma_f32_16x16x4f32 per octave and 16 x 16 sub-tile;
//  * P = 4, 8: four v_mfma_f32_4x4x1f32 (16 blocks of 4 x 4, each inside one cell); their
//    accumulator layout equals the 16x16x4 one, so every octave adds into the same registers;
//  * P = 1, 2: FP32 VALU in the same register layout.
// Octaves accumulate in FP32 in those registers; every sample is stored once.
//
// A workgroup (4 waves side by side, each 64 columns x 32 rows) walks tiles with a grid
// stride.  Once per workgroup it tabulates, in LDS, the 1D bases at every fraction an
// octave of period P <= kDyTabMaxP can take (the coordinate step), and a list of the
// hashing work of one tile.  Per tile it hashes the footprint nodes of every octave into
// LDS (K1 logic: column / row key prefixes, then one fmix32 per node, amplitude folded
// in); each lane then forms the row-side coefficients A of its cells from those
// gradients (K2 logic) and feeds the matrix cores.
#include <hip/hip_fp16.h>

#include "ptg_device.h"
#include "ptg_launch.h"

namespace ptg {

typedef float f32x4 __attribute__((ext_vector_type(4)));

template <typename T>
__device__ __forceinline__ T dy_out(float v);
template <>
__device__ __forceinline__ float dy_out<float>(float v)
{
    return v;
}
template <>
__device__ __forceinline__ __half dy_out<__half>(float v)
{
    return __float2half_rn(v);
}

// Monomial coefficients of the four 1D bases (rows: b0_0, b0_1, b1_0, b1_1), as arrays a
// lane can index with its own basis number (used for periods above the table size).
__constant__ float kBasisCubic[4][4] = {
    {1.f, 0.f, -3.f, 2.f}, {0.f, 0.f, 3.f, -2.f}, {0.f, 1.f, -2.f, 1.f}, {0.f, 0.f, -1.f, 1.f}};
__constant__ float kBasisQuintic[4][6] = {{1.f, 0.f, 0.f, -10.f, 15.f, -6.f},
                                          {0.f, 0.f, 0.f, 10.f, -15.f, 6.f},
                                          {0.f, 1.f, 0.f, -6.f, 8.f, -3.f},
                                          {0.f, 0.f, 0.f, -4.f, 7.f, -3.f}};

template <int M>
__device__ __forceinline__ float basis_horner(int k, float t)
{
    constexpr int N1 = 2 * M + 2;
    const float *c = (M == 1) ? &kBasisCubic[0][0] + 4 * k : &kBasisQuintic[0][0] + 6 * k;
    float v = c[N1 - 1];
#pragma unroll
    for (int e = N1 - 2; e >= 0; --e) v = v * t + c[e];
    return v;
}

// Sample fraction at world index W for period 2^s: (2 (W mod 2^s) + 1) * 2^-(s+1), exact.
__device__ __forceinline__ float dy_frac(int64_t W, uint32_t mask, float inv2p)
{
    return (float)(2u * ((uint32_t)W & mask) + 1u) * inv2p;
}

// Node blocks in LDS are column-major: node (i, j) of an octave's footprint sits at
// i * nny + j, so the two corners a row-side coefficient needs, (cx, cy) and (cx, cy+1),
// are adjacent.  nny is fixed by the tile height: (kDyTileY >> s) + 1, at least 2.
__host__ __device__ constexpr int dy_nny(int s) { return ((kDyTileY >> s) > 1 ? (kDyTileY >> s) : 1) + 1; }

// Per-workgroup shared state.
struct DyShared {
    float4 *tab;        // [tab_total] (b0_0, b0_1, b1_0, b1_1) at t = (2r+1)/(2P), per octave
    uint32_t *wl_pre;   // prefix work items: octave << 24 | axis << 23 | index
    uint32_t *wl_node;  // node work items: octave << 28 | ky offset << 14 | kx offset
    float2 *nodes;      // [nodes_total] amplitude-scaled (gx, gy), column-major per octave
    uint32_t *kx, *ky;  // key prefixes (per tile)
    float2 *wblk;       // this wave's block of the periods 2 and 1 ([wave_nodes])
};

// ---------------------------------------------------------------------------------
// Octaves of period >= 16: v_mfma_f32_16x16x4f32.  C = 0: period >= 64 (one cell across a
// wave's 64 columns), C = 1: period 32, C = 2: period 16.  Lane (m = lane%16, k = lane/16)
// supplies A[m][k] (row m, row-side coefficient k) and B[k][m] (basis k at column m).
// ---------------------------------------------------------------------------------
template <int M, int C>
__device__ __forceinline__ void mfma16_octave(f32x4 (&acc)[2][4], const Fbm2dDyadicArgs &a, const DyShared &sh,
                                              int o, int64_t Xw, int64_t Yt0, int lane, int xw)
{
    const int k = lane >> 4, m = lane & 15;
    const int s = a.shift[o];
    const uint32_t mask = (1u << s) - 1u;
    const int nny = a.nny[o];
    float B[4];          // basis k of the lane's column in sub-tiles c = 0..3 (16 apart)
    float ra[2], rb[2];  // the two row bases coefficient k needs at row m of groups g = 0, 1
    if (a.toff[o] >= 0) {
        const float *tb = reinterpret_cast<const float *>(sh.tab + a.toff[o]);
        // inside one cell a 16-sample move steps the table index by 16 (C = 0 for columns,
        // C <= 1 for rows); the period-32 and period-16 cases repeat an earlier index
        const int rx = (int)((uint32_t)Xw & mask) + m;
        const int ry = (int)((uint32_t)Yt0 & mask) + m;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int cc = (C == 0) ? c : (C == 1 ? (c & 1) : 0);
            B[c] = tb[4 * (rx + 16 * cc) + k];
        }
#pragma unroll
        for (int g = 0; g < 2; ++g) {
            const int gg = (C == 2) ? 0 : g;
            const float2 r2 = *reinterpret_cast<const float2 *>(tb + 4 * (ry + 16 * gg) + ((k < 2) ? 2 : 0));
            ra[g] = r2.x;
            rb[g] = r2.y;
        }
    } else {
        // period above the table (C = 0 only): Horner on the fly
        const float inv2p = a.inv2p[o];
        const float step = 32.0f * inv2p;
        const float tx0 = dy_frac(Xw + m, mask, inv2p);
        const float ty0 = dy_frac(Yt0 + m, mask, inv2p);
#pragma unroll
        for (int c = 0; c < 4; ++c) B[c] = basis_horner<M>(k, tx0 + (float)c * step);
#pragma unroll
        for (int g = 0; g < 2; ++g) {
            const float ty = ty0 + (float)g * step;
            ra[g] = basis_horner<M>(k < 2 ? 2 : 0, ty);
            rb[g] = basis_horner<M>(k < 2 ? 3 : 1, ty);
        }
    }
    // corners: G_k uses gy of node column cx + k, F_(k-2) uses gx of node column cx + k - 2
    const float *nf = reinterpret_cast<const float *>(sh.nodes + a.noff[o] + (k & 1) * nny) + ((k < 2) ? 1 : 0);
    constexpr int per = (C == 0) ? 4 : (C == 1 ? 2 : 1);  // sub-tiles per cell
#pragma unroll
    for (int g = 0; g < 2; ++g) {
        const int cyl = (C == 2) ? g : 0;  // y cell of the row group inside the tile
#pragma unroll
        for (int cp = 0; cp < 4 / per; ++cp) {
            const int cxl = (xw >> s) + cp;
            const float *pr = nf + 2 * (cxl * nny + cyl);
            const float A = pr[0] * ra[g] + pr[2] * rb[g];
#pragma unroll
            for (int q = 0; q < per; ++q) {
                const int c = cp * per + q;
                acc[g][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(A, B[c], acc[g][c], 0, 0, 0);
            }
        }
    }
}

// ---------------------------------------------------------------------------------
// Octaves of period P = 2^S (S = 2 or 3): v_mfma_f32_4x4x1f32 (16 blocks of 4 x 4).
// Block b = lane/4 covers rows 4*(lane/16).. and columns 4*((lane/4)&3).. of a 16 x 16
// sub-tile; A_b[i] comes from lane 4b+i (row i of the block), B_b[j] from lane 4b+j.
// P <= 8 divides the 16-aligned groups, so the bases depend on the lane only and a
// block's cell moves by 16/P columns per sub-tile and 16/P rows per row group.
// ---------------------------------------------------------------------------------
template <int M, int S>
__device__ __forceinline__ void mfma4_octave(f32x4 (&acc)[2][4], const Fbm2dDyadicArgs &a, const DyShared &sh,
                                             int o, int lane, int xw)
{
    constexpr int P = 1 << S;
    constexpr int NNY = dy_nny(S);
    const int rowA = 4 * (lane >> 4) + (lane & 3);        // row of this lane's A element
    const int colB = 4 * ((lane >> 2) & 3) + (lane & 3);  // column of this lane's B element
    const float4 bx = sh.tab[a.toff[o] + (colB & (P - 1))];
    const float4 yb = sh.tab[a.toff[o] + (rowA & (P - 1))];
    const float2 *base = sh.nodes + a.noff[o] + ((xw + 4 * ((lane >> 2) & 3)) >> S) * NNY + (rowA >> S);
#pragma unroll
    for (int g = 0; g < 2; ++g) {
        float A[4][4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const float2 *q = base + c * (16 / P) * NNY + g * (16 / P);
            const float2 n00 = q[0], n01 = q[1], n10 = q[NNY], n11 = q[NNY + 1];
            A[c][0] = n00.y * yb.z + n01.y * yb.w;
            A[c][1] = n10.y * yb.z + n11.y * yb.w;
            A[c][2] = n00.x * yb.x + n01.x * yb.y;
            A[c][3] = n10.x * yb.x + n11.x * yb.y;
        }
        // basis-major order: four independent accumulators between dependent MFMAs
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[g][c] = __builtin_amdgcn_mfma_f32_4x4x1f32(A[c][0], bx.x, acc[g][c], 0, 0, 0);
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[g][c] = __builtin_amdgcn_mfma_f32_4x4x1f32(A[c][1], bx.y, acc[g][c], 0, 0, 0);
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[g][c] = __builtin_amdgcn_mfma_f32_4x4x1f32(A[c][2], bx.z, acc[g][c], 0, 0, 0);
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[g][c] = __builtin_amdgcn_mfma_f32_4x4x1f32(A[c][3], bx.w, acc[g][c], 0, 0, 0);
    }
}

// ---------------------------------------------------------------------------------
// Octaves of period P = 2^S, S = 1 or 0: VALU, each lane its own 4 rows x 1 column per
// sub-tile.  Their nodes (about one per sample) are not held for the whole tile: per
// 16-row group each wave hashes the (64/P + 1) x (16/P + 1) nodes of its own columns
// into a private block (the same keys and amplitude-scaled gradients as the tile's
// shared block), then evaluates that group.
// ---------------------------------------------------------------------------------
__device__ __forceinline__ void dy_wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int M, int S>
__device__ __forceinline__ void valu_octave(f32x4 (&acc)[2][4], const Fbm2dDyadicArgs &a, const DyShared &sh, int o,
                                            float amp, int lane, int xw)
{
    constexpr int P = 1 << S;
    constexpr int NB = (16 >> S) + 1, NC = (64 >> S) + 1;  // block rows, columns
    const int k = lane >> 4, m = lane & 15;
    float2 *blk = sh.wblk + a.soff[o];
    const uint32_t *kx = sh.kx + a.pxoff[o] + (xw >> S), *ky = sh.ky + a.pyoff[o];
    const float4 bx = sh.tab[a.toff[o] + (m & (P - 1))];
#pragma unroll
    for (int g = 0; g < 2; ++g) {
        const int j0 = (16 * g) >> S;  // first node row of the group (tile-relative)
        dy_wave_sync();                 // the previous group has read the block
#pragma unroll 2
        for (int q = lane; q < NC * NB; q += 64) {
            const int i = q / NB, j = q - i * NB;  // column-major
            const float2 gr = grad2(key_combine(ky[j0 + j], kx[i]));
            blk[q] = make_float2(gr.x * amp, gr.y * amp);
        }
        dy_wave_sync();
#pragma unroll 2  // fully unrolled, the group's 64 node loads were all hoisted (228 VGPRs)
        for (int v = 0; v < 4; ++v) {
            const float4 yb = sh.tab[a.toff[o] + ((4 * k + v) & (P - 1))];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int cxl = (16 * c + m) >> S;  // column in the wave's block
                const float2 *q = blk + cxl * NB + (((16 * g + 4 * k + v) >> S) - j0);
                const float2 n00 = q[0], n01 = q[1], n10 = q[NB], n11 = q[NB + 1];
                const float G0 = n00.y * yb.z + n01.y * yb.w;
                const float G1 = n10.y * yb.z + n11.y * yb.w;
                const float F0 = n00.x * yb.x + n01.x * yb.y;
                const float F1 = n10.x * yb.x + n11.x * yb.y;
                acc[g][c][v] += G0 * bx.x + G1 * bx.y + F0 * bx.z + F1 * bx.w;
            }
        }
    }
}

template <int M, typename OutT>
__global__ __launch_bounds__(256) void k_fbm2d_dyadic(const Fbm2dDyadicArgs a)
{
    constexpr int TX = kDyTileX;  // 256: 4 waves x 64 columns
    constexpr int TY = kDyTileY;  // 32: 2 row groups of 16
    constexpr int NT = 256;
    extern __shared__ float4 lds4[];
    DyShared sh;
    sh.tab = lds4;
    sh.nodes = reinterpret_cast<float2 *>(lds4 + a.tab_total);
    sh.wl_pre = reinterpret_cast<uint32_t *>(sh.nodes + a.nodes_total);
    sh.wl_node = sh.wl_pre + (a.px_total + a.py_total);
    sh.kx = sh.wl_node + a.nodes_total;
    sh.ky = sh.kx + a.px_total;
    {  // per-wave blocks after the key prefixes, 8-byte aligned
        const int words = (int)(sh.ky + a.py_total - reinterpret_cast<uint32_t *>(lds4));
        sh.wblk = reinterpret_cast<float2 *>(reinterpret_cast<uint32_t *>(lds4) + ((words + 1) & ~1)) +
                  (threadIdx.x >> 6) * a.wave_nodes;
    }
    __shared__ uint32_t pre_key[kMaxOctaves];
    __shared__ int p_shift[kMaxOctaves], p_pxoff[kMaxOctaves], p_pyoff[kMaxOctaves];
    __shared__ float p_amp[kMaxOctaves];

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int N = a.octaves;
    const int xw = 64 * wave;  // first tile column of this wave
    const int k = lane >> 4, m = lane & 15;

    // ---- once per workgroup: basis tables, hashing work lists, key prefixes per octave ---
    // (the per-octave table offsets and steps are first staged in LDS: a lane-dependent
    // index into the kernel arguments would be a chain of dependent global loads)
    __shared__ int p_toff[kMaxOctaves];
    __shared__ float p_inv2p[kMaxOctaves];
    if (tid < N) {
        p_toff[tid] = a.toff[tid];
        p_inv2p[tid] = a.inv2p[tid];
    }
    __syncthreads();
    for (int q = tid; q < a.tab_total; q += NT) {
        int o = a.tab_first;  // every octave from tab_first on has a table, in order
        while (o + 1 < N && q >= p_toff[o + 1]) ++o;
        const int r = q - p_toff[o];
        float S, b10, b11;
        Basis<M>::eval((float)(2 * r + 1) * p_inv2p[o], S, b10, b11);
        sh.tab[q] = make_float4(1.0f - S, S, b10, b11);
    }
    for (int o = 0; o < N; ++o) {
        const int nnx = a.nnx[o], nny = a.nny[o];
        for (int i = tid; i < nnx + nny; i += NT)
            sh.wl_pre[a.pxoff[o] + a.pyoff[o] + i] =
                ((uint32_t)o << 24) | (i < nnx ? (uint32_t)i : ((1u << 23) | (uint32_t)(i - nnx)));
        if (a.shift[o] <= 1) continue;  // periods 2, 1: hashed per wave and row group
        for (int q = tid; q < nnx * nny; q += NT) {
            const int i = q / nny, j = q - i * nny;  // column-major
            sh.wl_node[a.noff[o] + q] =
                ((uint32_t)o << 28) | ((uint32_t)(a.pyoff[o] + j) << 14) | (uint32_t)(a.pxoff[o] + i);
        }
    }
    if (tid < N) {
        pre_key[tid] = key_prefix(a.seed, tid);
        p_shift[tid] = a.shift[tid];
        p_pxoff[tid] = a.pxoff[tid];
        p_pyoff[tid] = a.pyoff[tid];
        p_amp[tid] = a.amp[tid];
    }
    __syncthreads();

    const int npre = a.px_total + a.py_total;
    for (int64_t tile = blockIdx.x; tile < a.tiles; tile += gridDim.x) {
        const int64_t btx = tile % a.tiles_x, bty = tile / a.tiles_x;
        const int64_t Xt0 = a.tx_base + btx * TX, Yt0 = a.ty_base + bty * TY;

        // ---- per tile: key prefixes, then amplitude-scaled node gradients ----------------
        for (int q = tid; q < npre; q += NT) {
            const uint32_t it = sh.wl_pre[q];
            const int o = it >> 24;
            const int s = p_shift[o];
            const int idx = it & 0x7FFFFF;
            if (it & (1u << 23))
                sh.ky[p_pyoff[o] + idx] = absorb_index(pre_key[o], (Yt0 >> s) + idx);
            else
                sh.kx[p_pxoff[o] + idx] = key_xline((Xt0 >> s) + idx);
        }
        __syncthreads();
        for (int q = tid; q < a.nodes_total; q += NT) {
            const uint32_t it = sh.wl_node[q];
            const float amp = p_amp[it >> 28];
            const float2 g = grad2(key_combine(sh.ky[(it >> 14) & 0x3FFF], sh.kx[it & 0x3FFF]));
            sh.nodes[q] = make_float2(g.x * amp, g.y * amp);
        }
        __syncthreads();

        f32x4 acc[2][4];
#pragma unroll
        for (int g = 0; g < 2; ++g)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[g][c] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

        const int64_t Xw = Xt0 + xw;
        int o = 0;
        for (; o < N && a.shift[o] >= 6; ++o) mfma16_octave<M, 0>(acc, a, sh, o, Xw, Yt0, lane, xw);
        if (o < N && a.shift[o] == 5) mfma16_octave<M, 1>(acc, a, sh, o++, Xw, Yt0, lane, xw);
        if (o < N && a.shift[o] == 4) mfma16_octave<M, 2>(acc, a, sh, o++, Xw, Yt0, lane, xw);
        if (o < N && a.shift[o] == 3) mfma4_octave<M, 3>(acc, a, sh, o++, lane, xw);
        if (o < N && a.shift[o] == 2) mfma4_octave<M, 2>(acc, a, sh, o++, lane, xw);
        if (o < N && a.shift[o] == 1) valu_octave<M, 1>(acc, a, sh, o, p_amp[o], lane, xw), ++o;
        if (o < N && a.shift[o] == 0) valu_octave<M, 0>(acc, a, sh, o, p_amp[o], lane, xw), ++o;

        // ---- store: lane holds rows 4*(lane/16)+v of column lane%16 of each sub-tile -------
        OutT *out = reinterpret_cast<OutT *>(a.out);
        const int64_t xe = a.x0 + a.nx, ye = a.y0 + a.ny;
        const bool inside = Xt0 >= a.x0 && Xt0 + TX <= xe && Yt0 >= a.y0 && Yt0 + TY <= ye;
        if (inside) {
            OutT *col = out + (Yt0 - a.y0 + 4 * k) * a.pitch + (Xt0 - a.x0 + xw + m);
#pragma unroll
            for (int g = 0; g < 2; ++g)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    OutT *r = col + (16 * g + v) * a.pitch;
#pragma unroll
                    for (int c = 0; c < 4; ++c) r[16 * c] = dy_out<OutT>(acc[g][c][v]);
                }
        } else {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int64_t X = Xt0 + xw + 16 * c + m;
                if (X < a.x0 || X >= xe) continue;
#pragma unroll
                for (int g = 0; g < 2; ++g)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int64_t Y = Yt0 + 16 * g + 4 * k + v;
                        if (Y >= a.y0 && Y < ye)
                            out[(Y - a.y0) * a.pitch + (X - a.x0)] = dy_out<OutT>(acc[g][c][v]);
                    }
            }
        }
        __syncthreads();  // the next tile overwrites the prefixes and nodes
    }
}

template <int M, typename OutT>
static hipError_t launch_dy(const Fbm2dDyadicArgs &a, size_t lds, hipStream_t s)
{
    auto kern = k_fbm2d_dyadic<M, OutT>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    return launch_k(kern, dim3((unsigned)a.grid), dim3(256), lds, s, a);
}

hipError_t launch_fbm2d_dyadic(const Fbm2dDyadicArgs &a, int smooth, bool f16, size_t lds, hipStream_t s)
{
    if (smooth == 1) return f16 ? launch_dy<1, __half>(a, lds, s) : launch_dy<1, float>(a, lds, s);
    return f16 ? launch_dy<2, __half>(a, lds, s) : launch_dy<2, float>(a, lds, s);
}

}  // namespace ptg
