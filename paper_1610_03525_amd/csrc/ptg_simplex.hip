// ptg_simplex.hip -- comparison path: simplex-lattice gradient noise fBm (the stand-in for
// the OpenSimplex timings of the paper's Sec. 5.2, which the paper does not define).
//
// From the public mathematical description of 2D simplex noise: the lattice coordinate u =
// (X + 1/2) f is skewed by F2 = (sqrt 3 - 1) / 2 onto the square lattice, (i, j) =
// floor(u + (ux + uy) F2); the unskewed offsets (G2 = (3 - sqrt 3) / 6) pick the cell's
// lower or upper triangle; each of its three corners c adds max(0, 1/2 - |d|^2)^4 (g_c . d)
// with d the offset from the corner and g_c the unit gradient the lattice hash gives the
// skewed index (the same hash as the polynomial cells); the octave's sum is scaled by 70.
//
// World-aligned 64 x 64 sample tiles (so a crop of a field is computed by the same tiles as
// the field), 256 threads: lane = column, a wave per 16 rows.  Per octave each lane forms
// in FP64, at its wave's first row, its skewed coordinate split into the integer cell and
// a fraction, and the unskewed offsets from that cell's corner (u reaches 2^33 cells at the
// largest offsets); the wave's 16 rows then add the row offset in FP32 (at most 15 samples,
// so the rounding stays ~1e-6 of a cell: a sample that falls within that distance of a
// cell edge or the triangle diagonal may take the neighbouring simplex, whose value agrees
// there, the noise being continuous).  The tile's skewed footprint is
// hashed into LDS when it fits (every ladder whose finest cell spans two or more samples),
// else each corner is hashed where it is used.
#include "ptg.h"
#include "ptg_device.h"
#include "ptg_launch.h"

#include <hip/hip_fp16.h>

#include <algorithm>
#include <cmath>

namespace ptg {

namespace {

constexpr double kF2 = 0.36602540378443864676;  // (sqrt 3 - 1) / 2
constexpr double kG2 = 0.21132486540518711775;  // (3 - sqrt 3) / 6
constexpr float kF2f = 0.36602540378443864676f;
constexpr float kG2f = 0.21132486540518711775f;
constexpr int kSxTile = 64;

template <typename T>
__device__ __forceinline__ T sx_out(float v);
template <>
__device__ __forceinline__ float sx_out<float>(float v)
{
    return v;
}
template <>
__device__ __forceinline__ __half sx_out<__half>(float v)
{
    return __float2half_rn(v);
}

__host__ __device__ __forceinline__ int64_t sx_floor_div(int64_t a, int64_t b)
{
    const int64_t q = a / b;
    return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}

__device__ __forceinline__ float corner_term(float2 g, float dx, float dy)
{
    const float t = fmaxf(0.5f - dx * dx - dy * dy, 0.0f);
    const float t2 = t * t;
    return t2 * t2 * (g.x * dx + g.y * dy);
}

template <typename OutT>
__global__ __launch_bounds__(256) void k_simplex2d(const Fbm2dArgs a)
{
    extern __shared__ float4 lds4[];
    constexpr int T = kSxTile, RPW = kSxTile / 4;
    // LDS: [row and column keys | node gradients (capx nodes, sized by the launch)]
    uint32_t *kx = reinterpret_cast<uint32_t *>(lds4);
    uint32_t *ky = kx + kSimplexKeys;
    float2 *nodes = reinterpret_cast<float2 *>(ky + kSimplexKeys);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t bid = blockIdx.x;
    // world-aligned tile: origin (Xt, Yt), samples Xt + lane, Yt + row
    const int64_t Xt = (sx_floor_div(a.x0, T) + bid % a.tiles_x) * T;
    const int64_t Yt = (sx_floor_div(a.y0, T) + bid / a.tiles_x) * T;
    float acc[RPW];
#pragma unroll
    for (int r = 0; r < RPW; ++r) acc[r] = 0.0f;

    for (int o = 0; o < a.octaves; ++o) {
        const double f = a.freq[o];
        const float amp = a.amp[o] * 70.0f;
        const uint32_t pre = key_prefix(a.seed, o);
        // the tile's base cell (I0, J0): the skewed cell of its first sample (FP64, uniform);
        // skewed coordinates grow with both sample offsets, so every cell of the tile is at
        // (I0, J0) + [0, span - 3] (one cell of margin each way)
        const double tu = ((double)Xt + 0.5) * f, tv = ((double)Yt + 0.5) * f, ts = (tu + tv) * kF2;
        const double tbi = __builtin_floor(tu + ts), tbj = __builtin_floor(tv + ts);
        const int64_t I0 = (int64_t)tbi, J0 = (int64_t)tbj;
        const float ff = (float)f;
        const int span = (int)__builtin_floorf(1.0f + 63.0f * ff * (1.0f + 2.0f * kF2f)) + 3;
        const bool staged = span <= kSimplexKeys && span * span <= a.capx;
        __syncthreads();  // the previous octave is done with LDS
        if (staged) {
            for (int i = tid; i < span; i += 256) {
                kx[i] = key_xline(I0 - 1 + i);
                ky[i] = absorb_index(pre, J0 - 1 + i);
            }
            __syncthreads();
            for (int q = tid; q < span * span; q += 256) {
                const int j = q / span, i = q - j * span;
                const float2 g = grad2(key_combine(ky[j], kx[i]));
                nodes[q] = make_float2(g.x * amp, g.y * amp);
            }
            __syncthreads();
        }
        // per lane, in FP64 at the wave's first row: the skewed cell (bi, bj), the fraction
        // (rx, ry) and the unskewed offsets (cx, cy) from that cell's corner; the wave's rows
        // then add at most 15 samples in FP32
        const double ux = ((double)(Xt + lane) + 0.5) * f, uy = ((double)(Yt + wave * RPW) + 0.5) * f;
        const double s0 = (ux + uy) * kF2;
        const double bi = __builtin_floor(ux + s0), bj = __builtin_floor(uy + s0);
        const float rx = (float)(ux + s0 - bi), ry = (float)(uy + s0 - bj);  // in [0, 1]
        const double t0 = (bi + bj) * kG2;
        const float cx = (float)(ux - bi + t0), cy = (float)(uy - bj + t0);
        const int64_t LI = (int64_t)bi, LJ = (int64_t)bj;
        const int di = (int)(LI - I0), dj = (int)(LJ - J0);  // >= 0, within the footprint
        // one row's simplex: its cell (fi, fj) relative to (I0, J0), the corner offsets,
        // and the three corner terms from the gradients a node source gives
        auto row = [&](int r, auto &&grads) {
            const float ly = (float)r * ff;  // uniform
            const float ax = __builtin_fmaf(ly, kF2f, rx), ay = __builtin_fmaf(ly, 1.0f + kF2f, ry);
            const float fi = __builtin_floorf(ax), fj = __builtin_floorf(ay);
            const float tt = (fi + fj) * kG2f;
            const float x0 = cx - fi + tt, y0 = cy + ly - fj + tt;
            const int i1c = x0 > y0 ? 1 : 0;
            const float dx1 = x0 - (float)i1c + kG2f, dy1 = y0 - (float)(1 - i1c) + kG2f;
            const float dx2 = x0 - 1.0f + 2.0f * kG2f, dy2 = y0 - 1.0f + 2.0f * kG2f;
            float2 g0, g1, g2;
            grads(fi, fj, i1c, g0, g1, g2);
            acc[r] += corner_term(g0, x0, y0) + corner_term(g1, dx1, dy1) + corner_term(g2, dx2, dy2);
        };
        if (staged) {
            auto from_lds = [&](float fi, float fj, int i1c, float2 &g0, float2 &g1, float2 &g2) {
                // footprint index of (I0 + fi, J0 + fj); clamped so a rounding at the edge of
                // the range can never leave the staged block
                const int ii = min(max(di + (int)fi + 1, 0), span - 2), jj = min(max(dj + (int)fj + 1, 0), span - 2);
                const int q = jj * span + ii;
                g0 = nodes[q];
                g1 = nodes[q + i1c + (1 - i1c) * span];
                g2 = nodes[q + 1 + span];
            };
#pragma unroll
            for (int r = 0; r < RPW; ++r) row(r, from_lds);
        } else {
            auto hashed = [&](float fi, float fj, int i1c, float2 &g0, float2 &g1, float2 &g2) {
                const int64_t ci = LI + (int64_t)fi, cj = LJ + (int64_t)fj;
                const uint32_t kxa = key_xline(ci), kxb = key_xline(ci + 1);
                const uint32_t kya = absorb_index(pre, cj), kyb = absorb_index(pre, cj + 1);
                const float2 h0 = grad2(key_combine(kya, kxa));
                const float2 h1 = grad2(key_combine(i1c ? kya : kyb, i1c ? kxb : kxa));
                const float2 h2 = grad2(key_combine(kyb, kxb));
                g0 = make_float2(h0.x * amp, h0.y * amp);
                g1 = make_float2(h1.x * amp, h1.y * amp);
                g2 = make_float2(h2.x * amp, h2.y * amp);
            };
#pragma unroll
            for (int r = 0; r < RPW; ++r) row(r, hashed);
        }
    }
    const int64_t X = Xt + lane;
    if (X >= a.x0 && X < a.x0 + a.nx) {
        OutT *out = reinterpret_cast<OutT *>(a.out);
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
            const int64_t Y = Yt + wave * RPW + r;
            if (Y >= a.y0 && Y < a.y0 + a.ny) out[(Y - a.y0) * a.pitch + (X - a.x0)] = sx_out<OutT>(acc[r]);
        }
    }
}

}  // namespace

hipError_t launch_simplex2d(const Fbm2dArgs &args, bool f16, hipStream_t s)
{
    Fbm2dArgs a = args;
    const int64_t tx = sx_floor_div(a.x0 + a.nx - 1, kSxTile) - sx_floor_div(a.x0, kSxTile) + 1;
    const int64_t ty = sx_floor_div(a.y0 + a.ny - 1, kSxTile) - sx_floor_div(a.y0, kSxTile) + 1;
    a.tiles_x = (int32_t)tx;
    // node capacity: the largest footprint an octave stages (one row and column of margin
    // over the kernel's own estimate, which may round differently); octaves beyond
    // kSimplexCap hash their corners where they are used
    int cap = 1;
    for (int o = 0; o < a.octaves; ++o) {
        const float ff = (float)a.freq[o];
        const int span = (int)std::floor(1.0f + 63.0f * ff * (1.0f + 2.0f * kF2f)) + 4;
        if (span <= kSimplexKeys && span * span <= kSimplexCap) cap = std::max(cap, span * span);
    }
    a.capx = cap;
    const size_t lds = (size_t)2 * kSimplexKeys * 4 + (size_t)cap * 8;
    dim3 grid((unsigned)(tx * ty));
    return f16 ? launch_k(k_simplex2d<__half>, grid, dim3(256), lds, s, a)
               : launch_k(k_simplex2d<float>, grid, dim3(256), lds, s, a);
}

}  // namespace ptg
