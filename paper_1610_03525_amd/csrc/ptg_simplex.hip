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
// 64 x 64 sample tiles, 256 threads (lane = column, a wave per 16 rows).  Per octave the
// tile's skewed footprint is hashed into LDS when it fits (every ladder whose finest cell
// spans two or more samples), else each corner is hashed where it is used.  The skew runs
// in FP64 per sample (u reaches 2^33 cells at the largest offsets).
#include "ptg.h"
#include "ptg_device.h"
#include "ptg_launch.h"

#include <hip/hip_fp16.h>

namespace ptg {

namespace {

constexpr double kF2 = 0.36602540378443864676;  // (sqrt 3 - 1) / 2
constexpr double kG2 = 0.21132486540518711775;  // (3 - sqrt 3) / 6
constexpr float kG2f = 0.21132486540518711775f;

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
    constexpr int T = kTile2, RPW = kTile2 / 4;
    float2 *nodes = reinterpret_cast<float2 *>(lds4);
    uint32_t *kx = reinterpret_cast<uint32_t *>(nodes + kSimplexCap);
    uint32_t *ky = kx + kSimplexKeys;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t bid = blockIdx.x;
    const int64_t tx0 = (bid % a.tiles_x) * T, ty0 = (bid / a.tiles_x) * T;
    const int w = (int)min<int64_t>(T, a.nx - tx0), h = (int)min<int64_t>(T, a.ny - ty0);
    const int col = min(lane, w - 1);
    const int64_t X = a.x0 + tx0 + col, Xf = a.x0 + tx0, Xl = Xf + w - 1;
    const int64_t Yf = a.y0 + ty0, Yl = Yf + h - 1;
    float acc[RPW];
#pragma unroll
    for (int r = 0; r < RPW; ++r) acc[r] = 0.0f;

    for (int o = 0; o < a.octaves; ++o) {
        const double f = a.freq[o];
        const float amp = a.amp[o] * 70.0f;
        const uint32_t pre = key_prefix(a.seed, o);
        // the tile's skewed footprint (the skewed indices grow with ux and uy)
        const double ux0 = ((double)Xf + 0.5) * f, ux1 = ((double)Xl + 0.5) * f;
        const double uy0 = ((double)Yf + 0.5) * f, uy1 = ((double)Yl + 0.5) * f;
        const int64_t i0 = (int64_t)__builtin_floor(ux0 + (ux0 + uy0) * kF2);
        const int64_t j0 = (int64_t)__builtin_floor(uy0 + (ux0 + uy0) * kF2);
        const int64_t i1 = (int64_t)__builtin_floor(ux1 + (ux1 + uy1) * kF2) + 1;
        const int64_t j1 = (int64_t)__builtin_floor(uy1 + (ux1 + uy1) * kF2) + 1;
        const int ni = (int)(i1 - i0 + 1), nj = (int)(j1 - j0 + 1);
        const bool staged = ni <= kSimplexKeys && nj <= kSimplexKeys && ni * nj <= kSimplexCap;
        __syncthreads();  // the previous octave is done with LDS
        if (staged) {
            for (int i = tid; i < ni; i += 256) kx[i] = key_xline(i0 + i);
            for (int j = tid; j < nj; j += 256) ky[j] = absorb_index(pre, j0 + j);
            __syncthreads();
            for (int q = tid; q < ni * nj; q += 256) {
                const int j = q / ni, i = q - j * ni;
                const float2 g = grad2(key_combine(ky[j], kx[i]));
                nodes[q] = make_float2(g.x * amp, g.y * amp);
            }
            __syncthreads();
        }
        const double ux = ((double)X + 0.5) * f;
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
            const int row = min(wave * RPW + r, h - 1);
            const double uy = ((double)(Yf + row) + 0.5) * f;
            const double s = (ux + uy) * kF2;
            const double fi = __builtin_floor(ux + s), fj = __builtin_floor(uy + s);
            const double t = (fi + fj) * kG2;
            const float x0 = (float)(ux - (fi - t)), y0 = (float)(uy - (fj - t));
            const int i1c = x0 > y0 ? 1 : 0, j1c = 1 - i1c;
            const float dx1 = x0 - (float)i1c + kG2f, dy1 = y0 - (float)j1c + kG2f;
            const float dx2 = x0 - 1.0f + 2.0f * kG2f, dy2 = y0 - 1.0f + 2.0f * kG2f;
            const int64_t ci = (int64_t)fi, cj = (int64_t)fj;
            float2 g0, g1, g2;
            if (staged) {
                const int q = (int)(cj - j0) * ni + (int)(ci - i0);
                g0 = nodes[q];
                g1 = nodes[q + i1c + j1c * ni];
                g2 = nodes[q + 1 + ni];
            } else {
                const uint32_t kxa = key_xline(ci), kxb = key_xline(ci + 1);
                const uint32_t kya = absorb_index(pre, cj), kyb = absorb_index(pre, cj + 1);
                const float2 h0 = grad2(key_combine(kya, kxa));
                const float2 h1 = grad2(key_combine(i1c ? kya : kyb, i1c ? kxb : kxa));
                const float2 h2 = grad2(key_combine(kyb, kxb));
                g0 = make_float2(h0.x * amp, h0.y * amp);
                g1 = make_float2(h1.x * amp, h1.y * amp);
                g2 = make_float2(h2.x * amp, h2.y * amp);
            }
            acc[r] += corner_term(g0, x0, y0) + corner_term(g1, dx1, dy1) + corner_term(g2, dx2, dy2);
        }
    }
    if (lane < w) {
        OutT *out = reinterpret_cast<OutT *>(a.out);
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
            const int row = wave * RPW + r;
            if (row < h) out[(ty0 + row) * a.pitch + tx0 + lane] = sx_out<OutT>(acc[r]);
        }
    }
}

}  // namespace

hipError_t launch_simplex2d(const Fbm2dArgs &a, bool f16, hipStream_t s)
{
    const int64_t tiles = (int64_t)a.tiles_x * ((a.ny + kTile2 - 1) / kTile2);
    const size_t lds = (size_t)kSimplexCap * 8 + (size_t)2 * kSimplexKeys * 4;
    dim3 grid((unsigned)tiles);
    return f16 ? launch_k(k_simplex2d<__half>, grid, dim3(256), lds, s, a)
               : launch_k(k_simplex2d<float>, grid, dim3(256), lds, s, a);
}

}  // namespace ptg
