// ptg_stages.hip -- stand-alone stage kernels: a1 coordinate step, K1 lattice hash,
// K2 per-cell coefficients.  The dense-field kernels run the same device functions fused
// inside their workgroups; these launches expose each stage on its own (and K2 feeds the
// matrix-core form its per-cell coefficient matrices).
#include "ptg_device.h"
#include "ptg_launch.h"

namespace ptg {

// ---------------------------------------------------------------------------------
// a1: coordinate step for n samples x0.. and all octaves.
// ---------------------------------------------------------------------------------
struct CoordArgs {
    double freq[kMaxOctaves];
    int64_t x0, n;
    int64_t *cells;
    float *frac;
    int32_t octaves;
};

__global__ __launch_bounds__(256) void k_coords(const CoordArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int o = blockIdx.y;
    if (i >= a.n || o >= a.octaves) return;
    const Coord c = coord_step(a.x0 + i, a.freq[o]);
    a.cells[(int64_t)o * a.n + i] = c.cell;
    a.frac[(int64_t)o * a.n + i] = c.t;
}

hipError_t launch_coords(double f0, double lac, int octaves, int64_t x0, int64_t n, int64_t *cells, float *frac,
                         hipStream_t s)
{
    CoordArgs a{};
    double f = f0;
    for (int o = 0; o < octaves; ++o) {
        a.freq[o] = f;
        f = f * lac;
    }
    a.x0 = x0;
    a.n = n;
    a.cells = cells;
    a.frac = frac;
    a.octaves = octaves;
    dim3 grid((unsigned)((n + 255) / 256), (unsigned)octaves);
    hipLaunchKernelGGL(k_coords, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// K1: lattice hash -> unit gradient over a node box.  A workgroup covers 256 consecutive
// node columns of kLatRows consecutive node rows: each thread forms its column's x-line key
// once and walks the rows; a row's key prefix is the same for the whole workgroup (scalar
// unit), so a node costs one fmix32 and its gradient, and every store is one contiguous
// row segment per wave.
// ---------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_lattice2d(uint32_t seed, int octave, int64_t ix0, int64_t iy0, int64_t nx,
                                                   int64_t ny, uint32_t wgx, uint32_t *__restrict__ keys,
                                                   float *__restrict__ grad)
{
    const uint32_t by = blockIdx.x / wgx, bx = blockIdx.x - by * wgx;
    const int64_t i = (int64_t)bx * 256 + threadIdx.x;
    if (i >= nx) return;
    const int64_t n = nx * ny, j0 = (int64_t)by * kLatRows;
    const int rows = (int)min<int64_t>(kLatRows, ny - j0);
    const uint32_t pre = key_prefix(seed, octave), kx = key_xline(ix0 + i);
    for (int r = 0; r < rows; ++r) {
        const int64_t q = (j0 + r) * nx + i;
        const uint32_t key = key_combine(absorb_index(pre, iy0 + j0 + r), kx);
        if (keys) keys[q] = key;
        if (grad) {
            const float2 g = grad2(key);
            grad[q] = g.x;
            grad[n + q] = g.y;
        }
    }
}

// Zero-gradient model (Sec. 3.3): the node heights of a 2D node box (same layout).
__global__ __launch_bounds__(256) void k_heights2d(uint32_t seed, int octave, int64_t ix0, int64_t iy0, int64_t nx,
                                                   int64_t ny, uint32_t wgx, float *__restrict__ h)
{
    const uint32_t by = blockIdx.x / wgx, bx = blockIdx.x - by * wgx;
    const int64_t i = (int64_t)bx * 256 + threadIdx.x;
    if (i >= nx) return;
    const int64_t j0 = (int64_t)by * kLatRows;
    const int rows = (int)min<int64_t>(kLatRows, ny - j0);
    const uint32_t pre = key_prefix(seed, octave), kx = key_xline(ix0 + i);
    for (int r = 0; r < rows; ++r)
        h[(j0 + r) * nx + i] = height2(key_combine(absorb_index(pre, iy0 + j0 + r), kx));
}

// 3D: the node rows are the (j, k) pairs in k-major order, kLatRows of them per workgroup.
__global__ __launch_bounds__(256) void k_lattice3d(uint32_t seed, int octave, int64_t ix0, int64_t iy0, int64_t iz0,
                                                   int64_t nx, int64_t ny, int64_t nz, uint32_t wgx,
                                                   uint32_t *__restrict__ keys, uint32_t *__restrict__ second,
                                                   float *__restrict__ grad)
{
    const uint32_t by = blockIdx.x / wgx, bx = blockIdx.x - by * wgx;
    const int64_t i = (int64_t)bx * 256 + threadIdx.x;
    if (i >= nx) return;
    const int64_t n = nx * ny * nz, r0 = (int64_t)by * kLatRows;
    const int rows = (int)min<int64_t>(kLatRows, ny * nz - r0);
    int64_t k = r0 / ny, j = r0 - k * ny;
    const uint32_t pre = key_prefix(seed, octave), kx = key_xline(ix0 + i);
    uint32_t kz = absorb_index(pre, iz0 + k);
    for (int r = 0; r < rows; ++r) {
        const int64_t q = (r0 + r) * nx + i;  // ((k ny + j) nx + i)
        const uint32_t key = key_combine(absorb_index(kz, iy0 + j), kx);
        if (keys) keys[q] = key;
        if (second) second[q] = key3_second(key);
        if (grad) {
            const float3 g = grad3(key);
            grad[q] = g.x;
            grad[n + q] = g.y;
            grad[2 * n + q] = g.z;
        }
        if (++j == ny) {
            j = 0;
            ++k;
            kz = absorb_index(pre, iz0 + k);
        }
    }
}

hipError_t launch_lattice2d(uint32_t seed, int octave, int64_t ix0, int64_t iy0, int64_t nx, int64_t ny,
                            uint32_t *keys, float *grad, hipStream_t s)
{
    const uint32_t wgx = (uint32_t)((nx + 255) / 256);
    hipLaunchKernelGGL(k_lattice2d, dim3((unsigned)lattice_wgs(nx, ny)), dim3(256), 0, s, seed, octave, ix0, iy0, nx,
                       ny, wgx, keys, grad);
    return hipGetLastError();
}

hipError_t launch_heights2d(uint32_t seed, int octave, int64_t ix0, int64_t iy0, int64_t nx, int64_t ny,
                            float *heights, hipStream_t s)
{
    const uint32_t wgx = (uint32_t)((nx + 255) / 256);
    hipLaunchKernelGGL(k_heights2d, dim3((unsigned)lattice_wgs(nx, ny)), dim3(256), 0, s, seed, octave, ix0, iy0, nx,
                       ny, wgx, heights);
    return hipGetLastError();
}

hipError_t launch_lattice3d(uint32_t seed, int octave, int64_t ix0, int64_t iy0, int64_t iz0, int64_t nx,
                            int64_t ny, int64_t nz, uint32_t *keys, uint32_t *second, float *grad, hipStream_t s)
{
    const uint32_t wgx = (uint32_t)((nx + 255) / 256);
    hipLaunchKernelGGL(k_lattice3d, dim3((unsigned)lattice_wgs(nx, ny * nz)), dim3(256), 0, s, seed, octave, ix0,
                       iy0, iz0, nx, ny, nz, wgx, keys, second, grad);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// K2: per-cell monomial coefficients of h = sum c_ij x^i y^j (2D) / sum c_ijk x^i y^j z^k
// (3D).  A workgroup owns a row block of cells (2D: 64 x 4, 3D: 64 x 2 x 2; one wave per
// cell row) and stages the block's corner gradients in LDS once (each node is shared by
// 2^D cells).  The tensor Hermite form
//   c_ij = sum_corners [ gx b1_cx[i] b0_cy[j] + gy b0_cx[i] b1_cy[j] ]
// is expanded one axis at a time (sum factorisation: contract x, then y, then z), skipping
// the zero monomial coefficients of the bases.  Output: consecutive cells of a row are
// contiguous, so each wave writes its results to a private LDS buffer in output order and
// then stores the buffer as one contiguous span (16-byte vectors when the output allows):
// a cell's coefficients span 64 to 864 bytes, and stores of that stride per lane would
// leave most of each write request empty.
//   2D: lane = cell, 64 cells per pass.
//   3D: lane = (cell, i): each lane forms the slab c_i.. of one cell, 64 / (n+1) cells per
//       pass (16 cubic, 10 quintic), the wave's row in 4 or 7 passes.
// ---------------------------------------------------------------------------------

// acc + v * (basis coefficient k, e), the term dropped when the coefficient is zero
template <int M>
__device__ __forceinline__ float bterm(float acc, float v, int k, int e)
{
    const float b = BasisMono<M>::c(k, e);
    return b == 0.0f ? acc : __builtin_fmaf(v, b, acc);
}

// The wave's lanes write and read its LDS buffer: order the accesses within the wave.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// nf floats from the wave's LDS buffer to dst, consecutive lanes on consecutive 16-byte
// vectors (VEC: dst 16-byte aligned, nf a multiple of 4) or floats.
template <bool VEC>
__device__ __forceinline__ void store_span(float *dst, const float *buf, int nf, int lane)
{
    if (VEC) {
        const float4 *b4 = reinterpret_cast<const float4 *>(buf);
        float4 *d4 = reinterpret_cast<float4 *>(dst);
        for (int f = lane; f < nf / 4; f += 64) d4[f] = b4[f];
    } else {
        for (int f = lane; f < nf; f += 64) dst[f] = buf[f];
    }
}

template <int M, bool VEC>
__global__ __launch_bounds__(256) void k_cells2d(const float *__restrict__ grad, int64_t nnx, int64_t nny,
                                                 uint32_t wgx, float amp, float *__restrict__ coeff)
{
    constexpr int N1 = BasisMono<M>::N1, NC = N1 * N1;
    __shared__ float sgx[kCell2H + 1][kCell2W + 1];
    __shared__ float sgy[kCell2H + 1][kCell2W + 1];
    __shared__ __align__(16) float sbuf[kCell2H][kCell2W * NC];
    const uint32_t by = blockIdx.x / wgx, bx = blockIdx.x - by * wgx;
    const int64_t ncx = nnx - 1, ncy = nny - 1;
    const int64_t cx0 = (int64_t)bx * kCell2W, cy0 = (int64_t)by * kCell2H;
    const int64_t nn = nnx * nny;
    for (int q = threadIdx.x; q < (kCell2H + 1) * (kCell2W + 1); q += 256) {
        const int j = q / (kCell2W + 1), i = q - j * (kCell2W + 1);
        const int64_t gi = min(cx0 + i, nnx - 1), gj = min(cy0 + j, nny - 1);
        sgx[j][i] = grad[gj * nnx + gi];
        sgy[j][i] = grad[nn + gj * nnx + gi];
    }
    __syncthreads();
    const int li = threadIdx.x & 63, lj = threadIdx.x >> 6;
    const int64_t cj = cy0 + lj;
    if (cj >= ncy) return;  // the whole wave
    float gx[2][2], gy[2][2];  // [cy][cx]; lanes past the row's end compute a clamped cell
#pragma unroll
    for (int cy = 0; cy < 2; ++cy)
#pragma unroll
        for (int cx = 0; cx < 2; ++cx) {
            gx[cy][cx] = sgx[lj + cy][li + cx] * amp;
            gy[cy][cx] = sgy[lj + cy][li + cx] * amp;
        }
    float *mine = &sbuf[lj][li * NC];
#pragma unroll
    for (int i = 0; i < N1; ++i) {
        float U[2], V[2];  // x contracted: slope basis against gx, value basis against gy
#pragma unroll
        for (int cy = 0; cy < 2; ++cy) {
            U[cy] = bterm<M>(bterm<M>(0.0f, gx[cy][0], 2, i), gx[cy][1], 3, i);
            V[cy] = bterm<M>(bterm<M>(0.0f, gy[cy][0], 0, i), gy[cy][1], 1, i);
        }
#pragma unroll
        for (int j = 0; j < N1; ++j) {
            float c = 0.0f;
#pragma unroll
            for (int cy = 0; cy < 2; ++cy) c = bterm<M>(bterm<M>(c, U[cy], cy, j), V[cy], 2 + cy, j);
            mine[i * N1 + j] = c;
        }
    }
    wave_sync();
    const int nv = (int)min<int64_t>(kCell2W, ncx - cx0);  // cells of this row in the block
    store_span<VEC>(coeff + (cj * ncx + cx0) * NC, sbuf[lj], nv * NC, li);
}

template <int M, bool VEC>
__global__ __launch_bounds__(256) void k_cells3d(const float *__restrict__ grad, int64_t nnx, int64_t nny, int64_t nnz,
                                                 uint32_t wgx, uint32_t wgy, float amp, float *__restrict__ coeff)
{
    constexpr int N1 = BasisMono<M>::N1, NS = N1 * N1, NC = NS * N1;
    constexpr int CPP = 64 / N1;  // cells per pass
    constexpr int SX = kCell3W + 1;
    __shared__ float sg[3][3][3][SX];  // [axis][k][j][i]
    __shared__ __align__(16) float sbuf[4][CPP * NC];
    const uint32_t bz = blockIdx.x / (wgx * wgy), rem = blockIdx.x - bz * (wgx * wgy);
    const uint32_t by = rem / wgx, bx = rem - by * wgx;
    const int64_t ncx = nnx - 1, ncy = nny - 1, ncz = nnz - 1;
    const int64_t cx0 = (int64_t)bx * kCell3W, cy0 = (int64_t)by * 2, cz0 = (int64_t)bz * 2;
    const int64_t nn = nnx * nny * nnz;
    for (int q = threadIdx.x; q < 9 * SX; q += 256) {
        const int kj = q / SX, i = q - kj * SX, k = kj / 3, j = kj - 3 * k;
        const int64_t gi = min(cx0 + i, nnx - 1), gj = min(cy0 + j, nny - 1), gk = min(cz0 + k, nnz - 1);
        const int64_t g = (gk * nny + gj) * nnx + gi;
        sg[0][k][j][i] = grad[g];
        sg[1][k][j][i] = grad[nn + g];
        sg[2][k][j][i] = grad[2 * nn + g];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, lj = w & 1, lk = w >> 1;
    const int64_t cj = cy0 + lj, ck = cz0 + lk;
    if (cj >= ncy || ck >= ncz) return;  // the whole wave
    const int row_cells = (int)min<int64_t>(kCell3W, ncx - cx0);
    const int sub = lane / N1, i = lane - sub * N1;  // lanes >= CPP * N1 idle
    float *const rowdst = coeff + ((ck * ncy + cj) * ncx + cx0) * NC;
    for (int c0 = 0; c0 < row_cells; c0 += CPP) {
        if (lane < CPP * N1) {
            const int li = min(c0 + sub, kCell3W - 1);  // past the row's end: a clamped cell, not stored
            float g[3][2][2][2];  // [axis][cz][cy][cx]
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int cz = 0; cz < 2; ++cz)
#pragma unroll
                    for (int cy = 0; cy < 2; ++cy)
#pragma unroll
                        for (int cx = 0; cx < 2; ++cx) g[a][cz][cy][cx] = sg[a][lk + cz][lj + cy][li + cx] * amp;
            // contract x at this lane's i: the x gradient against the slope basis, y and z
            // against the value basis (the index i is per lane: select the coefficients)
            float X1[2][2], Y0[2][2], Z0[2][2];  // [cz][cy]
#pragma unroll
            for (int cz = 0; cz < 2; ++cz)
#pragma unroll
                for (int cy = 0; cy < 2; ++cy) {
                    X1[cz][cy] = Y0[cz][cy] = Z0[cz][cy] = 0.0f;
#pragma unroll
                    for (int e = 0; e < N1; ++e) {
                        if (e != i) continue;
                        X1[cz][cy] = bterm<M>(bterm<M>(0.0f, g[0][cz][cy][0], 2, e), g[0][cz][cy][1], 3, e);
                        Y0[cz][cy] = bterm<M>(bterm<M>(0.0f, g[1][cz][cy][0], 0, e), g[1][cz][cy][1], 1, e);
                        Z0[cz][cy] = bterm<M>(bterm<M>(0.0f, g[2][cz][cy][0], 0, e), g[2][cz][cy][1], 1, e);
                    }
                }
            float *mine = &sbuf[w][lane * NS];  // the slab of (cell sub, i): output order
#pragma unroll
            for (int j = 0; j < N1; ++j) {
                float P[2], R[2];  // contract y: P goes with the z value basis, R with the z slope basis
#pragma unroll
                for (int cz = 0; cz < 2; ++cz) {
                    float pv = 0.0f, rv = 0.0f;
#pragma unroll
                    for (int cy = 0; cy < 2; ++cy) {
                        pv = bterm<M>(bterm<M>(pv, X1[cz][cy], cy, j), Y0[cz][cy], 2 + cy, j);
                        rv = bterm<M>(rv, Z0[cz][cy], cy, j);
                    }
                    P[cz] = pv;
                    R[cz] = rv;
                }
#pragma unroll
                for (int k = 0; k < N1; ++k) {
                    float c = 0.0f;
#pragma unroll
                    for (int cz = 0; cz < 2; ++cz) c = bterm<M>(bterm<M>(c, P[cz], cz, k), R[cz], 2 + cz, k);
                    mine[j * N1 + k] = c;
                }
            }
        }
        wave_sync();
        const int nv = min(CPP, row_cells - c0);
        store_span<VEC>(rowdst + (int64_t)c0 * NC, sbuf[w], nv * NC, lane);
        wave_sync();  // the buffer is rewritten by the next pass
    }
}

hipError_t launch_cells2d(int smooth, const float *grad, int64_t nnx, int64_t nny, float amp, float *coeff,
                          hipStream_t s)
{
    const uint32_t wgx = (uint32_t)((nnx - 1 + kCell2W - 1) / kCell2W);
    const dim3 grid((unsigned)cells2_wgs(nnx - 1, nny - 1));
    const bool vec = (reinterpret_cast<uintptr_t>(coeff) & 15) == 0;
    if (smooth == 1) {
        if (vec)
            hipLaunchKernelGGL((k_cells2d<1, true>), grid, dim3(256), 0, s, grad, nnx, nny, wgx, amp, coeff);
        else
            hipLaunchKernelGGL((k_cells2d<1, false>), grid, dim3(256), 0, s, grad, nnx, nny, wgx, amp, coeff);
    } else {
        if (vec)
            hipLaunchKernelGGL((k_cells2d<2, true>), grid, dim3(256), 0, s, grad, nnx, nny, wgx, amp, coeff);
        else
            hipLaunchKernelGGL((k_cells2d<2, false>), grid, dim3(256), 0, s, grad, nnx, nny, wgx, amp, coeff);
    }
    return hipGetLastError();
}

hipError_t launch_cells3d(int smooth, const float *grad, int64_t nnx, int64_t nny, int64_t nnz, float amp,
                          float *coeff, hipStream_t s)
{
    const uint32_t wgx = (uint32_t)((nnx - 1 + kCell3W - 1) / kCell3W), wgy = (uint32_t)((nny - 1 + 1) / 2);
    const dim3 grid((unsigned)cells3_wgs(nnx - 1, nny - 1, nnz - 1));
    const bool vec = (reinterpret_cast<uintptr_t>(coeff) & 15) == 0;
    if (smooth == 1) {
        if (vec)
            hipLaunchKernelGGL((k_cells3d<1, true>), grid, dim3(256), 0, s, grad, nnx, nny, nnz, wgx, wgy, amp, coeff);
        else
            hipLaunchKernelGGL((k_cells3d<1, false>), grid, dim3(256), 0, s, grad, nnx, nny, nnz, wgx, wgy, amp, coeff);
    } else {
        if (vec)
            hipLaunchKernelGGL((k_cells3d<2, true>), grid, dim3(256), 0, s, grad, nnx, nny, nnz, wgx, wgy, amp, coeff);
        else
            hipLaunchKernelGGL((k_cells3d<2, false>), grid, dim3(256), 0, s, grad, nnx, nny, nnz, wgx, wgy, amp, coeff);
    }
    return hipGetLastError();
}

}  // namespace ptg
