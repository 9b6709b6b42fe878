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
// K1: lattice hash -> unit gradient over a node box (one node per thread).
// ---------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_lattice2d(uint32_t seed, int octave, int64_t ix0, int64_t iy0, int64_t nx,
                                                   int64_t ny, uint32_t *__restrict__ keys, float *__restrict__ grad)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t n = nx * ny;
    if (q >= n) return;
    const int64_t j = q / nx, i = q - j * nx;
    const uint32_t key = key_combine(absorb_index(key_prefix(seed, octave), iy0 + j), key_xline(ix0 + i));
    if (keys) keys[q] = key;
    if (grad) {
        const float2 g = grad2(key);
        grad[q] = g.x;
        grad[n + q] = g.y;
    }
}

// Zero-gradient model (Sec. 3.3): the node heights of a 2D node box.
__global__ __launch_bounds__(256) void k_heights2d(uint32_t seed, int octave, int64_t ix0, int64_t iy0, int64_t nx,
                                                   int64_t ny, float *__restrict__ h)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= nx * ny) return;
    const int64_t j = q / nx, i = q - j * nx;
    h[q] = height2(key_combine(absorb_index(key_prefix(seed, octave), iy0 + j), key_xline(ix0 + i)));
}

__global__ __launch_bounds__(256) void k_lattice3d(uint32_t seed, int octave, int64_t ix0, int64_t iy0, int64_t iz0,
                                                   int64_t nx, int64_t ny, int64_t nz, uint32_t *__restrict__ keys,
                                                   uint32_t *__restrict__ second, float *__restrict__ grad)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t n = nx * ny * nz;
    if (q >= n) return;
    const int64_t i = q % nx, jk = q / nx;
    const int64_t j = jk % ny, k = jk / ny;
    const uint32_t kzy = absorb_index(absorb_index(key_prefix(seed, octave), iz0 + k), iy0 + j);
    const uint32_t key = key_combine(kzy, key_xline(ix0 + i));
    if (keys) keys[q] = key;
    if (second) second[q] = key3_second(key);
    if (grad) {
        const float3 g = grad3(key);
        grad[q] = g.x;
        grad[n + q] = g.y;
        grad[2 * n + q] = g.z;
    }
}

hipError_t launch_lattice2d(uint32_t seed, int octave, int64_t ix0, int64_t iy0, int64_t nx, int64_t ny,
                            uint32_t *keys, float *grad, hipStream_t s)
{
    const int64_t n = nx * ny;
    hipLaunchKernelGGL(k_lattice2d, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, seed, octave, ix0, iy0, nx,
                       ny, keys, grad);
    return hipGetLastError();
}

hipError_t launch_heights2d(uint32_t seed, int octave, int64_t ix0, int64_t iy0, int64_t nx, int64_t ny,
                            float *heights, hipStream_t s)
{
    const int64_t n = nx * ny;
    hipLaunchKernelGGL(k_heights2d, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, seed, octave, ix0, iy0, nx,
                       ny, heights);
    return hipGetLastError();
}

hipError_t launch_lattice3d(uint32_t seed, int octave, int64_t ix0, int64_t iy0, int64_t iz0, int64_t nx,
                            int64_t ny, int64_t nz, uint32_t *keys, uint32_t *second, float *grad, hipStream_t s)
{
    const int64_t n = nx * ny * nz;
    hipLaunchKernelGGL(k_lattice3d, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, seed, octave, ix0, iy0,
                       iz0, nx, ny, nz, keys, second, grad);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// K2: per-cell monomial coefficients.  A workgroup owns a block of cells, stages the
// corner gradients of that block in LDS once (each node is shared by 2^D cells), and
// each thread expands its cell's tensor Hermite form into monomial coefficients:
//   c_ij = sum_corners [ gx * b1_cx[i] * b0_cy[j] + gy * b0_cx[i] * b1_cy[j] ].
// ---------------------------------------------------------------------------------
constexpr int kCell2 = 16;           // 16 x 16 cells per workgroup
constexpr int kCell3X = 8, kCell3Y = 8, kCell3Z = 4;

template <int M>
__global__ __launch_bounds__(256) void k_cells2d(const float *__restrict__ grad, int64_t nnx, int64_t nny, float amp,
                                                 float *__restrict__ coeff)
{
    constexpr int N1 = BasisMono<M>::N1;
    __shared__ float sgx[kCell2 + 1][kCell2 + 1];
    __shared__ float sgy[kCell2 + 1][kCell2 + 1];
    const int64_t ncx = nnx - 1, ncy = nny - 1;
    const int64_t bx = (int64_t)blockIdx.x * kCell2, by = (int64_t)blockIdx.y * kCell2;
    const int64_t nn = nnx * nny;
    for (int q = threadIdx.x; q < (kCell2 + 1) * (kCell2 + 1); q += 256) {
        const int j = q / (kCell2 + 1), i = q - j * (kCell2 + 1);
        const int64_t gi = min(bx + i, nnx - 1), gj = min(by + j, nny - 1);
        sgx[j][i] = grad[gj * nnx + gi];
        sgy[j][i] = grad[nn + gj * nnx + gi];
    }
    __syncthreads();
    const int li = threadIdx.x & (kCell2 - 1), lj = threadIdx.x / kCell2;
    const int64_t ci = bx + li, cj = by + lj;
    if (ci >= ncx || cj >= ncy) return;
    float gx[2][2], gy[2][2];  // [cy][cx]
    for (int cy = 0; cy < 2; ++cy)
        for (int cx = 0; cx < 2; ++cx) {
            gx[cy][cx] = sgx[lj + cy][li + cx] * amp;
            gy[cy][cx] = sgy[lj + cy][li + cx] * amp;
        }
    float *dst = coeff + (cj * ncx + ci) * (N1 * N1);
    for (int i = 0; i < N1; ++i)
        for (int j = 0; j < N1; ++j) {
            float c = 0.0f;
            for (int cy = 0; cy < 2; ++cy)
                for (int cx = 0; cx < 2; ++cx) {
                    c += gx[cy][cx] * BasisMono<M>::c(2 + cx, i) * BasisMono<M>::c(cy, j);
                    c += gy[cy][cx] * BasisMono<M>::c(cx, i) * BasisMono<M>::c(2 + cy, j);
                }
            dst[i * N1 + j] = c;
        }
}

template <int M>
__global__ __launch_bounds__(256) void k_cells3d(const float *__restrict__ grad, int64_t nnx, int64_t nny, int64_t nnz,
                                                 float amp, float *__restrict__ coeff)
{
    constexpr int N1 = BasisMono<M>::N1;
    constexpr int SX = kCell3X + 1, SY = kCell3Y + 1, SZ = kCell3Z + 1;
    __shared__ float sg[3][SZ][SY][SX];
    const int64_t ncx = nnx - 1, ncy = nny - 1, ncz = nnz - 1;
    const int64_t bx = (int64_t)blockIdx.x * kCell3X, by = (int64_t)blockIdx.y * kCell3Y,
                  bz = (int64_t)blockIdx.z * kCell3Z;
    const int64_t nn = nnx * nny * nnz;
    for (int q = threadIdx.x; q < SX * SY * SZ; q += 256) {
        const int i = q % SX, j = (q / SX) % SY, k = q / (SX * SY);
        const int64_t gi = min(bx + i, nnx - 1), gj = min(by + j, nny - 1), gk = min(bz + k, nnz - 1);
        const int64_t g = (gk * nny + gj) * nnx + gi;
        sg[0][k][j][i] = grad[g];
        sg[1][k][j][i] = grad[nn + g];
        sg[2][k][j][i] = grad[2 * nn + g];
    }
    __syncthreads();
    const int li = threadIdx.x % kCell3X, lj = (threadIdx.x / kCell3X) % kCell3Y, lk = threadIdx.x / (kCell3X * kCell3Y);
    const int64_t ci = bx + li, cj = by + lj, ck = bz + lk;
    if (ci >= ncx || cj >= ncy || ck >= ncz) return;
    float g[3][2][2][2];  // [axis][cz][cy][cx]
    for (int a = 0; a < 3; ++a)
        for (int cz = 0; cz < 2; ++cz)
            for (int cy = 0; cy < 2; ++cy)
                for (int cx = 0; cx < 2; ++cx) g[a][cz][cy][cx] = sg[a][lk + cz][lj + cy][li + cx] * amp;
    float *dst = coeff + ((ck * ncy + cj) * ncx + ci) * (N1 * N1 * N1);
    for (int i = 0; i < N1; ++i)
        for (int j = 0; j < N1; ++j)
            for (int k = 0; k < N1; ++k) {
                float c = 0.0f;
                for (int cz = 0; cz < 2; ++cz)
                    for (int cy = 0; cy < 2; ++cy)
                        for (int cx = 0; cx < 2; ++cx) {
                            const float bx0 = BasisMono<M>::c(cx, i), bx1 = BasisMono<M>::c(2 + cx, i);
                            const float by0 = BasisMono<M>::c(cy, j), by1 = BasisMono<M>::c(2 + cy, j);
                            const float bz0 = BasisMono<M>::c(cz, k), bz1 = BasisMono<M>::c(2 + cz, k);
                            c += g[0][cz][cy][cx] * bx1 * by0 * bz0;
                            c += g[1][cz][cy][cx] * bx0 * by1 * bz0;
                            c += g[2][cz][cy][cx] * bx0 * by0 * bz1;
                        }
                dst[(i * N1 + j) * N1 + k] = c;
            }
}

hipError_t launch_cells2d(int smooth, const float *grad, int64_t nnx, int64_t nny, float amp, float *coeff,
                          hipStream_t s)
{
    dim3 grid((unsigned)((nnx - 1 + kCell2 - 1) / kCell2), (unsigned)((nny - 1 + kCell2 - 1) / kCell2));
    if (smooth == 1)
        hipLaunchKernelGGL(k_cells2d<1>, grid, dim3(256), 0, s, grad, nnx, nny, amp, coeff);
    else
        hipLaunchKernelGGL(k_cells2d<2>, grid, dim3(256), 0, s, grad, nnx, nny, amp, coeff);
    return hipGetLastError();
}

hipError_t launch_cells3d(int smooth, const float *grad, int64_t nnx, int64_t nny, int64_t nnz, float amp,
                          float *coeff, hipStream_t s)
{
    dim3 grid((unsigned)((nnx - 1 + kCell3X - 1) / kCell3X), (unsigned)((nny - 1 + kCell3Y - 1) / kCell3Y),
              (unsigned)((nnz - 1 + kCell3Z - 1) / kCell3Z));
    if (smooth == 1)
        hipLaunchKernelGGL(k_cells3d<1>, grid, dim3(256), 0, s, grad, nnx, nny, nnz, amp, coeff);
    else
        hipLaunchKernelGGL(k_cells3d<2>, grid, dim3(256), 0, s, grad, nnx, nny, nnz, amp, coeff);
    return hipGetLastError();
}

}  // namespace ptg
