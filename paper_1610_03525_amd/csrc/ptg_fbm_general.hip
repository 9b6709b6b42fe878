// ptg_fbm_general.hip -- K3 launches for any octave parameters (the tile functions are in
// ptg_general_tile.h, shared with the persistent serving kernel).
#include "ptg.h"
#include "ptg_general_tile.h"

namespace ptg {

template <int M, typename OutT, int TH, int MD = 0>
__global__ __launch_bounds__(256) void k_fbm2d_general(const Fbm2dArgs a)
{
    extern __shared__ float4 lds4[];
    fbm2d_general_tile<M, OutT, TH, MD>(a, blockIdx.x, lds4);
}

// The field and its analytic gradient, 64 x 64 tiles.
template <int M, typename OutT, int MD>
__global__ __launch_bounds__(256) void k_fbm2d_general_grad(const Fbm2dArgs a)
{
    extern __shared__ float4 lds4[];
    fbm2d_general_tile<M, OutT, 64, MD, true>(a, blockIdx.x, lds4);
}

template <int M, typename OutT, int MD = 0>
__global__ __launch_bounds__(256) void k_fbm3d_general(const Fbm3dArgs a)
{
    extern __shared__ float4 lds4[];
    fbm3d_general_tile<M, OutT, MD>(a, blockIdx.x, lds4);
}

template <typename Args>
static hipError_t launch_dyn(void (*kernel)(Args), dim3 grid, size_t lds, hipStream_t s, const Args &a)
{
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    return launch_k(kernel, grid, dim3(256), lds, s, a);
}

// Orders 4..6 (64-row tiles; gradient or height-and-gradient model).
template <int M, int TH>
static hipError_t launch_2d_high_th(const Fbm2dArgs &a, bool f16, dim3 grid, size_t lds, hipStream_t s)
{
    if (a.model == 2)
        return f16 ? launch_dyn(k_fbm2d_general<M, __half, TH, 2>, grid, lds, s, a)
                   : launch_dyn(k_fbm2d_general<M, float, TH, 2>, grid, lds, s, a);
    return f16 ? launch_dyn(k_fbm2d_general<M, __half, TH>, grid, lds, s, a)
               : launch_dyn(k_fbm2d_general<M, float, TH>, grid, lds, s, a);
}

template <int M>
static hipError_t launch_2d_high(const Fbm2dArgs &a, bool f16, dim3 grid, size_t lds, hipStream_t s)
{
    return a.tile_h == 128 ? launch_2d_high_th<M, 128>(a, f16, grid, lds, s)
                           : launch_2d_high_th<M, 64>(a, f16, grid, lds, s);
}

template <int TH>
static hipError_t launch_2d_th(const Fbm2dArgs &a, int smooth, bool f16, dim3 grid, size_t lds, hipStream_t s)
{
    if (a.model == 3)  // Perlin's noise (fade S3 / S5: smoothness 1 / 2, validated)
        return smooth == 1 ? (f16 ? launch_dyn(k_fbm2d_general<1, __half, TH, 3>, grid, lds, s, a)
                                  : launch_dyn(k_fbm2d_general<1, float, TH, 3>, grid, lds, s, a))
                           : (f16 ? launch_dyn(k_fbm2d_general<2, __half, TH, 3>, grid, lds, s, a)
                                  : launch_dyn(k_fbm2d_general<2, float, TH, 3>, grid, lds, s, a));
    if (a.model == 1)  // zero-gradient model (smoothness 1, validated)
        return f16 ? launch_dyn(k_fbm2d_general<1, __half, TH, 1>, grid, lds, s, a)
                   : launch_dyn(k_fbm2d_general<1, float, TH, 1>, grid, lds, s, a);
    if (a.model == 2) {  // heights and weighted gradients
        if (smooth == 1)
            return f16 ? launch_dyn(k_fbm2d_general<1, __half, TH, 2>, grid, lds, s, a)
                       : launch_dyn(k_fbm2d_general<1, float, TH, 2>, grid, lds, s, a);
        if (smooth == 3)
            return f16 ? launch_dyn(k_fbm2d_general<3, __half, TH, 2>, grid, lds, s, a)
                       : launch_dyn(k_fbm2d_general<3, float, TH, 2>, grid, lds, s, a);
        return f16 ? launch_dyn(k_fbm2d_general<2, __half, TH, 2>, grid, lds, s, a)
                   : launch_dyn(k_fbm2d_general<2, float, TH, 2>, grid, lds, s, a);
    }
    if (smooth == 3)
        return f16 ? launch_dyn(k_fbm2d_general<3, __half, TH>, grid, lds, s, a)
                   : launch_dyn(k_fbm2d_general<3, float, TH>, grid, lds, s, a);
    if (smooth == 1)
        return f16 ? launch_dyn(k_fbm2d_general<1, __half, TH>, grid, lds, s, a)
                   : launch_dyn(k_fbm2d_general<1, float, TH>, grid, lds, s, a);
    return f16 ? launch_dyn(k_fbm2d_general<2, __half, TH>, grid, lds, s, a)
               : launch_dyn(k_fbm2d_general<2, float, TH>, grid, lds, s, a);
}

hipError_t launch_fbm2d_general(const Fbm2dArgs &a, int smooth, bool f16, size_t lds, hipStream_t s)
{
    const int64_t tiles = (int64_t)a.tiles_x * ((a.ny + a.tile_h - 1) / a.tile_h);
    dim3 grid((unsigned)tiles);
    if (smooth >= 4)  // the plan gives these orders 64- or 128-row tiles
        return smooth == 4 ? launch_2d_high<4>(a, f16, grid, lds, s)
             : smooth == 5 ? launch_2d_high<5>(a, f16, grid, lds, s)
                           : launch_2d_high<6>(a, f16, grid, lds, s);
    switch (a.tile_h) {
    case 16: return launch_2d_th<16>(a, smooth, f16, grid, lds, s);
    case 32: return launch_2d_th<32>(a, smooth, f16, grid, lds, s);
    case 128: return launch_2d_th<128>(a, smooth, f16, grid, lds, s);
    default: return launch_2d_th<64>(a, smooth, f16, grid, lds, s);
    }
}

template <typename OutT>
static hipError_t launch_grad_t(const Fbm2dArgs &a, int smooth, dim3 grid, size_t lds, hipStream_t s)
{
    if (a.model == 1) return launch_dyn(k_fbm2d_general_grad<1, OutT, 1>, grid, lds, s, a);
    if (a.model == 2) {
        if (smooth == 1) return launch_dyn(k_fbm2d_general_grad<1, OutT, 2>, grid, lds, s, a);
        if (smooth == 2) return launch_dyn(k_fbm2d_general_grad<2, OutT, 2>, grid, lds, s, a);
        return launch_dyn(k_fbm2d_general_grad<3, OutT, 2>, grid, lds, s, a);
    }
    if (smooth == 1) return launch_dyn(k_fbm2d_general_grad<1, OutT, 0>, grid, lds, s, a);
    if (smooth == 2) return launch_dyn(k_fbm2d_general_grad<2, OutT, 0>, grid, lds, s, a);
    return launch_dyn(k_fbm2d_general_grad<3, OutT, 0>, grid, lds, s, a);
}

hipError_t launch_fbm2d_general_grad(const Fbm2dArgs &a, int smooth, bool f16, size_t lds, hipStream_t s)
{
    const int64_t tiles = (int64_t)a.tiles_x * ((a.ny + 63) / 64);
    dim3 grid((unsigned)tiles);
    return f16 ? launch_grad_t<__half>(a, smooth, grid, lds, s) : launch_grad_t<float>(a, smooth, grid, lds, s);
}

template <int MD>
static hipError_t launch_3g(const Fbm3dArgs &a, int smooth, bool f16, dim3 grid, size_t lds, hipStream_t s)
{
    if (smooth == 1)
        return f16 ? launch_dyn(k_fbm3d_general<1, __half, MD>, grid, lds, s, a)
                   : launch_dyn(k_fbm3d_general<1, float, MD>, grid, lds, s, a);
    if (smooth == 3)
        return f16 ? launch_dyn(k_fbm3d_general<3, __half, MD>, grid, lds, s, a)
                   : launch_dyn(k_fbm3d_general<3, float, MD>, grid, lds, s, a);
    if (smooth == 4)
        return f16 ? launch_dyn(k_fbm3d_general<4, __half, MD>, grid, lds, s, a)
                   : launch_dyn(k_fbm3d_general<4, float, MD>, grid, lds, s, a);
    if (smooth == 5)
        return f16 ? launch_dyn(k_fbm3d_general<5, __half, MD>, grid, lds, s, a)
                   : launch_dyn(k_fbm3d_general<5, float, MD>, grid, lds, s, a);
    if (smooth == 6)
        return f16 ? launch_dyn(k_fbm3d_general<6, __half, MD>, grid, lds, s, a)
                   : launch_dyn(k_fbm3d_general<6, float, MD>, grid, lds, s, a);
    return f16 ? launch_dyn(k_fbm3d_general<2, __half, MD>, grid, lds, s, a)
               : launch_dyn(k_fbm3d_general<2, float, MD>, grid, lds, s, a);
}

hipError_t launch_fbm3d_general(const Fbm3dArgs &a, int smooth, bool f16, size_t lds, hipStream_t s)
{
    const int64_t tiles = (int64_t)a.tiles_x * a.tiles_y * ((a.nz + kTile3Z - 1) / kTile3Z);
    dim3 grid((unsigned)tiles);
    return a.model == PTG_MODEL_HEIGHT_GRADIENT ? launch_3g<2>(a, smooth, f16, grid, lds, s)
                                                : launch_3g<0>(a, smooth, f16, grid, lds, s);
}

}  // namespace ptg
