// ptg_fbm_strip_grad.hip -- the analytic gradient of a 2D dyadic field (the gradient maps
// of Sec. 5.1) on the strip kernel: H, dH/dX and dH/dY in one launch, in world units per
// sample.  Per strip, after one hashing of its footprint: the rows' values and their d/dY in
// one pass (d/dY differentiates each row segment's polynomial, w = (Y - centre) / 64, and
// takes the row-basis derivatives for the directly evaluated octaves), then dH/dX: H is
// linear in every lane's x-weights, so it is the same strip computation with the weights'
// t-derivatives (times 1/P per octave).
#include "ptg_strip_tile.h"

namespace ptg {

template <int M, typename OutT, int LO, int MD, int G>
__global__ __launch_bounds__(256) void k_fbm2d_strip_grad(const Fbm2dStripArgs a)
{
    extern __shared__ float4 lds4[];
    __shared__ StripShared sh;
    strip_field<M, OutT, LO, MD, 0, G>(a, reinterpret_cast<uint32_t *>(lds4), sh);
}

template <int M, typename OutT, int LO, int MD, int G>
static hipError_t launch_sg(const Fbm2dStripArgs &a, int grid, int waves, size_t lds, hipStream_t s)
{
    auto kern = k_fbm2d_strip_grad<M, OutT, LO, MD, G>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    return launch_k(kern, dim3(grid), dim3(64 * waves), lds, s, a);
}

template <int M, typename OutT, int LO, int MD, int G>
static int resident_sg(int waves, size_t lds)
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_fbm2d_strip_grad<M, OutT, LO, MD, G>, 64 * waves, lds) !=
        hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}

template <int M, typename OutT, int MD, int G>
static hipError_t launch_lo(const Fbm2dStripArgs &a, int grid, int waves, size_t lds, hipStream_t s)
{
    switch (a.lo) {
    case 0: return launch_sg<M, OutT, 0, MD, G>(a, grid, waves, lds, s);
    case 1: return launch_sg<M, OutT, 1, MD, G>(a, grid, waves, lds, s);
    case 2: return launch_sg<M, OutT, 2, MD, G>(a, grid, waves, lds, s);
    case 3: return launch_sg<M, OutT, 3, MD, G>(a, grid, waves, lds, s);
    case 4: return launch_sg<M, OutT, 4, MD, G>(a, grid, waves, lds, s);
    case 5: return launch_sg<M, OutT, 5, MD, G>(a, grid, waves, lds, s);
    default: return launch_sg<M, OutT, 6, MD, G>(a, grid, waves, lds, s);
    }
}

template <int M, typename OutT, int MD, int G>
static int resident_lo(int lo, int waves, size_t lds)
{
    switch (lo) {
    case 0: return resident_sg<M, OutT, 0, MD, G>(waves, lds);
    case 1: return resident_sg<M, OutT, 1, MD, G>(waves, lds);
    case 2: return resident_sg<M, OutT, 2, MD, G>(waves, lds);
    case 3: return resident_sg<M, OutT, 3, MD, G>(waves, lds);
    case 4: return resident_sg<M, OutT, 4, MD, G>(waves, lds);
    case 5: return resident_sg<M, OutT, 5, MD, G>(waves, lds);
    default: return resident_sg<M, OutT, 6, MD, G>(waves, lds);
    }
}

template <int M, int MD, int G>
static int resident_m(bool f16, int lo, int waves, size_t lds)
{
    return f16 ? resident_lo<M, __half, MD, G>(lo, waves, lds) : resident_lo<M, float, MD, G>(lo, waves, lds);
}

template <int M, int MD, int G>
static hipError_t launch_m(const Fbm2dStripArgs &a, bool f16, int grid, int waves, size_t lds, hipStream_t s)
{
    return f16 ? launch_lo<M, __half, MD, G>(a, grid, waves, lds, s) : launch_lo<M, float, MD, G>(a, grid, waves, lds, s);
}

template <int G>
static int resident_g(int smooth, int model, bool f16, int lo, int waves, size_t lds)
{
    if (model == 1) return resident_m<1, 1, G>(f16, lo, waves, lds);
    if (model == 2)
        return smooth == 1 ? resident_m<1, 2, G>(f16, lo, waves, lds)
             : smooth == 2 ? resident_m<2, 2, G>(f16, lo, waves, lds)
                           : resident_m<3, 2, G>(f16, lo, waves, lds);
    return smooth == 1 ? resident_m<1, 0, G>(f16, lo, waves, lds)
         : smooth == 2 ? resident_m<2, 0, G>(f16, lo, waves, lds)
                       : resident_m<3, 0, G>(f16, lo, waves, lds);
}

template <int G>
static hipError_t launch_g(const Fbm2dStripArgs &a, int smooth, int model, bool f16, int grid, int waves, size_t lds,
                           hipStream_t s)
{
    if (model == 1) return launch_m<1, 1, G>(a, f16, grid, waves, lds, s);
    if (model == 2)
        return smooth == 1 ? launch_m<1, 2, G>(a, f16, grid, waves, lds, s)
             : smooth == 2 ? launch_m<2, 2, G>(a, f16, grid, waves, lds, s)
                           : launch_m<3, 2, G>(a, f16, grid, waves, lds, s);
    return smooth == 1 ? launch_m<1, 0, G>(a, f16, grid, waves, lds, s)
         : smooth == 2 ? launch_m<2, 0, G>(a, f16, grid, waves, lds, s)
                       : launch_m<3, 0, G>(a, f16, grid, waves, lds, s);
}

// model 1 (zero-gradient) is smoothness 1 only; models 0 and 2 smoothness 1, 2 or 3
int strip_grad_wgs_per_cu(int smooth, int model, bool f16, int lo, int waves, size_t lds)
{
    return resident_g<4>(smooth, model, f16, lo, waves, lds);
}

hipError_t launch_fbm2d_strip_grad(const Fbm2dStripArgs &a, int smooth, int model, bool f16, int grid, int waves,
                                   size_t lds, hipStream_t s)
{
    return launch_g<4>(a, smooth, model, f16, grid, waves, lds, s);
}

}  // namespace ptg
