// ptg_fbm_strip.hip -- K3 for 2D dyadic octave ladders: the dense-field kernel (one wave
// per 64 x 64 strip, a grid-stride walk over the field's strips) and its launches; the
// per-strip code is in ptg_strip_tile.h.
#include "ptg_strip_tile.h"

namespace ptg {

template <int M, typename OutT, int LO, int MD, int PREC = 0>
__global__ __launch_bounds__(256) void k_fbm2d_strip(const Fbm2dStripArgs a)
{
    extern __shared__ float4 lds4[];
    __shared__ StripShared sh;
    strip_field<M, OutT, LO, MD, PREC, 0>(a, reinterpret_cast<uint32_t *>(lds4), sh);
}

template <int M, typename OutT, int LO, int MD, int PREC = 0>
static hipError_t launch_st(const Fbm2dStripArgs &a, int grid, int waves, size_t lds, hipStream_t s)
{
    auto kern = k_fbm2d_strip<M, OutT, LO, MD, PREC>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    return launch_k(kern, dim3(grid), dim3(64 * waves), lds, s, a);
}

template <int M, typename OutT, int MD>
static hipError_t launch_lo(const Fbm2dStripArgs &a, int grid, int waves, size_t lds, hipStream_t s)
{
    switch (a.lo) {
    case 0: return launch_st<M, OutT, 0, MD>(a, grid, waves, lds, s);
    case 1: return launch_st<M, OutT, 1, MD>(a, grid, waves, lds, s);
    case 2: return launch_st<M, OutT, 2, MD>(a, grid, waves, lds, s);
    case 3: return launch_st<M, OutT, 3, MD>(a, grid, waves, lds, s);
    case 4: return launch_st<M, OutT, 4, MD>(a, grid, waves, lds, s);
    case 5: return launch_st<M, OutT, 5, MD>(a, grid, waves, lds, s);
    default: return launch_st<M, OutT, 6, MD>(a, grid, waves, lds, s);
    }
}

template <int M, typename OutT, int LO, int MD, int PREC = 0>
static int resident_one(int waves, size_t lds)
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_fbm2d_strip<M, OutT, LO, MD, PREC>, 64 * waves, lds) !=
        hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}

template <int M, typename OutT, int MD>
static int resident_st(int lo, int waves, size_t lds)
{
    switch (lo) {
    case 0: return resident_one<M, OutT, 0, MD>(waves, lds);
    case 1: return resident_one<M, OutT, 1, MD>(waves, lds);
    case 2: return resident_one<M, OutT, 2, MD>(waves, lds);
    case 3: return resident_one<M, OutT, 3, MD>(waves, lds);
    case 4: return resident_one<M, OutT, 4, MD>(waves, lds);
    case 5: return resident_one<M, OutT, 5, MD>(waves, lds);
    default: return resident_one<M, OutT, 6, MD>(waves, lds);
    }
}

template <int M, int MD>
static int resident_m(bool f16, int lo, int waves, size_t lds)
{
    return f16 ? resident_st<M, __half, MD>(lo, waves, lds) : resident_st<M, float, MD>(lo, waves, lds);
}

// model 1 (zero-gradient) is smoothness 1 only; models 0 and 2 smoothness 1, 2 or 3
int strip_wgs_per_cu(int smooth, int model, bool f16, int lo, int waves, size_t lds)
{
    if (model == 1) return resident_m<1, 1>(f16, lo, waves, lds);
    if (model == 2)
        return smooth == 1 ? resident_m<1, 2>(f16, lo, waves, lds)
             : smooth == 2 ? resident_m<2, 2>(f16, lo, waves, lds)
                           : resident_m<3, 2>(f16, lo, waves, lds);
    return smooth == 1 ? resident_m<1, 0>(f16, lo, waves, lds)
         : smooth == 2 ? resident_m<2, 0>(f16, lo, waves, lds)
                       : resident_m<3, 0>(f16, lo, waves, lds);
}

template <int M, int MD>
static hipError_t launch_m(const Fbm2dStripArgs &a, bool f16, int grid, int waves, size_t lds, hipStream_t s)
{
    return f16 ? launch_lo<M, __half, MD>(a, grid, waves, lds, s) : launch_lo<M, float, MD>(a, grid, waves, lds, s);
}

hipError_t launch_fbm2d_strip(const Fbm2dStripArgs &a, int smooth, int model, bool f16, int grid, int waves,
                              size_t lds, hipStream_t s)
{
    if (model == 1) return launch_m<1, 1>(a, f16, grid, waves, lds, s);
    if (model == 2)
        return smooth == 1 ? launch_m<1, 2>(a, f16, grid, waves, lds, s)
             : smooth == 2 ? launch_m<2, 2>(a, f16, grid, waves, lds, s)
                           : launch_m<3, 2>(a, f16, grid, waves, lds, s);
    return smooth == 1 ? launch_m<1, 0>(a, f16, grid, waves, lds, s)
         : smooth == 2 ? launch_m<2, 0>(a, f16, grid, waves, lds, s)
                       : launch_m<3, 0>(a, f16, grid, waves, lds, s);
}

// The FP16 / BF16 precision form (cubic cells, gradient model, FP16 output).
template <int PREC>
static hipError_t launch_mx_lo(const Fbm2dStripArgs &a, int grid, int waves, size_t lds, hipStream_t s)
{
    switch (a.lo) {
    case 0: return launch_st<1, __half, 0, 0, PREC>(a, grid, waves, lds, s);
    case 1: return launch_st<1, __half, 1, 0, PREC>(a, grid, waves, lds, s);
    case 2: return launch_st<1, __half, 2, 0, PREC>(a, grid, waves, lds, s);
    case 3: return launch_st<1, __half, 3, 0, PREC>(a, grid, waves, lds, s);
    case 4: return launch_st<1, __half, 4, 0, PREC>(a, grid, waves, lds, s);
    case 5: return launch_st<1, __half, 5, 0, PREC>(a, grid, waves, lds, s);
    default: return launch_st<1, __half, 6, 0, PREC>(a, grid, waves, lds, s);
    }
}

template <int PREC>
static int resident_mx(int lo, int waves, size_t lds)
{
    switch (lo) {
    case 0: return resident_one<1, __half, 0, 0, PREC>(waves, lds);
    case 1: return resident_one<1, __half, 1, 0, PREC>(waves, lds);
    case 2: return resident_one<1, __half, 2, 0, PREC>(waves, lds);
    case 3: return resident_one<1, __half, 3, 0, PREC>(waves, lds);
    case 4: return resident_one<1, __half, 4, 0, PREC>(waves, lds);
    case 5: return resident_one<1, __half, 5, 0, PREC>(waves, lds);
    default: return resident_one<1, __half, 6, 0, PREC>(waves, lds);
    }
}

int strip_mx_wgs_per_cu(int prec, int lo, int waves, size_t lds)
{
    return prec == 1 ? resident_mx<1>(lo, waves, lds) : resident_mx<2>(lo, waves, lds);
}

hipError_t launch_fbm2d_strip_mx(const Fbm2dStripArgs &a, int prec, int grid, int waves, size_t lds, hipStream_t s)
{
    return prec == 1 ? launch_mx_lo<1>(a, grid, waves, lds, s) : launch_mx_lo<2>(a, grid, waves, lds, s);
}

}  // namespace ptg
