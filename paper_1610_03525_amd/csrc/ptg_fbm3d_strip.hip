// ptg_fbm3d_strip.hip -- K3 for 3D dyadic octave ladders: the dense-volume kernel (one wave
// per 64 x 8 x 16 block, each wave a run of consecutive blocks in z) and its launches; the
// per-block code is in ptg_strip3_tile.h.
#include "ptg.h"
#include "ptg_strip3_tile.h"

namespace ptg {

template <int M, typename OutT, int LO, int MD>
__global__ __launch_bounds__(256) void k_fbm3d_strip(const Fbm3dStripArgs a)
{
    extern __shared__ float4 lds4[];
    __shared__ Strip3Shared sh;
    const int tid = threadIdx.x, lane = tid & 63, nthreads = blockDim.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wpg = nthreads >> 6;
    // LDS: [basis table | wl_key | wl_node] shared, then per wave [gx | gy | gz | (h) | keys]
    const int listed = a.keys_col + 4 * a.n_coarse;
    uint32_t *wl_key = reinterpret_cast<uint32_t *>(lds4) + strip3_tab_words(a.tab_total);
    uint32_t *wl_node = wl_key + listed;
    const int shared_words = strip3_shared_words(a.tab_total, listed, a.nodes_listed);
    const int wave_words = strip3_wave_words(a.nodes_total, a.keys_total, MD == 2 ? 1 : 0);
    float *gx = reinterpret_cast<float *>(lds4) + shared_words + wave * wave_words;

    strip3_prologue<M>(a, sh, lds4, wl_key, wl_node, tid, nthreads);
    __syncthreads();
    Strip3Wave<M, OutT, LO, MD, true> w(a, sh, gx, lane);
    // each wave takes a run of consecutive blocks (z fastest), carrying the fine octaves'
    // node planes from a block to the next one above it
    const int64_t nwaves = (int64_t)gridDim.x * wpg, chunk = (a.blocks + nwaves - 1) / nwaves;
    const int64_t b0 = ((int64_t)blockIdx.x * wpg + wave) * chunk, b1 = min(b0 + chunk, a.blocks);
    for (int64_t blk = b0; blk < b1; ++blk)
        w.run(a, sh, lds4, wl_key, wl_node, blk, blk > b0 && blk % a.blocks_z != 0);
}

template <int M, typename OutT, int LO, int MD>
static hipError_t launch_s3(const Fbm3dStripArgs &a, int grid, int waves, size_t lds, hipStream_t s)
{
    auto kern = k_fbm3d_strip<M, OutT, LO, MD>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    return launch_k(kern, dim3(grid), dim3(64 * waves), lds, s, a);
}

template <int M, typename OutT, int MD>
static hipError_t launch_s3_lo(const Fbm3dStripArgs &a, int grid, int waves, size_t lds, hipStream_t s)
{
    switch (a.lo) {
    case 1: return launch_s3<M, OutT, 1, MD>(a, grid, waves, lds, s);
    case 2: return launch_s3<M, OutT, 2, MD>(a, grid, waves, lds, s);
    case 3: return launch_s3<M, OutT, 3, MD>(a, grid, waves, lds, s);
    default: return launch_s3<M, OutT, 4, MD>(a, grid, waves, lds, s);
    }
}

template <int M, typename OutT, int LO, int MD>
static int resident_s3_one(int waves, size_t lds)
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_fbm3d_strip<M, OutT, LO, MD>, 64 * waves, lds) !=
        hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}

template <int M, typename OutT, int MD>
static int resident_s3(int lo, int waves, size_t lds)
{
    switch (lo) {
    case 1: return resident_s3_one<M, OutT, 1, MD>(waves, lds);
    case 2: return resident_s3_one<M, OutT, 2, MD>(waves, lds);
    case 3: return resident_s3_one<M, OutT, 3, MD>(waves, lds);
    default: return resident_s3_one<M, OutT, 4, MD>(waves, lds);
    }
}

template <int MD>
static int resident_s3_md(int smooth, bool f16, int lo, int waves, size_t lds)
{
    if (smooth == 1)
        return f16 ? resident_s3<1, __half, MD>(lo, waves, lds) : resident_s3<1, float, MD>(lo, waves, lds);
    return f16 ? resident_s3<2, __half, MD>(lo, waves, lds) : resident_s3<2, float, MD>(lo, waves, lds);
}

int strip3_wgs_per_cu(int smooth, int model, bool f16, int lo, int waves, size_t lds)
{
    return model == PTG_MODEL_HEIGHT_GRADIENT ? resident_s3_md<2>(smooth, f16, lo, waves, lds)
                                              : resident_s3_md<0>(smooth, f16, lo, waves, lds);
}

template <int MD>
static hipError_t launch_s3_md(const Fbm3dStripArgs &a, int smooth, bool f16, int grid, int waves, size_t lds,
                               hipStream_t s)
{
    if (smooth == 1)
        return f16 ? launch_s3_lo<1, __half, MD>(a, grid, waves, lds, s)
                   : launch_s3_lo<1, float, MD>(a, grid, waves, lds, s);
    return f16 ? launch_s3_lo<2, __half, MD>(a, grid, waves, lds, s) : launch_s3_lo<2, float, MD>(a, grid, waves, lds, s);
}

hipError_t launch_fbm3d_strip(const Fbm3dStripArgs &a, int smooth, bool f16, int grid, int waves, size_t lds,
                              hipStream_t s)
{
    return a.model == PTG_MODEL_HEIGHT_GRADIENT ? launch_s3_md<2>(a, smooth, f16, grid, waves, lds, s)
                                                : launch_s3_md<0>(a, smooth, f16, grid, waves, lds, s);
}

}  // namespace ptg
