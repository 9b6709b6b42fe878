// ptg_launch.h -- host-side launch descriptors shared by the C-ABI layer and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ptg {

constexpr int kMaxOctaves = 16;

// Dense 2D field, general (any-parameter) K3: 64 x 64 sample tiles, 256 threads.
constexpr int kTile2 = 64;  // tile width, and the default (and the serving kernel's largest) tile height
// Dense 3D field, general K3: 64 x 8 x 8 sample tiles, 256 threads.
constexpr int kTile3X = 64;
constexpr int kTile3Y = 8;
constexpr int kTile3Z = 8;

// LDS of the general 2D tile beyond its row tables and one octave's node block: a footprint
// entry (kTileFootBytes) and the column and row keys of every octave.
constexpr int kTileFootBytes = 32;
__host__ __device__ inline size_t general2d_octave_lds(int octaves, int capx, int capy)
{
    return (size_t)octaves * ((size_t)kTileFootBytes + (size_t)(capx + capy) * 4);
}

// The 3D general tile's footprint entries and every octave's column and (z, y) row keys.
constexpr int kTileFoot3Bytes = 40;
__host__ __device__ inline size_t general3d_octave_lds(int octaves, int capx, int capy, int capz)
{
    return (size_t)octaves * ((size_t)kTileFoot3Bytes + (size_t)(capx + capy * capz) * 4);
}

struct Fbm2dArgs {
    int64_t x0, y0, nx, ny, pitch;
    void *out;
    double freq[kMaxOctaves];
    float amp[kMaxOctaves];
    int32_t octaves;
    uint32_t seed;
    int32_t capx, capy;  // LDS footprint capacity (nodes per axis) for every octave
    int32_t tiles_x;     // tiles per row of the tile grid
    int32_t tile_h;      // rows per tile: 16, 32 or 64 (tile shape chosen by the tuner)
    int32_t model;       // PTG_MODEL_*
    float gw;            // gradient weight (height-and-gradient model)
    void *out_dx, *out_dy;  // gradient outputs (ptg_fbm_2d_grad), same layout as out
};

struct Fbm3dArgs {
    int64_t x0, y0, z0, nx, ny, nz;
    void *out;
    double freq[kMaxOctaves];
    float amp[kMaxOctaves];
    int32_t octaves;
    uint32_t seed;
    int32_t capx, capy, capz;
    int32_t tiles_x, tiles_y;
    int32_t model;  // PTG_MODEL_GRADIENT or PTG_MODEL_HEIGHT_GRADIENT
    float gw;       // gradient weight (height-and-gradient model)
    int32_t pad;
};

// Dense 2D field, dyadic K3 (base frequency 2^-k, lacunarity 2): world-aligned tiles of
// kDyTileX x kDyTileY samples, 4 waves side by side, each 64 columns x 32 rows.
constexpr int kDyTileX = 256;
constexpr int kDyTileY = 32;
constexpr int kDyMaxShift = 22;  // period 2^s samples, s <= 22 keeps fractions exact in FP32

constexpr int kDyTabMaxP = 512;
constexpr size_t kDyMaxLds = 160 * 1024;  // LDS of one gfx950 compute unit  // octaves of period <= 512 read their bases from an LDS table

struct Fbm2dDyadicArgs {
    int64_t x0, y0, nx, ny, pitch;  // output window (world) and row pitch (elements)
    int64_t tx_base, ty_base;       // world origin of tile (0, 0), tile-aligned
    int64_t tiles;
    void *out;
    float amp[kMaxOctaves];
    float inv2p[kMaxOctaves];  // 2^-(s+1)
    int32_t shift[kMaxOctaves];
    int32_t nnx[kMaxOctaves], nny[kMaxOctaves];     // footprint nodes per axis
    int32_t noff[kMaxOctaves];                      // node-block offset of each octave
    int32_t soff[kMaxOctaves];                      // periods 2, 1: offset in a wave's block
    int32_t wave_nodes;                             // nodes of a wave's block (periods 2, 1)
    int32_t pxoff[kMaxOctaves], pyoff[kMaxOctaves]; // key-prefix offsets
    int32_t toff[kMaxOctaves];                      // basis-table offset, -1: no table
    int32_t nodes_total, px_total, py_total, tab_total, tab_first;
    int32_t octaves;
    uint32_t seed;
    int32_t tiles_x;
    int32_t grid;
    int32_t n_c0;   // leading octaves of period >= 64
};

// Dyadic ladders, plain FP32 form on the vector ALUs: world-aligned strips of
// kStripW x kStripH samples, one wave each (lane = column).  Per-octave node footprints of
// a strip do not depend on its position, so the node / key layout is fixed per launch.
constexpr int kStripW = 64;
constexpr int kStripH = 64;
constexpr int kStripWavesPerWg = 4;  // at most; fewer when a wave's nodes need more LDS

struct Fbm2dStripArgs {
    int64_t x0, y0, nx, ny, pitch;  // output window (world) and row pitch (elements)
    int64_t sx_base, sy_base;       // world origin of strip (0, 0), strip-aligned
    int64_t strips;
    void *out;
    void *out_dx, *out_dy;                          // gradient outputs of the fused gradient kernel
    float amp[kMaxOctaves];
    float inv2p[kMaxOctaves];                       // 2^-(shift + 1)
    int32_t shift[kMaxOctaves];                     // period 2^shift; shift[o] = shift[0] - o
    int32_t nnx[kMaxOctaves], nny[kMaxOctaves];     // node columns / rows of a strip's footprint
    int32_t noff[kMaxOctaves];                      // node block (column-major, nbr rows)
    int32_t nbr[kMaxOctaves];                       // rows of the node block: nny, or for the
                                                    // streamed periods (<= 2 in a ladder that
                                                    // reaches them) one row segment's, R / P + 1
    int32_t kxoff[kMaxOctaves], kyoff[kMaxOctaves]; // column / row key offsets (all column keys first)
    int32_t nodes_total, keys_total, keys_col;      // keys [0, keys_col) are column keys
    int32_t nodes_hashed;                           // nodes [0, nodes_hashed) are hashed per strip
    float gw;                                       // gradient weight (height-and-gradient model)
    int32_t octaves;
    uint32_t seed;
    int32_t strips_x;
    int32_t n_generic;                // octaves 0 .. n_generic-1 have period >= 128
    int32_t o64, o32, o16, o8, o4, o2, o1;  // octave of period 64, 32, ..., 1, or -1
    int32_t lo;                       // min(finest shift, 6): selects the kernel's row loop
    int32_t basis;                    // precision form: PTG_BASIS_* of the MFMA terms
};

// 3D dyadic ladders, plain FP32 form on the vector ALUs: world-aligned blocks of
// k3BlockX x k3BlockY x k3BlockZ samples, one wave each (lane = x column, a walk over the
// block's slices in z).  Octaves of period >= k3BlockZ are "coarse" (one cell over the
// block in y and z); periods 8, 4, 2 are "fine" (their node planes are hashed as the walk
// enters their z cells).
constexpr int k3BlockX = 64;
constexpr int k3BlockY = 8;
constexpr int k3BlockZ = 16;
constexpr int k3TabMaxP = 256;  // coarse octaves of period <= 256 take their block bases from an LDS table

struct Fbm3dStripArgs {
    int64_t x0, y0, z0, nx, ny, nz;  // output volume (world), dense [nz][ny][nx]
    int64_t bx_base, by_base, bz_base;
    int64_t blocks;
    void *out;
    float amp[kMaxOctaves];
    float inv2p[kMaxOctaves];       // 2^-(shift + 1)
    int32_t shift[kMaxOctaves];     // period 2^shift; shift[o] = shift[0] - o
    int32_t nnx[kMaxOctaves];       // node columns of a block's footprint
    int32_t kxoff[kMaxOctaves];     // column keys of octave o in a wave's key block
    int32_t coff[kMaxOctaves];      // coarse octave: its nnx x 2 x 2 nodes (4 i + 2 k + j) from here
    int32_t poff[kMaxOctaves];      // fine octave: its z-plane slots (slot, then i * nny + j) from here
    int32_t ytoff[kMaxOctaves], ztoff[kMaxOctaves];  // coarse octave: basis table (floats), or -1
    int32_t tab_total;              // floats of the basis table
    int32_t fwl[3];                 // fine octaves of period 8, 4, 2: their plane list in the node work list
    int32_t nodes_total;            // nodes of a wave's block: coarse nodes, then the fine planes
    int32_t coarse_nodes;           // coarse nodes (hashed per block from the work list)
    int32_t nodes_listed;           // entries of the node work list (coarse nodes, fine planes)
    int32_t keys_col;               // column keys of every octave
    int32_t keys_total;             // + 4 row keys per coarse octave + the fine planes' row keys
    int32_t octaves;
    uint32_t seed;
    int32_t blocks_x, blocks_y, blocks_z;  // block index = (by * blocks_x + bx) * blocks_z + bz
    int32_t n_coarse;               // octaves 0 .. n_coarse-1 have period >= k3BlockZ
    int32_t o8, o4, o2;             // octave of period 8, 4, 2, or -1
    int32_t lo;                     // min(finest shift, 4): selects the kernel's fine classes
    int32_t model;                  // PTG_MODEL_GRADIENT or PTG_MODEL_HEIGHT_GRADIENT
    float gw;                       // gradient weight (height-and-gradient model)
};

// ---- launch recording (HIP graphs) --------------------------------------------------
// Every dense-field driver launches exactly one kernel whose only argument is one of the
// argument structs above.  Inside a batch recording (ptg_batch_add_*) on this thread the
// launch is recorded instead -- function, shape, dynamic LDS and a copy of the argument
// bytes -- and the batch later launches its records as the kernel nodes of one HIP graph.
constexpr int kLaunchArgMax = 1024;

struct LaunchRec {
    const void *func;
    dim3 grid, block;
    uint32_t lds;
    uint32_t arg_bytes;
    alignas(16) unsigned char args[kLaunchArgMax];
};

struct LaunchSink {
    LaunchRec rec;
    int n;  // launches recorded (a driver makes one)
};

// This thread's sink (NULL: launch at once).
LaunchSink *&launch_sink();

template <typename Args>
inline hipError_t launch_k(void (*kern)(Args), dim3 grid, dim3 block, size_t lds, hipStream_t s, const Args &a)
{
    static_assert(sizeof(Args) <= kLaunchArgMax, "kernel argument struct too large to record");
    if (LaunchSink *k = launch_sink()) {
        if (k->n++ != 0) return hipErrorInvalidValue;  // a driver records one launch
        k->rec.func = reinterpret_cast<const void *>(kern);
        k->rec.grid = grid;
        k->rec.block = block;
        k->rec.lds = (uint32_t)lds;
        k->rec.arg_bytes = (uint32_t)sizeof(Args);
        __builtin_memcpy(k->rec.args, &a, sizeof(Args));
        return hipSuccess;
    }
    hipLaunchKernelGGL(kern, grid, block, lds, s, a);
    return hipGetLastError();
}

// Launch wrappers (defined in the .hip translation units).  They assume validated
// arguments and return the HIP status of the launch.
hipError_t launch_fbm2d_general(const Fbm2dArgs &a, int smooth, bool f16, size_t lds_bytes, hipStream_t s);
hipError_t launch_fbm2d_dyadic(const Fbm2dDyadicArgs &a, int smooth, bool f16, size_t lds_bytes, hipStream_t s);
// LDS words of the strip kernel's work lists (shared by a workgroup) and of one wave's
// private node block (node gradients, then keys).
__host__ __device__ inline int strip_shared_words(int nodes_hashed, int keys_total)
{
    return (keys_total + nodes_hashed + 3) & ~3;
}
// hw = 1: a node height (float) per node besides its gradient (height-and-gradient model)
__host__ __device__ inline int strip_wave_words(int nodes_total, int keys_total, int hw = 0)
{
    return ((2 + hw) * nodes_total + keys_total + 3) & ~3;
}

// LDS words of the 3D strip kernel's shared part (basis table, key list, node list of the
// coarse nodes and the fine planes; the lists start at word tab_words(tab_total)) and of one
// wave's block (gx, gy, gz[, h], then keys).
__host__ __device__ inline int strip3_tab_words(int tab_total) { return (tab_total + 3) & ~3; }
__host__ __device__ inline int strip3_shared_words(int tab_total, int keys_listed, int nodes_listed)
{
    return strip3_tab_words(tab_total) + ((keys_listed + nodes_listed + 3) & ~3);
}
__host__ __device__ inline int strip3_wave_words(int nodes_total, int keys_total, int hw = 0)
{
    return ((3 + hw) * nodes_total + keys_total + 3) & ~3;
}

hipError_t launch_fbm2d_strip(const Fbm2dStripArgs &a, int smooth, int model, bool f16, int grid, int waves, size_t lds_bytes,
                              hipStream_t s);
int strip_wgs_per_cu(int smooth, int model, bool f16, int lo, int waves, size_t lds_bytes);  // resident WGs per CU
// The field and its analytic gradient on the strip kernel, one launch: H to a.out, dH/dX to
// a.out_dx, dH/dY to a.out_dy.
hipError_t launch_fbm2d_strip_grad(const Fbm2dStripArgs &a, int smooth, int model, bool f16, int grid, int waves,
                                   size_t lds_bytes, hipStream_t s);
int strip_grad_wgs_per_cu(int smooth, int model, bool f16, int lo, int waves, size_t lds_bytes);
// The FP16 / BF16 precision form on the strip kernel (prec 1 / 2; cubic cells, FP16 output).
hipError_t launch_fbm2d_strip_mx(const Fbm2dStripArgs &a, int prec, int grid, int waves, size_t lds_bytes,
                                 hipStream_t s);
int strip_mx_wgs_per_cu(int prec, int lo, int waves, size_t lds_bytes);
hipError_t launch_fbm3d_general(const Fbm3dArgs &a, int smooth, bool f16, size_t lds_bytes, hipStream_t s);
hipError_t launch_fbm2d_general_grad(const Fbm2dArgs &a, int smooth, bool f16, size_t lds_bytes, hipStream_t s);
// Simplex-lattice comparison path (ptg_simplex.hip): 64 x 64 tiles; a tile's skewed lattice
// footprint is staged in LDS when it has at most kSimplexKeys nodes per axis and
// kSimplexCap nodes.
constexpr int kSimplexCap = 6144;
constexpr int kSimplexKeys = 128;
hipError_t launch_simplex2d(const Fbm2dArgs &a, bool f16, hipStream_t s);
hipError_t launch_fbm3d_strip(const Fbm3dStripArgs &a, int smooth, bool f16, int grid, int waves, size_t lds_bytes,
                              hipStream_t s);
int strip3_wgs_per_cu(int smooth, int model, bool f16, int lo, int waves, size_t lds_bytes);

// Stand-alone stage kernels (ptg_stages.hip): one-dimensional grids of these workgroups;
// the entry points reject boxes whose workgroup count exceeds 2^31 - 1.
constexpr int kLatRows = 16;  // K1: a workgroup covers 256 node columns x kLatRows node rows
constexpr int kCell2W = 64, kCell2H = 4;  // K2 2D: 64 x 4 cells per workgroup (a wave per row)
constexpr int kCell3W = 64;               // K2 3D: 64 x 2 x 2 cells per workgroup
__host__ __device__ inline int64_t lattice_wgs(int64_t nx, int64_t rows)
{
    return ((nx + 255) / 256) * ((rows + kLatRows - 1) / kLatRows);
}
__host__ __device__ inline int64_t cells2_wgs(int64_t ncx, int64_t ncy)
{
    return ((ncx + kCell2W - 1) / kCell2W) * ((ncy + kCell2H - 1) / kCell2H);
}
__host__ __device__ inline int64_t cells3_wgs(int64_t ncx, int64_t ncy, int64_t ncz)
{
    return ((ncx + kCell3W - 1) / kCell3W) * ((ncy + 1) / 2) * ((ncz + 1) / 2);
}

hipError_t launch_coords(double f0, double lac, int octaves, int64_t x0, int64_t n, int64_t *cells, float *frac,
                         hipStream_t s);
hipError_t launch_lattice2d(uint32_t seed, int octave, int64_t ix0, int64_t iy0, int64_t nx, int64_t ny,
                            uint32_t *keys, float *grad, hipStream_t s);
hipError_t launch_heights2d(uint32_t seed, int octave, int64_t ix0, int64_t iy0, int64_t nx, int64_t ny,
                            float *heights, hipStream_t s);
hipError_t launch_lattice3d(uint32_t seed, int octave, int64_t ix0, int64_t iy0, int64_t iz0, int64_t nx,
                            int64_t ny, int64_t nz, uint32_t *keys, uint32_t *second, float *grad, hipStream_t s);
hipError_t launch_cells2d(int smooth, const float *grad, int64_t nnx, int64_t nny, float amp, float *coeff,
                          hipStream_t s);
hipError_t launch_cells3d(int smooth, const float *grad, int64_t nnx, int64_t nny, int64_t nnz, float amp,
                          float *coeff, hipStream_t s);

}  // namespace ptg
