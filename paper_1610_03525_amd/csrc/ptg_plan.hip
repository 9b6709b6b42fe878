// ptg_plan.hip -- octave plan and kernel choice for the dense fields.
#include <algorithm>
#include <cmath>

#include "ptg_internal.h"
#include "ptg_launch.h"

namespace ptg {

// Base frequency 2^-k with 0 <= k <= kDyMaxShift and lacunarity exactly 2 (every octave
// period then a power of two >= 1, checked by the caller's frequency validation).
bool dyadic_shift(const ptg_params *p, int *k_out)
{
    if (p->lacunarity != 2.0) return false;
    int e = 0;
    const double m = std::frexp(p->base_freq, &e);  // base_freq = m * 2^e, m in [0.5, 1)
    if (m != 0.5) return false;
    const int k = 1 - e;  // base_freq = 2^-k
    if (k < 0 || k > kDyMaxShift || k - (p->octaves - 1) < 0) return false;
    *k_out = k;
    return true;
}

static int64_t floor_to(int64_t a, int64_t b)  // largest multiple of b <= a (b > 0)
{
    int64_t q = a / b;
    if (q * b > a) --q;
    return q * b;
}

static int device_cus()
{
    static int cus[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (cus[dev] == 0) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
        cus[dev] = n;
    }
    return cus[dev];
}

static int fbm2d_dyadic(const ptg_params *p, int k, int64_t x0, int64_t y0, int64_t nx, int64_t ny, void *out,
                        int64_t pitch, hipStream_t s)
{
    constexpr int TX = kDyTileX, TY = kDyTileY;
    Fbm2dDyadicArgs a{};
    a.x0 = x0;
    a.y0 = y0;
    a.nx = nx;
    a.ny = ny;
    a.pitch = pitch;
    a.out = out;
    a.tx_base = floor_to(x0, TX);
    a.ty_base = floor_to(y0, TY);
    const int64_t tiles_x = (x0 + nx - a.tx_base + TX - 1) / TX;
    const int64_t tiles_y = (y0 + ny - a.ty_base + TY - 1) / TY;
    a.tiles_x = (int32_t)tiles_x;
    a.tiles = tiles_x * tiles_y;
    double freq[kMaxOctaves];
    octave_tables(p, freq, a.amp);
    a.octaves = p->octaves;
    a.seed = p->seed;
    int nodes = 0, px = 0, py = 0, tab = 0, wnodes = 0;
    a.tab_first = p->octaves;
    for (int o = 0; o < p->octaves; ++o) {
        const int sh = k - o;
        a.shift[o] = sh;
        if (sh >= 6) a.n_c0 = o + 1;
        a.inv2p[o] = std::ldexp(1.0f, -(sh + 1));
        a.nnx[o] = std::max(TX >> sh, 1) + 1;
        a.nny[o] = std::max(TY >> sh, 1) + 1;
        a.noff[o] = nodes;
        a.pxoff[o] = px;
        a.pyoff[o] = py;
        a.soff[o] = wnodes;
        if (sh <= 1)  // periods 2, 1: each wave hashes its 64 columns one 16-row group at a time
            wnodes += ((64 >> sh) + 1) * ((16 >> sh) + 1);
        else
            nodes += a.nnx[o] * a.nny[o];
        px += a.nnx[o];
        py += a.nny[o];
        if ((1 << sh) <= kDyTabMaxP) {
            if (a.tab_first == p->octaves) a.tab_first = o;
            a.toff[o] = tab;
            tab += 1 << sh;
        } else {
            a.toff[o] = -1;
        }
    }
    a.nodes_total = nodes;
    a.wave_nodes = wnodes;
    a.px_total = px;
    a.py_total = py;
    a.tab_total = tab;
    // workgroups: a few per compute unit, each walking tiles with a grid stride
    a.grid = (int32_t)std::min<int64_t>(a.tiles, (int64_t)device_cus() * 4);
    const size_t lds = (size_t)tab * 16 + (size_t)nodes * 8 + (size_t)(px + py) * 4 + (size_t)nodes * 4 +
                       (size_t)(px + py) * 4 + 8 + (size_t)(kDyTileX / 64) * wnodes * 8;
    if (lds > kDyMaxLds) return 1;  // footprint too large for one workgroup: caller falls back
    (void)tune_pick(TuneKey{PTG_TUNE_DYADIC_2D, p->smoothness, p->out_dtype == PTG_F16, size_class(nx * ny), k}, 0);
    if (tune_dry()) return PTG_OK;
    hipError_t e = launch_fbm2d_dyadic(a, p->smoothness, p->out_dtype == PTG_F16, lds, s);
    return e == hipSuccess ? PTG_OK : hip_fail(e, "fbm2d dyadic launch");
}

int strip_args_2d(const ptg_params *p, int k, int64_t x0, int64_t y0, int64_t nx, int64_t ny, void *out,
                  int64_t pitch, Fbm2dStripArgs *ap)
{
    constexpr int SW = kStripW, SH = kStripH;
    Fbm2dStripArgs &a = *ap;
    a = Fbm2dStripArgs{};
    a.x0 = x0;
    a.y0 = y0;
    a.nx = nx;
    a.ny = ny;
    a.pitch = pitch;
    a.out = out;
    a.sx_base = floor_to(x0, SW);
    a.sy_base = floor_to(y0, SH);
    const int64_t strips_x = (x0 + nx - a.sx_base + SW - 1) / SW;
    const int64_t strips_y = (y0 + ny - a.sy_base + SH - 1) / SH;
    if (strips_x > 0x7FFFFFFFLL) return 1;
    a.strips_x = (int32_t)strips_x;
    a.strips = strips_x * strips_y;
    double freq[kMaxOctaves];
    octave_tables(p, freq, a.amp);
    a.octaves = p->octaves;
    a.seed = p->seed;
    a.gw = (float)p->gradient_weight;
    a.basis = p->basis;
    a.o64 = a.o32 = a.o16 = a.o8 = a.o4 = a.o2 = a.o1 = -1;
    const int smin = k - (p->octaves - 1);
    // the row loop assumes every period from 32 down to the finest is present
    if (smin <= 5 && k < 5) return 1;
    a.lo = std::min(smin, 6);
    int nodes = 0, keys = 0, kcol = 0;
    // periods 2 and 1 (ladders that reach them) are streamed: their node rows are hashed per
    // row segment (8 rows for cubic cells, in every form; 16 for higher orders) into a block
    // of that height, instead of per strip (65 x 65 nodes at period 1 would hold 34 KB of LDS
    // per wave)
    const int seg_rows = p->smoothness == 1 ? 8 : 16;
    const bool stream = a.lo <= 1;
    for (int o = 0; o < p->octaves; ++o)  // column keys of every octave first, then row keys
        kcol += std::max(SW >> std::min(k - o, 30), 1) + 1;
    a.keys_col = kcol;
    kcol = 0;
    for (int o = 0; o < p->octaves; ++o) {
        const int sh = k - o;
        a.shift[o] = sh;
        a.inv2p[o] = std::ldexp(1.0f, -(sh + 1));
        if (sh >= 7) a.n_generic = o + 1;
        if (sh == 6) a.o64 = o;
        if (sh == 5) a.o32 = o;
        if (sh == 4) a.o16 = o;
        if (sh == 3) a.o8 = o;
        if (sh == 2) a.o4 = o;
        if (sh == 1) a.o2 = o;
        if (sh == 0) a.o1 = o;
        a.nnx[o] = std::max(SW >> std::min(sh, 30), 1) + 1;
        a.nny[o] = std::max(SH >> std::min(sh, 30), 1) + 1;
        const bool streamed = stream && sh <= 1;  // the finest octaves: they come last
        a.nbr[o] = streamed ? (seg_rows >> sh) + 1 : a.nny[o];
        a.noff[o] = nodes;
        a.kxoff[o] = kcol;
        a.kyoff[o] = a.keys_col + (keys - kcol);
        nodes += a.nnx[o] * a.nbr[o];
        if (!streamed) a.nodes_hashed = nodes;
        kcol += a.nnx[o];
        keys += a.nnx[o] + a.nny[o];
    }
    a.nodes_total = nodes;
    a.keys_total = keys;
    if (keys >= (1 << 14)) return 1;
    return 0;
}

// The strip kernel's arguments and launch shape for a dyadic field; returns 1 when a strip's
// node footprint does not fit the workgroup's LDS.
static int strip_plan(const ptg_params *p, int k, int64_t x0, int64_t y0, int64_t nx, int64_t ny, void *out,
                      int64_t pitch, Fbm2dStripArgs *a, int *waves_out, size_t *lds_out)
{
    if (strip_args_2d(p, k, x0, y0, nx, ny, out, pitch, a)) return 1;
    const size_t shared_words = (size_t)strip_shared_words(a->nodes_hashed, a->keys_total);
    const size_t wave_words =
        (size_t)strip_wave_words(a->nodes_total, a->keys_total, p->model == PTG_MODEL_HEIGHT_GRADIENT);
    // waves per workgroup: the tuned count (default 4), at most what the private node
    // blocks allow in LDS
    int waves = tune_pick(TuneKey{PTG_TUNE_STRIP_2D, p->smoothness + 2 * p->model, p->out_dtype == PTG_F16,
                                  size_class(nx * ny), a->lo},
                          kStripWavesPerWg);
    while (waves > 1 && (shared_words + waves * wave_words) * 4 > kDyMaxLds) --waves;
    const size_t lds = (shared_words + waves * wave_words) * 4;
    if (lds > kDyMaxLds) return 1;
    *waves_out = waves;
    *lds_out = lds;
    return 0;
}

// A persistent grid of exactly the resident workgroups (a partial second round would leave
// most of the chip idle at the end).
static int strip_grid(const Fbm2dStripArgs &a, int waves, int per_cu)
{
    const int64_t wgs = (a.strips + waves - 1) / waves;
    return (int)std::min<int64_t>(wgs, (int64_t)device_cus() * per_cu);
}

// Plain FP32 dyadic field through the strip kernel; returns 1 when a strip's node
// footprint does not fit the workgroup's LDS (the caller falls back).
static int fbm2d_strip(const ptg_params *p, int k, int64_t x0, int64_t y0, int64_t nx, int64_t ny, void *out,
                       int64_t pitch, hipStream_t s)
{
    Fbm2dStripArgs a;
    int waves = 0;
    size_t lds = 0;
    if (strip_plan(p, k, x0, y0, nx, ny, out, pitch, &a, &waves, &lds)) return 1;
    if (tune_dry()) return PTG_OK;
    const bool f16 = p->out_dtype == PTG_F16;
    const int grid = strip_grid(a, waves, strip_wgs_per_cu(p->smoothness, p->model, f16, a.lo, waves, lds));
    hipError_t e = launch_fbm2d_strip(a, p->smoothness, p->model, f16, grid, waves, lds, s);
    return e == hipSuccess ? PTG_OK : hip_fail(e, "fbm2d strip launch");
}

size_t general_args_2d(const ptg_params *p, int64_t x0, int64_t y0, int64_t nx, int64_t ny, void *out,
                       int64_t pitch, int tile_h, Fbm2dArgs *a)
{
    *a = Fbm2dArgs{};
    a->x0 = x0;
    a->y0 = y0;
    a->nx = nx;
    a->ny = ny;
    a->pitch = pitch;
    a->out = out;
    octave_tables(p, a->freq, a->amp);
    a->octaves = p->octaves;
    a->seed = p->seed;
    a->tile_h = tile_h;
    a->model = p->model;
    a->gw = (float)p->gradient_weight;
    a->capx = footprint_cap(a->freq, p->octaves, kTile2);
    a->capy = footprint_cap(a->freq, p->octaves, tile_h);
    a->tiles_x = (int32_t)((nx + kTile2 - 1) / kTile2);
    const size_t node_bytes = p->model == PTG_MODEL_HEIGHT_GRADIENT ? 12 : p->model == PTG_MODEL_ZERO_GRADIENT ? 4 : 8;
    return (size_t)tile_h * 16 + (size_t)a->capx * a->capy * node_bytes +
           general2d_octave_lds(p->octaves, a->capx, a->capy);
}

size_t general_args_3d(const ptg_params *p, int64_t x0, int64_t y0, int64_t z0, int64_t nx, int64_t ny, int64_t nz,
                       void *out, Fbm3dArgs *a)
{
    *a = Fbm3dArgs{};
    a->x0 = x0;
    a->y0 = y0;
    a->z0 = z0;
    a->nx = nx;
    a->ny = ny;
    a->nz = nz;
    a->out = out;
    octave_tables(p, a->freq, a->amp);
    a->octaves = p->octaves;
    a->seed = p->seed;
    a->capx = footprint_cap(a->freq, p->octaves, kTile3X);
    a->capy = footprint_cap(a->freq, p->octaves, kTile3Y);
    a->capz = footprint_cap(a->freq, p->octaves, kTile3Z);
    a->tiles_x = (int32_t)((nx + kTile3X - 1) / kTile3X);
    a->tiles_y = (int32_t)((ny + kTile3Y - 1) / kTile3Y);
    a->model = p->model;
    a->gw = (float)p->gradient_weight;
    return (size_t)(kTile3Y + kTile3Z) * 16 +
           (size_t)a->capx * a->capy * a->capz * (p->model == PTG_MODEL_HEIGHT_GRADIENT ? 16 : 12) +
           general3d_octave_lds(p->octaves, a->capx, a->capy, a->capz);
}

int fbm2d_plain(const ptg_params *p, int64_t x0, int64_t y0, int64_t nx, int64_t ny, void *out, int64_t pitch,
                hipStream_t s)
{
    if (p->model == PTG_MODEL_SIMPLEX) {  // comparison path: its own kernel for any ladder
        Fbm2dArgs a{};
        (void)general_args_2d(p, x0, y0, nx, ny, out, pitch, kTile2, &a);
        (void)tune_pick(TuneKey{PTG_TUNE_GENERAL_2D, p->smoothness + 2 * p->model, p->out_dtype == PTG_F16, size_class(nx * ny), 0},
                        kTile2);
        if (tune_dry()) return PTG_OK;
        hipError_t e = launch_simplex2d(a, p->out_dtype == PTG_F16, s);
        return e == hipSuccess ? PTG_OK : hip_fail(e, "simplex launch");
    }
    int k = 0;
    const bool dy = dyadic_shift(p, &k);
    if (p->path == PTG_PATH_DYADIC && !dy)
        return fail(PTG_EINVAL, "the dyadic kernel needs base_freq = 2^-k (k <= %d) and lacunarity 2", kDyMaxShift);
    if (p->path == PTG_PATH_DYADIC && p->smoothness > 3)
        return fail(PTG_EINVAL, "smoothness orders above 3 run on the general kernel only");
    if (dy && p->path != PTG_PATH_GENERAL && p->smoothness <= 3 && p->model != PTG_MODEL_PERLIN) {
        int rc = fbm2d_strip(p, k, x0, y0, nx, ny, out, pitch, s);
        if (rc <= 0) return rc;
        // the tile kernel (the strip kernel's fallback when a strip's footprint does not fit
        // LDS) has gradient-model C1 / C2 cells only
        if (p->model == PTG_MODEL_GRADIENT && p->smoothness <= 2) {
            rc = fbm2d_dyadic(p, k, x0, y0, nx, ny, out, pitch, s);
            if (rc <= 0) return rc;
        }
        if (p->path == PTG_PATH_DYADIC && p->model != PTG_MODEL_GRADIENT)
            return fail(PTG_EINVAL, "the dyadic path of this model is the strip kernel, which needs a ladder whose "
                                    "coarsest period is >= 32 (or finest >= 64) and a footprint that fits LDS");
        if (p->path == PTG_PATH_DYADIC)
            return fail(PTG_EINVAL, "the dyadic kernel's lattice footprint exceeds the workgroup's LDS");
    }
    Fbm2dArgs a{};
    double freq[kMaxOctaves];
    float amp[kMaxOctaves];
    octave_tables(p, freq, amp);
    // untuned: 128-row tiles for tall fields (each octave's set-up per tile is amortised over
    // twice the rows) while a tile's LDS block stays small enough for eight workgroups per
    // compute unit; else 64 (on fine ladders the larger block would cost more occupancy)
    Fbm2dArgs probe{};
    const bool tall_ok = ny >= 1024 && general_args_2d(p, x0, y0, nx, ny, out, pitch, 2 * kTile2, &probe) <= 20 * 1024;
    const int dflt = tall_ok ? 2 * kTile2 : kTile2;
    // (orders above 3 have 64- and 128-row tiles only)
    const int picked = tune_pick(TuneKey{PTG_TUNE_GENERAL_2D, p->smoothness + 2 * p->model, p->out_dtype == PTG_F16,
                                         size_class(nx * ny), ladder_class(freq, p->octaves)},
                                 dflt);
    int tile_h = p->smoothness >= 4 ? (picked >= 2 * kTile2 ? 2 * kTile2 : kTile2) : picked;
    size_t lds = general_args_2d(p, x0, y0, nx, ny, out, pitch, tile_h, &a);
    // ladders whose cells are finer than a sample: shorter tiles until a tile's lattice
    // footprint fits the workgroup's LDS
    while (lds > kDyMaxLds && tile_h > (p->smoothness >= 4 ? kTile2 : 16)) {
        tile_h /= 2;
        lds = general_args_2d(p, x0, y0, nx, ny, out, pitch, tile_h, &a);
    }
    if (lds > kDyMaxLds)
        return fail(PTG_EINVAL, "the ladder's finest cells are too small for a tile's lattice footprint in LDS "
                                "(%zu bytes)", lds);
    if (tune_dry()) return PTG_OK;
    hipError_t e = launch_fbm2d_general(a, p->smoothness, p->out_dtype == PTG_F16, lds, s);
    return e == hipSuccess ? PTG_OK : hip_fail(e, "fbm2d launch");
}

// The field and its analytic gradient.  Dyadic ladders (unless the general path is asked
// for) take the strip kernel in one launch: per strip the field and dH/dY in one pass, then
// dH/dX (the field's arithmetic is that of ptg_fbm_2d's strip launch, bit for bit).
// Otherwise, or when a strip's footprint does not fit LDS, the general kernel with 64-row
// tiles (any model, any ladder) and a second row table for the row-basis derivatives writes
// all three in one pass.
int fbm2d_grad(const ptg_params *p, int64_t x0, int64_t y0, int64_t nx, int64_t ny, void *out, void *out_dx,
               void *out_dy, int64_t pitch, hipStream_t s)
{
    int k = 0;
    if (dyadic_shift(p, &k) && p->path != PTG_PATH_GENERAL) {
        Fbm2dStripArgs a;
        int waves = 0;
        size_t lds = 0;
        if (!strip_plan(p, k, x0, y0, nx, ny, out, pitch, &a, &waves, &lds)) {
            const bool f16 = p->out_dtype == PTG_F16;
            const int sm = p->smoothness, md = p->model;
            a.out_dx = out_dx;
            a.out_dy = out_dy;
            const int grid = strip_grid(a, waves, strip_grad_wgs_per_cu(sm, md, f16, a.lo, waves, lds));
            hipError_t e = launch_fbm2d_strip_grad(a, sm, md, f16, grid, waves, lds, s);
            return e == hipSuccess ? PTG_OK : hip_fail(e, "fbm2d strip gradient launch");
        }
    }
    Fbm2dArgs a{};
    const size_t lds = general_args_2d(p, x0, y0, nx, ny, out, pitch, kTile2, &a) + (size_t)kTile2 * 16;
    if (lds > kDyMaxLds)
        return fail(PTG_EINVAL, "the ladder's finest cells are too small for a tile's lattice footprint in LDS "
                                "(%zu bytes)", lds);
    a.out_dx = out_dx;
    a.out_dy = out_dy;
    hipError_t e = launch_fbm2d_general_grad(a, p->smoothness, p->out_dtype == PTG_F16, lds, s);
    return e == hipSuccess ? PTG_OK : hip_fail(e, "fbm2d grad launch");
}

int strip3_args(const ptg_params *p, int k, int64_t x0, int64_t y0, int64_t z0, int64_t nx, int64_t ny, int64_t nz,
                void *out, Fbm3dStripArgs *ap, bool ahead_all)
{
    constexpr int BX = k3BlockX, BY = k3BlockY, BZ = k3BlockZ;
    Fbm3dStripArgs &a = *ap;
    a = Fbm3dStripArgs{};
    a.x0 = x0;
    a.y0 = y0;
    a.z0 = z0;
    a.nx = nx;
    a.ny = ny;
    a.nz = nz;
    a.out = out;
    a.bx_base = floor_to(x0, BX);
    a.by_base = floor_to(y0, BY);
    a.bz_base = floor_to(z0, BZ);
    const int64_t bxn = (x0 + nx - a.bx_base + BX - 1) / BX;
    const int64_t byn = (y0 + ny - a.by_base + BY - 1) / BY;
    const int64_t bzn = (z0 + nz - a.bz_base + BZ - 1) / BZ;
    if (bxn > 0x7FFFFFFFLL || byn > 0x7FFFFFFFLL || bzn > 0x7FFFFFFFLL) return 1;
    a.blocks_x = (int32_t)bxn;
    a.blocks_y = (int32_t)byn;
    a.blocks_z = (int32_t)bzn;
    a.blocks = bxn * byn * bzn;
    double freq[kMaxOctaves];
    octave_tables(p, freq, a.amp);
    a.octaves = p->octaves;
    a.seed = p->seed;
    a.model = p->model;
    a.gw = (float)p->gradient_weight;
    a.o8 = a.o4 = a.o2 = -1;
    const int smin = k - (p->octaves - 1);
    if (smin < 1) return 1;            // period 1: the general kernel
    if (smin <= 3 && k < 3) return 1;  // the fine classes assume every period from 8 down to the finest
    a.lo = std::min(smin, 4);
    int kcol = 0, cnodes = 0, tab = 0;
    for (int o = 0; o < p->octaves; ++o) {
        const int sh = k - o;
        a.shift[o] = sh;
        a.inv2p[o] = std::ldexp(1.0f, -(sh + 1));
        const int c = std::min(sh, 30);
        a.nnx[o] = std::max(BX >> c, 1) + 1;
        a.kxoff[o] = kcol;
        kcol += a.nnx[o];
        a.coff[o] = a.poff[o] = a.ytoff[o] = a.ztoff[o] = -1;
        if ((1 << std::min(sh, 30)) >= BZ) {
            a.n_coarse = o + 1;
            a.coff[o] = cnodes;
            cnodes += 4 * a.nnx[o];
            if ((1 << std::min(sh, 30)) <= k3TabMaxP) {  // block bases from the table
                const int E = 3 * (2 * p->smoothness + 2), P = 1 << sh;
                a.ytoff[o] = tab;
                tab += (P / BY) * E;
                a.ztoff[o] = tab;
                tab += (P / BZ) * E;
            }
        }
        if (sh == 3) a.o8 = o;
        if (sh == 2) a.o4 = o;
        if (sh == 1) a.o2 = o;
    }
    a.keys_col = kcol;
    a.coarse_nodes = cnodes;
    a.tab_total = tab;
    int nodes = cnodes, listed = cnodes;
    const int fine[3] = {a.o8, a.o4, a.o2};
    for (int f = 0; f < 3; ++f) {
        const int o = fine[f];
        a.fwl[f] = listed;
        if (o < 0) continue;
        const int P = 8 >> f, plane = (BX / P + 1) * (BY / P + 1);
        a.poff[o] = nodes;
        // plane slots: two, four for period 2 when its planes are hashed two ahead
        nodes += (f == 2 && (ahead_all || p->model != PTG_MODEL_HEIGHT_GRADIENT) ? 4 : 2) * plane;
        listed += plane;
    }
    a.nodes_total = nodes;
    a.nodes_listed = listed;
    // + the fine octaves' row keys of the block's planes (periods 8, 4, 2: 3 x 2, 5 x 3, 9 x 5)
    a.keys_total = kcol + 4 * a.n_coarse + 66;
    if (a.keys_total >= (1 << 14) || cnodes >= (1 << 14)) return 1;
    return 0;
}

// Plain FP32 dyadic volume through the 3D strip kernel; returns 1 when it does not apply
// (a ladder starting below period 4, or a node block larger than LDS): the caller falls back.
static int fbm3d_strip(const ptg_params *p, int k, int64_t x0, int64_t y0, int64_t z0, int64_t nx, int64_t ny,
                       int64_t nz, void *out, hipStream_t s)
{
    Fbm3dStripArgs a;
    if (strip3_args(p, k, x0, y0, z0, nx, ny, nz, out, &a, true)) return 1;
    const int hw = p->model == PTG_MODEL_HEIGHT_GRADIENT ? 1 : 0;
    const size_t shared_words =
        (size_t)strip3_shared_words(a.tab_total, a.keys_col + 4 * a.n_coarse, a.nodes_listed);
    const size_t wave_words = (size_t)strip3_wave_words(a.nodes_total, a.keys_total, hw);
    int waves = tune_pick(TuneKey{PTG_TUNE_STRIP_3D, p->smoothness + 2 * hw, p->out_dtype == PTG_F16,
                                  size_class(nx * ny * nz), a.lo},
                          4);
    while (waves > 1 && (shared_words + waves * wave_words) * 4 > kDyMaxLds) --waves;
    const size_t lds = (shared_words + waves * wave_words) * 4;
    if (lds > kDyMaxLds) return 1;
    if (tune_dry()) return PTG_OK;
    const int64_t per_cu = strip3_wgs_per_cu(p->smoothness, p->model, p->out_dtype == PTG_F16, a.lo, waves, lds);
    const int64_t wgs = (a.blocks + waves - 1) / waves;
    const int grid = (int)std::min<int64_t>(wgs, (int64_t)device_cus() * per_cu);
    hipError_t e = launch_fbm3d_strip(a, p->smoothness, p->out_dtype == PTG_F16, grid, waves, lds, s);
    return e == hipSuccess ? PTG_OK : hip_fail(e, "fbm3d strip launch");
}

int fbm3d_plain(const ptg_params *p, int64_t x0, int64_t y0, int64_t z0, int64_t nx, int64_t ny, int64_t nz,
                void *out, hipStream_t s)
{
    int k = 0;
    const bool dy = dyadic_shift(p, &k);
    if (p->path == PTG_PATH_DYADIC && !dy)
        return fail(PTG_EINVAL, "the dyadic kernel needs base_freq = 2^-k (k <= %d) and lacunarity 2", kDyMaxShift);
    if (p->path == PTG_PATH_DYADIC && p->smoothness >= 3)
        return fail(PTG_EINVAL, "3D smoothness orders above 2 run on the general kernel only");
    if (dy && p->path != PTG_PATH_GENERAL && p->smoothness <= 2) {
        const int rc = fbm3d_strip(p, k, x0, y0, z0, nx, ny, nz, out, s);
        if (rc <= 0) return rc;
        if (p->path == PTG_PATH_DYADIC)
            return fail(PTG_EINVAL, "the 3D dyadic kernel does not apply (a ladder reaching period 1, finer than 8 "
                                    "with a coarsest period below 8, or LDS)");
    }
    Fbm3dArgs a{};
    const size_t lds = general_args_3d(p, x0, y0, z0, nx, ny, nz, out, &a);
    (void)tune_pick(TuneKey{PTG_TUNE_GENERAL_3D, p->smoothness, p->out_dtype == PTG_F16, size_class(nx * ny * nz),
                            ladder_class(a.freq, p->octaves)},
                    0);
    if (lds > kDyMaxLds)
        return fail(PTG_EINVAL, "the ladder's finest cells are too small for a tile's lattice footprint in LDS "
                                "(%zu bytes)", lds);
    if (tune_dry()) return PTG_OK;
    hipError_t e = launch_fbm3d_general(a, p->smoothness, p->out_dtype == PTG_F16, lds, s);
    return e == hipSuccess ? PTG_OK : hip_fail(e, "fbm3d launch");
}

int fbm2d_mfma(const ptg_params *p, int64_t x0, int64_t y0, int64_t nx, int64_t ny, void *out, int64_t pitch,
               hipStream_t s)
{
    int k = 0;
    if (!dyadic_shift(p, &k))
        return fail(PTG_EINVAL, "the FP16/BF16 matrix-core form needs base_freq = 2^-k (k <= %d) and lacunarity 2",
                    kDyMaxShift);
    Fbm2dStripArgs a;
    if (strip_args_2d(p, k, x0, y0, nx, ny, out, pitch, &a))
        return fail(PTG_EINVAL, "the matrix-core form needs a ladder whose coarsest period is >= 32 (or whose finest "
                                "is >= 64) and a footprint that fits LDS");
    const int prec = p->form == PTG_FORM_MFMA_F16 ? 1 : 2;
    const size_t shared_words = (size_t)strip_shared_words(a.nodes_hashed, a.keys_total);
    const size_t wave_words = (size_t)strip_wave_words(a.nodes_total, a.keys_total, 0);
    int waves = tune_pick(TuneKey{PTG_TUNE_STRIP_2D, 8 + prec, 1, size_class(nx * ny), a.lo}, kStripWavesPerWg);
    while (waves > 1 && (shared_words + waves * wave_words) * 4 > kDyMaxLds) --waves;
    const size_t lds = (shared_words + waves * wave_words) * 4;
    if (lds > kDyMaxLds) return fail(PTG_EINVAL, "the lattice footprint exceeds the workgroup's LDS");
    if (tune_dry()) return PTG_OK;
    const int64_t per_cu = strip_mx_wgs_per_cu(prec, a.lo, waves, lds);
    const int64_t wgs = (a.strips + waves - 1) / waves;
    const int grid = (int)std::min<int64_t>(wgs, (int64_t)device_cus() * per_cu);
    hipError_t e = launch_fbm2d_strip_mx(a, prec, grid, waves, lds, s);
    return e == hipSuccess ? PTG_OK : hip_fail(e, "fbm2d precision-form launch");
}

}  // namespace ptg
