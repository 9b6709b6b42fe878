// ptg_api.hip -- the C ABI (include/ptg.h): argument validation, octave plan, launches.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>

#include "../../include/ptg.h"
#include "ptg_internal.h"
#include "ptg_launch.h"

namespace ptg {

static thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(PTG_EHIP, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

static bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

int validate_params(const ptg_params *p, int dim)
{
    if (!p) return fail(PTG_EINVAL, "params is NULL");
    if (p->dim != dim) return fail(PTG_EINVAL, "params.dim is %d, this entry point takes %d", p->dim, dim);
    if (p->smoothness < 1 || p->smoothness > PTG_MAX_SMOOTHNESS)
        return fail(PTG_EINVAL, "smoothness must be 1 (C1 cubic), 2 (C2 quintic), 3 (C3 septic) .. %d, got %d",
                    PTG_MAX_SMOOTHNESS, p->smoothness);
    if (p->octaves < 1 || p->octaves > PTG_MAX_OCTAVES)
        return fail(PTG_EINVAL, "octaves must be in 1..%d, got %d", PTG_MAX_OCTAVES, p->octaves);
    if (p->out_dtype != PTG_F32 && p->out_dtype != PTG_F16)
        return fail(PTG_EINVAL, "out_dtype must be PTG_F32 or PTG_F16, got %d", p->out_dtype);
    if (!finite_pos(p->persistence)) return fail(PTG_EINVAL, "persistence must be finite and > 0");
    if (!finite_pos(p->lacunarity)) return fail(PTG_EINVAL, "lacunarity must be finite and > 0");
    if (!finite_pos(p->base_freq)) return fail(PTG_EINVAL, "base_freq must be finite and > 0");
    if (p->form != PTG_FORM_PLAIN && p->form != PTG_FORM_MFMA_F16 && p->form != PTG_FORM_MFMA_BF16)
        return fail(PTG_EINVAL, "unknown form %d", p->form);
    if (p->form != PTG_FORM_PLAIN && (dim != 2 || p->smoothness != 1))
        return fail(PTG_EINVAL, "the matrix-core forms are 2D C1 only");
    if (p->basis != PTG_BASIS_MONOMIAL && p->basis != PTG_BASIS_CENTRED && p->basis != PTG_BASIS_HERMITE)
        return fail(PTG_EINVAL, "unknown basis %d", p->basis);
    if (p->form != PTG_FORM_PLAIN && p->out_dtype != PTG_F16)
        return fail(PTG_EINVAL, "the matrix-core forms write FP16 output");
    if (p->path != PTG_PATH_AUTO && p->path != PTG_PATH_GENERAL && p->path != PTG_PATH_DYADIC)
        return fail(PTG_EINVAL, "unknown path %d", p->path);
    if (p->model != PTG_MODEL_GRADIENT && p->model != PTG_MODEL_ZERO_GRADIENT && p->model != PTG_MODEL_HEIGHT_GRADIENT &&
        p->model != PTG_MODEL_PERLIN && p->model != PTG_MODEL_SIMPLEX)
        return fail(PTG_EINVAL, "unknown model %d", p->model);
    if (p->model == PTG_MODEL_SIMPLEX &&
        (dim != 2 || p->smoothness != 1 || p->form != PTG_FORM_PLAIN || p->path == PTG_PATH_DYADIC))
        return fail(PTG_EINVAL, "the simplex-lattice noise is 2D, smoothness 1, plain form, its own kernel");
    if (p->model == PTG_MODEL_PERLIN &&
        (dim != 2 || p->smoothness > 2 || p->form != PTG_FORM_PLAIN || p->path == PTG_PATH_DYADIC))
        return fail(PTG_EINVAL, "Perlin's noise is 2D, fade S3 or S5 (smoothness 1, 2), plain form, general kernel");
    if (p->model == PTG_MODEL_HEIGHT_GRADIENT && p->form != PTG_FORM_PLAIN)
        return fail(PTG_EINVAL, "the height-and-gradient model is plain form");
    if (p->model == PTG_MODEL_HEIGHT_GRADIENT && !std::isfinite(p->gradient_weight))
        return fail(PTG_EINVAL, "gradient_weight must be finite");
    if (p->model == PTG_MODEL_ZERO_GRADIENT && (dim != 2 || p->smoothness != 1 || p->form != PTG_FORM_PLAIN))
        return fail(PTG_EINVAL, "the zero-gradient model is 2D, smoothness 1, plain form");
    double f = p->base_freq, a = 1.0;
    for (int o = 0; o < p->octaves; ++o) {
        if (!(f <= 1.0) || !(f > 0.0))
            return fail(PTG_EINVAL, "octave %d frequency %.17g is outside (0, 1] cells per sample", o, f);
        if (!std::isfinite(a) || a == 0.0) return fail(PTG_EINVAL, "octave %d amplitude is not finite/non-zero", o);
        f = f * p->lacunarity;
        a = a * p->persistence;
    }
    return PTG_OK;
}

int validate_extent(const char *axis, int64_t x0, int64_t n)
{
    if (n < 0) return fail(PTG_EINVAL, "%s extent is negative", axis);
    if (n >= PTG_MAX_WORLD_ABS || x0 <= -PTG_MAX_WORLD_ABS || x0 >= PTG_MAX_WORLD_ABS)
        return fail(PTG_EINVAL, "%s origin/extent outside +-2^52", axis);
    const int64_t last = x0 + n;  // no overflow: both bounded by 2^52
    if (last <= -PTG_MAX_WORLD_ABS || last >= PTG_MAX_WORLD_ABS)
        return fail(PTG_EINVAL, "%s origin + extent outside +-2^52", axis);
    return PTG_OK;
}

void octave_tables(const ptg_params *p, double *freq, float *amp)
{
    double f = p->base_freq, a = 1.0;
    for (int o = 0; o < p->octaves; ++o) {
        freq[o] = f;
        amp[o] = (float)a;
        f = f * p->lacunarity;
        a = a * p->persistence;
    }
}

// Largest number of lattice nodes one tile of `extent` samples touches along an axis:
// floor(a + d) - floor(a) <= floor(d) + 1 with d = (extent-1) f, plus the far corner,
// plus one node of margin for the rounding of the two FP64 products.
int footprint_cap(const double *freq, int octaves, int extent)
{
    int cap = 2;
    for (int o = 0; o < octaves; ++o) {
        const int c = (int)std::floor((double)(extent - 1) * freq[o]) + 4;
        if (c > cap) cap = c;
    }
    return cap;
}

}  // namespace ptg

using namespace ptg;

extern "C" {

const char *ptg_version(void) { return "ptg 0.1 (gfx950)"; }

const char *ptg_last_error(void) { return g_last_error.c_str(); }

void ptg_params_default(ptg_params *p)
{
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->dim = 2;
    p->smoothness = 1;
    p->octaves = 8;
    p->out_dtype = PTG_F32;
    p->persistence = 0.5;
    p->lacunarity = 2.0;
    p->base_freq = 1.0 / 512.0;
    p->seed = 1;
    p->form = PTG_FORM_PLAIN;
    p->basis = PTG_BASIS_MONOMIAL;
    p->gradient_weight = 0.01;
}

int ptg_fbm_2d(const ptg_params *p, int64_t x0, int64_t y0, int64_t nx, int64_t ny, void *out_dev,
               int64_t row_pitch, void *stream)
{
    int rc = validate_params(p, 2);
    if (rc) return rc;
    if ((rc = validate_extent("x", x0, nx))) return rc;
    if ((rc = validate_extent("y", y0, ny))) return rc;
    if (nx == 0 || ny == 0) return PTG_OK;
    if (!out_dev) return fail(PTG_EINVAL, "out_dev is NULL");
    if (row_pitch < nx) return fail(PTG_EINVAL, "row_pitch %lld < nx %lld", (long long)row_pitch, (long long)nx);
    // the general kernel's smallest tiles are 64 x 16
    const int64_t tiles_x = (nx + kTile2 - 1) / kTile2, tiles_y = (ny + 15) / 16;
    if (tiles_x * tiles_y > 0x7FFFFFFFLL) return fail(PTG_EINVAL, "field too large for one launch");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (p->form != PTG_FORM_PLAIN) return fbm2d_mfma(p, x0, y0, nx, ny, out_dev, row_pitch, s);
    return fbm2d_plain(p, x0, y0, nx, ny, out_dev, row_pitch, s);
}

int ptg_fbm_2d_grad(const ptg_params *p, int64_t x0, int64_t y0, int64_t nx, int64_t ny, void *out_dev,
                    void *dx_dev, void *dy_dev, int64_t row_pitch, void *stream)
{
    int rc = validate_params(p, 2);
    if (rc) return rc;
    if (p->form != PTG_FORM_PLAIN) return fail(PTG_EINVAL, "the gradient output is computed in the plain form");
    if (p->smoothness > 3) return fail(PTG_EINVAL, "the gradient output takes smoothness 1..3");
    if (p->model == PTG_MODEL_PERLIN || p->model == PTG_MODEL_SIMPLEX)
        return fail(PTG_EINVAL, "the gradient output takes the cell models");
    if ((rc = validate_extent("x", x0, nx))) return rc;
    if ((rc = validate_extent("y", y0, ny))) return rc;
    if (nx == 0 || ny == 0) return PTG_OK;
    if (!out_dev || !dx_dev || !dy_dev) return fail(PTG_EINVAL, "an output pointer is NULL");
    if (row_pitch < nx) return fail(PTG_EINVAL, "row_pitch %lld < nx %lld", (long long)row_pitch, (long long)nx);
    const int64_t tiles_x = (nx + kTile2 - 1) / kTile2, tiles_y = (ny + kTile2 - 1) / kTile2;
    if (tiles_x * tiles_y > 0x7FFFFFFFLL) return fail(PTG_EINVAL, "field too large for one launch");
    return fbm2d_grad(p, x0, y0, nx, ny, out_dev, dx_dev, dy_dev, row_pitch, reinterpret_cast<hipStream_t>(stream));
}

int ptg_fbm_3d(const ptg_params *p, int64_t x0, int64_t y0, int64_t z0, int64_t nx, int64_t ny, int64_t nz,
               void *out_dev, void *stream)
{
    int rc = validate_params(p, 3);
    if (rc) return rc;
    if ((rc = validate_extent("x", x0, nx))) return rc;
    if ((rc = validate_extent("y", y0, ny))) return rc;
    if ((rc = validate_extent("z", z0, nz))) return rc;
    if (nx == 0 || ny == 0 || nz == 0) return PTG_OK;
    if (!out_dev) return fail(PTG_EINVAL, "out_dev is NULL");
    const int64_t tx = (nx + kTile3X - 1) / kTile3X, ty = (ny + kTile3Y - 1) / kTile3Y,
                  tz = (nz + kTile3Z - 1) / kTile3Z;
    if (tx > 0x7FFFFFFFLL || ty > 0x7FFFFFFFLL || tx * ty * tz > 0x7FFFFFFFLL)
        return fail(PTG_EINVAL, "volume too large for one launch");
    return fbm3d_plain(p, x0, y0, z0, nx, ny, nz, out_dev, reinterpret_cast<hipStream_t>(stream));
}

int ptg_coords(double base_freq, double lacunarity, int32_t octaves, int64_t x0, int64_t n, int64_t *cells_dev,
               float *frac_dev, void *stream)
{
    if (!finite_pos(base_freq) || !finite_pos(lacunarity)) return fail(PTG_EINVAL, "bad base_freq / lacunarity");
    if (octaves < 1 || octaves > PTG_MAX_OCTAVES) return fail(PTG_EINVAL, "octaves out of range");
    int rc = validate_extent("x", x0, n);
    if (rc) return rc;
    if (n == 0) return PTG_OK;
    if (!cells_dev || !frac_dev) return fail(PTG_EINVAL, "NULL output");
    if ((n + 255) / 256 > 0x7FFFFFFFLL) return fail(PTG_EINVAL, "n too large");
    hipError_t e = launch_coords(base_freq, lacunarity, octaves, x0, n, cells_dev, frac_dev,
                                 reinterpret_cast<hipStream_t>(stream));
    return e == hipSuccess ? PTG_OK : hip_fail(e, "coords launch");
}

int ptg_lattice_2d(uint32_t seed, int32_t octave, int64_t ix0, int64_t iy0, int64_t nx, int64_t ny,
                   uint32_t *keys_dev, float *grad_dev, void *stream)
{
    if (octave < 0) return fail(PTG_EINVAL, "octave < 0");
    if (nx < 0 || ny < 0) return fail(PTG_EINVAL, "negative node box");
    if (nx == 0 || ny == 0) return PTG_OK;
    if (!keys_dev && !grad_dev) return fail(PTG_EINVAL, "both outputs NULL");
    if (nx > (1LL << 40) / ny || lattice_wgs(nx, ny) > 0x7FFFFFFFLL) return fail(PTG_EINVAL, "box too large");
    hipError_t e = launch_lattice2d(seed, octave, ix0, iy0, nx, ny, keys_dev, grad_dev,
                                    reinterpret_cast<hipStream_t>(stream));
    return e == hipSuccess ? PTG_OK : hip_fail(e, "lattice2d launch");
}

int ptg_heights_2d(uint32_t seed, int32_t octave, int64_t ix0, int64_t iy0, int64_t nx, int64_t ny,
                   float *heights_dev, void *stream)
{
    if (octave < 0) return fail(PTG_EINVAL, "octave < 0");
    if (nx < 0 || ny < 0) return fail(PTG_EINVAL, "negative node box");
    if (nx == 0 || ny == 0) return PTG_OK;
    if (!heights_dev) return fail(PTG_EINVAL, "heights_dev is NULL");
    if (nx > (1LL << 40) / ny || lattice_wgs(nx, ny) > 0x7FFFFFFFLL) return fail(PTG_EINVAL, "box too large");
    hipError_t e = launch_heights2d(seed, octave, ix0, iy0, nx, ny, heights_dev, reinterpret_cast<hipStream_t>(stream));
    return e == hipSuccess ? PTG_OK : hip_fail(e, "heights2d launch");
}

int ptg_lattice_3d(uint32_t seed, int32_t octave, int64_t ix0, int64_t iy0, int64_t iz0, int64_t nx, int64_t ny,
                   int64_t nz, uint32_t *keys_dev, uint32_t *second_dev, float *grad_dev, void *stream)
{
    if (octave < 0) return fail(PTG_EINVAL, "octave < 0");
    if (nx < 0 || ny < 0 || nz < 0) return fail(PTG_EINVAL, "negative node box");
    if (nx == 0 || ny == 0 || nz == 0) return PTG_OK;
    if (!keys_dev && !second_dev && !grad_dev) return fail(PTG_EINVAL, "all outputs NULL");
    if (nx > (1LL << 40) / ny || nx * ny > (1LL << 40) / nz || lattice_wgs(nx, ny * nz) > 0x7FFFFFFFLL)
        return fail(PTG_EINVAL, "box too large");
    hipError_t e = launch_lattice3d(seed, octave, ix0, iy0, iz0, nx, ny, nz, keys_dev, second_dev, grad_dev,
                                    reinterpret_cast<hipStream_t>(stream));
    return e == hipSuccess ? PTG_OK : hip_fail(e, "lattice3d launch");
}

int ptg_cells_2d(int32_t smoothness, const float *grad_dev, int64_t nnx, int64_t nny, float amplitude,
                 float *coeff_dev, void *stream)
{
    if (smoothness != 1 && smoothness != 2) return fail(PTG_EINVAL, "smoothness must be 1 or 2");
    if (nnx < 2 || nny < 2) return fail(PTG_EINVAL, "a node box needs at least 2 x 2 nodes");
    if (!grad_dev || !coeff_dev) return fail(PTG_EINVAL, "NULL buffer");
    if (nnx > (1LL << 40) / nny || cells2_wgs(nnx - 1, nny - 1) > 0x7FFFFFFFLL)
        return fail(PTG_EINVAL, "box too large");
    if (!std::isfinite(amplitude)) return fail(PTG_EINVAL, "amplitude not finite");
    hipError_t e = launch_cells2d(smoothness, grad_dev, nnx, nny, amplitude, coeff_dev,
                                  reinterpret_cast<hipStream_t>(stream));
    return e == hipSuccess ? PTG_OK : hip_fail(e, "cells2d launch");
}

int ptg_cells_3d(int32_t smoothness, const float *grad_dev, int64_t nnx, int64_t nny, int64_t nnz, float amplitude,
                 float *coeff_dev, void *stream)
{
    if (smoothness != 1 && smoothness != 2) return fail(PTG_EINVAL, "smoothness must be 1 or 2");
    if (nnx < 2 || nny < 2 || nnz < 2) return fail(PTG_EINVAL, "a node box needs at least 2 nodes per axis");
    if (!grad_dev || !coeff_dev) return fail(PTG_EINVAL, "NULL buffer");
    if (nnx > (1LL << 40) / nny || nnx * nny > (1LL << 40) / nnz || cells3_wgs(nnx - 1, nny - 1, nnz - 1) > 0x7FFFFFFFLL)
        return fail(PTG_EINVAL, "box too large");
    if (!std::isfinite(amplitude)) return fail(PTG_EINVAL, "amplitude not finite");
    hipError_t e = launch_cells3d(smoothness, grad_dev, nnx, nny, nnz, amplitude, coeff_dev,
                                  reinterpret_cast<hipStream_t>(stream));
    return e == hipSuccess ? PTG_OK : hip_fail(e, "cells3d launch");
}

}  // extern "C"
