// ptg_internal.h -- host-side helpers shared by the C-ABI translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdint.h>

#include "../../include/ptg.h"
#include "ptg_launch.h"

namespace ptg {

int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
int validate_params(const ptg_params *p, int dim);
int validate_extent(const char *axis, int64_t x0, int64_t n);
void octave_tables(const ptg_params *p, double *freq, float *amp);
int footprint_cap(const double *freq, int octaves, int extent);

// Kernel arguments of the general K3 for one field; return the dynamic LDS bytes.
size_t general_args_2d(const ptg_params *p, int64_t x0, int64_t y0, int64_t nx, int64_t ny, void *out,
                       int64_t pitch, int tile_h, Fbm2dArgs *a);
size_t general_args_3d(const ptg_params *p, int64_t x0, int64_t y0, int64_t z0, int64_t nx, int64_t ny, int64_t nz,
                       void *out, Fbm3dArgs *a);

// base_freq = 2^-k with lacunarity 2 and every octave within one cell per sample.
bool dyadic_shift(const ptg_params *p, int *k_out);
// Kernel arguments of the 2D strip kernel for a dyadic field (k from dyadic_shift);
// returns 1 when the strip kernel does not apply (a ladder it cannot take, too many keys).
int strip_args_2d(const ptg_params *p, int k, int64_t x0, int64_t y0, int64_t nx, int64_t ny, void *out,
                  int64_t pitch, Fbm2dStripArgs *a);

// Kernel arguments of the 3D strip kernel for a dyadic volume; returns 1 when it does not
// apply (a ladder starting below period 4, too many keys).
// ahead_all: period-2 plane slots for the period-2 planes hashed two ahead in every model
// (the dense kernel); otherwise in the gradient model only (a serving workgroup).
int strip3_args(const ptg_params *p, int k, int64_t x0, int64_t y0, int64_t z0, int64_t nx, int64_t ny, int64_t nz,
                void *out, Fbm3dStripArgs *a, bool ahead_all = false);

// ---- tile-shape tuning (a6) -----------------------------------------------------
// A launch class: which kernel a call runs (PTG_TUNE_*), its cell order, output type,
// size class (ceil log2 of the samples) and ladder class (finest period, log2, capped).
struct TuneKey {
    int32_t kernel, smooth, f16, size_class, ladder;
    bool operator<(const TuneKey &o) const;
};
// The shape a launch of class k uses: the value forced by the tuner on this thread, else
// the recorded choice, else dflt.  Also remembers k and dflt as this thread's last class.
int tune_pick(const TuneKey &k, int dflt);
// Dry run on this thread: the drivers choose their kernel and shape, then return PTG_OK
// without launching (tune queries); and the value the tuner forces (0 = none).
bool tune_dry();
// Scope of one tuned or queried call on this thread (not nestable).
struct TuneScope {
    TuneScope(bool dry, int force);
    ~TuneScope();
    bool picked() const;  // a driver chose its class inside the scope
    TuneKey key() const;  // the class it chose
    int value() const;    // and the shape it used
    int dflt() const;     // and the shape it uses untuned
};
int size_class(int64_t samples);
int ladder_class(const double *freq, int octaves);

// Dense-field drivers (arguments already validated, field non-empty).
int fbm2d_plain(const ptg_params *p, int64_t x0, int64_t y0, int64_t nx, int64_t ny, void *out, int64_t pitch,
                hipStream_t s);
int fbm3d_plain(const ptg_params *p, int64_t x0, int64_t y0, int64_t z0, int64_t nx, int64_t ny, int64_t nz,
                void *out, hipStream_t s);
int fbm2d_mfma(const ptg_params *p, int64_t x0, int64_t y0, int64_t nx, int64_t ny, void *out, int64_t pitch,
               hipStream_t s);
int fbm2d_grad(const ptg_params *p, int64_t x0, int64_t y0, int64_t nx, int64_t ny, void *out, void *out_dx,
               void *out_dy, int64_t pitch, hipStream_t s);

}  // namespace ptg
