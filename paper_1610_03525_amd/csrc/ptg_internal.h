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
                       int64_t pitch, Fbm2dArgs *a);
size_t general_args_3d(const ptg_params *p, int64_t x0, int64_t y0, int64_t z0, int64_t nx, int64_t ny, int64_t nz,
                       void *out, Fbm3dArgs *a);

// Dense-field drivers (arguments already validated, field non-empty).
int fbm2d_plain(const ptg_params *p, int64_t x0, int64_t y0, int64_t nx, int64_t ny, void *out, int64_t pitch,
                hipStream_t s);
int fbm3d_plain(const ptg_params *p, int64_t x0, int64_t y0, int64_t z0, int64_t nx, int64_t ny, int64_t nz,
                void *out, hipStream_t s);
int fbm2d_mfma(const ptg_params *p, int64_t x0, int64_t y0, int64_t nx, int64_t ny, void *out, int64_t pitch,
               hipStream_t s);

}  // namespace ptg
