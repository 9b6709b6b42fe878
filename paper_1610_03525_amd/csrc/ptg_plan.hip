// ptg_plan.hip -- octave plan and kernel choice for the dense fields.
#include <algorithm>

#include "ptg_internal.h"
#include "ptg_launch.h"

namespace ptg {

int fbm2d_plain(const ptg_params *p, int64_t x0, int64_t y0, int64_t nx, int64_t ny, void *out, int64_t pitch,
                hipStream_t s)
{
    Fbm2dArgs a{};
    a.x0 = x0;
    a.y0 = y0;
    a.nx = nx;
    a.ny = ny;
    a.pitch = pitch;
    a.out = out;
    octave_tables(p, a.freq, a.amp);
    a.octaves = p->octaves;
    a.seed = p->seed;
    a.capx = footprint_cap(a.freq, p->octaves, kTile2);
    a.capy = a.capx;
    a.tiles_x = (int32_t)((nx + kTile2 - 1) / kTile2);
    const size_t lds = (size_t)kTile2 * 16 + (size_t)a.capx * a.capy * 8 + (size_t)(a.capx + a.capy) * 4;
    hipError_t e = launch_fbm2d_general(a, p->smoothness, p->out_dtype == PTG_F16, lds, s);
    return e == hipSuccess ? PTG_OK : hip_fail(e, "fbm2d launch");
}

int fbm3d_plain(const ptg_params *p, int64_t x0, int64_t y0, int64_t z0, int64_t nx, int64_t ny, int64_t nz,
                void *out, hipStream_t s)
{
    Fbm3dArgs a{};
    a.x0 = x0;
    a.y0 = y0;
    a.z0 = z0;
    a.nx = nx;
    a.ny = ny;
    a.nz = nz;
    a.out = out;
    octave_tables(p, a.freq, a.amp);
    a.octaves = p->octaves;
    a.seed = p->seed;
    a.capx = footprint_cap(a.freq, p->octaves, kTile3X);
    a.capy = footprint_cap(a.freq, p->octaves, kTile3Y);
    a.capz = footprint_cap(a.freq, p->octaves, kTile3Z);
    a.tiles_x = (int32_t)((nx + kTile3X - 1) / kTile3X);
    a.tiles_y = (int32_t)((ny + kTile3Y - 1) / kTile3Y);
    const size_t lds = (size_t)(kTile3Y + kTile3Z) * 16 + (size_t)a.capx * a.capy * a.capz * 12 +
                       (size_t)(a.capx + a.capy * a.capz) * 4;
    hipError_t e = launch_fbm3d_general(a, p->smoothness, p->out_dtype == PTG_F16, lds, s);
    return e == hipSuccess ? PTG_OK : hip_fail(e, "fbm3d launch");
}

int fbm2d_mfma(const ptg_params *, int64_t, int64_t, int64_t, int64_t, void *, int64_t, hipStream_t)
{
    return fail(PTG_EINVAL, "matrix-core form not available in this build");
}

}  // namespace ptg
