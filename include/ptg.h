/*
 * ptg.h -- C ABI of libptg: polynomial gradient-noise fBm on AMD Instinct MI355X (gfx950).
 *
 * Method: Thorimbert & Chopard, "Polynomial methods for fast Procedural Terrain
 * Generation" (arXiv:1610.03525).  Per octave the library
 *   a1. maps every sample to a lattice cell and a local fraction (FP64 coordinate step),
 *   a2. hashes the lattice nodes to unit gradients (K1),
 *   a3. forms each cell's boundary-constrained polynomial from its corner gradients (K2;
 *       Sec. 2, eqs. mixedderiv / independance / polynomial; Sec. 3.1, 3.4),
 *   a4. evaluates that polynomial at every sample (K3), and
 *   a5. accumulates the octaves with amplitude p^o and frequency f0 * L^o (Sec. 4).
 *
 * Conventions (the readings taken where the paper is silent):
 *   - Cell polynomial: tensor polynomial of degree n = 2M+1 per axis (M = smoothness)
 *     whose value is 0 at each corner, whose gradient equals the corner's lattice
 *     gradient, and whose other mixed derivatives h^d, 0 <= d_k <= M, are 0.  M = 1 gives
 *     C1 cubic cells (D2M1N3 / D3M1N3 with zero twist), M = 2 C2 quintic cells, M = 3
 *     C3 septic cells, up to M = 6; the 1D bases of any M are the closed forms of
 *     two-point Taylor interpolation, S(t) = t^(M+1) sum_{k<=M} C(M+k,k) (1-t)^k,
 *     b10(t) = t (1-t)^(M+1) sum_{k<M} C(M+k,k) t^k, b11(t) = -b10(1-t).  Two more cell models (ptg_params.model): the zero-gradient
 *     model (2D), whose nodes carry heights and zero gradients (Sec. 3.3), and the
 *     height-and-gradient model (2D and 3D), whose nodes carry both (Sec. 3.1; D3M1N3 of
 *     Sec. 3.4 with heights; gradient weight w, Sec. 4).
 *   - Optional output: the analytic gradient of the field (ptg_fbm_2d_grad, Sec. 5.1).
 *   - Octave o = 0..N-1: frequency f_o = base_freq * lacunarity^o and amplitude
 *     a_o = persistence^o, each by repeated FP64 multiplication; no normalisation.
 *   - Sample at int64 world index X sits at X + 1/2: u = (X + 1/2) * f_o (FP64),
 *     cell = floor(u), fraction t = u - cell rounded to FP32.
 *   - Lattice hash (all arithmetic mod 2^32), fmix32 = MurmurHash3 finalizer:
 *       prefix  = fmix32(fmix32(seed ^ 0x9E3779B9) ^ octave)
 *       line(k, i) = fmix32(fmix32(k ^ lo32(i)) ^ hi32(i))      (i as two's complement)
 *       key2    = fmix32(line(prefix, iy) ^ line(0x27D4EB2F, ix))
 *       key3    = fmix32(line(line(prefix, iz), iy) ^ line(0x27D4EB2F, ix))
 *       second3 = fmix32(key3 ^ 0x165667B1)
 *     2D gradient: angle 2*pi*(key >> 8)/2^24.  3D gradient: z = 1 - (2*(key>>8)+1)/2^24,
 *     azimuth 2*pi*(second3 >> 8)/2^24, radius sqrt(1 - z^2).
 *
 * Memory: every `void *` buffer argument named *_dev is device memory (e.g. a torch CUDA
 * tensor's data_ptr on ROCm) owned by the caller; `stream` is a hipStream_t (NULL = the
 * default stream).  Calls are asynchronous on that stream unless stated otherwise.
 * Errors: every entry point returns PTG_OK (0) or a negative PTG_E* code.  All argument
 * checks happen before any launch, so a rejected call writes nothing.  The message of
 * the last failure on the calling thread is returned by ptg_last_error().  No C++
 * exception crosses this interface.
 */
#ifndef PTG_H
#define PTG_H

#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define PTG_API __attribute__((visibility("default")))
#else
#define PTG_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------------ */
#define PTG_OK 0
#define PTG_EINVAL (-1)     /* an argument is out of range or a pointer is NULL        */
#define PTG_ENOMEM (-2)     /* a device or host allocation failed                      */
#define PTG_E2BIG (-3)      /* a request is larger than the whole serving budget       */
#define PTG_EAGAIN (-4)     /* non-blocking submit: no room now                        */
#define PTG_ETIMEDOUT (-5)  /* wait timed out; the request is still pending            */
#define PTG_ESHUTDOWN (-6)  /* server is shutting down / was destroyed                 */
#define PTG_EHIP (-7)       /* a HIP runtime call failed (text in ptg_last_error)      */
#define PTG_ENOENT (-8)     /* unknown or already released ticket                      */

/* ---- limits ------------------------------------------------------------------ */
#define PTG_MAX_OCTAVES 16
#define PTG_MAX_SMOOTHNESS 6 /* cell order M: derivatives up to M prescribed, degree 2M+1   */
/* |world index| + extent must stay below 2^52 so X + 1/2 is exact in FP64 */
#define PTG_MAX_WORLD_ABS 4503599627370496LL

/* ---- output element types ---------------------------------------------------- */
#define PTG_F32 0
#define PTG_F16 1

/* ---- evaluation forms -------------------------------------------------------- */
#define PTG_FORM_PLAIN 0      /* FP32 VALU evaluation, any parameters                  */
#define PTG_FORM_MFMA_F16 1   /* 2D only: V_x C V_y^T on FP16 MFMA, FP32 accumulate    */
#define PTG_FORM_MFMA_BF16 2  /* 2D only: same on BF16 MFMA                            */

/* ---- kernel choice for the plain form ----------------------------------------- */
#define PTG_PATH_AUTO 0     /* dyadic kernel when it applies, else the general kernel    */
#define PTG_PATH_GENERAL 1  /* any base frequency / lacunarity / origin                  */
#define PTG_PATH_DYADIC 2   /* base_freq = 2^-k (k <= 22), lacunarity = 2 (in 3D the     */
                            /* ladder must also start at period >= 4 when it reaches   */
                            /* period 4); PTG_EINVAL when the parameters are otherwise  */

/* ---- bases for the MFMA forms (Vandermonde rows fed to the matrix cores) ------ */
/* Every 4 rows x 64 columns of the field are one MFMA: per column the octaves of period */
/* >= 16 summed as one cubic per 16-row quarter, the period-8 cell and the period-4 cell */
/* holding the rows; the constant terms and the octaves of period 2 and 1 stay FP32.      */
#define PTG_BASIS_MONOMIAL 0  /* V(t) = [1, t, t^2, t^3], t = the cell's (quarter's) own  */
                              /* corner coordinate, C = monomial coefficients            */
#define PTG_BASIS_CENTRED 1   /* V(t) = [1, s, s^2, s^3] with s = t - 1/2 (centred)       */
#define PTG_BASIS_HERMITE 2   /* cells in their 1D Hermite bases [1, S, b10, b11] (C = the */
                              /* corner data itself); the quarter's cubic centred         */

/* ---- cell models ------------------------------------------------------------ */
#define PTG_MODEL_GRADIENT 0       /* value 0 and the lattice gradient at every corner     */
                                   /* (Sec. 2 with zero heights; C1 or C2 across faces)    */
#define PTG_MODEL_ZERO_GRADIENT 1  /* zero-gradient D2M1N3 (Sec. 3.3): a random height per */
                                   /* node (uniform on [-1, 1) from the node's key: top 24  */
                                   /* bits / 2^23 - 1), zero gradients at the corners;      */
                                   /* continuous across faces, its gradient pinned at the   */
                                   /* nodes only.  2D, smoothness 1, plain form; fields and  */
                                   /* served tiles                                          */
#define PTG_MODEL_HEIGHT_GRADIENT 2 /* tensor Hermite cells with a random height per node    */
                                   /* (uniform on [-1, 1): in 2D from the node's second     */
                                   /* hash word, in 3D from its third, fmix32(second3 ^     */
                                   /* 0x165667B1)) and the lattice gradient times           */
                                   /* gradient_weight w (Sec. 3.1 heights, Sec. 3.4, Sec. 4 */
                                   /* w); C1 / C2 / C3 across faces.  2D and 3D, plain     */
                                   /* form; fields and served tiles                         */

#define PTG_MODEL_PERLIN 3          /* comparison path: Perlin's gradient noise (Sec. 3.2)  */
                                   /* on the same hashed unit gradients, corner            */
                                   /* contributions g . (t - c) blended with the fade S3    */
                                   /* (smoothness 1) or S5 (smoothness 2).  2D, plain form, */
                                   /* general kernel, fields only (not served)              */
#define PTG_MODEL_SIMPLEX 4         /* comparison path standing for the paper's OpenSimplex  */
                                   /* timings (Sec. 5.2; the paper does not define it):     */
                                   /* 2D simplex-lattice gradient noise written from its    */
                                   /* public mathematical description -- skew (sqrt3-1)/2,  */
                                   /* unskew (3-sqrt3)/6, corner kernel max(0, 1/2 -        */
                                   /* |d|^2)^4 (g . d), g the hashed unit gradient of the   */
                                   /* skewed index, sum x 70.  2D, smoothness 1, plain form, */
                                   /* fields only (not served)                              */

/* Problem parameters (Sec. 2.2 DdMmNn naming: dim = d, smoothness = m, n = 2m+1;
 * Sec. 4: octaves, persistence, lacunarity). */
typedef struct ptg_params {
    int32_t dim;          /* 2 or 3                                                    */
    int32_t smoothness;   /* M = 1 C1 cubic, 2 C2 quintic, 3 C3 septic .. 6 (C6, degree */
                          /* 13; Sec. 2.2 eq. nconstraints, the Conclusion's arbitrary  */
                          /* smoothness).  1, 2: every kernel; 3: the 2D strip and the  */
                          /* general kernels; 4..6: the general kernels.  Served tiles  */
                          /* take 1, 2; the matrix-core form 1; the gradient output 1..3 */
    int32_t octaves;      /* 1 .. PTG_MAX_OCTAVES                                      */
    int32_t out_dtype;    /* PTG_F32 or PTG_F16                                        */
    double persistence;   /* amplitude ratio per octave, finite, > 0                   */
    double lacunarity;    /* frequency ratio per octave, finite, > 0                   */
    double base_freq;     /* lattice cells per sample at octave 0, finite, > 0; every  */
                          /* octave's frequency must be <= 1 cell per sample           */
    uint32_t seed;        /* lattice seed                                              */
    int32_t form;         /* PTG_FORM_*                                                */
    int32_t basis;        /* PTG_BASIS_* (MFMA forms only)                             */
    int32_t path;         /* PTG_PATH_*: kernel choice for the plain form              */
    int32_t model;        /* PTG_MODEL_*                                               */
    double gradient_weight; /* w of PTG_MODEL_HEIGHT_GRADIENT (finite; default 0.01, the */
                          /* paper's h0 / 100 with h0 = 1); ignored by the other models */
} ptg_params;

/* Library version string (static storage). */
PTG_API const char *ptg_version(void);

/* Message of the last failing call on this thread ("" if none).  Thread-local storage,
 * valid until the next failing call on the same thread. */
PTG_API const char *ptg_last_error(void);

/* Fill a ptg_params with the defaults: dim 2, smoothness 1, 8 octaves, persistence 0.5,
 * lacunarity 2, base_freq 1/512, seed 1, FP32, plain form, gradient model (w = 0.01). */
PTG_API void ptg_params_default(ptg_params *p);

/* ---- a1-a5: dense fields ----------------------------------------------------- */

/* 2D fBm heightmap H(X, Y) = sum_o a_o h_o((X+1/2) f_o, (Y+1/2) f_o) for the samples
 * X = x0 + i, Y = y0 + j, 0 <= i < nx, 0 <= j < ny (Sec. 4 octave sum of Sec. 2 cells).
 * out_dev: device buffer of element type p->out_dtype, row-major; sample (i, j) at
 *   out_dev[j * row_pitch + i]; row_pitch >= nx (elements).  nx or ny == 0 is a no-op.
 * p->dim must be 2.  Asynchronous on `stream`.
 * Errors: PTG_EINVAL (bad parameters, NULL out_dev with a non-empty field, |x0|, |x0+nx|,
 *   |y0| or |y0+ny| >= PTG_MAX_WORLD_ABS, an MFMA form with smoothness 2 or dim 3),
 *   PTG_ENOMEM (workspace), PTG_EHIP (launch failure). */
PTG_API int ptg_fbm_2d(const ptg_params *p, int64_t x0, int64_t y0, int64_t nx, int64_t ny,
               void *out_dev, int64_t row_pitch, void *stream);

/* The 2D field of ptg_fbm_2d and its analytic gradient (the gradient maps of Sec. 5.1):
 * out_dev[j*row_pitch + i] = H(X, Y), dx_dev[...] = dH/dX, dy_dev[...] = dH/dY in world
 * units (per sample: sum_o a_o f_o dh_o/dt), the three buffers of p->out_dtype with the same
 * layout.  The cell models at smoothness 1..3; plain form.  Dyadic ladders that the strip
 * kernel takes (p->path not PTG_PATH_GENERAL) run one strip launch for the three outputs
 * (out_dev bit-identical to ptg_fbm_2d's strip launch).  Other ladders, and p->path ==
 * PTG_PATH_GENERAL, run the general kernel, which writes the three in one pass.
 * Errors: as ptg_fbm_2d (PTG_EINVAL also for a NULL output or a matrix-core form). */
PTG_API int ptg_fbm_2d_grad(const ptg_params *p, int64_t x0, int64_t y0, int64_t nx, int64_t ny, void *out_dev,
                    void *dx_dev, void *dy_dev, int64_t row_pitch, void *stream);

/* 3D fBm volume over X = x0+i, Y = y0+j, Z = z0+k; out_dev dense row-major
 * [nz][ny][nx] of p->out_dtype (D3M1N3 / D3M2N5 cells, Sec. 3.4).  p->dim must be 3 and
 * p->form PTG_FORM_PLAIN.  Errors as ptg_fbm_2d. */
PTG_API int ptg_fbm_3d(const ptg_params *p, int64_t x0, int64_t y0, int64_t z0, int64_t nx, int64_t ny,
               int64_t nz, void *out_dev, void *stream);

/* ---- stage entry points (the same device code the fields run, exposed per stage) */

/* a1. Coordinate step (Sec. 4: octave o at frequency base_freq * lacunarity^o, by repeated
 * FP64 multiplication) for n consecutive world samples x0 .. x0+n-1 and octaves
 * 0 .. octaves-1, each sample at its centre: u = (X + 1/2) f_o in FP64, cell = floor(u),
 * fraction u - cell: cells_dev[o*n + i] (int64) and frac_dev[o*n + i] (float, rounded to
 * nearest).  Device buffers of octaves*n entries, owned by the caller.
 * Errors: PTG_EINVAL, PTG_EHIP. */
PTG_API int ptg_coords(double base_freq, double lacunarity, int32_t octaves, int64_t x0, int64_t n,
               int64_t *cells_dev, float *frac_dev, void *stream);

/* a2. K1 for the zero-gradient model (Sec. 3.3, random node heights): node heights of the node box
 * ix0 <= ix < ix0+nx, iy0 <= iy < iy0+ny of octave `octave`, heights_dev[j*nx + i]
 * (FP32, exact: top 24 key bits / 2^23 - 1).  Errors: PTG_EINVAL, PTG_EHIP. */
PTG_API int ptg_heights_2d(uint32_t seed, int32_t octave, int64_t ix0, int64_t iy0, int64_t nx, int64_t ny,
                   float *heights_dev, void *stream);

/* a2. K1 lattice kernel, 2D (Sec. 3.2: the grid of random gradients each octave's cells
 * interpolate; the hash and the gradient map are stated above): for the node box
 * ix0 <= ix < ix0+nx, iy0 <= iy < iy0+ny of octave `octave`: keys_dev[j*nx + i] (uint32,
 * may be NULL) and the unit gradient,
 * SoA: grad_dev[j*nx + i] = x component, grad_dev[nx*ny + j*nx + i] = y component
 * (may be NULL).  Errors: PTG_EINVAL (negative sizes, octave < 0), PTG_EHIP. */
PTG_API int ptg_lattice_2d(uint32_t seed, int32_t octave, int64_t ix0, int64_t iy0, int64_t nx,
                   int64_t ny, uint32_t *keys_dev, float *grad_dev, void *stream);

/* a2. K1, 3D (Sec. 3.2 lattice, Sec. 3.4 D3 cells): node box of nx*ny*nz nodes, index
 * q = (k*ny + j)*nx + i; keys_dev[q], second words second_dev[q] (may be NULL), unit
 * gradients SoA grad_dev[c*nx*ny*nz + q] (may be NULL).  Device buffers owned by the
 * caller.  Errors: PTG_EINVAL (negative sizes, octave < 0), PTG_EHIP. */
PTG_API int ptg_lattice_3d(uint32_t seed, int32_t octave, int64_t ix0, int64_t iy0, int64_t iz0,
                   int64_t nx, int64_t ny, int64_t nz, uint32_t *keys_dev, uint32_t *second_dev,
                   float *grad_dev, void *stream);

/* a3. K2 per-cell coefficient kernel, 2D (Sec. 2.2, the cell's polynomial from its corner
 * constraints): from a node-gradient box in the layout K1
 * writes (nnx*nny nodes, SoA), the monomial coefficients c_ij of h = sum c_ij x^i y^j
 * (eq. polynomial, D = 2, n = 2*smoothness+1) of every cell of the box:
 * coeff_dev[(cj*(nnx-1) + ci)*(n+1)^2 + i*(n+1) + j], scaled by `amplitude`.
 * Each workgroup stages its corner gradients in LDS.  nnx, nny >= 2.
 * Errors: PTG_EINVAL, PTG_EHIP. */
PTG_API int ptg_cells_2d(int32_t smoothness, const float *grad_dev, int64_t nnx, int64_t nny,
                 float amplitude, float *coeff_dev, void *stream);

/* a3. K2, 3D (Sec. 2.2, Sec. 3.4): coefficient c_ijk of x^i y^j z^k at
 * coeff_dev[cell*(n+1)^3 + (i*(n+1) + j)*(n+1) + k], cell = (ck*(nny-1) + cj)*(nnx-1) + ci. */
PTG_API int ptg_cells_3d(int32_t smoothness, const float *grad_dev, int64_t nnx, int64_t nny,
                 int64_t nnz, float amplitude, float *coeff_dev, void *stream);

/* ---- a6: tile-shape autotuner ------------------------------------------------
 * Each dense-field call runs one kernel class; some classes have a free launch shape that
 * changes neither the arithmetic nor the result (every sample is computed by the same
 * operations whatever the shape):
 *   PTG_TUNE_GENERAL_2D  general 2D kernel: tile height in rows, 16, 32, 64 or 128 (tiles
 *                        are 64 wide; served tiles take at most 64); a shorter tile hashes
 *                        more duplicated footprint nodes and repeats each octave's set-up
 *                        more often, but gives small fields more workgroups (untuned: 128
 *                        for fields of 1024 rows or more, except the height-and-gradient
 *                        model, else 64);
 *   PTG_TUNE_STRIP_2D    dyadic 2D kernel (64 x 64 strips, one per wave): waves per
 *                        workgroup, 1, 2 or 4;
 *   PTG_TUNE_STRIP_3D    dyadic 3D kernel (64 x 8 x 16 blocks, one per wave): waves per
 *                        workgroup, 1, 2 or 4;
 *   PTG_TUNE_GENERAL_3D, PTG_TUNE_DYADIC_2D (precision forms, dyadic 2D tiles): fixed.
 * A class is keyed by (kernel, smoothness, output type, ceil(log2(samples)), ladder class:
 * log2 of the finest period for the dyadic kernels, of 1 / the largest frequency, capped
 * at 8, for the general ones).  The library keeps one table per process (thread-safe);
 * untuned classes use the defaults (64 rows, 4 waves). */
#define PTG_TUNE_GENERAL_2D 1
#define PTG_TUNE_STRIP_2D 2
#define PTG_TUNE_GENERAL_3D 3
#define PTG_TUNE_STRIP_3D 4
#define PTG_TUNE_DYADIC_2D 5
#define PTG_TUNE_MAX_CANDIDATES 4

typedef struct ptg_tune_result {
    int32_t kernel;          /* PTG_TUNE_* class the call runs                          */
    int32_t value;           /* shape now recorded for it (0: nothing to tune)          */
    int32_t n;               /* candidates timed (1 when the class has no free shape)   */
    int32_t default_value;   /* the untuned shape                                       */
    int32_t candidates[PTG_TUNE_MAX_CANDIDATES];
    double us[PTG_TUNE_MAX_CANDIDATES]; /* mean launch time of each candidate, us       */
} ptg_tune_result;

/* Time every candidate shape of the class that ptg_fbm_2d(p, x0, y0, nx, ny, out_dev,
 * row_pitch, stream) runs (one warm-up, then `reps` back-to-back launches bracketed by HIP
 * events, per candidate; reps <= 0 means 5), record the fastest for that class and fill
 * *res.  out_dev receives the field (every candidate writes the same values).  Synchronous:
 * returns after the timings.  Errors: as ptg_fbm_2d, PTG_EINVAL for a NULL res. */
PTG_API int ptg_tune_2d(const ptg_params *p, int64_t x0, int64_t y0, int64_t nx, int64_t ny, void *out_dev,
                        int64_t row_pitch, void *stream, int32_t reps, ptg_tune_result *res);
PTG_API int ptg_tune_3d(const ptg_params *p, int64_t x0, int64_t y0, int64_t z0, int64_t nx, int64_t ny,
                        int64_t nz, void *out_dev, void *stream, int32_t reps, ptg_tune_result *res);

/* The class and shape a call with these parameters and extents would use now, without
 * launching anything (host only; origins do not affect the choice).  *kernel and *value
 * as in ptg_tune_result.  Errors: PTG_EINVAL (parameters, NULL outputs). */
PTG_API int ptg_tune_query_2d(const ptg_params *p, int64_t nx, int64_t ny, int32_t *kernel, int32_t *value);
PTG_API int ptg_tune_query_3d(const ptg_params *p, int64_t nx, int64_t ny, int64_t nz, int32_t *kernel,
                              int32_t *value);

/* Record a shape for the class of such a call (e.g. one tuned in an earlier process).
 * Errors: PTG_EINVAL (parameters, or value not a candidate of the class). */
PTG_API int ptg_tune_set_2d(const ptg_params *p, int64_t nx, int64_t ny, int32_t value);
PTG_API int ptg_tune_set_3d(const ptg_params *p, int64_t nx, int64_t ny, int64_t nz, int32_t value);

/* Forget every recorded shape. */
PTG_API void ptg_tune_reset(void);

/* Persist the recorded shapes: a text file whose first line names the current device
 * (architecture name and compute-unit count; "none" without a device), then one line per
 * class.  ptg_tune_load adds the file's shapes to the table when it was written for the
 * same device, and skips it otherwise (*loaded, optional, receives the number of shapes
 * taken: 0 for another device).  Errors: PTG_EINVAL (NULL path, not a table, a malformed
 * or invalid entry: nothing is taken), PTG_ENOENT (the file cannot be opened or written). */
PTG_API int ptg_tune_save(const char *path);
PTG_API int ptg_tune_load(const char *path, int32_t *loaded);

/* ---- a6: HIP-graph batches of dense fields ------------------------------------
 * A batch collects dense-field calls -- the one kernel launch each ptg_fbm_2d / ptg_fbm_3d
 * call makes, with its arguments -- and launches them together as the kernel nodes of one
 * HIP graph (the plain path of the tile stream, or a terrain engine's per-frame tile set).
 * The graph of a batch shape (the same kernels with the same workgroup sizes in the same
 * order) is instantiated once; a later batch of that shape updates the instance's kernel
 * nodes in place (grid, dynamic LDS size and arguments, hipGraphExecKernelNodeSetParams) and
 * relaunches it, e.g. tiles of other sizes at new origins, seeds or output buffers; if the
 * runtime refuses an update the instance is instantiated again.  Up to 4 instances of a shape are
 * kept so that no instance is updated while a launch of it may still run; up to 64 shapes
 * per batch object are cached, the least recently used dropped first.  The calls of one
 * batch may run concurrently: their outputs must not overlap.  A batch object is used by
 * one thread at a time.  Results equal the direct calls bit for bit (same kernels, same
 * arguments). */
typedef struct ptg_batch ptg_batch;

typedef struct ptg_batch_stats {
    int64_t launches;        /* graph launches                                              */
    int64_t nodes;           /* kernel nodes launched (dense-field calls)                   */
    int64_t instantiations;  /* graphs instantiated (new shapes, or a 2nd..4th instance)    */
    int64_t updates;         /* launches that reused an instance with updated arguments     */
    int64_t instances;       /* instances cached now                                        */
    int64_t pending;         /* calls recorded and not launched yet                         */
} ptg_batch_stats;

/* A batch of at most max_calls (1..4096) calls.  Errors: PTG_EINVAL, PTG_ENOMEM. */
PTG_API int ptg_batch_create(int32_t max_calls, ptg_batch **out);

/* Record the launch of ptg_fbm_2d(p, x0, y0, nx, ny, out_dev, row_pitch, -) (validated as
 * that call; an empty field records nothing).  Nothing runs until ptg_batch_launch.
 * Errors: as ptg_fbm_2d, PTG_EINVAL when the batch is full. */
PTG_API int ptg_batch_add_2d(ptg_batch *b, const ptg_params *p, int64_t x0, int64_t y0, int64_t nx, int64_t ny,
                             void *out_dev, int64_t row_pitch);
/* The same for ptg_fbm_3d. */
PTG_API int ptg_batch_add_3d(ptg_batch *b, const ptg_params *p, int64_t x0, int64_t y0, int64_t z0, int64_t nx,
                             int64_t ny, int64_t nz, void *out_dev);

/* Launch the recorded calls as one graph on `stream` (asynchronous; may wait for an earlier
 * launch of the same shape when all 4 of its instances are in flight) and empty the batch.
 * An empty batch is a no-op.  Errors: PTG_EINVAL, PTG_EHIP (the recorded calls are
 * dropped). */
PTG_API int ptg_batch_launch(ptg_batch *b, void *stream);

/* Drop the recorded calls without launching them. */
PTG_API int ptg_batch_clear(ptg_batch *b);

PTG_API int ptg_batch_stats_get(const ptg_batch *b, ptg_batch_stats *st);

/* Wait for the batch's graph launches to finish and free everything. */
PTG_API int ptg_batch_destroy(ptg_batch *b);

/* ---- a6: serving (continuous batching of terrain tiles) ----------------------- */
/* A server owns an output arena of hbm_budget_bytes and one persistent kernel.  Requests
 * (terrain tiles of any size, 2D or 3D, any octave parameters, FP32 output, plain form, the
 * gradient or height-and-gradient cells at C1, C2 or C3 or the zero-gradient cells (2D C1);
 * not the comparison paths) are
 * queued by ptg_tiles_submit, admitted while arena bytes and request slots are free, cut
 * into work items and published into a ring that the persistent kernel's workgroups drain
 * while earlier requests are still running.  A 2D request whose ladder is dyadic (base_freq
 * 2^-k, lacunarity 2, finest period >= 2) and whose 64 x 64 strip footprint fits a serving
 * workgroup runs as strips, one per wave, with the same device code as ptg_fbm_2d with
 * PTG_PATH_DYADIC; a 3D C1 / C2 request with a dyadic ladder of finest period >= 2 whose
 * footprint fits runs as 64 x 8 x 16 blocks with the device code of ptg_fbm_3d with
 * PTG_PATH_DYADIC; every other request runs
 * as 64 x tile_h (2D) or 64 x 8 x 8 (3D) sample tiles with the device code of
 * PTG_PATH_GENERAL.  A served tile equals the corresponding stand-alone call bit for bit
 * (ptg_tile_result.kernel says which).  With cfg->lattice_cache the general 2D tiles read
 * their node gradients (the K1 output of ptg_lattice_2d) from blocks cached in the arena
 * across requests of the same seed. */

typedef struct ptg_server ptg_server;

#define PTG_EXEC_GPU 0   /* persistent kernel on cfg->device                             */
#define PTG_EXEC_HOST 1  /* test-only: no GPU; each tile "completes" after fake_tile_ns   */
                         /* on a host thread and the arena is host memory (outputs are   */
                         /* not computed): admission, budget and shutdown logic only     */

typedef struct ptg_server_cfg {
    int64_t hbm_budget_bytes; /* output arena (owned by the server), > 0                   */
    int32_t max_items;        /* work-item ring entries, >= 64                              */
    int32_t workgroups;       /* persistent workgroups, 0 = 1 per compute unit              */
    int32_t device;           /* HIP device ordinal                                         */
    int32_t executor;         /* PTG_EXEC_GPU or PTG_EXEC_HOST                              */
    int64_t fake_tile_ns;     /* PTG_EXEC_HOST only: simulated time per tile                */
    int32_t tiles_per_item;   /* sample tiles per work item, 1..16 (strip requests: 4 strips */
                              /* or 3D blocks per tile, one per wave); 0 = from the load:   */
                              /* the tiles in flight and pending plus the request's own     */
                              /* (enough items for every workgroup, at most 16 tiles)       */
    int32_t autotune;         /* 1: at creation (PTG_EXEC_GPU) time the 2D tile heights on  */
                              /* a 512 x 512, 8-octave field per cell order (ptg_tune_2d,   */
                              /* general kernel; needs a budget >= 1 MiB) and use the best  */
    int32_t tile_h;           /* 2D tile height in rows: 16, 32 or 64; 0 = the tuned one    */
                              /* (autotune), else 64.  3D tiles are 64 x 8 x 8              */
    int32_t lattice_cache;    /* 1: device-resident lattice cache for 2D requests served as */
                              /* general tiles: the FP32 node gradients of each octave in    */
                              /* blocks of 32 x 32 nodes keyed by (seed, octave, block),     */
                              /* 8 KiB each in the arena (counted in the budget).  A request */
                              /* references the blocks of its footprint at admission; the    */
                              /* missing ones are first filled by the persistent kernel (K1),*/
                              /* then its tiles read the gradients instead of hashing them   */
                              /* (same results bit for bit).  Blocks stay resident after     */
                              /* use and are evicted, least recently used first, when arena  */
                              /* bytes are needed.  Requests whose footprint needs more than */
                              /* 2048 blocks hash.  Budget at most 1 TiB.  0: no cache       */
} ptg_server_cfg;

typedef struct ptg_tile_req {
    ptg_params params;        /* dim 2 or 3, PTG_FORM_PLAIN, PTG_F32; path is ignored       */
    int64_t origin[3];        /* world sample index of element (0,0,0); origin[2] = 0 in 2D */
    int64_t extent[3];        /* nx, ny, nz >= 1; nz = 1 in 2D                              */
    uint64_t user_tag;        /* returned unchanged                                         */
} ptg_tile_req;

typedef struct ptg_tile_result {
    int32_t status;           /* PTG_OK, PTG_ESHUTDOWN or PTG_EHIP                          */
    int32_t kernel;           /* code that computed it: PTG_TUNE_STRIP_2D / _STRIP_3D (the  */
                              /* dyadic strip code; equals ptg_fbm_2d / _3d with            */
                              /* PTG_PATH_DYADIC bit for bit), PTG_TUNE_GENERAL_2D / _3D     */
                              /* (equals PTG_PATH_GENERAL)                                   */
    void *out_dev;            /* the tile, dense row-major FP32 [nz][ny][nx], valid until   */
                              /* ptg_tile_release (device memory; host memory for           */
                              /* PTG_EXEC_HOST)                                              */
    int64_t bytes;
    uint64_t user_tag;
    int64_t t_submit_ns, t_admit_ns, t_done_ns; /* steady clock, ns                         */
} ptg_tile_result;

/* Create a server: allocates the arena, the pinned work-item ring and request table, and
 * starts the scheduler thread; the persistent kernel runs on a stream of its own, is
 * launched when work is published and it is not running, and is parked (its workgroups
 * leave) after 5 ms with nothing in flight.  A device-wide synchronisation (e.g.
 * hipDeviceSynchronize) therefore returns only once the server's in-flight work is done
 * and the kernel has parked; synchronise streams instead where that matters.
 * Errors: PTG_EINVAL, PTG_ENOMEM, PTG_EHIP. */
PTG_API int ptg_server_create(const ptg_server_cfg *cfg, ptg_server **out);

/* Queue n requests (thread-safe, never blocks); tickets_out[i] receives request i's
 * ticket.  Admission is in arrival order, except that a request that does not fit the
 * free arena bytes yet lets later ones pass until it has waited 50 ms.
 * Errors (none of the n is queued): PTG_EINVAL (a request fails validation), PTG_E2BIG (a
 * request's output exceeds the whole budget), PTG_ESHUTDOWN. */
PTG_API int ptg_tiles_submit(ptg_server *s, const ptg_tile_req *reqs, int32_t n, uint64_t *tickets_out);

/* Wait up to timeout_ns (0: poll, < 0: forever) for a ticket and fill *res.
 * Errors: PTG_ETIMEDOUT (still pending), PTG_ENOENT (unknown or released ticket),
 * PTG_EAGAIN (the request cannot be admitted until the caller releases completed outputs:
 * it is pending, nothing is in flight, and the arena bytes it needs are held by completed
 * requests not yet released -- reported once that state has lasted a few milliseconds;
 * release some, then wait again). */
PTG_API int ptg_tiles_wait(ptg_server *s, uint64_t ticket, int64_t timeout_ns, ptg_tile_result *res);

/* Wait up to timeout_ns (0: poll, < 0: forever) for the next request to complete, in
 * completion order, whatever its ticket: *ticket_out and *res receive it.  Each completion
 * is returned once (completions released through ptg_tile_release before they were
 * returned are skipped); the ticket stays valid for ptg_tiles_wait and ptg_tile_release.
 * Errors: PTG_ETIMEDOUT (none completed in time), PTG_ENOENT (no request is pending or in
 * flight: nothing can complete), PTG_EAGAIN (the pending requests wait for arena bytes held
 * by completed outputs that have not been released; as for ptg_tiles_wait). */
PTG_API int ptg_tiles_wait_any(ptg_server *s, int64_t timeout_ns, uint64_t *ticket_out, ptg_tile_result *res);

/* Return a completed ticket's arena bytes to the server (its out_dev becomes invalid).
 * Errors: PTG_ENOENT, PTG_EAGAIN (not complete yet). */
PTG_API int ptg_tile_release(ptg_server *s, uint64_t ticket);

typedef struct ptg_server_stats {
    int64_t submitted, admitted, completed, released;
    int64_t tiles_done;       /* sample tiles (or strips / 3D blocks) finished              */
    int64_t pending, in_flight;
    int64_t bytes_in_use, bytes_peak, budget;
    int64_t kernel_launches;  /* persistent-kernel launches (it exits after idling)         */
    int32_t tile_h[2];        /* 2D tile height used for C1 / C2 requests                    */
    int64_t lat_blocks;       /* lattice-cache blocks resident (referenced or not)           */
    int64_t lat_bytes;        /* their arena bytes (part of bytes_in_use)                    */
    int64_t lat_hits;         /* blocks admitted requests found resident                     */
    int64_t lat_misses;       /* blocks admitted requests had to fill                        */
    int64_t lat_evictions;    /* unreferenced blocks freed for other allocations             */
} ptg_server_stats;

PTG_API int ptg_server_stats_get(ptg_server *s, ptg_server_stats *st);

/* Stop admitting; queued requests complete with PTG_ESHUTDOWN, admitted ones run to the
 * end; then the kernel is stopped and everything is freed (outputs of unreleased tickets
 * too).  s is invalid afterwards. */
PTG_API int ptg_server_destroy(ptg_server *s);

#ifdef __cplusplus
}
#endif
#endif /* PTG_H */
