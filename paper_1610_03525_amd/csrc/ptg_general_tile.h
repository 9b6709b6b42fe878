// ptg_general_tile.h -- K3 tile functions for any octave
// parameters (any base frequency, lacunarity, persistence, world origin).
//
// One workgroup owns a tile of samples; its 64 lanes of each wave own 64 consecutive
// columns (coalesced stores) and each wave walks a band of rows.  Per octave the
// workgroup
//   1. computes the tile's lattice footprint (first/last cell on each axis, FP64 step),
//   2. hashes every footprint node once into LDS (K1 logic: per-row / per-column key
//      prefixes, then one fmix32 per node), with the octave amplitude folded in,
//   3. tabulates the row (and slab) basis values of the tile in LDS,
//   4. and every lane forms, whenever its row band enters a new cell, the column form of
//      that cell's polynomial (K2 logic: the Hermite tensor form collapsed along x),
//      then evaluates one cubic / quintic per sample (3 FMA + 1 add) into registers.
// Octaves accumulate in registers; each sample is stored once.
//
// Cell polynomial (Sec. 2, Sec. 3.4): h = sum_corners [gx b1_cx(x) b0_cy(y) + gy b0_cx(x) b1_cy(y)]
// (2D) with b0_0 = 1 - s, b0_1 = s.  For a fixed column x it is the 1D Hermite form in y
//   h(y) = E0 + (E1 - E0) s(y) + Q0 b10(y) + Q1 b11(y),
//   E_cy = sum_cx gx_{cx,cy} b1_cx(x),   Q_cy = gy_{0,cy} + s(x) (gy_{1,cy} - gy_{0,cy}).
#pragma once

#include <hip/hip_fp16.h>

#include "ptg_device.h"
#include "ptg_launch.h"

namespace ptg {

template <typename T>
__device__ __forceinline__ T to_out(float v);
template <>
__device__ __forceinline__ float to_out<float>(float v)
{
    return v;
}
template <>
__device__ __forceinline__ __half to_out<__half>(float v)
{
    return __float2half_rn(v);
}

// Materialise v here, in program order.  Without it the compiler sinks every row's
// accumulate to the end of the octave and keeps all rows' column forms live across the
// row loop (2D tile of 64 rows: 174 VGPRs instead of 54, two waves per SIMD instead of
// eight).  The statement emits no instruction.
__device__ __forceinline__ void keep_here(float &v) { asm volatile("" : "+v"(v)); }
typedef float f32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ f32x4 load_here4(const float4 *p)
{
    f32x4 v = *reinterpret_cast<const f32x4 *>(p);
    asm volatile("" : "+v"(v));
    return v;
}

// Device-resident lattice cache (serving): the unit gradients of one octave's nodes in
// blocks of kLatBlk x kLatBlk nodes, SoA per block (x components at [(iy & 31) * 32 +
// (ix & 31)], y components kLatBlk^2 floats further), anywhere in the arena.  A request
// sees the blocks that cover its footprint as a table per octave: block (bx, by) =
// (ix >> 5, iy >> 5) is entry tbl0[o] + (by - by0[o]) * nbx[o] + (bx - bx0[o]), whose
// value is the block's arena offset in 256-byte units.  The blocks hold the K1 output for
// their nodes, so loading them gives the same gradients as hashing them.
constexpr int kLatBlkLog = 5;
constexpr int kLatBlk = 1 << kLatBlkLog;
constexpr int kLatBlkFloats = 2 * kLatBlk * kLatBlk;
struct LatCache {
    const char *base;       // arena
    const uint32_t *tbl;    // table entries (LDS copy)
    int32_t n;              // entries
    const int64_t *bx0, *by0;
    const int32_t *nbx, *tbl0;
};

// ---------------------------------------------------------------------------------
// 2D: tile 64 x TH samples (TH = 16, 32, 64 or 128 rows), 4 waves x TH/4 rows.
// LDS: row table float4[TH] | (GRAD) row-derivative table float4[TH] | every octave's
// footprint TileFoot[octaves] | gx[capx*capy] | gy[capx*capy] | (MD = 2) gh[capx*capy] |
// every octave's keys kx[octaves*capx] | ky[octaves*capy]
// ---------------------------------------------------------------------------------
// Once per tile: the octaves' footprints (one lane per octave, FP64) and the keys of their
// node columns and rows.  Per octave, between two barriers: the row table and the node
// block; then each wave's rows, where a ballot over the row table marks the rows that
// enter a new cell (a uniform bit test per row, no per-row lane-to-scalar move).
// MD = 1: the zero-gradient model (Sec. 3.3; M = 1): gx holds the node heights, and a
// cell at the lane's column x is E0 + dE S(y) + dQ (y - S(y)) with, per node row j,
// E_j = h0j + S(x) D_j, Q_j = (S(x) - x) D_j, D_j = h1j - h0j; y - S(y) = b10(y) + b11(y),
// so the row evaluation is the gradient model's with Q0 = Q1 = dQ.
// MD = 2: heights and w-weighted gradients (tensor Hermite): gh holds the heights, gx / gy
// the gradients times w, and a node row's value term gains h0j (1 - S(x)) + h1j S(x).
// MD = 3: Perlin's gradient noise (Sec. 3.2; the comparison path), fade S3 (M = 1) or S5
// (M = 2): v_c = g_c . (t - c), h = lerp_y(lerp_x(v00, v10, S(x)), lerp_x(v01, v11, S(x)), S(y)).
// At the lane's column h = a0 + a1 y + S(y) (b0 - b1 - a0) + S(y) y (b1 - a1) with
// h0 = a0 + a1 y and h1 = b0 + b1 (y - 1) the x-lerps of the node rows, so the row table
// holds (S(y), y, S(y) y) and the row evaluation keeps its shape.
// GRAD: also the analytic gradient dH/dX, dH/dY (to a.out_dx, a.out_dy): per octave the
// cell's derivatives in its local coordinates times the octave frequency; the x-derivative
// is the same row form with the x-bases differentiated, the y-derivative the row form with
// the row bases differentiated (a second row table in LDS).
struct TileFoot {  // one octave's lattice footprint over a tile: first node and node counts
    int64_t cxf, cyf;
    int32_t nnx, nny, pad0, pad1;
};
static_assert(sizeof(TileFoot) == kTileFootBytes, "footprint table entry size");

__device__ __forceinline__ int uniform_i32(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uniform_i64(int64_t v)
{
    const uint64_t u = (uint64_t)v;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

template <int M, typename OutT, int TH, int MD = 0, bool GRAD = false>
__device__ __forceinline__ void fbm2d_general_tile(const Fbm2dArgs &a, int64_t bid, float4 *lds4,
                                                   const LatCache *lat_in = nullptr)
{
    // the lattice cache holds unit gradients: the gradient model only (the others hash)
    const LatCache *const lat = MD == 0 ? lat_in : nullptr;
    constexpr int T = kTile2;
    constexpr int RPT = TH / 4;
    static_assert(RPT <= 64, "a wave's rows are one ballot");
    float4 *rowt = lds4;
    float4 *rowd = lds4 + TH;  // GRAD only: row-basis derivatives
    TileFoot *foot = reinterpret_cast<TileFoot *>(lds4 + (GRAD ? 2 * TH : TH));
    const int cap = a.capx * a.capy;
    float *gx = reinterpret_cast<float *>(foot + a.octaves);
    float *gy = gx + cap;
    float *gh = gy + cap;  // MD = 2 only
    // (the zero-gradient model's nodes hold a height only: no gy block)
    uint32_t *kx_all = reinterpret_cast<uint32_t *>(MD == 2 ? gh + cap : MD == 1 ? gx + cap : gy + cap);
    uint32_t *ky_all = kx_all + a.octaves * a.capx;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t tx0 = (bid % a.tiles_x) * T, ty0 = (bid / a.tiles_x) * TH;
    const int w = (int)min<int64_t>(T, a.nx - tx0);
    const int h = (int)min<int64_t>(TH, a.ny - ty0);
    const int col = min(lane, w - 1);  // lanes past the edge shadow the last column
    const int64_t X = a.x0 + tx0 + col;
    const int64_t Xf = a.x0 + tx0, Xl = a.x0 + tx0 + w - 1;
    const int64_t Yf = a.y0 + ty0, Yl = a.y0 + ty0 + h - 1;

    // ---- once per tile: every octave's footprint, then its column and row keys ----------
    if (tid < a.octaves) {
        const double f = a.freq[tid];
        TileFoot ft;
        ft.cxf = cell_of(Xf, f);
        ft.cyf = cell_of(Yf, f);
        ft.nnx = (int)(cell_of(Xl, f) - ft.cxf) + 2;
        ft.nny = (int)(cell_of(Yl, f) - ft.cyf) + 2;
        ft.pad0 = ft.pad1 = 0;
        foot[tid] = ft;
    }
    __syncthreads();
    if (!lat) {  // octaves spread over the waves (the coarse ones have a few keys each)
        for (int o = wave; o < a.octaves; o += 4) {
            const TileFoot ft = foot[o];
            const int nnx = uniform_i32(ft.nnx), nny = uniform_i32(ft.nny);
            const int64_t cxf = uniform_i64(ft.cxf), cyf = uniform_i64(ft.cyf);
            uint32_t *kx = kx_all + o * a.capx, *ky = ky_all + o * a.capy;
            const uint32_t pre = key_prefix(a.seed, o);
            for (int q = lane; q < nnx + nny; q += 64) {  // column keys, then row keys
                const bool c = q < nnx;  // a column key is the x index absorbed under its salt
                const uint32_t key = absorb_index(c ? kXSalt : pre, c ? cxf + q : cyf + (q - nnx));
                (c ? kx + q : ky + (q - nnx))[0] = key;
            }
        }
    }

    float acc[RPT], accx[GRAD ? RPT : 1], accy[GRAD ? RPT : 1];
#pragma unroll
    for (int r = 0; r < RPT; ++r) acc[r] = 0.0f;
#pragma unroll
    for (int r = 0; r < (GRAD ? RPT : 1); ++r) accx[r] = accy[r] = 0.0f;

    for (int o = 0; o < a.octaves; ++o) {
        const double f = a.freq[o];
        const float amp = a.amp[o];
        const TileFoot ft = foot[o];
        const int64_t cxf = uniform_i64(ft.cxf), cyf = uniform_i64(ft.cyf);
        const int nnx = uniform_i32(ft.nnx), nny = uniform_i32(ft.nny);
        const uint32_t *kx = kx_all + o * a.capx, *ky = ky_all + o * a.capy;

        __syncthreads();  // the previous octave is done with the row table and node block
        if (tid < TH) {
            const int r = min(tid, h - 1);
            const Coord c = coord_step(Yf + r, f);
            float s, b10, b11;
            Basis<M>::eval(c.t, s, b10, b11);
            if (MD == 3) {  // Perlin: (S(y), y, S(y) y)
                b10 = c.t;
                b11 = s * c.t;
            }
            rowt[tid] = make_float4(__int_as_float((int)(c.cell - cyf)), s, b10, b11);
            if constexpr (GRAD) {
                float ds, db10, db11;
                BasisD<M>::eval(c.t, ds, db10, db11);
                rowd[tid] = make_float4(ds, db10, db11, 0.0f);
            }
        }
        if (lat) {  // gradients from the cached lattice blocks
            // node (cxf + i, cyf + j) relative to the origin of the octave's first block
            const int ox = (int)(cxf - (lat->bx0[o] << kLatBlkLog)), oy = (int)(cyf - (lat->by0[o] << kLatBlkLog));
            const int nb = lat->nbx[o], e0 = lat->tbl0[o], nn = nnx * nny;
            // kLatIlp nodes per thread per pass, their loads issued together (a gather's
            // latency is paid once per pass, not once per node)
            constexpr int kLatIlp = 4;
            for (int q0 = tid; q0 < nn; q0 += kLatIlp * 256) {
                float vx[kLatIlp], vy[kLatIlp];
#pragma unroll
                for (int k = 0; k < kLatIlp; ++k) {
                    const int q = min(q0 + k * 256, nn - 1);  // past the end: reload the last node
                    const int j = q / nnx, i = q - j * nnx;
                    const int X = ox + i, Y = oy + j;
                    int e = e0 + (Y >> kLatBlkLog) * nb + (X >> kLatBlkLog);
                    e = min(max(e, 0), lat->n - 1);  // in range by construction; never read outside the table
                    const float *blk = reinterpret_cast<const float *>(lat->base + (size_t)lat->tbl[e] * 256);
                    const int w = (Y & (kLatBlk - 1)) * kLatBlk + (X & (kLatBlk - 1));
                    vx[k] = blk[w];
                    vy[k] = blk[kLatBlk * kLatBlk + w];
                }
#pragma unroll
                for (int k = 0; k < kLatIlp; ++k) {
                    const int q = q0 + k * 256;
                    if (q < nn) {
                        gx[q] = vx[k] * amp;
                        gy[q] = vy[k] * amp;
                    }
                }
            }
        } else {
            // node q = j nnx + i; a thread's nodes step by 256 = dj rows and di columns
            const int nn = nnx * nny, dj = 256 / nnx, di = 256 - dj * nnx;
            // tid / nnx from the reciprocal (within one of the quotient), then corrected
            int j = (int)(((float)tid + 0.5f) * __builtin_amdgcn_rcpf((float)nnx));
            j -= j * nnx > tid ? 1 : 0;
            j += (j + 1) * nnx <= tid ? 1 : 0;
            int i = tid - j * nnx;
            const float aw = MD == 2 ? amp * a.gw : amp;
            for (int q = tid; q < nn; q += 256) {
                const uint32_t key = key_combine(ky[j], kx[i]);
                if (MD == 1) {
                    gx[q] = height2(key) * amp;
                } else {
                    const float2 g = grad2(key);
                    gx[q] = g.x * aw;
                    gy[q] = g.y * aw;
                    if (MD == 2) gh[q] = height2_second(key) * amp;
                }
                i += di;
                j += dj;
                if (i >= nnx) {
                    i -= nnx;
                    ++j;
                }
            }
        }
        const Coord cc = coord_step(X, f);
        const int lcx = (int)(cc.cell - cxf);
        float sx, b10x, b11x, dsx = 0.0f, db10x = 0.0f, db11x = 0.0f;
        Basis<M>::eval(cc.t, sx, b10x, b11x);
        if constexpr (GRAD) BasisD<M>::eval(cc.t, dsx, db10x, db11x);
        const float fo = (float)f;  // d/dX = f d/dt
        __syncthreads();

        // rows of this wave that enter a new cell (the first always does)
        uint64_t fresh;
        {
            const int rr = wave * RPT + min(lane, RPT - 1);
            const int cy = __float_as_int(rowt[rr].x);
            const int cp = (lane > 0 && lane < RPT) ? __float_as_int(rowt[rr - 1].x) : -1;
            fresh = __ballot(lane < RPT && cy != cp);
        }

        // A node row collapsed along x at the lane's column (adjacent cells share one): value
        // term E and y-slope term Q (zero-gradient model: Q = (S(x) - x) D, the cell's slope
        // being the difference of its rows'; Perlin: the x-lerps A, B of the x- and
        // y-gradient ramps), and their x-derivatives (GRAD).
        struct NodeRow {
            float E, Q, Ex, Qx;
        };
        auto node_row = [&](int q) {
            NodeRow n{0.0f, 0.0f, 0.0f, 0.0f};
            if (MD == 1) {
                const float h0 = gx[q], d = gx[q + 1] - h0;
                n.E = h0 + sx * d;
                n.Q = (sx - cc.t) * d;
                if (GRAD) {
                    n.Ex = dsx * d;
                    n.Qx = (dsx - 1.0f) * d;
                }
            } else if (MD == 3) {
                const float fx0 = gx[q], fx1 = gx[q + 1], fy0 = gy[q], fy1 = gy[q + 1];
                n.E = fx0 * cc.t + sx * (fx1 * (cc.t - 1.0f) - fx0 * cc.t);
                n.Q = fy0 + sx * (fy1 - fy0);
            } else {
                const float fx0 = gx[q], fx1 = gx[q + 1], fy0 = gy[q], fy1 = gy[q + 1];
                n.E = fx0 * b10x + fx1 * b11x;
                if (MD == 2) n.E += gh[q] + sx * (gh[q + 1] - gh[q]);  // the heights' value term
                n.Q = fy0 + sx * (fy1 - fy0);
                if (GRAD) {
                    n.Ex = fx0 * db10x + fx1 * db11x;
                    if (MD == 2) n.Ex += dsx * (gh[q + 1] - gh[q]);
                    n.Qx = dsx * (fy1 - fy0);
                }
            }
            return n;
        };
        float E0 = 0.0f, dE = 0.0f, Q0 = 0.0f, Q1 = 0.0f;
        float E0x = 0.0f, dEx = 0.0f, Q0x = 0.0f, Q1x = 0.0f;  // the x-derivative's row form (GRAD)
        NodeRow lo{}, hi{};
        int prev = -2;  // the current cell's row (uniform)
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            // one 16-byte read per row (the cell index is used on fresh rows only)
            const f32x4 re = load_here4(rowt + wave * RPT + r);
            if ((fresh >> r) & 1u) {
                const int lcy = __builtin_amdgcn_readfirstlane(__float_as_int(re.x));
                const int q = lcy * nnx + lcx;
                lo = lcy == prev + 1 ? hi : node_row(q);  // the next cell up shares its lower row
                hi = node_row(q + nnx);
                prev = lcy;
                if (MD == 1) {
                    E0 = lo.E;
                    dE = hi.E - lo.E;
                    Q0 = Q1 = hi.Q - lo.Q;
                    if (GRAD) {
                        E0x = lo.Ex;
                        dEx = hi.Ex - lo.Ex;
                        Q0x = Q1x = hi.Qx - lo.Qx;
                    }
                } else if (MD == 3) {  // Perlin: E0 = A0, dE = A1 - B1 - A0, Q0 = B0, Q1 = B1 - B0
                    E0 = lo.E;
                    dE = hi.E - hi.Q - lo.E;
                    Q0 = lo.Q;
                    Q1 = hi.Q - lo.Q;
                } else {
                    E0 = lo.E;
                    dE = hi.E - lo.E;
                    Q0 = lo.Q;
                    Q1 = hi.Q;
                    if (GRAD) {
                        E0x = lo.Ex;
                        dEx = hi.Ex - lo.Ex;
                        Q0x = lo.Qx;
                        Q1x = hi.Qx;
                    }
                }
            }
            acc[r] += E0 + dE * re.y + Q0 * re.z + Q1 * re.w;
            keep_here(acc[r]);
            if (GRAD) {
                const float4 rd = rowd[wave * RPT + r];
                accx[r] += fo * (E0x + dEx * re.y + Q0x * re.z + Q1x * re.w);
                accy[r] += fo * (dE * rd.x + Q0 * rd.y + Q1 * rd.z);
                keep_here(accx[r]);
                keep_here(accy[r]);
            }
        }
    }

    if (lane < w) {
        OutT *out = reinterpret_cast<OutT *>(a.out);
        OutT *odx = reinterpret_cast<OutT *>(a.out_dx), *ody = reinterpret_cast<OutT *>(a.out_dy);
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const int row = wave * RPT + r;
            if (row >= h) continue;
            const int64_t at = (ty0 + row) * a.pitch + tx0 + lane;
            out[at] = to_out<OutT>(acc[r]);
            if (GRAD) {
                odx[at] = to_out<OutT>(accx[r]);
                ody[at] = to_out<OutT>(accy[r]);
            }
        }
    }
}

// ---------------------------------------------------------------------------------
// 3D: tile 64 x 8 x TZ samples; wave w owns TZ / 4 slabs, all 8 rows of each.
// For a fixed column the cell is collapsed along x (a, b, c per (cy, cz) corner pair),
// then along z, leaving the 1D Hermite form in y evaluated per sample.
// LDS: y table float4[8] | z table float4[TZ] | every octave's footprint TileFoot3[octaves] |
// g{x,y,z}[cap] | (MD = 2) h[cap] | every octave's keys kx[octaves*capx] | kzy[octaves*capy*capz]
// ---------------------------------------------------------------------------------
// Once per tile: the octaves' footprints (one lane per octave, FP64) and the keys of their
// node columns and (z, y) node rows; per octave, between two barriers, the y and z tables
// and the node block (node indices stepped, not divided); then each wave's slabs.
// MD = 2: node heights (third key word) and w-weighted gradients; the x collapse adds the
// heights' value term to each corner's a.
struct TileFoot3 {  // one octave's lattice footprint over a 3D tile
    int64_t cxf, cyf, czf;
    int32_t nnx, nny, nnz, pad;
};
static_assert(sizeof(TileFoot3) == kTileFoot3Bytes, "3D footprint table entry size");

template <int M, typename OutT, int MD = 0>
__device__ __forceinline__ void fbm3d_general_tile(const Fbm3dArgs &a, int64_t bid, float4 *lds4)
{
    constexpr int TX = kTile3X, TY = kTile3Y, TZ = kTile3Z;
    constexpr int ZPW = TZ / 4;  // slabs per wave
    constexpr int RPT = ZPW * TY;
    float4 *yt = lds4;
    float4 *zt = lds4 + TY;
    TileFoot3 *foot = reinterpret_cast<TileFoot3 *>(lds4 + TY + TZ);
    const int cap = a.capx * a.capy * a.capz, capzy = a.capy * a.capz;
    float *gxs = reinterpret_cast<float *>(foot + a.octaves);
    float *gys = gxs + cap;
    float *gzs = gys + cap;
    float *hs = gzs + cap;  // node heights (MD = 2)
    uint32_t *kx_all = reinterpret_cast<uint32_t *>(gzs + (MD == 2 ? 2 : 1) * cap);
    uint32_t *kzy_all = kx_all + a.octaves * a.capx;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t tpl = (int64_t)a.tiles_x * a.tiles_y;
    const int64_t tz = bid / tpl, rem = bid - tz * tpl;
    const int64_t ty = rem / a.tiles_x, tx = rem - ty * a.tiles_x;
    const int64_t tx0 = tx * TX, ty0 = ty * TY, tz0 = tz * TZ;
    const int w = (int)min<int64_t>(TX, a.nx - tx0);
    const int hy = (int)min<int64_t>(TY, a.ny - ty0);
    const int hz = (int)min<int64_t>(TZ, a.nz - tz0);
    const int col = min(lane, w - 1);
    const int64_t X = a.x0 + tx0 + col;
    const int64_t Xf = a.x0 + tx0, Yf = a.y0 + ty0, Zf = a.z0 + tz0;

    // ---- once per tile: every octave's footprint, then its column and (z, y) row keys -----
    if (tid < a.octaves) {
        const double f = a.freq[tid];
        TileFoot3 ft;
        ft.cxf = cell_of(Xf, f);
        ft.cyf = cell_of(Yf, f);
        ft.czf = cell_of(Zf, f);
        ft.nnx = (int)(cell_of(Xf + w - 1, f) - ft.cxf) + 2;
        ft.nny = (int)(cell_of(Yf + hy - 1, f) - ft.cyf) + 2;
        ft.nnz = (int)(cell_of(Zf + hz - 1, f) - ft.czf) + 2;
        ft.pad = 0;
        foot[tid] = ft;
    }
    __syncthreads();
    const int wave_u = __builtin_amdgcn_readfirstlane(wave);
    for (int o = wave_u; o < a.octaves; o += 4) {  // octaves spread over the waves
        const TileFoot3 ft = foot[o];
        const int nnx = uniform_i32(ft.nnx), nny = uniform_i32(ft.nny), nnz = uniform_i32(ft.nnz);
        const int64_t cxf = uniform_i64(ft.cxf), cyf = uniform_i64(ft.cyf), czf = uniform_i64(ft.czf);
        uint32_t *kx = kx_all + o * a.capx, *kzy = kzy_all + o * capzy;
        const uint32_t pre = key_prefix(a.seed, o);
        for (int i = lane; i < nnx; i += 64) kx[i] = key_xline(cxf + i);
        for (int q = lane; q < nny * nnz; q += 64) {
            const int k = q / nny, j = q - k * nny;
            kzy[q] = absorb_index(absorb_index(pre, czf + k), cyf + j);
        }
    }

    float acc[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) acc[r] = 0.0f;

    for (int o = 0; o < a.octaves; ++o) {
        const double f = a.freq[o];
        const float amp = a.amp[o];
        const TileFoot3 ft = foot[o];
        const int nnx = uniform_i32(ft.nnx), nny = uniform_i32(ft.nny), nnz = uniform_i32(ft.nnz);
        const int64_t cxf = uniform_i64(ft.cxf), cyf = uniform_i64(ft.cyf), czf = uniform_i64(ft.czf);
        const uint32_t *kx = kx_all + o * a.capx, *kzy = kzy_all + o * capzy;

        __syncthreads();  // the previous octave is done with the tables and node block
        if (tid < TY) {
            const int r = min(tid, hy - 1);
            const Coord c = coord_step(Yf + r, f);
            float s, b10, b11;
            Basis<M>::eval(c.t, s, b10, b11);
            yt[tid] = make_float4(__int_as_float((int)(c.cell - cyf)), s, b10, b11);
        } else if (tid >= 64 && tid < 64 + TZ) {
            const int r = min(tid - 64, hz - 1);
            const Coord c = coord_step(Zf + r, f);
            float s, b10, b11;
            Basis<M>::eval(c.t, s, b10, b11);
            zt[tid - 64] = make_float4(__int_as_float((int)(c.cell - czf)), s, b10, b11);
        }
        {
            // node q = row nnx + i (row = k nny + j); a thread's nodes step by 256
            const int plane = nnx * nny, nn = plane * nnz, drow = 256 / nnx, di = 256 - drow * nnx;
            int row = tid / nnx, i = tid - row * nnx;
            const float gsc = MD == 2 ? amp * a.gw : amp;
            for (int q = tid; q < nn; q += 256) {
                const uint32_t key = key_combine(kzy[row], kx[i]), second = key3_second(key);
                const float3 g = grad3_of(key, second);
                gxs[q] = g.x * gsc;
                gys[q] = g.y * gsc;
                gzs[q] = g.z * gsc;
                if (MD == 2) hs[q] = height3_of_second(second) * amp;
                i += di;
                row += drow;
                if (i >= nnx) {
                    i -= nnx;
                    ++row;
                }
            }
        }
        const Coord cc = coord_step(X, f);
        const int lcx = (int)(cc.cell - cxf);
        float sx, b10x, b11x;
        Basis<M>::eval(cc.t, sx, b10x, b11x);
        __syncthreads();

        // rows of the y table that enter a new y cell (the first always does)
        uint64_t yfresh;
        {
            const int r = min(lane, TY - 1);
            const int cy = __float_as_int(yt[r].x);
            const int cp = (lane > 0 && lane < TY) ? __float_as_int(yt[r - 1].x) : -1;
            yfresh = __ballot(lane < TY && cy != cp);
        }
        int prev_cell = -1;
        float ca[2][2], cb[2][2], cc2[2][2];  // x-collapsed coefficients [cy][cz]
#pragma unroll
        for (int zz = 0; zz < ZPW; ++zz) {
            const float4 ze = zt[wave * ZPW + zz];
            const int lcz = __builtin_amdgcn_readfirstlane(__float_as_int(ze.x));
            float E0 = 0.0f, dE = 0.0f, Q0 = 0.0f, Q1 = 0.0f;
#pragma unroll
            for (int yy = 0; yy < TY; ++yy) {
                const f32x4 ye = load_here4(yt + yy);
                if ((yfresh >> yy) & 1u) {  // a new y cell (or the slab's first row)
                    const int lcy = __builtin_amdgcn_readfirstlane(__float_as_int(ye.x));
                    const int cell = lcz * 65536 + lcy;
                    if (cell != prev_cell) {
                        prev_cell = cell;
#pragma unroll
                        for (int cz = 0; cz < 2; ++cz)
#pragma unroll
                            for (int cy = 0; cy < 2; ++cy) {
                                const int q = ((lcz + cz) * nny + (lcy + cy)) * nnx + lcx;
                                ca[cy][cz] = gxs[q] * b10x + gxs[q + 1] * b11x;
                                if (MD == 2) ca[cy][cz] += hs[q] + sx * (hs[q + 1] - hs[q]);
                                cb[cy][cz] = gys[q] + sx * (gys[q + 1] - gys[q]);
                                cc2[cy][cz] = gzs[q] + sx * (gzs[q + 1] - gzs[q]);
                            }
                    }
                    float Ev[2], Bq[2];
#pragma unroll
                    for (int cy = 0; cy < 2; ++cy) {
                        const float A = ca[cy][0] + ze.y * (ca[cy][1] - ca[cy][0]);
                        const float C = cc2[cy][0] * ze.z + cc2[cy][1] * ze.w;
                        Bq[cy] = cb[cy][0] + ze.y * (cb[cy][1] - cb[cy][0]);
                        Ev[cy] = A + C;
                    }
                    E0 = Ev[0];
                    dE = Ev[1] - Ev[0];
                    Q0 = Bq[0];
                    Q1 = Bq[1];
                }
                acc[zz * TY + yy] += E0 + dE * ye.y + Q0 * ye.z + Q1 * ye.w;
                keep_here(acc[zz * TY + yy]);
            }
        }
    }

    if (lane < w) {
        OutT *out = reinterpret_cast<OutT *>(a.out);
#pragma unroll
        for (int zz = 0; zz < ZPW; ++zz) {
            const int z = wave * ZPW + zz;
            if (z >= hz) continue;
#pragma unroll
            for (int yy = 0; yy < TY; ++yy) {
                if (yy >= hy) continue;
                out[((tz0 + z) * a.ny + (ty0 + yy)) * a.nx + tx0 + lane] = to_out<OutT>(acc[zz * TY + yy]);
            }
        }
    }
}

}  // namespace ptg
