// ptg_device.h -- device-side building blocks shared by the libptg kernels (gfx950).
//
// Lattice hash, gradient maps, FP64 coordinate step and the 1D Hermite bases of the
// boundary-constrained cell polynomials (Thorimbert & Chopard, Sec. 2-4).  The exact
// conventions (hash words, salts, sample-centre coordinates) are stated in include/ptg.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ptg {

// ---------------------------------------------------------------------------------
// Lattice hash (a2).  fmix32 is the MurmurHash3 32-bit finalizer.
// ---------------------------------------------------------------------------------
__host__ __device__ __forceinline__ uint32_t fmix32(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}

// Absorb an int64 lattice index: low word, then high word (two's complement).
__host__ __device__ __forceinline__ uint32_t absorb_index(uint32_t k, int64_t i)
{
    const uint64_t u = (uint64_t)i;
    k = fmix32(k ^ (uint32_t)u);
    k = fmix32(k ^ (uint32_t)(u >> 32));
    return k;
}

__host__ __device__ __forceinline__ uint32_t key_prefix(uint32_t seed, int32_t octave)
{
    return fmix32(fmix32(seed ^ 0x9E3779B9u) ^ (uint32_t)octave);
}

// Per-column part of every key (x index under its own salt).
constexpr uint32_t kXSalt = 0x27D4EB2Fu;
__host__ __device__ __forceinline__ uint32_t key_xline(int64_t ix) { return absorb_index(kXSalt, ix); }

// key2 = fmix32(ky ^ kx) with ky = absorb_index(prefix, iy), kx = key_xline(ix);
// key3 = fmix32(kzy ^ kx) with kzy = absorb_index(absorb_index(prefix, iz), iy).
__host__ __device__ __forceinline__ uint32_t key_combine(uint32_t krow, uint32_t kx) { return fmix32(krow ^ kx); }

__host__ __device__ __forceinline__ uint32_t key3_second(uint32_t key) { return fmix32(key ^ 0x165667B1u); }

// 2D unit gradient from a key: angle = (key >> 8) / 2^24 turns.  v_sin/v_cos take their
// argument in turns, so no range reduction is needed on [0, 1).
__device__ __forceinline__ float2 grad2(uint32_t key)
{
    const float turns = (float)(key >> 8) * (1.0f / 16777216.0f);
    return make_float2(__builtin_amdgcn_cosf(turns), __builtin_amdgcn_sinf(turns));
}

// Node height of the zero-gradient model (Sec. 3.3): m / 2^23 - 1 with m the key's top 24
// bits, uniform on [-1, 1) and exact in FP32.
__device__ __forceinline__ float height2(uint32_t key) { return (float)(key >> 8) * (1.0f / 8388608.0f) - 1.0f; }

// Node height of the height-and-gradient model: the same map on the node's second word
// (its gradient angle takes the first word's top bits).
__device__ __forceinline__ float height2_second(uint32_t key) { return height2(key3_second(key)); }

// 3D unit gradient: z = 1 - (2m+1)/2^24 (exact in FP32), azimuth from the second word,
// radius sqrt((1-z)(1+z)) (the hardware square root, within 1 ulp).
__device__ __forceinline__ float3 grad3_of(uint32_t key, uint32_t second)
{
    const uint32_t m1 = key >> 8;
    const uint32_t m2 = second >> 8;
    const float k = (float)(2u * m1 + 1u) * (1.0f / 16777216.0f);
    const float z = 1.0f - k;
    const float r = __builtin_amdgcn_sqrtf(fmaxf(k * (2.0f - k), 0.0f));
    const float turns = (float)m2 * (1.0f / 16777216.0f);
    return make_float3(r * __builtin_amdgcn_cosf(turns), r * __builtin_amdgcn_sinf(turns), z);
}

__device__ __forceinline__ float3 grad3(uint32_t key) { return grad3_of(key, key3_second(key)); }

// Node height of the 3D height-and-gradient model: the height map on the key's third word
// (the second-word map applied to the second word; the first two give the gradient).
__device__ __forceinline__ float height3_of_second(uint32_t second) { return height2(key3_second(second)); }

// ---------------------------------------------------------------------------------
// Coordinate step (a1): u = (X + 1/2) * f in FP64, cell = floor(u), t = u - cell.
// Contraction is off so the device computes exactly the IEEE operations written.
// ---------------------------------------------------------------------------------
struct Coord {
    int64_t cell;
    float t;
};

__device__ __forceinline__ Coord coord_step(int64_t X, double f)
{
#pragma clang fp contract(off)
    const double u = ((double)X + 0.5) * f;
    const double c = __builtin_floor(u);
    Coord r;
    r.cell = (int64_t)c;
    r.t = (float)(u - c);
    return r;
}

__host__ __device__ __forceinline__ int64_t cell_of(int64_t X, double f)
{
#pragma clang fp contract(off)
    return (int64_t)__builtin_floor(((double)X + 0.5) * f);
}

// ---------------------------------------------------------------------------------
// 1D Hermite bases on [0,1] (M = 1 cubic, M = 2 quintic).
//   s   = value basis of the far corner (S3 = 3t^2 - 2t^3, S5 = 6t^5 - 15t^4 + 10t^3);
//         the near corner's value basis is 1 - s.
//   b10 = slope basis of the near corner, b11 = slope basis of the far corner.
// ---------------------------------------------------------------------------------
// Any order M >= 4 (the value and first M derivatives prescribed at both ends): the closed
// forms of two-point Taylor interpolation, evaluated in factored form (every term of each sum
// is non-negative on [0, 1], so no cancellation):
//   S(t)   = t^(M+1) sum_{k=0..M} C(M+k, k) (1-t)^k,
//   b10(t) = t (1-t)^(M+1) sum_{k=0..M-1} C(M+k, k) t^k,
//   b11(t) = -(1-t) t^(M+1) sum_{k=0..M-1} C(M+k, k) (1-t)^k.
__host__ __device__ constexpr float binom_f(int n, int k)
{
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (double)(n - k + i) / (double)i;
    return (float)r;
}

template <int M>
struct Basis {
    static_assert(M >= 4 && M <= 6, "orders 1..3 have explicit forms below; the API allows up to 6");
    __device__ __forceinline__ static void eval(float t, float &s, float &b10, float &b11)
    {
        const float u = 1.0f - t;
        float pu = binom_f(2 * M - 1, M - 1), pt = pu;  // sums over k <= M-1, Horner from the top
#pragma unroll
        for (int k = M - 2; k >= 0; --k) {
            pu = __builtin_fmaf(pu, u, binom_f(M + k, k));
            pt = __builtin_fmaf(pt, t, binom_f(M + k, k));
        }
        float tm = 1.0f, um = 1.0f;  // t^M, (1-t)^M
#pragma unroll
        for (int k = 0; k < M; ++k) {
            tm *= t;
            um *= u;
        }
        const float tp = tm * t, up = um * u;
        s = tp * __builtin_fmaf(binom_f(2 * M, M), um, pu);  // the k = M term joins the sum
        b10 = t * up * pt;
        b11 = -u * tp * pu;
    }
};

template <>
struct Basis<1> {
    __device__ __forceinline__ static void eval(float t, float &s, float &b10, float &b11)
    {
        const float t2 = t * t;
        const float u = 1.0f - t;
        s = t2 * (3.0f - 2.0f * t);
        b10 = t * u * u;
        b11 = -t2 * u;
    }
};

template <>
struct Basis<2> {
    __device__ __forceinline__ static void eval(float t, float &s, float &b10, float &b11)
    {
        const float t2 = t * t;
        const float t3 = t2 * t;
        s = t3 * (10.0f + t * (-15.0f + 6.0f * t));
        b10 = t + t3 * (-6.0f + t * (8.0f - 3.0f * t));
        b11 = t3 * (-4.0f + t * (7.0f - 3.0f * t));
    }
};

// Septic cells (M = 3: derivatives up to third order constrained): the degree-7
// smoothstep and the two slope bases with zero second and third end derivatives.
template <>
struct Basis<3> {
    __device__ __forceinline__ static void eval(float t, float &s, float &b10, float &b11)
    {
        const float t2 = t * t;
        const float t4 = t2 * t2;
        s = t4 * (35.0f + t * (-84.0f + t * (70.0f - 20.0f * t)));
        b10 = t + t4 * (-20.0f + t * (45.0f + t * (-36.0f + 10.0f * t)));
        b11 = t4 * (-15.0f + t * (39.0f + t * (-34.0f + 10.0f * t)));
    }
};

// Derivatives d/dt of the bases above (the analytic gradient of the height field).
template <int M>
struct BasisD;

template <>
struct BasisD<1> {
    __device__ __forceinline__ static void eval(float t, float &ds, float &db10, float &db11)
    {
        ds = 6.0f * t * (1.0f - t);
        db10 = 1.0f + t * (-4.0f + 3.0f * t);
        db11 = t * (-2.0f + 3.0f * t);
    }
};

template <>
struct BasisD<2> {
    __device__ __forceinline__ static void eval(float t, float &ds, float &db10, float &db11)
    {
        const float t2 = t * t;
        ds = t2 * (30.0f + t * (-60.0f + 30.0f * t));
        db10 = 1.0f + t2 * (-18.0f + t * (32.0f - 15.0f * t));
        db11 = t2 * (-12.0f + t * (28.0f - 15.0f * t));
    }
};

template <>
struct BasisD<3> {
    __device__ __forceinline__ static void eval(float t, float &ds, float &db10, float &db11)
    {
        const float t3 = t * t * t;
        ds = t3 * (140.0f + t * (-420.0f + t * (420.0f - 140.0f * t)));
        db10 = 1.0f + t3 * (-80.0f + t * (225.0f + t * (-216.0f + 70.0f * t)));
        db11 = t3 * (-60.0f + t * (195.0f + t * (-204.0f + 70.0f * t)));
    }
};

// Monomial coefficients of the four 1D bases, rows: 1-s, s, b10, b11; column e = t^e.
// Used by the per-cell coefficient kernel (K2) to expand the tensor form.
template <int M>
struct BasisMono;

template <>
struct BasisMono<1> {
    static constexpr int N1 = 4;
    __device__ __forceinline__ static float c(int k, int e)
    {
        // 1 - 3t^2 + 2t^3 | 3t^2 - 2t^3 | t - 2t^2 + t^3 | -t^2 + t^3
        constexpr float tab[4][4] = {{1.f, 0.f, -3.f, 2.f}, {0.f, 0.f, 3.f, -2.f},
                                     {0.f, 1.f, -2.f, 1.f}, {0.f, 0.f, -1.f, 1.f}};
        return tab[k][e];
    }
};

template <>
struct BasisMono<2> {
    static constexpr int N1 = 6;
    __device__ __forceinline__ static float c(int k, int e)
    {
        constexpr float tab[4][6] = {{1.f, 0.f, 0.f, -10.f, 15.f, -6.f},
                                     {0.f, 0.f, 0.f, 10.f, -15.f, 6.f},
                                     {0.f, 1.f, 0.f, -6.f, 8.f, -3.f},
                                     {0.f, 0.f, 0.f, -4.f, 7.f, -3.f}};
        return tab[k][e];
    }
};

}  // namespace ptg
