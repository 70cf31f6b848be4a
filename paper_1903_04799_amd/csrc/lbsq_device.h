// lbsq_device.h -- device-side definitions shared by the gfx950 kernels of the
// lattice Boltzmann squirmer library (arXiv:1903.04799).
//
// Lattice, storage formats, the body table and the small device functions
// that more than one kernel must evaluate identically (inside test, wall
// velocity, bounce-back shift, refill density).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbsq {

constexpr int Q = 19;
constexpr int BLOCK = 256;
constexpr int MAXB = 253;

// Cell owner codes.  Fluid cells carry a flag telling the fused kernel
// whether any of their 18 neighbours is solid (the slow path).
constexpr uint8_t OWN_FLUID = 0;
constexpr uint8_t OWN_FLUID_NB = 254;
constexpr uint8_t OWN_WALL = 255;

__host__ __device__ constexpr bool is_fluid(uint8_t o) { return o == OWN_FLUID || o == OWN_FLUID_NB; }
__host__ __device__ constexpr bool is_body(uint8_t o) { return o >= 1 && o <= MAXB; }

// D3Q19 in the canonical order of the C ABI (rest, faces, edges; for odd i
// the opposite direction is i+1).
__host__ __device__ constexpr int cx(int i)
{
    return (i == 1 || i == 7 || i == 9 || i == 11 || i == 13) ? 1
           : (i == 2 || i == 8 || i == 10 || i == 12 || i == 14) ? -1 : 0;
}
__host__ __device__ constexpr int cy(int i)
{
    return (i == 3 || i == 7 || i == 10 || i == 15 || i == 17) ? 1
           : (i == 4 || i == 8 || i == 9 || i == 16 || i == 18) ? -1 : 0;
}
__host__ __device__ constexpr int cz(int i)
{
    return (i == 5 || i == 11 || i == 14 || i == 15 || i == 18) ? 1
           : (i == 6 || i == 12 || i == 13 || i == 16 || i == 17) ? -1 : 0;
}
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
__host__ __device__ constexpr double wgt(int i) { return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0); }
__host__ __device__ constexpr float wgtf(int i) { return i == 0 ? 1.0f / 3.0f : (i <= 6 ? 1.0f / 18.0f : 1.0f / 36.0f); }

// ---------------------------------------------------------------------------
// Population storage: deviations d_i = f_i - w_i rho0, times 2^k.

struct StF32 {
    using T = float;
    static __device__ __forceinline__ float ld(T v, float) { return v; }
    static __device__ __forceinline__ T st(float v, float) { return v; }
};

struct StF16 {
    using T = _Float16;
    static __device__ __forceinline__ float ld(T v, float inv) { return static_cast<float>(v) * inv; }
    // float -> half conversion rounds to nearest even
    static __device__ __forceinline__ T st(float v, float scale) { return static_cast<_Float16>(v * scale); }
};

struct StBF16 {
    using T = uint16_t;
    static __device__ __forceinline__ float ld(T v, float inv)
    {
        return __uint_as_float(static_cast<uint32_t>(v) << 16) * inv;
    }
    // round to nearest even on the upper 16 bits; NaN stays NaN
    static __device__ __forceinline__ T st(float v, float scale)
    {
        uint32_t u = __float_as_uint(v * scale);
        if ((u & 0x7fffffffu) > 0x7f800000u) return static_cast<T>((u >> 16) | 0x40u);
        u += 0x7fffu + ((u >> 16) & 1u);
        return static_cast<T>(u >> 16);
    }
};

// ---------------------------------------------------------------------------
// Rigid bodies (FP64), one record per body, resident on the device.

struct DevBody {
    double pos[3], e[3], v[3], w[3];
    double R, B1, beta, m, I;
    double F[3], T[3], Fbb[3], Tbb[3], Fc[3], Tc[3], Fwca[3];
    int mode;  // 0 free, 1 fixed, 2 prescribed
    int H;     // half width of the body's bounding box in cells
    int64_t Rq;  // radius in 2^-20 quanta
};

struct Box {
    int nx, ny, nz;
    uint32_t n;       // cells
    uint64_t stride;  // elements between population planes
};

// Minimum image of a real difference in a box of length L (|d| < 1.5 L).
__device__ __forceinline__ double min_image(double d, int L)
{
    if (d >= 0.5 * L) d -= L;
    else if (d < -0.5 * L) d += L;
    return d;
}

__device__ __forceinline__ int wrap(int a, int n)
{
    a %= n;
    return a < 0 ? a + n : a;
}

// Lever arm from the body centre to the centre of cell (x, y, z).
__device__ __forceinline__ void lever_arm(const Box &b, const DevBody &B, int x, int y, int z, double d[3])
{
    d[0] = min_image((x + 0.5) - B.pos[0], b.nx);
    d[1] = min_image((y + 0.5) - B.pos[1], b.ny);
    d[2] = min_image((z + 0.5) - B.pos[2], b.nz);
}

// Inside test in int64 fixed point (2^-20 quanta, centres at i + 1/2, ties
// inside, positions rounded half to even).
__device__ __forceinline__ bool inside_body(const Box &b, const DevBody &B, int x, int y, int z)
{
    const int64_t ONE = int64_t(1) << 20;
    const int n[3] = {b.nx, b.ny, b.nz};
    const int c[3] = {x, y, z};
    int64_t sum = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int64_t X = (2 * int64_t(c[k]) + 1) * (ONE / 2);
        const int64_t P = __double2ll_rn(B.pos[k] * double(ONE));
        const int64_t L = int64_t(n[k]) * ONE;
        int64_t D = (X - P) % L;
        if (D < 0) D += L;
        if (D >= L / 2) D -= L;
        sum += D * D;
    }
    return sum <= B.Rq * B.Rq;
}

// Bounding box of a body: cells floor(pos) - H ... floor(pos) + H per axis.
__device__ __forceinline__ void bbox_origin(const DevBody &B, int o[3])
{
#pragma unroll
    for (int k = 0; k < 3; ++k) o[k] = static_cast<int>(floor(B.pos[k])) - B.H;
}

__device__ __forceinline__ bool in_bbox(const Box &b, const DevBody &B, int x, int y, int z)
{
    int o[3];
    bbox_origin(B, o);
    const int side = 2 * B.H + 1;
    return wrap(x - o[0], b.nx) < side && wrap(y - o[1], b.ny) < side && wrap(z - o[2], b.nz) < side;
}

// Wall velocity of the solid node of body B centred at cell s, eq. (vb) plus
// the slip of eq. (squirmer): v + w x d + B1 (1 + beta e.n)((e.n) n - e).
__device__ __forceinline__ void wall_velocity(const DevBody &B, const double d[3], double vb[3])
{
    vb[0] = B.v[0] + B.w[1] * d[2] - B.w[2] * d[1];
    vb[1] = B.v[1] + B.w[2] * d[0] - B.w[0] * d[2];
    vb[2] = B.v[2] + B.w[0] * d[1] - B.w[1] * d[0];
    if (B.B1 != 0.0) {
        const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        const double n[3] = {d[0] / r, d[1] / r, d[2] / r};
        const double en = B.e[0] * n[0] + B.e[1] * n[1] + B.e[2] * n[2];
        const double a = B.B1 * (1.0 + B.beta * en);
#pragma unroll
        for (int k = 0; k < 3; ++k) vb[k] += a * (en * n[k] - B.e[k]);
    }
}

// Shift of the reflected population for the link (x, i) whose source node s
// = x - c_i belongs to body B: 6 w_i rho_w c_i.v_b (moving-wall rule).
__device__ __forceinline__ float bounce_shift(int i, float rho_w, const DevBody &B, const double d[3])
{
    double vb[3];
    wall_velocity(B, d, vb);
    const double cv = cx(i) * vb[0] + cy(i) * vb[1] + cz(i) * vb[2];
    return static_cast<float>(6.0 * wgt(i) * static_cast<double>(rho_w) * cv);
}

}  // namespace lbsq
