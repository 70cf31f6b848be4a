// lbsq_device.h -- device-side definitions shared by the gfx950 kernels of the
// lattice Boltzmann squirmer library (arXiv:1903.04799).
//
// Lattice, storage formats, the body table and the small device functions
// that more than one kernel must evaluate identically (inside test, box
// geometry, lever arms).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbsq {

// Pointers known to address device global memory.  Pointers read from a
// descriptor in memory are generic otherwise, which costs flat loads and
// 64-bit address arithmetic on the hot path.
template <class T>
using gptr = T __attribute__((address_space(1))) *;
template <class T>
__device__ __forceinline__ gptr<T> as_global(T *p)
{
    return (gptr<T>)p;
}

constexpr int Q = 19;
constexpr int BLOCK = 256;
constexpr int MAXB = 252;
// cells per block of the kernels that work on the bodies' boxes with one
// thread per (cell, direction): 13 x 19 = 247 of 256 threads
constexpr int CPB = 13;

// Cell owner codes.  Fluid cells carry a flag saying which of their 18
// neighbours are solid: none (the streaming kernel's fast path), static
// walls only (the streaming kernel reflects them), or at least one body
// cell (the boundary kernel takes the cell).
constexpr uint8_t OWN_FLUID = 0;
constexpr uint8_t OWN_NB_WALL = 253;
constexpr uint8_t OWN_NB_BODY = 254;
constexpr uint8_t OWN_WALL = 255;

__host__ __device__ constexpr bool is_fluid(uint8_t o) { return o == OWN_FLUID || o == OWN_NB_WALL || o == OWN_NB_BODY; }
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

// The same lattice for a direction index known only at run time: bit masks
// of the directions whose component is +1 and -1 (compact code for loops
// that are not unrolled).
__host__ __device__ constexpr int rcx(int i) { return int((0x2a82u >> i) & 1u) - int((0x5504u >> i) & 1u); }
__host__ __device__ constexpr int rcy(int i) { return int((0x28488u >> i) & 1u) - int((0x50310u >> i) & 1u); }
__host__ __device__ constexpr int rcz(int i) { return int((0x4c820u >> i) & 1u) - int((0x33040u >> i) & 1u); }

__host__ __device__ constexpr bool lattice_tables_agree(int i)
{
    return i == Q || (rcx(i) == cx(i) && rcy(i) == cy(i) && rcz(i) == cz(i) && lattice_tables_agree(i + 1));
}
static_assert(lattice_tables_agree(0), "run-time D3Q19 masks disagree with the lattice");

// ---------------------------------------------------------------------------
// Population storage: deviations d_i = f_i - w_i rho0, times 2^k.

struct StF32 {
    using T = float;
    // waves per SIMD the fluid kernel is compiled for (its register budget;
    // the steps with the fused audit take 4)
    static constexpr int waves = 5;
    // stored values are the deviations themselves (no scale)
    static constexpr bool scaled = false;
    static __device__ __forceinline__ float dec(T v) { return v; }
    static __device__ __forceinline__ T enc(float v) { return v; }
    static __device__ __forceinline__ float ld(T v, float) { return v; }
    static __device__ __forceinline__ T st(float v, float) { return v; }
};

struct StF16 {
    using T = _Float16;
    // waves per SIMD the fluid kernel is compiled for: half-width elements
    // move half the bytes per load, so more waves keep enough in flight
    static constexpr int waves = 6;
    // stored values are the deviations times the scale 2^k
    static constexpr bool scaled = true;
    static __device__ __forceinline__ float dec(T v) { return static_cast<float>(v); }
    // float -> half conversion rounds to nearest even
    static __device__ __forceinline__ T enc(float v) { return static_cast<_Float16>(v); }
    static __device__ __forceinline__ float ld(T v, float inv) { return dec(v) * inv; }
    static __device__ __forceinline__ T st(float v, float scale) { return enc(v * scale); }
};

struct StBF16 {
    using T = uint16_t;
    static constexpr int waves = 6;
    static constexpr bool scaled = true;
    static __device__ __forceinline__ float dec(T v) { return __uint_as_float(static_cast<uint32_t>(v) << 16); }
    // round to nearest even on the upper 16 bits; NaN stays NaN
    static __device__ __forceinline__ T enc(float v)
    {
        uint32_t u = __float_as_uint(v);
        if ((u & 0x7fffffffu) > 0x7f800000u) return static_cast<T>((u >> 16) | 0x40u);
        u += 0x7fffu + ((u >> 16) & 1u);
        return static_cast<T>(u >> 16);
    }
    static __device__ __forceinline__ float ld(T v, float inv) { return dec(v) * inv; }
    static __device__ __forceinline__ T st(float v, float scale) { return enc(v * scale); }
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

// What the geometry kernel needs of a body at its new position (kept in
// LDS): floor of the position, the position's offset from it in 2^-20
// quanta (rounded half to even), the squared radius in quanta, and the
// rigid-body velocity for refills.
struct GeoBody {
    double pos[3], v[3], w[3];
    int ip[3], pq[3];
    int64_t Rq2;
    int H;
};

// What the boundary kernel needs of a body for its links (kept in LDS),
// relative to the floor of the position.
struct LinkBody {
    int ip[3];
    int H;
    float fr[3], v[3], w[3], e[3];
    float B1, beta;
};

// Forces and torques are accumulated in integers, so that the sums are
// bit-identical in any order.  Per body:
//   [0..2]   momentum exchange without the pressure part, 2^-44 fixed point
//   [3..5]   its torque, 2^-44 fixed point
//   [6..8]   conversion force, 2^-44 fixed point
//   [9..11]  conversion torque, 2^-44 fixed point
//   [12..14] Kf = sum over links of k_i c_i (k = 2 on faces, 1 on edges)
//   [15..17] Kr = sum over links of k_i (2 r + 1) x c_i, r the source cell
//            relative to the floor of the body position
// The pressure part of the momentum exchange, -c_i 2 w_i rho0 per link, is
// -(rho0/18) Kf in total, and its torque -(rho0/18)(Kr/2 - p x Kf) with p
// the position minus its floor: both exact up to one final rounding, so the
// pressure terms of a closed surface cancel exactly.  Three sets rotate over
// the steps (written, read, cleared).
constexpr int NACC = 18;
constexpr int NACCSET = 3;
// each set keeps NCOPY copies, picked by block index, so that the atomics of
// many blocks do not pile up on the same addresses; the body update sums them
constexpr int NCOPY = 16;
constexpr int ACCSET_SIZE = NCOPY * MAXB * NACC;  // integers per set
// up to this many bodies the last boundary block of the fluid launch does the
// body update (staged in LDS); more bodies take a separate one-block launch
constexpr int FUSE_MAX = 8;

// Population layouts.  In place (one buffer): after an even step f*_j(x) is
// in plane jbar at x, after an odd step (and initially) in plane j at x + c_j.
// Pull (two buffers): step t reads buffer t & 1 and writes the other, and
// f*_j(x) is in plane j at x of the buffer last written.
constexpr int LAY_AA_ODD = 0, LAY_AA_EVEN = 1, LAY_AB = 2;
// how a step streams: in place with an even or odd index, or pull
constexpr int STEP_AA_EVEN = 0, STEP_AA_ODD = 1, STEP_AB = 2;
constexpr double FX_SCALE = 17592186044416.0;  // 2^44
__device__ __forceinline__ long long to_fx(double v) { return __double2ll_rn(v * FX_SCALE); }
__device__ __forceinline__ double from_fx(unsigned long long v) { return double(static_cast<long long>(v)) / FX_SCALE; }

// Wrap an integer difference in (-2n, 2n) into [0, n).
__device__ __forceinline__ int wrap_small(int a, int n)
{
    if (a < 0) a += n;
    if (a >= n) a -= n;
    return a;
}

struct Box {
    int nx, ny, nz;
    uint32_t n;       // cells
    uint64_t stride;  // elements between population planes (buffer size / 19)
    // Where population i of cell c sits in a buffer: i * dstride + c +
    // (c >> 8) * tmul (see pop_slot).
    uint64_t dstride;
    uint32_t tmul;
    // division by nx and ny as a multiply and shift, exact for dividends
    // below 2^31: q = umulhi(v, m) >> s
    uint32_t mx, sx, my, sy;
};

__device__ __forceinline__ uint32_t div_magic(uint32_t v, uint32_t m, uint32_t s) { return __umulhi(v, m) >> s; }

// Population layout within a buffer.  Tiled (tmul = 18 * 256, dstride =
// 256): the cells form groups of 256 consecutive cells, and the 19
// directions of a group are stored one after another, 256 elements each, so
// group g starts at element g * 19 * 256.  A block of 256 cells then writes
// one contiguous run of 19 * 256 elements and reads from a handful of
// neighbouring runs.  Planes (tmul = 0, dstride = stride): direction i is
// one plane; taken where a tiled buffer would outgrow the 32-bit byte
// offsets of the step kernels.  pop_off is the part that depends on the
// cell (it fits 32 bits in either form); pop_slot the whole index.
__host__ __device__ __forceinline__ uint32_t pop_off(const Box &b, uint32_t c) { return c + (c >> 8) * b.tmul; }
__host__ __device__ __forceinline__ uint64_t pop_slot(const Box &b, int i, uint32_t c)
{
    return uint64_t(i) * b.dstride + pop_off(b, c);
}

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
template <class BT>
__device__ __forceinline__ void lever_arm(const Box &b, const BT &B, int x, int y, int z, double d[3])
{
    d[0] = min_image((x + 0.5) - B.pos[0], b.nx);
    d[1] = min_image((y + 0.5) - B.pos[1], b.ny);
    d[2] = min_image((z + 0.5) - B.pos[2], b.nz);
}

// Inside test in int64 fixed point (2^-20 quanta, centres at i + 1/2, ties
// inside, positions rounded half to even).  Body positions are kept in
// [0, n), so X - P lies in (-L, L) and one conditional wrap gives the
// minimum image.
template <class BT>
__device__ __forceinline__ bool inside_body(const Box &b, const BT &B, int x, int y, int z)
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
        int64_t D = X - P;
        if (D >= L / 2) D -= L;
        else if (D < -(L / 2)) D += L;
        sum += D * D;
    }
    return sum <= B.Rq * B.Rq;
}

// Bounding box of a body: cells floor(pos) - H - g ... floor(pos) + H + g per
// axis (g = 0, or 1 for the box that also covers the next position).
template <class BT>
__device__ __forceinline__ void bbox_origin(const BT &B, int o[3], int g = 0)
{
#pragma unroll
    for (int k = 0; k < 3; ++k) o[k] = static_cast<int>(floor(B.pos[k])) - B.H - g;
}

template <class BT>
__device__ __forceinline__ bool in_bbox(const Box &b, const BT &B, int x, int y, int z, int g = 0)
{
    int o[3];
    bbox_origin(B, o, g);
    const int side = 2 * (B.H + g) + 1;
    return wrap(x - o[0], b.nx) < side && wrap(y - o[1], b.ny) < side && wrap(z - o[2], b.nz) < side;
}

}  // namespace lbsq
