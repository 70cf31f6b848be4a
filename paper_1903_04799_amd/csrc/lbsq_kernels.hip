// lbsq_kernels.hip -- gfx950 kernels of the lattice Boltzmann squirmer library
// (arXiv:1903.04799).
//
// A time step t is two launches on one stream, each covering every
// simulation of a batch (one simulation is a batch of one):
//   k_fluid           every fluid cell, in place on one population buffer
//                     (the AA pattern described below) or, per simulation,
//                     pulling from one of two buffers into the other; FP32
//                     arithmetic on stored deviations, non-temporal stores.
//                     Its leading blocks
//                     take the cells next to a body, found in the bodies'
//                     boxes, one thread per (cell, direction): pull streaming
//                     and the TRT collision of eq. (lb) with moving-wall
//                     bounce-back carrying
//                     the rigid-body velocity eq. (vb) plus the squirmer slip
//                     eq. (squirmer), and the momentum exchange of their
//                     links, eqs. (bbforce), (bbtorque), accumulated as
//                     fixed-point integers.  The other blocks take every
//                     remaining fluid cell, one thread per cell: pull
//                     streaming and the collision (static walls reflected in
//                     place).  The last boundary block of a simulation to
//                     finish does the body update (decode of the integer
//                     force sums, WCA eq. (wca), symplectic Euler) while the
//                     streaming blocks still run; for many bodies the
//                     one-block k_body does it after the launch;
//   k_geoconv         over each moving body's box, the integer inside test
//                     at the new positions gives new owners and neighbour
//                     flags, and the cell conversion of Sec. "Numerical
//                     Method" refills uncovered cells and accumulates the
//                     conversion force eq. (consforce) for the next
//                     integration.
// Owners and the body table are double-buffered (time t is read while time
// t+1 is written); force sums rotate over three accumulator sets.
#include "lbsq_device.h"
#include "lbsq_launch.h"

#include <hip/hip_ext.h>

namespace lbsq {

// ---------------------------------------------------------------------------
// reductions

// FP64 block reduction in a fixed order (xor-shuffle tree inside each wave,
// then the wave results in wave order); result in out[0..K) from threads < K.
template <int K>
__device__ __forceinline__ void block_reduce(double (&v)[K], double *out)
{
    __shared__ double red[BLOCK / 64][K];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double x = v[k];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        v[k] = x;
    }
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) red[wid][k] = v[k];
    __syncthreads();
    if (threadIdx.x < K) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < BLOCK / 64; ++w) s += red[w][threadIdx.x];
        out[threadIdx.x] = s;
    }
}

// Integer block reduction of N values; result in out[0..N) from threads < N
// (integer sums: any order gives the same result).
template <int N>
__device__ __forceinline__ void block_reduce_i64(long long (&v)[N], long long *out)
{
    __shared__ long long red[BLOCK / 64][N];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        long long x = v[k];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        v[k] = x;
    }
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < N; ++k) red[wid][k] = v[k];
    __syncthreads();
    if (threadIdx.x < N) {
        long long s = 0;
#pragma unroll
        for (int w = 0; w < BLOCK / 64; ++w) s += red[w][threadIdx.x];
        out[threadIdx.x] = s;
    }
}

// Add the integer vectors v of all lanes with the same key (a body index;
// key < 0 = nothing) into acc[key * NACC + slot[k]].  Called by whole waves;
// one atomic per component and distinct key in the wave.
template <int N>
__device__ __forceinline__ void wave_accumulate(int key, const long long (&v)[N], const int (&slot)[N],
                                                unsigned long long *acc)
{
    unsigned long long pending = __ballot(key >= 0);
    const int lane = threadIdx.x & 63;
    while (pending) {
        const int leader = __ffsll(static_cast<long long>(pending)) - 1;
        const int kb = __shfl(key, leader, 64);
        const bool mine = key == kb;
        long long s[N];
#pragma unroll
        for (int k = 0; k < N; ++k) {
            s[k] = mine ? v[k] : 0;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) s[k] += __shfl_xor(s[k], o, 64);
        }
        if (lane == leader)
#pragma unroll
            for (int k = 0; k < N; ++k) atomicAdd(&acc[kb * NACC + slot[k]], static_cast<unsigned long long>(s[k]));
        pending &= ~__ballot(mine);
    }
}

__device__ __forceinline__ uint32_t cell_of(const Box &bx, int x, int y, int z)
{
    return uint32_t(x) + uint32_t(bx.nx) * (uint32_t(y) + uint32_t(bx.ny) * uint32_t(z));
}

// ---------------------------------------------------------------------------
// the collision, shared by the streaming and boundary kernels

// Neighbour offsets (mod 2^32) of cell idx in a periodic box.
struct Nbr {
    uint32_t idx, x, y, z;
    uint32_t oxm, oxp, oym, oyp, ozm, ozp;
    __device__ __forceinline__ Nbr(const Box &bx, uint32_t i) : idx(i)
    {
        const uint32_t nx = bx.nx, ny = bx.ny, nz = bx.nz, pl = nx * ny;
        const uint32_t yz = div_magic(i, bx.mx, bx.sx);
        x = i - yz * nx;
        z = div_magic(yz, bx.my, bx.sy);
        y = yz - z * ny;
        oxm = x == 0 ? nx - 1 : uint32_t(-1);
        oxp = x == nx - 1 ? uint32_t(1) - nx : 1u;
        oym = y == 0 ? (ny - 1) * nx : uint32_t(0) - nx;
        oyp = y == ny - 1 ? uint32_t(0) - (ny - 1) * nx : nx;
        ozm = z == 0 ? (nz - 1) * pl : uint32_t(0) - pl;
        ozp = z == nz - 1 ? uint32_t(0) - (nz - 1) * pl : pl;
    }
    // source cell x - c_i of the pull
    __device__ __forceinline__ uint32_t src(int i) const
    {
        uint32_t s = idx;
        if (cx(i) == 1) s += oxm;
        else if (cx(i) == -1) s += oxp;
        if (cy(i) == 1) s += oym;
        else if (cy(i) == -1) s += oyp;
        if (cz(i) == 1) s += ozm;
        else if (cz(i) == -1) s += ozp;
        return s;
    }
};

// TRT collision of the incoming deviations f into out, both as stored (times
// the storage scale s, which is 1 in FP32).  Per pair (i, ibar) the
// symmetric part relaxes with lam_e towards w_i (drho + rho (4.5 (c_i.u)^2 -
// 1.5 u^2)) and the antisymmetric part with lam_o towards 3 w_i rho c_i.u.
// Written with the pair sum sp = f_i + f_ibar and difference dm = f_i -
// f_ibar, which also give the moments:
//   out_i    = (1 - lam_e)/2 sp + s lam_e eq+ + (1 - lam_o)/2 dm + s lam_o eq-
//   out_ibar = (1 - lam_e)/2 sp + s lam_e eq+ - (1 - lam_o)/2 dm - s lam_o eq-
// with the products of lam, w_i and s taken once per simulation.
template <class S, bool FORCE>
__device__ __forceinline__ void collide(const StepArgs &a, const float (&f)[Q], float (&out)[Q])
{
    float sp[Q], dm[Q];  // indexed by the odd member of each pair
    float drs = f[0], jxs = 0.0f, jys = 0.0f, jzs = 0.0f;
#pragma unroll
    for (int i = 1; i < Q; i += 2) {
        sp[i] = f[i] + f[i + 1];
        dm[i] = f[i] - f[i + 1];
        drs += sp[i];
        if (cx(i)) jxs += cx(i) * dm[i];
        if (cy(i)) jys += cy(i) * dm[i];
        if (cz(i)) jzs += cz(i) * dm[i];
    }
    const float drho = S::scaled ? drs * a.c_is : drs;
    const float rho = a.rho0 + drho;
    // one reciprocal (within 1 ulp) instead of a correctly rounded division
    const float ir = __builtin_amdgcn_rcpf(rho);
    float ux, uy, uz;
    if (FORCE) {
        const float is = S::scaled ? a.c_is : 1.0f;
        ux = fmaf(jxs, is, 0.5f * a.g[0]) * ir;
        uy = fmaf(jys, is, 0.5f * a.g[1]) * ir;
        uz = fmaf(jzs, is, 0.5f * a.g[2]) * ir;
    } else {
        const float q = S::scaled ? a.c_is * ir : ir;
        ux = jxs * q;
        uy = jys * q;
        uz = jzs * q;
    }
    const float h = 1.5f * (ux * ux + uy * uy + uz * uz);
    // s lam_e w_k (drho + rho X) = A_k + B_k X;  s lam_o 3 w_k rho c.u = C_k c.u
    const float A0 = a.c_lew[0] * drs, A1 = a.c_lew[1] * drs, A2 = a.c_lew[2] * drs;
    const float B0 = a.c_lews[0] * rho, B1 = a.c_lews[1] * rho, B2 = a.c_lews[2] * rho;
    const float C1 = a.c_low3s[1] * rho, C2 = a.c_low3s[2] * rho;
    out[0] = fmaf(a.c_1mle, f[0], fmaf(-B0, h, A0));
#pragma unroll
    for (int i = 1; i < Q; i += 2) {
        const bool axis = i <= 6;
        const float cu = cx(i) * ux + cy(i) * uy + cz(i) * uz;
        const float X = fmaf(4.5f * cu, cu, -h);
        const float ep = fmaf(axis ? B1 : B2, X, axis ? A1 : A2);
        const float em = (axis ? C1 : C2) * cu;
        const float P = fmaf(a.c_k1, sp[i], ep);
        const float M = fmaf(a.c_k2, dm[i], em);
        out[i] = P + M;
        out[i + 1] = P - M;
    }
    if (FORCE) {
        // Guo forcing, times s like the populations
        const float sc = S::scaled ? a.c_s : 1.0f;
        const float ug = ux * a.g[0] + uy * a.g[1] + uz * a.g[2];
        const float ce = (1.0f - 0.5f * a.lam_e) * sc, co = (1.0f - 0.5f * a.lam_o) * sc;
        out[0] += ce * wgtf(0) * (-3.0f * ug);
#pragma unroll
        for (int i = 1; i < Q; i += 2) {
            const float cu = cx(i) * ux + cy(i) * uy + cz(i) * uz;
            const float cg = cx(i) * a.g[0] + cy(i) * a.g[1] + cz(i) * a.g[2];
            const float se = wgtf(i) * (9.0f * cu * cg - 3.0f * ug);
            const float so = 3.0f * wgtf(i) * cg;
            out[i] += ce * se + co * so;
            out[i + 1] += ce * se - co * so;
        }
    }
}

// The audit adds what is stored (as it will be read back); out is in the
// stored form (times the storage scale).
template <class S>
__device__ __forceinline__ void audit_add(const StepArgs &a, const float (&out)[Q], double (&am)[5])
{
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double v = S::scaled ? double(S::dec(S::enc(out[i])) * a.c_is) : double(out[i]);
        am[0] += v;
        am[1] += cx(i) * v;
        am[2] += cy(i) * v;
        am[3] += cz(i) * v;
    }
    am[4] = 1.0;
}

// The same TRT collision for one direction i of a cell, by the thread that
// owns that direction (the boundary kernel's layout); f holds the cell's 19
// incoming populations in shared memory.  For the pair (i, ibar) both
// threads evaluate the shared symmetric part identically and the
// antisymmetric part with opposite signs.
template <bool FORCE>
__device__ __forceinline__ float collide_one(const StepArgs &a, const float *f, int i)
{
    float drho = 0.0f, jx = 0.0f, jy = 0.0f, jz = 0.0f;
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        const float v = f[k];
        drho += v;
        if (cx(k)) jx += cx(k) * v;
        if (cy(k)) jy += cy(k) * v;
        if (cz(k)) jz += cz(k) * v;
    }
    if (FORCE) {
        jx += 0.5f * a.g[0];
        jy += 0.5f * a.g[1];
        jz += 0.5f * a.g[2];
    }
    const float rho = a.rho0 + drho;
    const float ir = 1.0f / rho;
    const float ux = jx * ir, uy = jy * ir, uz = jz * ir;
    const float usq = ux * ux + uy * uy + uz * uz;
    const float le = a.lam_e, lo = a.lam_o;
    const float w = i == 0 ? wgtf(0) : (i <= 6 ? wgtf(1) : wgtf(7));
    const float fi = f[i];
    float out;
    if (i == 0) {
        out = fi - le * (fi - w * (drho - 1.5f * rho * usq));
    } else {
        const float fb = f[opp(i)];
        const float cu = rcx(i) * ux + rcy(i) * uy + rcz(i) * uz;
        const float ep = w * (drho + rho * (4.5f * cu * cu - 1.5f * usq));
        const float em = w * rho * 3.0f * cu;
        const float fp = 0.5f * (fi + fb), fm = 0.5f * (fi - fb);
        out = fi - le * (fp - ep) - lo * (fm - em);
    }
    if (FORCE) {
        const float ug = ux * a.g[0] + uy * a.g[1] + uz * a.g[2];
        const float ce = 1.0f - 0.5f * le, co = 1.0f - 0.5f * lo;
        if (i == 0) {
            out += ce * w * (-3.0f * ug);
        } else {
            const float cu = rcx(i) * ux + rcy(i) * uy + rcz(i) * uz;
            const float cg = rcx(i) * a.g[0] + rcy(i) * a.g[1] + rcz(i) * a.g[2];
            out += ce * (w * (9.0f * cu * cg - 3.0f * ug)) + co * (3.0f * w * cg);
        }
    }
    return out;
}

// ---------------------------------------------------------------------------
// In-place (AA) streaming on one population buffer F.  A step t reads the
// incoming populations of every fluid cell and writes its post-collision
// populations where the next step will read them:
//   t even: f_i^in(x) = F[i][x];          f*_i(x) -> F[ibar][x]
//   t odd:  f_i^in(x) = F[ibar][x - c_i];  f*_i(x) -> F[i][x + c_i]
// so that between steps the post-collision population f*_j(x) sits in
// F[jbar][x] after an even step and in F[j][x + c_j] after an odd one.  Every
// slot is read and then written by the one cell that owns it in that step.
// Bounce-back from a solid source s = x - c_i takes the cell's own f*_ibar(x),
// which sits in F[ibar][s] before an even step and in F[i][x] before an odd
// one; neither slot is written by anyone else in the step.
//
// Pull streaming on two buffers (chosen per simulation): step t reads buffer
// A = t & 1 and writes the other, B:
//   f_i^in(x) = A[i][x - c_i] (A[ibar][x] from a solid source);
//   f*_i(x) -> B[i][x].

// Element idx of a population plane P, addressed by a 32-bit byte offset from
// the plane's (uniform) base: the loads and stores then take the scalar-base,
// vector-offset form.  Planes are below 4 GiB (checked at creation).  Values
// are in the stored form (times the storage scale).
template <class S>
__device__ __forceinline__ float ld_plane(gptr<const typename S::T> P, uint32_t idx)
{
    using T = typename S::T;
    return S::dec(*(gptr<const T>)((gptr<const char>)P + idx * uint32_t(sizeof(T))));
}
// The same load, non-temporal: the pull layout reads each population once
// per step and never rewrites the lines it reads, so they need not stay in
// the caches.
template <class S>
__device__ __forceinline__ float ld_plane_nt(gptr<const typename S::T> P, uint32_t idx)
{
    using T = typename S::T;
    return S::dec(__builtin_nontemporal_load((gptr<const T>)((gptr<const char>)P + idx * uint32_t(sizeof(T)))));
}
template <class S>
__device__ __forceinline__ void st_plane_nt(gptr<typename S::T> P, uint32_t idx, float v)
{
    using T = typename S::T;
    __builtin_nontemporal_store(S::enc(v), (gptr<T>)((gptr<char>)P + idx * uint32_t(sizeof(T))));
}

// The Q plane bases of the buffer, computed in uniform control flow and
// pinned in scalar registers by an empty asm (otherwise the compiler folds
// them into per-lane 64-bit addresses).
template <class T>
struct Planes {
    gptr<T> p[Q];
    __device__ __forceinline__ Planes(gptr<T> F, uint64_t st)
    {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            gptr<char> b = (gptr<char>)(F + i * st);
            asm volatile("" : "+s"(b));
            p[i] = (gptr<T>)b;
        }
    }
};

// Slot of the post-collision population f*_j of cell (x, y, z) between steps,
// by layout: in place after an odd step (LAY_AA_ODD) or an even one
// (LAY_AA_EVEN), or in the buffer the last step wrote in the two-buffer pull
// layout (LAY_AB).
__device__ __forceinline__ uint64_t post_slot(const Box &bx, int j, int x, int y, int z, int lay)
{
    if (lay == LAY_AB) return pop_slot(bx, j, cell_of(bx, x, y, z));
    if (lay == LAY_AA_EVEN) return pop_slot(bx, opp(j), cell_of(bx, x, y, z));
    return pop_slot(bx, j, cell_of(bx, wrap_small(x + rcx(j), bx.nx), wrap_small(y + rcy(j), bx.ny),
                                wrap_small(z + rcz(j), bx.nz)));
}

// ---------------------------------------------------------------------------
// the hot loop: every fluid cell without a body neighbour

template <class S, bool AUDIT, bool FORCE, int MODE>
__device__ __forceinline__ void stream_collide_block(const StepArgs &a, gptr<typename S::T> F, int64_t to_write,
                                                     gptr<const uint8_t> own, gptr<const uint32_t> wmask,
                                                     double *__restrict__ audit_part, uint32_t grp, uint32_t part)
{
    // cells grp * BLOCK ... of the box; the audit partial goes to entry
    // part.  F is the buffer read (and, in place, written); the pull layout
    // writes the other buffer, to_write bytes away
    const Box &bx = a.box;
    const Planes<typename S::T> P(F, bx.dstride);
    const uint32_t idx = grp * BLOCK + threadIdx.x;
    const uint8_t o = idx < bx.n ? own[idx] : OWN_WALL;
    double am[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (o == OWN_FLUID || o == OWN_NB_WALL) {
        const Nbr nb(bx, idx);
        const uint32_t oi = pop_off(bx, idx);
        float f[Q];
        if (!__any(o == OWN_NB_WALL)) {
            // no cell of the wave is next to a static wall: plain pulls (a
            // wave-uniform branch, so that boxes without walls, and most
            // waves of boxes with them, keep every load unconditional)
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                if (MODE == STEP_AA_ODD) f[i] = ld_plane<S>(P.p[opp(i)], pop_off(bx, nb.src(i)));
                else if (MODE == STEP_AB) f[i] = ld_plane_nt<S>(P.p[i], pop_off(bx, nb.src(i)));
                else f[i] = ld_plane<S>(P.p[i], oi);
            }
        } else {
            // no-slip walls: a population that would come from a wall is the
            // cell's own opposite post-collision population.  Wall-adjacent
            // cells take their sources' wall bits from the static mask, so
            // they run the same loads as the other cells plus one load per
            // wall link.
            const uint32_t wm = o == OWN_NB_WALL ? wmask[idx] : 0u;
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                // either load, never both: one destination per direction
                const bool wall = (wm >> i) & 1u;
                if (MODE == STEP_AA_ODD)
                    f[i] = wall ? ld_plane<S>(P.p[i], oi) : ld_plane<S>(P.p[opp(i)], pop_off(bx, nb.src(i)));
                else if (MODE == STEP_AB)
                    f[i] = wall ? ld_plane_nt<S>(P.p[opp(i)], oi) : ld_plane_nt<S>(P.p[i], pop_off(bx, nb.src(i)));
                else
                    f[i] = wall ? ld_plane<S>(P.p[opp(i)], pop_off(bx, nb.src(i))) : ld_plane<S>(P.p[i], oi);
            }
        }
        float out[Q];
        collide<S, FORCE>(a, f, out);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            if (MODE == STEP_AA_ODD) st_plane_nt<S>(P.p[i], pop_off(bx, nb.src(opp(i))), out[i]);
            else if (MODE == STEP_AB)
                st_plane_nt<S>((gptr<typename S::T>)((gptr<char>)P.p[i] + to_write), oi, out[i]);
            else st_plane_nt<S>(P.p[opp(i)], oi, out[i]);
        }
        if (AUDIT) audit_add<S>(a, out, am);
    }
    if (AUDIT) block_reduce<5>(am, audit_part + size_t(part) * 5);
}

// ---------------------------------------------------------------------------
// rigid bodies

__device__ void rotate_by(double e[3], const double w[3])
{
    const double th = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    if (th == 0.0) return;
    const double k[3] = {w[0] / th, w[1] / th, w[2] / th};
    const double kxe[3] = {k[1] * e[2] - k[2] * e[1], k[2] * e[0] - k[0] * e[2], k[0] * e[1] - k[1] * e[0]};
    const double ke = k[0] * e[0] + k[1] * e[1] + k[2] * e[2];
    // the per-step angle is tiny: a short series gives sin, cos and 1 - cos
    // to double precision without the library's argument reduction
    double s, c, omc;
    if (th < 1e-2) {
        const double t2 = th * th;
        s = th * (1.0 - t2 / 6.0 * (1.0 - t2 / 20.0 * (1.0 - t2 / 42.0 * (1.0 - t2 / 72.0))));
        omc = t2 / 2.0 * (1.0 - t2 / 12.0 * (1.0 - t2 / 30.0 * (1.0 - t2 / 56.0)));
        c = 1.0 - omc;
    } else {
        s = sin(th);
        c = cos(th);
        omc = 1.0 - c;
    }
    double o[3];
    for (int a = 0; a < 3; ++a) o[a] = e[a] * c + kxe[a] * s + k[a] * ke * omc;
    const double nn = sqrt(o[0] * o[0] + o[1] * o[1] + o[2] * o[2]);
    for (int a = 0; a < 3; ++a) e[a] = o[a] / nn;
}

__device__ double wca_magnitude(double r, double sigma, double eps)
{
    const double rc = 1.122462048309373 * sigma;  // 2^(1/6) sigma
    if (r >= rc) return 0.0;
    if (r < 0.05 * sigma) r = 0.05 * sigma;
    const double s2 = (sigma / r) * (sigma / r);
    const double sr6 = s2 * s2 * s2;
    return 24.0 * eps / r * (2.0 * sr6 * sr6 - sr6);
}

// State of body b at t+1, in place in B (which holds its state at t), from
// the step's integer force sums q (NACC values) and WCA against every other
// body of the table cur (time t).
__device__ void advance_body(const Box &bx, const DevBody *__restrict__ cur, int nbody, int b, const long long *q,
                             double rho0, double sigma, double eps, DevBody &B, int *__restrict__ err)
{
    const int nn[3] = {bx.nx, bx.ny, bx.nz};
    double kf[3], kr[3], p[3];
    for (int k = 0; k < 3; ++k) {
        kf[k] = double(q[12 + k]);
        kr[k] = double(q[15 + k]);
        p[k] = B.pos[k] - floor(B.pos[k]);
    }
    const double pr = rho0 / 18.0;
    const double pxk[3] = {p[1] * kf[2] - p[2] * kf[1], p[2] * kf[0] - p[0] * kf[2], p[0] * kf[1] - p[1] * kf[0]};
    for (int k = 0; k < 3; ++k) {
        B.Fbb[k] = double(q[k]) / FX_SCALE - pr * kf[k];
        B.Tbb[k] = double(q[3 + k]) / FX_SCALE - pr * (0.5 * kr[k] - pxk[k]);
        B.Fc[k] = double(q[6 + k]) / FX_SCALE;
        B.Tc[k] = double(q[9 + k]) / FX_SCALE;
        B.Fwca[k] = 0.0;
    }
    for (int j = 0; j < nbody; ++j) {
        if (j == b) continue;
        double dv[3];
        for (int k = 0; k < 3; ++k) dv[k] = min_image(B.pos[k] - cur[j].pos[k], nn[k]);
        const double dist = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
        const double fm = wca_magnitude(dist - B.R - cur[j].R, sigma, eps);
        if (fm == 0.0) continue;
        for (int k = 0; k < 3; ++k) B.Fwca[k] += fm * dv[k] / dist;
    }
    for (int k = 0; k < 3; ++k) {
        B.F[k] = B.Fbb[k] + B.Fc[k] + B.Fwca[k];
        B.T[k] = B.Tbb[k] + B.Tc[k];
    }
    if (B.mode == 0) {
        for (int k = 0; k < 3; ++k) {
            B.v[k] += B.F[k] / B.m;
            B.w[k] += B.T[k] / B.I;
        }
    }
    if (B.mode == 0 || B.mode == 2) {
        for (int k = 0; k < 3; ++k) {
            if (!(fabs(B.v[k]) < 1.0)) err[2] = 1;
            double x = B.pos[k] + B.v[k];
            if (x >= nn[k]) x -= nn[k];
            if (x < 0.0) x += nn[k];
            // positions stay in [0, n) even after a flagged runaway
            if (!(x >= 0.0 && x < nn[k])) x = 0.0;
            B.pos[k] = x;
        }
        rotate_by(B.e, B.w);
    }
}

// The step's integer sums of every body: the NCOPY copies of an
// accumulator set added up into s_q[body][k].  The loads are device-coherent
// so that a block of the launch that produced the sums can read them once
// every producer has arrived.
__device__ void gather_sums(int nbody, unsigned long long *acc, long long (*s_q)[NACC])
{
    for (int j = threadIdx.x; j < nbody * NACC; j += BLOCK) {
        long long t = 0;
#pragma unroll
        for (int c = 0; c < NCOPY; ++c)
            t += static_cast<long long>(
                __hip_atomic_load(&acc[c * (MAXB * NACC) + j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        s_q[j / NACC][j % NACC] = t;
    }
    __syncthreads();
}

// Zero the first nbody entries of every copy of an accumulator set.
__device__ __forceinline__ void clear_set(int nbody, unsigned long long *__restrict__ acc)
{
    for (int j = threadIdx.x; j < NCOPY * nbody * NACC; j += BLOCK) {
        const int c = j / (nbody * NACC);
        acc[c * (MAXB * NACC) + (j - c * nbody * NACC)] = 0ull;
    }
}

// the accumulator set of step t
__device__ __forceinline__ unsigned long long *acc_set(unsigned long long *acc, int64_t t)
{
    return acc + size_t(t % NACCSET) * ACCSET_SIZE;
}

// Body update of one simulation (descriptor D[0]) by one block, for more
// bodies than the fluid launch updates itself; also clears the accumulator
// set of the step after next.
__global__ __launch_bounds__(BLOCK) void k_body(const SimDesc *__restrict__ D, int64_t k)
{
    __shared__ long long s_q[MAXB][NACC];
    const SimDesc &d = D[0];
    const int64_t t = d.t0 + k;
    if (t >= d.t_end) return;
    const int c = int(t & 1);
    gather_sums(d.nbody, acc_set(d.acc, t), s_q);
    for (int b = threadIdx.x; b < d.nbody; b += BLOCK) {
        DevBody B = d.bodies[c][b];
        advance_body(d.a.box, d.bodies[c], d.nbody, b, s_q[b], d.a.rho0d, d.wca_sigma, d.wca_eps, B, d.err);
        d.bodies[c ^ 1][b] = B;
    }
    clear_set(d.nbody, acc_set(d.acc, t + 2));
}

// the simulation of a batched launch that block blk belongs to
__device__ __forceinline__ int find_sim(const uint32_t *start, int nsim, uint32_t blk)
{
    int s = 0;
    while (s + 1 < nsim && blk >= start[s + 1]) ++s;
    return s;
}

// ---------------------------------------------------------------------------
// work layout of the boundary and geometry kernels: a block takes CPB
// consecutive cells of one body's box (grown by g cells on each side), one
// thread per (cell, direction); blocks [start[m], start[m+1]) belong to the
// m-th listed body

struct Slot {
    int m;      // position in the body list
    int cl, i;  // cell slot in the block, direction
    int x, y, z;
    bool valid;
};

template <class BT>
__device__ __forceinline__ Slot slot_of(const Box &bx, const BT *bodies, const int *ids, const int *start, int nlist,
                                        int g, int blk)
{
    Slot r;
    r.cl = threadIdx.x / Q;
    r.i = threadIdx.x - r.cl * Q;
    int m = 0;
    while (m + 1 < nlist && blk >= start[m + 1]) ++m;
    r.m = m;
    const BT &B = bodies[ids[m]];
    const int side = 2 * (B.H + g) + 1;
    const uint32_t l = uint32_t(blk - start[m]) * CPB + r.cl;
    r.valid = r.cl < CPB && l < uint32_t(side) * side * side;
    int o[3];
    bbox_origin(B, o, g);
    r.x = wrap(o[0] + int(l % side), bx.nx);
    r.y = wrap(o[1] + int((l / side) % side), bx.ny);
    r.z = wrap(o[2] + int(l / (side * side)), bx.nz);
    return r;
}

// the lowest-listed body whose box contains the cell handles it, so every
// cell is processed once
template <class BT>
__device__ __forceinline__ bool first_box(const Box &bx, const BT *bodies, const int *ids, int m, int x, int y, int z,
                                          int g)
{
    for (int mm = 0; mm < m; ++mm)
        if (in_bbox(bx, bodies[ids[mm]], x, y, z, g)) return false;
    return true;
}

// ---------------------------------------------------------------------------
// cells next to a body: moving-wall bounce-back and momentum exchange

// The link of cell (x, y, z) in direction i whose source s = x - c_i is a
// cell of body B: returns f_i^in = f_ibar*(x) + 6 w_i rho_w c_i.v_b, with the
// wall velocity eq. (vb) plus the slip of eq. (squirmer) taken at the link
// midpoint (centre of s + c_i/2), where the halfway bounce-back wall lies.
// The momentum handed to the body, -c_i (f_ibar*(x) + f_i^in(x)), is split
// into its small part (FP32 force and torque in fv, lever arm to the centre
// of s as in eq. (bbtorque)) and the pressure part -c_i 2 w_i rho0 (integer
// counts kf, kr).
__device__ __forceinline__ float body_link(const Box &bx, const LinkBody &B, int i, int x, int y, int z, float fob,
                                           float rho_w, float (&fv)[6], int (&kf)[3], int (&kr)[3])
{
    const int c[3] = {rcx(i), rcy(i), rcz(i)};
    const int k = i <= 6 ? 2 : 1;  // 36 w_i
    const int sc[3] = {x - c[0], y - c[1], z - c[2]};
    const int n[3] = {bx.nx, bx.ny, bx.nz};
    int r[3];
    float d[3], m[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        r[a] = wrap_small(sc[a] - (B.ip[a] - B.H), n[a]) - B.H;  // source relative to floor(pos)
        d[a] = (float(r[a]) + 0.5f) - B.fr[a];
        m[a] = d[a] + 0.5f * float(c[a]);
    }
    float vb[3] = {B.v[0] + B.w[1] * m[2] - B.w[2] * m[1], B.v[1] + B.w[2] * m[0] - B.w[0] * m[2],
                   B.v[2] + B.w[0] * m[1] - B.w[1] * m[0]};
    if (B.B1 != 0.0f) {
        const float ir = rsqrtf(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
        const float nn[3] = {m[0] * ir, m[1] * ir, m[2] * ir};
        const float en = B.e[0] * nn[0] + B.e[1] * nn[1] + B.e[2] * nn[2];
        const float am = B.B1 * (1.0f + B.beta * en);
#pragma unroll
        for (int a = 0; a < 3; ++a) vb[a] += am * (en * nn[a] - B.e[a]);
    }
    const float w = k == 2 ? 1.0f / 18.0f : 1.0f / 36.0f;
    const float sh = 6.0f * w * rho_w * (c[0] * vb[0] + c[1] * vb[1] + c[2] * vb[2]);
    const float fin = fob + sh;
    const float var = fob + fin;
    const float dp[3] = {-c[0] * var, -c[1] * var, -c[2] * var};
    fv[0] = dp[0];
    fv[1] = dp[1];
    fv[2] = dp[2];
    fv[3] = d[1] * dp[2] - d[2] * dp[1];
    fv[4] = d[2] * dp[0] - d[0] * dp[2];
    fv[5] = d[0] * dp[1] - d[1] * dp[0];
#pragma unroll
    for (int a = 0; a < 3; ++a) kf[a] = k * c[a];
    const int q[3] = {2 * r[0] + 1, 2 * r[1] + 1, 2 * r[2] + 1};
    kr[0] = k * (q[1] * c[2] - q[2] * c[1]);
    kr[1] = k * (q[2] * c[0] - q[0] * c[2]);
    kr[2] = k * (q[0] * c[1] - q[1] * c[0]);
    return fin;
}

// Every fluid cell with a body neighbour: pull streaming where the source is
// fluid, reflection at walls, moving-wall bounce-back at bodies, then the
// collision.  Momentum exchange: integer sums, reduced over the block for
// the box's own body.
// Add v to *p at device scope and wait until the addition has been
// performed, so that anything the thread does afterwards (an arrival at the
// boundary blocks' counter) is ordered after it without a cache flush.
__device__ __forceinline__ void add_performed(unsigned long long *p, unsigned long long v)
{
    const unsigned long long old = __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    asm volatile("" ::"v"(old));
}

template <class S, bool AUDIT, bool FORCE, int MODE>
__device__ __forceinline__ void boundary_block(const StepArgs &a, gptr<typename S::T> F, int64_t to_write,
                                               gptr<const uint8_t> own,
                                               const DevBody *__restrict__ cur, int nbody,
                                               const int4 *__restrict__ blkinfo, const uint32_t *__restrict__ shell,
                                               unsigned long long *__restrict__ acc, gptr<const float> dens_prev,
                                               gptr<float> dens_cur, double *__restrict__ audit_part, int blk)
{
    extern __shared__ double lds_dyn[];  // nbody LinkBody entries
    LinkBody *lb = reinterpret_cast<LinkBody *>(lds_dyn);
    __shared__ float s_f[CPB][Q + 1], s_o[CPB][Q + 1];
    __shared__ int s_minb[CPB];
    const Box &bx = a.box;
    // the block's body and first shell cell (precomputed), the thread's
    // (shell cell, direction)
    const int4 bi = blkinfo[blk];
    const int home = bi.x;
    const int cl = threadIdx.x / Q, i = threadIdx.x - cl * Q;
    const bool valid = cl < bi.z;
    const uint32_t e = valid ? shell[bi.y + cl] : 0x20080200u;  // offset (0, 0, 0) when unused
    // the bodies' link data, staged once per block
    for (int b = threadIdx.x; b < nbody; b += BLOCK) {
        const DevBody &D = cur[b];
        LinkBody &L = lb[b];
        for (int k = 0; k < 3; ++k) {
            const double flo = floor(D.pos[k]);
            L.ip[k] = int(flo);
            L.fr[k] = float(D.pos[k] - flo);
            L.v[k] = float(D.v[k]);
            L.w[k] = float(D.w[k]);
            L.e[k] = float(D.e[k]);
        }
        L.H = D.H;
        L.B1 = float(D.B1);
        L.beta = float(D.beta);
    }
    if (threadIdx.x < CPB) s_minb[threadIdx.x] = 0x7fffffff;
    __syncthreads();
    const int x = wrap_small(lb[home].ip[0] + int(e & 1023u) - 512, bx.nx);
    const int y = wrap_small(lb[home].ip[1] + int((e >> 10) & 1023u) - 512, bx.ny);
    const int z = wrap_small(lb[home].ip[2] + int((e >> 20) & 1023u) - 512, bx.nz);
    const uint32_t c = cell_of(bx, x, y, z);
    const uint32_t s = cell_of(bx, wrap_small(x - rcx(i), bx.nx), wrap_small(y - rcy(i), bx.ny),
                               wrap_small(z - rcz(i), bx.nz));
    // the owners, both candidate populations and the cell's link density
    // are loaded together, so that no load waits for another: the incoming
    // population where the source is fluid, the cell's own f*_ibar (for a
    // reflection) otherwise
    const uint8_t oc = valid ? own[c] : OWN_WALL;
    const uint8_t os = (valid && i > 0) ? own[s] : OWN_FLUID;
    float f_in = 0.0f, f_ref = 0.0f, dprev = 0.0f;
    if (valid) {
        constexpr bool ODD = MODE == STEP_AA_ODD;
        if (MODE == STEP_AB) {
            f_in = S::ld(F[pop_slot(bx, i, s)], a.inv_scale);
            f_ref = S::ld(F[pop_slot(bx, opp(i), c)], a.inv_scale);
        } else {
            f_in = S::ld(F[ODD ? pop_slot(bx, opp(i), s) : pop_slot(bx, i, c)], a.inv_scale);
            f_ref = S::ld(F[ODD ? pop_slot(bx, i, c) : pop_slot(bx, opp(i), s)], a.inv_scale);
        }
        dprev = dens_prev[c];
    }
    const bool cand = oc == OWN_NB_BODY;
    const float fl = is_fluid(os) ? f_in : f_ref;
    // a cell next to several bodies is taken by the smallest of them (the
    // shell lists of all of them contain it)
    if (cand && is_body(os)) atomicMin(&s_minb[cl], int(os) - 1);
    __syncthreads();
    const bool active = cand && s_minb[cl] == home;
    int key = -1;  // body of this thread's link
    long long v[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (active) {
        float fin = fl;
        if (is_body(os)) {
            // local density of the cell's post-collision populations, kept
            // from the previous step (its slots are rewritten in place)
            const float rw = a.rho0 + dprev;
            key = os - 1;
            float fv[6];
            int kf[3], kr[3];
            fin = body_link(bx, lb[key], i, x, y, z, fl, rw, fv, kf, kr);
            for (int k = 0; k < 6; ++k) v[k] = to_fx(fv[k]);
            for (int k = 0; k < 3; ++k) {
                v[6 + k] = kf[k];
                v[9 + k] = kr[k];
            }
        }
        s_f[cl][i] = fin;
    }
    __syncthreads();
    // collision, one direction per thread; the stored (rounded) values are
    // summed for the link density of the next step and for the audit
    double am[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (active) {
        const typename S::T o = S::st(collide_one<FORCE>(a, s_f[cl], i), a.scale);
        s_o[cl][i] = S::ld(o, a.inv_scale);
        if (MODE == STEP_AA_ODD) {
            const uint64_t at = pop_slot(bx, i, cell_of(bx, wrap_small(x + rcx(i), bx.nx),
                                                        wrap_small(y + rcy(i), bx.ny), wrap_small(z + rcz(i), bx.nz)));
            __builtin_nontemporal_store(o, &F[at]);
        } else if (MODE == STEP_AB) {
            const gptr<typename S::T> W = (gptr<typename S::T>)((gptr<char>)F + to_write);
            __builtin_nontemporal_store(o, &W[pop_slot(bx, i, c)]);
        } else {
            __builtin_nontemporal_store(o, &F[pop_slot(bx, opp(i), c)]);
        }
    }
    __syncthreads();
    if (active && i == 0) {
        float dr = 0.0f;
#pragma unroll
        for (int j = 0; j < Q; ++j) dr += s_o[cl][j];
        dens_cur[c] = dr;
        if (AUDIT) {
#pragma unroll
            for (int j = 0; j < Q; ++j) {
                const double v = s_o[cl][j];
                am[0] += v;
                am[1] += cx(j) * v;
                am[2] += cy(j) * v;
                am[3] += cz(j) * v;
            }
            am[4] = 1.0;
        }
    }
    // links into the box's own body: reduced over the block, then one atomic
    // per component into the block's copy of the sums (blocks without such a
    // link skip this); links into another body (a cell touching two bodies)
    // are added directly
    constexpr int slot[12] = {0, 1, 2, 3, 4, 5, 12, 13, 14, 15, 16, 17};
    unsigned long long *copy = acc + (blk % NCOPY) * (MAXB * NACC);
    if (key >= 0 && key != home) {
        for (int k = 0; k < 12; ++k) add_performed(&copy[key * NACC + slot[k]], static_cast<unsigned long long>(v[k]));
        for (int k = 0; k < 12; ++k) v[k] = 0;
    }
    if (__syncthreads_or(key == home)) {
        __shared__ long long s_sum[12];
        block_reduce_i64<12>(v, s_sum);
        if (threadIdx.x < 12)
            add_performed(&copy[home * NACC + slot[threadIdx.x]], static_cast<unsigned long long>(s_sum[threadIdx.x]));
    }
    if (AUDIT) block_reduce<5>(am, audit_part + size_t(blk) * 5);
}

// Body update of a simulation with at most FUSE_MAX bodies, by the last of
// its boundary blocks to finish.  Every boundary block has added its link
// momentum to the step's sums (the conversion force of the previous move is
// already there), waited until those device-scope additions were performed,
// and then arrives at the counter with one more device-scope addition.  The
// block that arrives last therefore finds every sum in place: it reads them
// with device-coherent loads, advances the bodies into the other table and
// clears the accumulator set of the step after next, while the streaming
// blocks still run.  No cache is flushed or invalidated (that would cost
// the streaming blocks their cached neighbours).  It leaves the counter at
// zero for the next step.  The new state is staged in LDS, which keeps the
// update's registers within those of the streaming path.
__device__ __forceinline__ void arrive_and_update(const SimDesc &d, int c, int64_t t)
{
    __shared__ long long s_q[FUSE_MAX][NACC];
    __shared__ DevBody s_nb[FUSE_MAX];
    __shared__ int s_last;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned prev = __hip_atomic_fetch_add(d.arrive, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_last = prev == unsigned(d.nblk_b - 1);
    }
    __syncthreads();
    if (!s_last) return;
    // the bodies' states at t, copied in 8-byte words by the whole block
    static_assert(sizeof(DevBody) % sizeof(double) == 0, "body table copied in 8-byte words");
    constexpr int W = int(sizeof(DevBody) / sizeof(double));
    double *nb = reinterpret_cast<double *>(s_nb);
    const double *cur = reinterpret_cast<const double *>(d.bodies[c]);
    for (int j = threadIdx.x; j < d.nbody * W; j += BLOCK) nb[j] = cur[j];
    gather_sums(d.nbody, acc_set(d.acc, t), s_q);
    if (int(threadIdx.x) < d.nbody)
        advance_body(d.a.box, d.bodies[c], d.nbody, threadIdx.x, s_q[threadIdx.x], d.a.rho0d, d.wca_sigma,
                     d.wca_eps, s_nb[threadIdx.x], d.err);
    __syncthreads();
    double *nxt = reinterpret_cast<double *>(d.bodies[c ^ 1]);
    for (int j = threadIdx.x; j < d.nbody * W; j += BLOCK) nxt[j] = nb[j];
    clear_set(d.nbody, acc_set(d.acc, t + 2));
    if (threadIdx.x == 0) __hip_atomic_store(d.arrive, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The update of every fluid cell of every simulation of a batch, one launch
// per step.  A simulation's blocks are contiguous; its first nblk_b blocks
// take the cells next to a body (listed first so that their longer latency
// overlaps the streaming blocks), the rest stream and collide the remaining
// cells, BLOCK consecutive cells per block (with static walls, only the
// groups of BLOCK cells that hold a cell other than a wall).  Audit
// partials: streaming block j writes slot j, boundary block j writes slot
// nblk_s + j.
template <class S, bool AUDIT, bool FORCE>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(AUDIT ? 4 : S::waves))) void k_fluid(const SimDesc *__restrict__ D, BatchMap m, int64_t k)
{
    using T = typename S::T;
    const int si = find_sim(m.fluid0, m.nsim, blockIdx.x);
    const SimDesc &d = D[si];
    const int64_t t = d.t0 + k;
    if (t >= d.t_end) return;
    const int c = int(t & 1);
    // in place the step's parity picks the streaming direction; the pull
    // layout reads buffer c and writes the other.  Either is the same for
    // every block of a simulation.
    const bool ab = d.f2 != nullptr;
    const gptr<T> F = as_global(static_cast<T *>(ab && c ? d.f2 : d.f));
    const int64_t to_write = ab ? (c ? static_cast<const char *>(d.f) - static_cast<const char *>(d.f2)
                                     : static_cast<const char *>(d.f2) - static_cast<const char *>(d.f))
                                : 0;
    const gptr<const uint8_t> own = as_global(static_cast<const uint8_t *>(d.own[c]));
    const gptr<const uint32_t> wmask = as_global(d.wmask);
    const int blk = int(blockIdx.x - m.fluid0[si]);
    if (blk < d.nblk_b) {
        const gptr<const float> dp = as_global(static_cast<const float *>(d.dens[c ^ 1]));
        const gptr<float> dc = as_global(d.dens[c]);
        double *ap = d.audit_part + size_t(d.nblk_s) * 5;
        if (ab)
            boundary_block<S, AUDIT, FORCE, STEP_AB>(d.a, F, to_write, own, d.bodies[c], d.nbody, d.blkinfo, d.shell,
                                                     acc_set(d.acc, t), dp, dc, ap, blk);
        else if (c)
            boundary_block<S, AUDIT, FORCE, STEP_AA_ODD>(d.a, F, 0, own, d.bodies[c], d.nbody, d.blkinfo, d.shell,
                                                         acc_set(d.acc, t), dp, dc, ap, blk);
        else
            boundary_block<S, AUDIT, FORCE, STEP_AA_EVEN>(d.a, F, 0, own, d.bodies[c], d.nbody, d.blkinfo, d.shell,
                                                          acc_set(d.acc, t), dp, dc, ap, blk);
        if (d.nbody <= FUSE_MAX) arrive_and_update(d, c, t);
    } else {
        // streaming block j takes the j-th group of BLOCK cells, or with
        // static walls the j-th group that holds a cell other than a wall
        const uint32_t j = uint32_t(blk - d.nblk_b);
        const uint32_t g = d.sgrp ? d.sgrp[j] : j;
        if (ab)
            stream_collide_block<S, AUDIT, FORCE, STEP_AB>(d.a, F, to_write, own, wmask, d.audit_part, g, j);
        else if (c)
            stream_collide_block<S, AUDIT, FORCE, STEP_AA_ODD>(d.a, F, 0, own, wmask, d.audit_part, g, j);
        else
            stream_collide_block<S, AUDIT, FORCE, STEP_AA_EVEN>(d.a, F, 0, own, wmask, d.audit_part, g, j);
    }
}

// ---------------------------------------------------------------------------
// geometry and cell conversion at the new positions.  Owners of every cell
// of the moving bodies' boxes are recomputed into the other owner buffer;
// cells outside the boxes did not change and are equal in both buffers.

// Inside test against a body staged in LDS: the same predicate as the
// fixed-point test on absolute positions (cell centre minus rounded position,
// minimum image, squared length <= Rq^2), evaluated relative to the floor of
// the position, where the difference of a cell within the box needs no wrap
// and fits 32 bits.
__device__ __forceinline__ bool inside_geo(const Box &bx, const GeoBody &B, int x, int y, int z)
{
    const int c[3] = {x, y, z};
    const int n[3] = {bx.nx, bx.ny, bx.nz};
    int64_t sum = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int r = wrap_small(c[k] - (B.ip[k] - B.H), n[k]) - B.H;
        if (r < -B.H || r > B.H) return false;
        const int D = (2 * r + 1) * (1 << 19) - B.pq[k];
        sum += int64_t(D) * int64_t(D);
    }
    return sum <= B.Rq2;
}

// owner of cell (x, y, z) at the new positions, given its old owner
// (static walls stay; first body that contains it; clash if two do)
__device__ __forceinline__ uint8_t new_owner(const Box &bx, const GeoBody *gb, int nbody, uint8_t old, int x, int y,
                                             int z, bool &clash)
{
    if (old == OWN_WALL) return OWN_WALL;
    uint8_t nw = OWN_FLUID;
    for (int b = 0; b < nbody; ++b) {
        if (!inside_geo(bx, gb[b], x, y, z)) continue;
        if (nw != OWN_FLUID) clash = true;
        else nw = uint8_t(b + 1);
    }
    return nw;
}

// new body state in the form the inside test and the refill use
__device__ __forceinline__ void stage_geo(const DevBody &D, GeoBody &G)
{
    for (int k = 0; k < 3; ++k) {
        G.pos[k] = D.pos[k];
        G.v[k] = D.v[k];
        G.w[k] = D.w[k];
        const double fl = floor(D.pos[k]);
        G.ip[k] = int(fl);
        G.pq[k] = int(__double2ll_rn(D.pos[k] * 1048576.0) - int64_t(fl) * 1048576);
    }
    G.Rq2 = D.Rq * D.Rq;
    G.H = D.H;
}

// One thread per (cell, neighbour): the cells are those of the moving
// bodies' boxes around their old positions (table cur), grown by one cell so
// that they contain the boxes around the new positions (table nxt, written
// by the body update of the fluid launch or by k_body).
template <class S>
__device__ __forceinline__ void geoconv_block(const StepArgs &a, const DevBody *__restrict__ cur,
                                              const DevBody *__restrict__ nxt, int nbody,
                                              const int *__restrict__ ids, const int *__restrict__ start, int nlist,
                                              unsigned long long *__restrict__ acc_conv,
                                              gptr<const uint8_t> own_old, gptr<uint8_t> own_new,
                                              gptr<typename S::T> A, int lay, gptr<float> dens,
                                              int *__restrict__ err, int blk)
{
    extern __shared__ double lds_dyn[];  // nbody GeoBody
    GeoBody *gb = reinterpret_cast<GeoBody *>(lds_dyn);
    __shared__ uint8_t s_on[CPB][Q + 1], s_oo[CPB][Q + 1];
    __shared__ double s_rho[CPB][Q + 1];
    if (nlist == 0) return;
    const Box &bx = a.box;
    const Slot sl = slot_of(bx, cur, ids, start, nlist, 1, blk);
    const int i = sl.i;
    const bool mine = sl.valid && first_box(bx, cur, ids, sl.m, sl.x, sl.y, sl.z, 1);
    // neighbour i of the cell (i = 0: the cell itself)
    const int nxc = wrap_small(sl.x + rcx(i), bx.nx), nyc = wrap_small(sl.y + rcy(i), bx.ny),
              nzc = wrap_small(sl.z + rcz(i), bx.nz);
    const uint32_t ncell = cell_of(bx, nxc, nyc, nzc);
    const uint8_t oo = mine ? own_old[ncell] : uint8_t(0);
    for (int b = threadIdx.x; b < nbody; b += BLOCK) stage_geo(nxt[b], gb[b]);
    __syncthreads();
    bool clash = false;
    if (mine) {
        s_on[sl.cl][i] = new_owner(bx, gb, nbody, oo, nxc, nyc, nzc, clash);
        s_oo[sl.cl][i] = oo;
    }
    __syncthreads();
    if (mine) {
        // densities of the neighbours that are fluid at both time levels,
        // needed where the cell is uncovered
        double r = -1.0;
        const bool uncovered = is_body(s_oo[sl.cl][0]) && s_on[sl.cl][0] == OWN_FLUID;
        if (uncovered && i > 0 && s_on[sl.cl][i] == OWN_FLUID && is_fluid(oo)) {
            r = 0.0;
            for (int j = 0; j < Q; ++j) r += double(S::ld(A[post_slot(bx, j, nxc, nyc, nzc, lay)], a.inv_scale));
            r += a.rho0d;
        }
        s_rho[sl.cl][i] = r;
    }
    __syncthreads();
    int key = -1;
    long long fx[6] = {0, 0, 0, 0, 0, 0};
    if (mine && i == 0) {
        const uint32_t c = ncell;
        const uint8_t old = oo, nw = s_on[sl.cl][0];
        double p[3] = {0.0, 0.0, 0.0}, sg = 0.0;
        int eb = -1;  // body of a conversion event
        if (is_body(nw)) {
            own_new[c] = nw;
            if (is_fluid(old)) {
                // covered: the body swallows the cell's populations
                for (int j = 1; j < Q; ++j) {
                    const double fj = S::ld(A[post_slot(bx, j, sl.x, sl.y, sl.z, lay)], a.inv_scale);
                    p[0] += rcx(j) * fj;
                    p[1] += rcy(j) * fj;
                    p[2] += rcz(j) * fj;
                }
                sg = 1.0;
                eb = nw - 1;
            }
        } else if (nw == OWN_WALL) {
            own_new[c] = OWN_WALL;
        } else {
            bool nb_body = false, nb_wall = false;
            double rsum = 0.0;
            int rcnt = 0;
            for (int j = 1; j < Q; ++j) {
                const uint8_t on = s_on[sl.cl][j];
                nb_body |= is_body(on);
                nb_wall |= on == OWN_WALL;
                const double rj = s_rho[sl.cl][j];
                if (rj >= 0.0) {
                    rsum += rj;
                    ++rcnt;
                }
            }
            own_new[c] = nb_body ? OWN_NB_BODY : (nb_wall ? OWN_NB_WALL : OWN_FLUID);
            if (is_body(old)) {
                // uncovered: refill with f^eq(rho_bar, v + w x d); its
                // momentum comes from the body that left
                eb = old - 1;
                const GeoBody &B = gb[eb];
                double d[3], u[3];
                lever_arm(bx, B, sl.x, sl.y, sl.z, d);
                u[0] = B.v[0] + B.w[1] * d[2] - B.w[2] * d[1];
                u[1] = B.v[1] + B.w[2] * d[0] - B.w[0] * d[2];
                u[2] = B.v[2] + B.w[0] * d[1] - B.w[1] * d[0];
                const double rb = rcnt ? rsum / rcnt : a.rho0d;
                const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
                for (int j = 0; j < Q; ++j) {
                    const double cu = rcx(j) * u[0] + rcy(j) * u[1] + rcz(j) * u[2];
                    const double w = j == 0 ? 1.0 / 3.0 : (j <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
                    const double dev = w * (rb - a.rho0d) + w * rb * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
                    A[post_slot(bx, j, sl.x, sl.y, sl.z, lay)] = S::st(float(dev), a.scale);
                }
                p[0] = rb * u[0];
                p[1] = rb * u[1];
                p[2] = rb * u[2];
                sg = -1.0;
            }
            if (nb_body && old != OWN_NB_BODY) {
                // a cell that becomes a body neighbour (or is uncovered next
                // to one): the density its links will use in the next step,
                // summed as the boundary kernel sums what it stores
                float dr = 0.0f;
                for (int j = 0; j < Q; ++j) dr += S::ld(A[post_slot(bx, j, sl.x, sl.y, sl.z, lay)], a.inv_scale);
                dens[c] = dr;
            }
        }
        if (eb >= 0) {
            double d[3];
            lever_arm(bx, gb[eb], sl.x, sl.y, sl.z, d);
            key = eb;
            fx[0] = to_fx(sg * p[0]);
            fx[1] = to_fx(sg * p[1]);
            fx[2] = to_fx(sg * p[2]);
            fx[3] = to_fx(sg * (d[1] * p[2] - d[2] * p[1]));
            fx[4] = to_fx(sg * (d[2] * p[0] - d[0] * p[2]));
            fx[5] = to_fx(sg * (d[0] * p[1] - d[1] * p[0]));
        }
    }
    if (clash) err[0] = 1;
    constexpr int slot[6] = {6, 7, 8, 9, 10, 11};
    if (__any(key >= 0)) wave_accumulate<6>(key, fx, slot, acc_conv + (blk % NCOPY) * (MAXB * NACC));
}

// Geometry and conversion of every simulation of a batch, one launch per
// step (blocks of a simulation contiguous).
template <class S>
__global__ __launch_bounds__(BLOCK) void k_geoconv(const SimDesc *__restrict__ D, BatchMap m, int64_t k)
{
    const int si = find_sim(m.geo0, m.nsim, blockIdx.x);
    const SimDesc &d = D[si];
    const int64_t t = d.t0 + k;
    if (t >= d.t_end) return;
    const int c = int(t & 1);
    // the populations after step t: in place in the one buffer, or in the
    // buffer step t wrote
    const bool ab = d.f2 != nullptr;
    void *post = ab && c == 0 ? d.f2 : d.f;
    const int lay = ab ? LAY_AB : (c == 0 ? LAY_AA_EVEN : LAY_AA_ODD);
    geoconv_block<S>(d.a, d.bodies[c], d.bodies[c ^ 1], d.nbody, d.mov_ids, d.mov_start, d.nmov,
                     acc_set(d.acc, t + 1), as_global(static_cast<const uint8_t *>(d.own[c])), as_global(d.own[c ^ 1]),
                     as_global(static_cast<typename S::T *>(post)), lay, as_global(d.dens[c]), d.err,
                     int(blockIdx.x - m.geo0[si]));
}

// ---------------------------------------------------------------------------
// set-up, audit and readout kernels (outside the timed step)

// Owner flags of the fluid cells (which of their neighbours are solid), and,
// where static walls exist, every non-wall cell's wall mask: bit i set when
// the source x - c_i of its direction i is a wall.  The mask depends on the
// static walls only, so it is also right for body cells that later turn
// fluid.
__global__ __launch_bounds__(BLOCK) void k_classify(Box bx, uint8_t *__restrict__ own, uint32_t *__restrict__ wmask,
                                                    int set_flags)
{
    const uint32_t c = blockIdx.x * BLOCK + threadIdx.x;
    if (c >= bx.n) return;
    const uint8_t o = own[c];
    if (o == OWN_WALL) return;
    const int x = c % bx.nx, y = (c / bx.nx) % bx.ny, z = c / (uint32_t(bx.nx) * bx.ny);
    bool nb_body = false;
    uint32_t wm = 0;
    for (int i = 1; i < Q; ++i) {
        const uint8_t on = own[cell_of(bx, wrap(x + cx(i), bx.nx), wrap(y + cy(i), bx.ny), wrap(z + cz(i), bx.nz))];
        nb_body |= is_body(on);
        // the neighbour x + c_i is the source of the opposite direction
        if (on == OWN_WALL) wm |= 1u << opp(i);
    }
    if (wmask) wmask[c] = wm;
    if (set_flags && is_fluid(o)) own[c] = nb_body ? OWN_NB_BODY : (wm ? OWN_NB_WALL : OWN_FLUID);
}

// mark (or, with check_only, test) the cells of body b
__global__ __launch_bounds__(BLOCK) void k_body_cells(Box bx, const DevBody *__restrict__ bodies, int b,
                                                      uint8_t *__restrict__ own, int check_only,
                                                      int *__restrict__ err)
{
    const DevBody &B = bodies[b];
    const int side = 2 * B.H + 1;
    const uint32_t l = blockIdx.x * BLOCK + threadIdx.x;
    if (l >= uint32_t(side) * side * side) return;
    int o[3];
    bbox_origin(B, o);
    const int x = wrap(o[0] + int(l % side), bx.nx), y = wrap(o[1] + int((l / side) % side), bx.ny),
              z = wrap(o[2] + int(l / (side * side)), bx.nz);
    if (!inside_body(bx, B, x, y, z)) return;
    const uint32_t c = cell_of(bx, x, y, z);
    if (check_only) {
        if (!is_fluid(own[c])) err[0] = 1;
    } else {
        own[c] = uint8_t(b + 1);
    }
}

// coordinates of cell c
__device__ __forceinline__ void coords(const Box &bx, uint32_t c, int &x, int &y, int &z)
{
    x = int(c % uint32_t(bx.nx));
    const uint32_t yz = c / uint32_t(bx.nx);
    y = int(yz % uint32_t(bx.ny));
    z = int(yz / uint32_t(bx.ny));
}

template <class S>
__global__ __launch_bounds__(BLOCK) void k_audit(StepArgs a, const typename S::T *__restrict__ A,
                                                 const uint8_t *__restrict__ own, int lay,
                                                 double *__restrict__ part)
{
    const uint32_t c = blockIdx.x * BLOCK + threadIdx.x;
    double am[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (c < a.box.n && is_fluid(own[c])) {
        int x, y, z;
        coords(a.box, c, x, y, z);
        for (int i = 0; i < Q; ++i) {
            const double v = S::ld(A[post_slot(a.box, i, x, y, z, lay)], a.inv_scale);
            am[0] += v;
            am[1] += cx(i) * v;
            am[2] += cy(i) * v;
            am[3] += cz(i) * v;
        }
        am[4] = 1.0;
    }
    block_reduce<5>(am, part + size_t(blockIdx.x) * 5);
}

// sum nblk partials of 5 doubles in a fixed order; flag non-finite results
__global__ __launch_bounds__(BLOCK) void k_audit_final(const double *__restrict__ part, int nblk,
                                                       double *__restrict__ out, int *__restrict__ err)
{
    __shared__ double red[BLOCK][5];
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nblk; b += BLOCK)
        for (int k = 0; k < 5; ++k) acc[k] += part[size_t(b) * 5 + k];
    for (int k = 0; k < 5; ++k) red[threadIdx.x][k] = acc[k];
    __syncthreads();
    for (int h = BLOCK / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h)
            for (int k = 0; k < 5; ++k) red[threadIdx.x][k] += red[threadIdx.x + h][k];
        __syncthreads();
    }
    if (threadIdx.x < 5) {
        const double v = red[0][threadIdx.x];
        out[threadIdx.x] = v;
        if (!isfinite(v)) err[1] = 1;
    }
}

template <class S>
__global__ __launch_bounds__(BLOCK) void k_fields(StepArgs a, const typename S::T *__restrict__ A,
                                                  const uint8_t *__restrict__ own, int lay, uint32_t c0,
                                                  uint32_t cnt, double *__restrict__ rho,
                                                  double *__restrict__ u, uint8_t *__restrict__ own_out)
{
    // cells [c0, c0 + cnt) into slots 0..cnt-1; u holds three planes of cnt
    const uint32_t q = blockIdx.x * BLOCK + threadIdx.x;
    if (q >= cnt) return;
    const uint32_t c = c0 + q;
    const uint8_t o = own[c];
    own_out[q] = is_fluid(o) ? 0 : o;
    if (!is_fluid(o)) {
        rho[q] = 0.0;
        u[q] = u[cnt + q] = u[2 * size_t(cnt) + q] = 0.0;
        return;
    }
    double r = 0.0, j[3] = {0.0, 0.0, 0.0};
    int x, y, z;
    coords(a.box, c, x, y, z);
    for (int i = 0; i < Q; ++i) {
        const double v = S::ld(A[post_slot(a.box, i, x, y, z, lay)], a.inv_scale);
        r += v;
        j[0] += cx(i) * v;
        j[1] += cy(i) * v;
        j[2] += cz(i) * v;
    }
    r += a.rho0d;
    rho[q] = r;
    for (int k = 0; k < 3; ++k) u[k * size_t(cnt) + q] = (j[k] - 0.5 * double(a.g[k])) / r;
}

// Population i of every cell as FP64 (solid cells read 0), and back.  Each
// (i, cell) pair owns one slot of the buffer in either layout, so these are
// permutations of it.
template <class S>
__global__ __launch_bounds__(BLOCK) void k_plane_to_f64(StepArgs a, const typename S::T *__restrict__ A,
                                                        const uint8_t *__restrict__ own, int lay, int i,
                                                        double *__restrict__ out)
{
    const uint32_t c = blockIdx.x * BLOCK + threadIdx.x;
    if (c >= a.box.n) return;
    int x, y, z;
    coords(a.box, c, x, y, z);
    out[c] = is_fluid(own[c])
                 ? wgt(i) * a.rho0d + double(S::ld(A[post_slot(a.box, i, x, y, z, lay)], a.inv_scale))
                 : 0.0;
}

template <class S>
__global__ __launch_bounds__(BLOCK) void k_plane_from_f64(StepArgs a, typename S::T *__restrict__ A,
                                                          const uint8_t *__restrict__ own, int lay, int i,
                                                          const double *__restrict__ in)
{
    const uint32_t c = blockIdx.x * BLOCK + threadIdx.x;
    if (c >= a.box.n) return;
    int x, y, z;
    coords(a.box, c, x, y, z);
    A[post_slot(a.box, i, x, y, z, lay)] =
        is_fluid(own[c]) ? S::st(float(in[c] - wgt(i) * a.rho0d), a.scale) : S::st(0.0f, a.scale);
}

// Densities (sum of stored deviations, in the boundary kernel's order) of
// every cell next to a body, for the links of the next step.
template <class S>
__global__ __launch_bounds__(BLOCK) void k_dens(StepArgs a, const typename S::T *__restrict__ A,
                                                const uint8_t *__restrict__ own, int lay,
                                                float *__restrict__ dens)
{
    const uint32_t c = blockIdx.x * BLOCK + threadIdx.x;
    if (c >= a.box.n || own[c] != OWN_NB_BODY) return;
    int x, y, z;
    coords(a.box, c, x, y, z);
    float dr = 0.0f;
    for (int i = 0; i < Q; ++i) dr += S::ld(A[post_slot(a.box, i, x, y, z, lay)], a.inv_scale);
    dens[c] = dr;
}

// bit i of mask[c] set when fluid cell c has a solid source c - c_i
__global__ __launch_bounds__(BLOCK) void k_link_mask(Box bx, const uint8_t *__restrict__ own,
                                                     uint32_t *__restrict__ mask)
{
    const uint32_t c = blockIdx.x * BLOCK + threadIdx.x;
    if (c >= bx.n) return;
    uint32_t m = 0;
    if (is_fluid(own[c])) {
        const int x = c % bx.nx, y = (c / bx.nx) % bx.ny, z = c / (uint32_t(bx.nx) * bx.ny);
        for (int i = 1; i < Q; ++i)
            if (!is_fluid(own[cell_of(bx, wrap(x - cx(i), bx.nx), wrap(y - cy(i), bx.ny), wrap(z - cz(i), bx.nz))]))
                m |= 1u << i;
    }
    mask[c] = m;
}

// ---------------------------------------------------------------------------
// host-side launchers (storage type resolved here)

#define LB_TRY(x)                        \
    do {                                 \
        const hipError_t e_ = (x);       \
        if (e_ != hipSuccess) return e_; \
    } while (0)

template <class S>
static hipError_t launch_batch_t(const BatchLaunch &L)
{
    const BatchMap &m = L.map;
    const uint32_t nf = m.fluid0[m.nsim], ng = m.geo0[m.nsim];
    if (nf > 0) {
        auto kf = L.audit ? (L.force ? k_fluid<S, true, true> : k_fluid<S, true, false>)
                          : (L.force ? k_fluid<S, false, true> : k_fluid<S, false, false>);
        const uint32_t lds = uint32_t(size_t(L.nbody_max) * sizeof(LinkBody));
        // timing events, when asked for, are stamped with the launch's own
        // start and end (not with markers queued around it)
        if (L.ev_start && L.ev_stop)
            hipExtLaunchKernelGGL(kf, dim3(nf), dim3(BLOCK), lds, L.stream, L.ev_start, L.ev_stop, 0u, L.desc, m, L.k);
        else
            hipLaunchKernelGGL(kf, dim3(nf), dim3(BLOCK), lds, L.stream, L.desc, m, L.k);
        LB_TRY(hipGetLastError());
    } else if (L.ev_start && L.ev_stop) {
        LB_TRY(hipEventRecord(L.ev_start, L.stream));
        LB_TRY(hipEventRecord(L.ev_stop, L.stream));
    }
    if (L.audit) {
        hipLaunchKernelGGL(k_audit_final, dim3(1), dim3(BLOCK), 0, L.stream, L.audit_part, L.npart, L.audit_out,
                           L.err);
        LB_TRY(hipGetLastError());
    }
    if (L.body_kernel) {
        hipLaunchKernelGGL(k_body, dim3(1), dim3(BLOCK), 0, L.stream, L.desc, L.k);
        LB_TRY(hipGetLastError());
    }
    if (ng > 0) {
        const size_t lds = size_t(L.nbody_max) * sizeof(GeoBody);  // staged bodies
        hipLaunchKernelGGL(k_geoconv<S>, dim3(ng), dim3(BLOCK), lds, L.stream, L.desc, m, L.k);
        LB_TRY(hipGetLastError());
    }
    return hipSuccess;
}

hipError_t launch_batch_step(int storage, const BatchLaunch &L)
{
    switch (storage) {
    case 1: return launch_batch_t<StF16>(L);
    case 2: return launch_batch_t<StBF16>(L);
    default: return launch_batch_t<StF32>(L);
    }
}

hipError_t launch_classify(const Box &bx, uint8_t *own, uint32_t *wmask, int set_flags, hipStream_t s)
{
    hipLaunchKernelGGL(k_classify, dim3((bx.n + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, bx, own, wmask, set_flags);
    return hipGetLastError();
}

hipError_t launch_body_cells(const Box &bx, const DevBody *bodies, int b, int side, uint8_t *own, int check,
                             int *err, hipStream_t s)
{
    const uint32_t cells = uint32_t(side) * side * side;
    hipLaunchKernelGGL(k_body_cells, dim3((cells + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, bx, bodies, b, own,
                       check, err);
    return hipGetLastError();
}

template <class S>
static hipError_t launch_audit_t(const StepArgs &a, const void *A, const uint8_t *own, int lay, double *part,
                                 double *out, int *err, hipStream_t s)
{
    const int nblk = int((a.box.n + BLOCK - 1) / BLOCK);
    hipLaunchKernelGGL(k_audit<S>, dim3(nblk), dim3(BLOCK), 0, s, a, static_cast<const typename S::T *>(A), own,
                       lay, part);
    hipLaunchKernelGGL(k_audit_final, dim3(1), dim3(BLOCK), 0, s, part, nblk, out, err);
    return hipGetLastError();
}

hipError_t launch_audit(int storage, const StepArgs &a, const void *A, const uint8_t *own, int lay,
                        double *part, double *out, int *err, hipStream_t s)
{
    switch (storage) {
    case 1: return launch_audit_t<StF16>(a, A, own, lay, part, out, err, s);
    case 2: return launch_audit_t<StBF16>(a, A, own, lay, part, out, err, s);
    default: return launch_audit_t<StF32>(a, A, own, lay, part, out, err, s);
    }
}

template <class S>
static hipError_t launch_fields_t(const StepArgs &a, const void *A, const uint8_t *own, int lay, uint32_t c0,
                                  uint32_t cnt, double *rho, double *u, uint8_t *own_out, hipStream_t s)
{
    if (cnt == 0 || c0 > a.box.n || cnt > a.box.n - c0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_fields<S>, dim3((cnt + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, a,
                       static_cast<const typename S::T *>(A), own, lay, c0, cnt, rho, u, own_out);
    return hipGetLastError();
}

hipError_t launch_fields(int storage, const StepArgs &a, const void *A, const uint8_t *own, int lay, uint32_t c0,
                         uint32_t cnt, double *rho, double *u, uint8_t *own_out, hipStream_t s)
{
    switch (storage) {
    case 1: return launch_fields_t<StF16>(a, A, own, lay, c0, cnt, rho, u, own_out, s);
    case 2: return launch_fields_t<StBF16>(a, A, own, lay, c0, cnt, rho, u, own_out, s);
    default: return launch_fields_t<StF32>(a, A, own, lay, c0, cnt, rho, u, own_out, s);
    }
}

template <class S>
static hipError_t launch_plane_t(const StepArgs &a, void *A, const uint8_t *own, int lay, int i, double *buf,
                                 int to_f64, hipStream_t s)
{
    using T = typename S::T;
    const dim3 g((a.box.n + BLOCK - 1) / BLOCK);
    if (to_f64)
        hipLaunchKernelGGL(k_plane_to_f64<S>, g, dim3(BLOCK), 0, s, a, static_cast<const T *>(A), own, lay, i,
                           buf);
    else
        hipLaunchKernelGGL(k_plane_from_f64<S>, g, dim3(BLOCK), 0, s, a, static_cast<T *>(A), own, lay, i,
                           static_cast<const double *>(buf));
    return hipGetLastError();
}

hipError_t launch_plane(int storage, const StepArgs &a, void *A, const uint8_t *own, int lay, int i,
                        double *buf, int to_f64, hipStream_t s)
{
    switch (storage) {
    case 1: return launch_plane_t<StF16>(a, A, own, lay, i, buf, to_f64, s);
    case 2: return launch_plane_t<StBF16>(a, A, own, lay, i, buf, to_f64, s);
    default: return launch_plane_t<StF32>(a, A, own, lay, i, buf, to_f64, s);
    }
}

template <class S>
static hipError_t launch_dens_t(const StepArgs &a, const void *A, const uint8_t *own, int lay, float *dens,
                                hipStream_t s)
{
    hipLaunchKernelGGL(k_dens<S>, dim3((a.box.n + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, a,
                       static_cast<const typename S::T *>(A), own, lay, dens);
    return hipGetLastError();
}

hipError_t launch_dens(int storage, const StepArgs &a, const void *A, const uint8_t *own, int lay, float *dens,
                       hipStream_t s)
{
    switch (storage) {
    case 1: return launch_dens_t<StF16>(a, A, own, lay, dens, s);
    case 2: return launch_dens_t<StBF16>(a, A, own, lay, dens, s);
    default: return launch_dens_t<StF32>(a, A, own, lay, dens, s);
    }
}

hipError_t launch_link_mask(const Box &bx, const uint8_t *own, uint32_t *mask, hipStream_t s)
{
    hipLaunchKernelGGL(k_link_mask, dim3((bx.n + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, bx, own, mask);
    return hipGetLastError();
}

}  // namespace lbsq
