// lbsq_kernels.hip -- gfx950 kernels of the lattice Boltzmann squirmer library
// (arXiv:1903.04799).
//
// One time step is five launches on the handle's stream:
//   k_geom      integer inside test over each moving body's bounding box:
//               new owners and covered/uncovered events (fixed point, exact);
//   k_refill    neighbour-solid flags and the refill of uncovered cells with
//               the equilibrium at the mean neighbour density and the rigid
//               body velocity (cell conversion, Sec. "Numerical Method");
//   k_force     momentum exchange eqs. (bbforce), (bbtorque) over the links
//               of every body plus the conversion force eq. (consforce), as
//               FP64 per-block partials;
//   k_stream_collide  the hot loop: pull streaming with moving-wall
//               bounce-back and the TRT collision of eq. (lb), FP32 math on
//               stored deviations;
//   k_body      fixed-order FP64 reduction of the partials, WCA eq. (wca),
//               symplectic Euler.
#include "lbsq_device.h"
#include "lbsq_launch.h"

namespace lbsq {

constexpr uint16_t EV_COVERED = 0x100;
constexpr uint16_t EV_UNCOVERED = 0x200;

// ---------------------------------------------------------------------------
// block reductions in FP64 (fixed order: xor-shuffle tree inside a wave, then
// wave 0 sums the per-wave results in wave order)

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

// ---------------------------------------------------------------------------
// bounding-box work distribution: blocks [start[m], start[m+1]) cover the
// (2H+1)^3 cells of the m-th listed body

struct BoxCell {
    int m;  // position in the body list
    int x, y, z;
    bool valid;
};

__device__ __forceinline__ BoxCell box_cell(const Box &bx, const DevBody *bodies, const int *ids,
                                            const int *start, int nlist)
{
    BoxCell r;
    const int blk = blockIdx.x;
    int m = 0;
    while (m + 1 < nlist && blk >= start[m + 1]) ++m;
    r.m = m;
    const DevBody &B = bodies[ids[m]];
    const int side = 2 * B.H + 1;
    const uint32_t l = uint32_t(blk - start[m]) * BLOCK + threadIdx.x;
    r.valid = l < uint32_t(side) * side * side;
    int o[3];
    bbox_origin(B, o);
    const int lx = l % side, ly = (l / side) % side, lz = l / (side * side);
    r.x = wrap(o[0] + lx, bx.nx);
    r.y = wrap(o[1] + ly, bx.ny);
    r.z = wrap(o[2] + lz, bx.nz);
    return r;
}

__device__ __forceinline__ uint32_t cell_of(const Box &bx, int x, int y, int z)
{
    return uint32_t(x) + uint32_t(bx.nx) * (uint32_t(y) + uint32_t(bx.ny) * uint32_t(z));
}

// the lowest-listed moving body whose box contains the cell does the
// per-cell (not per-body) work, so every cell is written by one thread only
__device__ __forceinline__ bool first_box(const Box &bx, const DevBody *bodies, const int *ids, int m,
                                          int x, int y, int z)
{
    for (int mm = 0; mm < m; ++mm)
        if (in_bbox(bx, bodies[ids[mm]], x, y, z)) return false;
    return true;
}

// ---------------------------------------------------------------------------
// geometry

__global__ __launch_bounds__(BLOCK) void k_geom(Box bx, const DevBody *__restrict__ bodies, int nbody,
                                                const int *__restrict__ ids, const int *__restrict__ start,
                                                int nlist, uint8_t *__restrict__ own,
                                                uint16_t *__restrict__ ev, int *__restrict__ err)
{
    const BoxCell bc = box_cell(bx, bodies, ids, start, nlist);
    if (!bc.valid || !first_box(bx, bodies, ids, bc.m, bc.x, bc.y, bc.z)) return;
    const uint32_t c = cell_of(bx, bc.x, bc.y, bc.z);
    const uint8_t old = own[c];
    if (old == OWN_WALL) {
        ev[c] = 0;
        return;
    }
    uint8_t nw = OWN_FLUID;
    bool clash = false;
    for (int b = 0; b < nbody; ++b) {
        if (!in_bbox(bx, bodies[b], bc.x, bc.y, bc.z)) continue;
        if (inside_body(bx, bodies[b], bc.x, bc.y, bc.z)) {
            if (nw != OWN_FLUID) clash = true;
            else nw = uint8_t(b + 1);
        }
    }
    if (clash) err[0] = 1;
    uint16_t e = 0;
    if (nw != OWN_FLUID) {
        if (is_fluid(old)) e = EV_COVERED | nw;
        if (old != nw) own[c] = nw;
    } else if (is_body(old)) {
        e = EV_UNCOVERED | old;
        own[c] = OWN_FLUID;
    }
    ev[c] = e;
}

// density of cell c from stored deviations, FP64
template <class S>
__device__ __forceinline__ double cell_density(const typename S::T *A, uint64_t stride, uint32_t c,
                                               double rho0, float inv)
{
    double r = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) r += double(S::ld(A[i * stride + c], inv));
    return rho0 + r;
}

// mean density of the D3Q19 neighbours that are fluid at both time levels
template <class S>
__device__ __forceinline__ double refill_density(const Box &bx, const typename S::T *A, const uint8_t *own,
                                                 const uint16_t *ev, int x, int y, int z, double rho0,
                                                 float inv)
{
    double sum = 0.0;
    int cnt = 0;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const uint32_t n = cell_of(bx, wrap(x + cx(i), bx.nx), wrap(y + cy(i), bx.ny), wrap(z + cz(i), bx.nz));
        if (is_fluid(own[n]) && !(ev[n] & EV_UNCOVERED)) {
            sum += cell_density<S>(A, bx.stride, n, rho0, inv);
            ++cnt;
        }
    }
    return cnt ? sum / cnt : rho0;
}

template <class S>
__global__ __launch_bounds__(BLOCK) void k_refill(StepArgs a, const DevBody *__restrict__ bodies,
                                                  const int *__restrict__ ids, const int *__restrict__ start,
                                                  int nlist, uint8_t *__restrict__ own,
                                                  const uint16_t *__restrict__ ev, typename S::T *__restrict__ A)
{
    const Box &bx = a.box;
    const BoxCell bc = box_cell(bx, bodies, ids, start, nlist);
    if (!bc.valid || !first_box(bx, bodies, ids, bc.m, bc.x, bc.y, bc.z)) return;
    const uint32_t c = cell_of(bx, bc.x, bc.y, bc.z);
    const uint8_t o = own[c];
    if (!is_fluid(o)) return;
    bool nb = false;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const uint32_t n = cell_of(bx, wrap(bc.x + cx(i), bx.nx), wrap(bc.y + cy(i), bx.ny), wrap(bc.z + cz(i), bx.nz));
        nb |= !is_fluid(own[n]);
    }
    const uint8_t flag = nb ? OWN_FLUID_NB : OWN_FLUID;
    if (flag != o) own[c] = flag;
    const uint16_t e = ev[c];
    if (!(e & EV_UNCOVERED)) return;
    const DevBody &B = bodies[(e & 0xff) - 1];
    const double rb = refill_density<S>(bx, A, own, ev, bc.x, bc.y, bc.z, a.rho0d, a.inv_scale);
    double d[3], u[3];
    lever_arm(bx, B, bc.x, bc.y, bc.z, d);
    u[0] = B.v[0] + B.w[1] * d[2] - B.w[2] * d[1];
    u[1] = B.v[1] + B.w[2] * d[0] - B.w[0] * d[2];
    u[2] = B.v[2] + B.w[0] * d[1] - B.w[1] * d[0];
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double cu = cx(i) * u[0] + cy(i) * u[1] + cz(i) * u[2];
        const double dev = wgt(i) * (rb - a.rho0d) + wgt(i) * rb * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
        A[i * bx.stride + c] = S::st(float(dev), a.scale);
    }
}

// ---------------------------------------------------------------------------
// momentum exchange and conversion force, per-block FP64 partials
// partial layout: Fbb[3] Tbb[3] Fc[3] Tc[3]

template <class S>
__global__ __launch_bounds__(BLOCK) void k_force(StepArgs a, const DevBody *__restrict__ bodies,
                                                 const int *__restrict__ ids, const int *__restrict__ start,
                                                 int nlist, const uint8_t *__restrict__ own,
                                                 const uint16_t *__restrict__ ev,
                                                 const typename S::T *__restrict__ A, double *__restrict__ part)
{
    const Box &bx = a.box;
    const BoxCell bc = box_cell(bx, bodies, ids, start, nlist);
    const int b = ids[bc.m];
    const DevBody &B = bodies[b];
    double acc[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = 0.0;
    if (bc.valid) {
        const uint32_t c = cell_of(bx, bc.x, bc.y, bc.z);
        const uint8_t o = own[c];
        const uint8_t me = uint8_t(b + 1);
        if (o == OWN_FLUID_NB) {
            float fo[Q];
            float rw = 0.0f;
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                fo[i] = S::ld(A[i * bx.stride + c], a.inv_scale);
                rw += fo[i];
            }
            rw += a.rho0;
#pragma unroll
            for (int i = 1; i < Q; ++i) {
                const int sx = wrap(bc.x - cx(i), bx.nx), sy = wrap(bc.y - cy(i), bx.ny), sz = wrap(bc.z - cz(i), bx.nz);
                if (own[cell_of(bx, sx, sy, sz)] != me) continue;
                double d[3];
                lever_arm(bx, B, sx, sy, sz, d);
                const float fin = fo[opp(i)] + bounce_shift(i, rw, B, d);
                const double s = 2.0 * wgt(i) * a.rho0d + double(fo[opp(i)]) + double(fin);
                const double dp[3] = {-cx(i) * s, -cy(i) * s, -cz(i) * s};
                acc[0] += dp[0];
                acc[1] += dp[1];
                acc[2] += dp[2];
                acc[3] += d[1] * dp[2] - d[2] * dp[1];
                acc[4] += d[2] * dp[0] - d[0] * dp[2];
                acc[5] += d[0] * dp[1] - d[1] * dp[0];
            }
        }
        if (B.mode != 1) {
            const uint16_t e = ev[c];
            if ((e & 0xff) == me && (e & (EV_COVERED | EV_UNCOVERED))) {
                double d[3], p[3];
                lever_arm(bx, B, bc.x, bc.y, bc.z, d);
                double sg;
                if (e & EV_COVERED) {
                    // the populations the body swallows (still in A)
                    p[0] = p[1] = p[2] = 0.0;
#pragma unroll
                    for (int i = 1; i < Q; ++i) {
                        const double fi = S::ld(A[i * bx.stride + c], a.inv_scale);
                        p[0] += cx(i) * fi;
                        p[1] += cy(i) * fi;
                        p[2] += cz(i) * fi;
                    }
                    sg = 1.0;
                } else {
                    // momentum of the refill, taken from the body
                    const double rb = refill_density<S>(bx, A, own, ev, bc.x, bc.y, bc.z, a.rho0d, a.inv_scale);
                    p[0] = rb * (B.v[0] + B.w[1] * d[2] - B.w[2] * d[1]);
                    p[1] = rb * (B.v[1] + B.w[2] * d[0] - B.w[0] * d[2]);
                    p[2] = rb * (B.v[2] + B.w[0] * d[1] - B.w[1] * d[0]);
                    sg = -1.0;
                }
                acc[6] += sg * p[0];
                acc[7] += sg * p[1];
                acc[8] += sg * p[2];
                acc[9] += sg * (d[1] * p[2] - d[2] * p[1]);
                acc[10] += sg * (d[2] * p[0] - d[0] * p[2]);
                acc[11] += sg * (d[0] * p[1] - d[1] * p[0]);
            }
        }
    }
    block_reduce<12>(acc, part + size_t(blockIdx.x) * 12);
}

// ---------------------------------------------------------------------------
// the hot loop: pull streaming + bounce-back + TRT collision

template <class S, bool AUDIT, bool FORCE>
__global__ __launch_bounds__(BLOCK) void k_stream_collide(StepArgs a, const typename S::T *__restrict__ A,
                                                          typename S::T *__restrict__ Bf,
                                                          const uint8_t *__restrict__ own,
                                                          const DevBody *__restrict__ bodies,
                                                          double *__restrict__ audit_part)
{
    const Box &bx = a.box;
    const uint32_t idx = blockIdx.x * BLOCK + threadIdx.x;
    const uint64_t st = bx.stride;
    const uint8_t o = idx < bx.n ? own[idx] : OWN_WALL;
    double am[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (is_fluid(o)) {
        const uint32_t nx = bx.nx, ny = bx.ny, nz = bx.nz;
        const uint32_t x = idx % nx, yz = idx / nx, y = yz % ny, z = yz / ny;
        const uint32_t pl = nx * ny;
        // unsigned offsets (mod 2^32) to the -1 / +1 neighbour on each axis
        const uint32_t oxm = x == 0 ? nx - 1 : uint32_t(-1), oxp = x == nx - 1 ? uint32_t(1) - nx : 1u;
        const uint32_t oym = y == 0 ? (ny - 1) * nx : uint32_t(0) - nx, oyp = y == ny - 1 ? uint32_t(0) - (ny - 1) * nx : nx;
        const uint32_t ozm = z == 0 ? (nz - 1) * pl : uint32_t(0) - pl, ozp = z == nz - 1 ? uint32_t(0) - (nz - 1) * pl : pl;
        auto src = [&](int i) -> uint32_t {
            uint32_t s = idx;
            if (cx(i) == 1) s += oxm;
            else if (cx(i) == -1) s += oxp;
            if (cy(i) == 1) s += oym;
            else if (cy(i) == -1) s += oyp;
            if (cz(i) == 1) s += ozm;
            else if (cz(i) == -1) s += ozp;
            return s;
        };
        float f[Q];
        if (o == OWN_FLUID) {
#pragma unroll
            for (int i = 0; i < Q; ++i) f[i] = S::ld(A[i * st + src(i)], a.inv_scale);
        } else {
            float fo[Q];
            float rw = 0.0f;
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                fo[i] = S::ld(A[i * st + idx], a.inv_scale);
                rw += fo[i];
            }
            rw += a.rho0;
            f[0] = fo[0];
#pragma unroll
            for (int i = 1; i < Q; ++i) {
                const uint32_t s = src(i);
                const uint8_t os = own[s];
                if (is_fluid(os)) {
                    f[i] = S::ld(A[i * st + s], a.inv_scale);
                } else if (os == OWN_WALL) {
                    f[i] = fo[opp(i)];
                } else {
                    double d[3];
                    const DevBody &B = bodies[os - 1];
                    lever_arm(bx, B, int(wrap(int(x) - cx(i), nx)), int(wrap(int(y) - cy(i), ny)),
                              int(wrap(int(z) - cz(i), nz)), d);
                    f[i] = fo[opp(i)] + bounce_shift(i, rw, B, d);
                }
            }
        }
        // moments of the incoming deviations
        float drho = 0.0f, jx = 0.0f, jy = 0.0f, jz = 0.0f;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            drho += f[i];
            if (cx(i)) jx += cx(i) * f[i];
            if (cy(i)) jy += cy(i) * f[i];
            if (cz(i)) jz += cz(i) * f[i];
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
        float out[Q];
        out[0] = f[0] - le * (f[0] - wgtf(0) * (drho - 1.5f * rho * usq));
#pragma unroll
        for (int i = 1; i < Q; i += 2) {
            const int ib = i + 1;
            const float cu = cx(i) * ux + cy(i) * uy + cz(i) * uz;
            const float ep = wgtf(i) * (drho + rho * (4.5f * cu * cu - 1.5f * usq));
            const float em = wgtf(i) * rho * 3.0f * cu;
            const float fp = 0.5f * (f[i] + f[ib]), fm = 0.5f * (f[i] - f[ib]);
            const float de = le * (fp - ep), dodd = lo * (fm - em);
            out[i] = f[i] - de - dodd;
            out[ib] = f[ib] - de + dodd;
        }
        if (FORCE) {
            const float ug = ux * a.g[0] + uy * a.g[1] + uz * a.g[2];
            const float ce = 1.0f - 0.5f * le, co = 1.0f - 0.5f * lo;
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
#pragma unroll
        for (int i = 0; i < Q; ++i) Bf[i * st + idx] = S::st(out[i], a.scale);
        if (AUDIT) {
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                // what was stored, as it will be read back
                const double v = S::ld(S::st(out[i], a.scale), a.inv_scale);
                am[0] += v;
                am[1] += cx(i) * v;
                am[2] += cy(i) * v;
                am[3] += cz(i) * v;
            }
            am[4] = 1.0;
        }
    }
    if (AUDIT) block_reduce<5>(am, audit_part + size_t(blockIdx.x) * 5);
}

// ---------------------------------------------------------------------------
// body update: reduce partials, WCA, symplectic Euler (one block)

__device__ void rotate_by(double e[3], const double w[3])
{
    const double th = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    if (th == 0.0) return;
    const double k[3] = {w[0] / th, w[1] / th, w[2] / th};
    const double kxe[3] = {k[1] * e[2] - k[2] * e[1], k[2] * e[0] - k[0] * e[2], k[0] * e[1] - k[1] * e[0]};
    const double ke = k[0] * e[0] + k[1] * e[1] + k[2] * e[2];
    const double c = cos(th), s = sin(th);
    double o[3];
    for (int a = 0; a < 3; ++a) o[a] = e[a] * c + kxe[a] * s + k[a] * ke * (1.0 - c);
    const double nn = sqrt(o[0] * o[0] + o[1] * o[1] + o[2] * o[2]);
    for (int a = 0; a < 3; ++a) e[a] = o[a] / nn;
}

__device__ double wca_magnitude(double r, double sigma, double eps)
{
    const double rc = pow(2.0, 1.0 / 6.0) * sigma;
    if (r >= rc) return 0.0;
    if (r < 0.05 * sigma) r = 0.05 * sigma;
    const double sr6 = pow(sigma / r, 6.0);
    return 24.0 * eps / r * (2.0 * sr6 * sr6 - sr6);
}

__global__ __launch_bounds__(BLOCK) void k_body(Box bx, DevBody *__restrict__ bodies, int nbody,
                                                const int *__restrict__ start, const double *__restrict__ part,
                                                double wca_sigma, double wca_eps, int *__restrict__ err)
{
    __shared__ double red[BLOCK][12];
    __shared__ double tot[MAXB > 64 ? 64 : MAXB][12];
    for (int b0 = 0; b0 < nbody; b0 += 64) {
        const int bn = min(64, nbody - b0);
        for (int bi = 0; bi < bn; ++bi) {
            const int b = b0 + bi;
            double acc[12];
            for (int k = 0; k < 12; ++k) acc[k] = 0.0;
            for (int blk = start[b] + threadIdx.x; blk < start[b + 1]; blk += BLOCK)
                for (int k = 0; k < 12; ++k) acc[k] += part[size_t(blk) * 12 + k];
            for (int k = 0; k < 12; ++k) red[threadIdx.x][k] = acc[k];
            __syncthreads();
            for (int h = BLOCK / 2; h > 0; h >>= 1) {
                if (threadIdx.x < h)
                    for (int k = 0; k < 12; ++k) red[threadIdx.x][k] += red[threadIdx.x + h][k];
                __syncthreads();
            }
            if (threadIdx.x < 12) tot[bi][threadIdx.x] = red[0][threadIdx.x];
            __syncthreads();
        }
        if (threadIdx.x < bn) {
            DevBody &B = bodies[b0 + threadIdx.x];
            for (int k = 0; k < 3; ++k) {
                B.Fbb[k] = tot[threadIdx.x][k];
                B.Tbb[k] = tot[threadIdx.x][3 + k];
                B.Fc[k] = tot[threadIdx.x][6 + k];
                B.Tc[k] = tot[threadIdx.x][9 + k];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const int nn[3] = {bx.nx, bx.ny, bx.nz};
    for (int b = 0; b < nbody; ++b)
        for (int k = 0; k < 3; ++k) bodies[b].Fwca[k] = 0.0;
    for (int a = 0; a < nbody; ++a)
        for (int b = a + 1; b < nbody; ++b) {
            DevBody &A = bodies[a], &Bb = bodies[b];
            double dv[3];
            for (int k = 0; k < 3; ++k) dv[k] = min_image(Bb.pos[k] - A.pos[k], nn[k]);
            const double dist = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
            const double fm = wca_magnitude(dist - A.R - Bb.R, wca_sigma, wca_eps);
            if (fm == 0.0) continue;
            for (int k = 0; k < 3; ++k) {
                Bb.Fwca[k] += fm * dv[k] / dist;
                A.Fwca[k] -= fm * dv[k] / dist;
            }
        }
    for (int b = 0; b < nbody; ++b) {
        DevBody &B = bodies[b];
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
                double p = B.pos[k] + B.v[k];
                if (p >= nn[k]) p -= nn[k];
                if (p < 0.0) p += nn[k];
                B.pos[k] = p;
            }
            rotate_by(B.e, B.w);
        }
    }
}

// ---------------------------------------------------------------------------
// set-up, audit and readout kernels (outside the timed step)

__global__ __launch_bounds__(BLOCK) void k_classify(Box bx, uint8_t *__restrict__ own)
{
    const uint32_t c = blockIdx.x * BLOCK + threadIdx.x;
    if (c >= bx.n) return;
    const uint8_t o = own[c];
    if (!is_fluid(o)) return;
    const int x = c % bx.nx, y = (c / bx.nx) % bx.ny, z = c / (uint32_t(bx.nx) * bx.ny);
    bool nb = false;
    for (int i = 1; i < Q; ++i)
        nb |= !is_fluid(own[cell_of(bx, wrap(x + cx(i), bx.nx), wrap(y + cy(i), bx.ny), wrap(z + cz(i), bx.nz))]);
    own[c] = nb ? OWN_FLUID_NB : OWN_FLUID;
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

template <class S>
__global__ __launch_bounds__(BLOCK) void k_audit(StepArgs a, const typename S::T *__restrict__ A,
                                                 const uint8_t *__restrict__ own, double *__restrict__ part)
{
    const uint32_t c = blockIdx.x * BLOCK + threadIdx.x;
    double am[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (c < a.box.n && is_fluid(own[c])) {
        for (int i = 0; i < Q; ++i) {
            const double v = S::ld(A[i * a.box.stride + c], a.inv_scale);
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
                                                  const uint8_t *__restrict__ own, double *__restrict__ rho,
                                                  double *__restrict__ u, uint8_t *__restrict__ own_out)
{
    const uint32_t c = blockIdx.x * BLOCK + threadIdx.x;
    if (c >= a.box.n) return;
    const uint8_t o = own[c];
    own_out[c] = is_fluid(o) ? 0 : o;
    if (!is_fluid(o)) {
        rho[c] = 0.0;
        u[c] = u[a.box.n + c] = u[2 * size_t(a.box.n) + c] = 0.0;
        return;
    }
    double r = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < Q; ++i) {
        const double v = S::ld(A[i * a.box.stride + c], a.inv_scale);
        r += v;
        j[0] += cx(i) * v;
        j[1] += cy(i) * v;
        j[2] += cz(i) * v;
    }
    r += a.rho0d;
    rho[c] = r;
    for (int k = 0; k < 3; ++k) u[k * size_t(a.box.n) + c] = (j[k] - 0.5 * double(a.g[k])) / r;
}

template <class S>
__global__ __launch_bounds__(BLOCK) void k_plane_to_f64(StepArgs a, const typename S::T *__restrict__ A,
                                                        const uint8_t *__restrict__ own, int i,
                                                        double *__restrict__ out)
{
    const uint32_t c = blockIdx.x * BLOCK + threadIdx.x;
    if (c >= a.box.n) return;
    out[c] = is_fluid(own[c]) ? wgt(i) * a.rho0d + double(S::ld(A[i * a.box.stride + c], a.inv_scale)) : 0.0;
}

template <class S>
__global__ __launch_bounds__(BLOCK) void k_plane_from_f64(StepArgs a, typename S::T *__restrict__ A,
                                                          const uint8_t *__restrict__ own, int i,
                                                          const double *__restrict__ in)
{
    const uint32_t c = blockIdx.x * BLOCK + threadIdx.x;
    if (c >= a.box.n) return;
    A[i * a.box.stride + c] = is_fluid(own[c]) ? S::st(float(in[c] - wgt(i) * a.rho0d), a.scale) : S::st(0.0f, a.scale);
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

template <class S>
static hipError_t launch_step_t(const StepLaunch &L)
{
    using T = typename S::T;
    const StepArgs &a = L.args;
    const int nblk = int((a.box.n + BLOCK - 1) / BLOCK);
    T *A = static_cast<T *>(L.A);
    T *B = static_cast<T *>(L.B);
    if (L.nmov > 0) {
        hipLaunchKernelGGL(k_geom, dim3(L.nblk_mov), dim3(BLOCK), 0, L.stream, a.box, L.bodies, L.nbody,
                           L.mov_ids, L.mov_start, L.nmov, L.own, L.ev, L.err);
        hipLaunchKernelGGL(k_refill<S>, dim3(L.nblk_mov), dim3(BLOCK), 0, L.stream, a, L.bodies, L.mov_ids,
                           L.mov_start, L.nmov, L.own, L.ev, A);
    }
    if (L.nbody > 0)
        hipLaunchKernelGGL(k_force<S>, dim3(L.nblk_all), dim3(BLOCK), 0, L.stream, a, L.bodies, L.all_ids,
                           L.all_start, L.nbody, L.own, L.ev, A, L.part);
    if (L.ev_start && hipEventRecord(L.ev_start, L.stream) != hipSuccess) return hipErrorUnknown;
    const bool force = a.g[0] != 0.0f || a.g[1] != 0.0f || a.g[2] != 0.0f;
    if (L.audit) {
        if (force)
            hipLaunchKernelGGL((k_stream_collide<S, true, true>), dim3(nblk), dim3(BLOCK), 0, L.stream, a, A, B,
                               L.own, L.bodies, L.audit_part);
        else
            hipLaunchKernelGGL((k_stream_collide<S, true, false>), dim3(nblk), dim3(BLOCK), 0, L.stream, a, A,
                               B, L.own, L.bodies, L.audit_part);
    } else {
        if (force)
            hipLaunchKernelGGL((k_stream_collide<S, false, true>), dim3(nblk), dim3(BLOCK), 0, L.stream, a, A,
                               B, L.own, L.bodies, L.audit_part);
        else
            hipLaunchKernelGGL((k_stream_collide<S, false, false>), dim3(nblk), dim3(BLOCK), 0, L.stream, a, A,
                               B, L.own, L.bodies, L.audit_part);
    }
    if (L.ev_stop && hipEventRecord(L.ev_stop, L.stream) != hipSuccess) return hipErrorUnknown;
    if (L.audit)
        hipLaunchKernelGGL(k_audit_final, dim3(1), dim3(BLOCK), 0, L.stream, L.audit_part, nblk, L.audit_out,
                           L.err);
    if (L.nbody > 0)
        hipLaunchKernelGGL(k_body, dim3(1), dim3(BLOCK), 0, L.stream, a.box, L.bodies, L.nbody, L.all_start,
                           L.part, L.wca_sigma, L.wca_eps, L.err);
    return hipGetLastError();
}

hipError_t launch_step(int storage, const StepLaunch &L)
{
    switch (storage) {
    case 1: return launch_step_t<StF16>(L);
    case 2: return launch_step_t<StBF16>(L);
    default: return launch_step_t<StF32>(L);
    }
}

hipError_t launch_classify(const Box &bx, uint8_t *own, hipStream_t s)
{
    hipLaunchKernelGGL(k_classify, dim3((bx.n + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, bx, own);
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
static hipError_t launch_audit_t(const StepArgs &a, const void *A, const uint8_t *own, double *part, double *out,
                                 int *err, hipStream_t s)
{
    const int nblk = int((a.box.n + BLOCK - 1) / BLOCK);
    hipLaunchKernelGGL(k_audit<S>, dim3(nblk), dim3(BLOCK), 0, s, a, static_cast<const typename S::T *>(A), own,
                       part);
    hipLaunchKernelGGL(k_audit_final, dim3(1), dim3(BLOCK), 0, s, part, nblk, out, err);
    return hipGetLastError();
}

hipError_t launch_audit(int storage, const StepArgs &a, const void *A, const uint8_t *own, double *part,
                        double *out, int *err, hipStream_t s)
{
    switch (storage) {
    case 1: return launch_audit_t<StF16>(a, A, own, part, out, err, s);
    case 2: return launch_audit_t<StBF16>(a, A, own, part, out, err, s);
    default: return launch_audit_t<StF32>(a, A, own, part, out, err, s);
    }
}

template <class S>
static hipError_t launch_fields_t(const StepArgs &a, const void *A, const uint8_t *own, double *rho, double *u,
                                  uint8_t *own_out, hipStream_t s)
{
    hipLaunchKernelGGL(k_fields<S>, dim3((a.box.n + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, a,
                       static_cast<const typename S::T *>(A), own, rho, u, own_out);
    return hipGetLastError();
}

hipError_t launch_fields(int storage, const StepArgs &a, const void *A, const uint8_t *own, double *rho, double *u,
                         uint8_t *own_out, hipStream_t s)
{
    switch (storage) {
    case 1: return launch_fields_t<StF16>(a, A, own, rho, u, own_out, s);
    case 2: return launch_fields_t<StBF16>(a, A, own, rho, u, own_out, s);
    default: return launch_fields_t<StF32>(a, A, own, rho, u, own_out, s);
    }
}

template <class S>
static hipError_t launch_plane_t(const StepArgs &a, void *A, const uint8_t *own, int i, double *buf, int to_f64,
                                 hipStream_t s)
{
    using T = typename S::T;
    const dim3 g((a.box.n + BLOCK - 1) / BLOCK);
    if (to_f64)
        hipLaunchKernelGGL(k_plane_to_f64<S>, g, dim3(BLOCK), 0, s, a, static_cast<const T *>(A), own, i, buf);
    else
        hipLaunchKernelGGL(k_plane_from_f64<S>, g, dim3(BLOCK), 0, s, a, static_cast<T *>(A), own, i,
                           static_cast<const double *>(buf));
    return hipGetLastError();
}

hipError_t launch_plane(int storage, const StepArgs &a, void *A, const uint8_t *own, int i, double *buf, int to_f64,
                        hipStream_t s)
{
    switch (storage) {
    case 1: return launch_plane_t<StF16>(a, A, own, i, buf, to_f64, s);
    case 2: return launch_plane_t<StBF16>(a, A, own, i, buf, to_f64, s);
    default: return launch_plane_t<StF32>(a, A, own, i, buf, to_f64, s);
    }
}

hipError_t launch_link_mask(const Box &bx, const uint8_t *own, uint32_t *mask, hipStream_t s)
{
    hipLaunchKernelGGL(k_link_mask, dim3((bx.n + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, bx, own, mask);
    return hipGetLastError();
}

}  // namespace lbsq
