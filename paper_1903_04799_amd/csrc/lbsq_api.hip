// lbsq_api.hip -- the C ABI of include/lbsq.h: handle life cycle, argument
// validation, device memory, step scheduling and readout.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "lbsq_sim.h"

using namespace lbsq;

namespace {

constexpr int NERR = 4;  // error flags 0..2, then the arrival counter of the boundary blocks

int nblocks(uint64_t n) { return int((n + BLOCK - 1) / BLOCK); }

// population plane stride: whole 256-element groups plus one extra group, so
// that the 19 planes do not start at the same offset modulo large powers of
// two
uint64_t plane_stride(uint64_t n) { return ((n + 255) / 256) * 256 + 256; }

void *dev_alloc(lb_sim *s, size_t bytes)
{
    void *p = nullptr;
    if (bytes == 0) bytes = 1;
    if (s->p.alloc) {
        p = s->p.alloc(bytes, s->p.alloc_ctx);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        p = nullptr;
    }
    return p;
}

void dev_free(lb_sim *s, void *p)
{
    if (!p) return;
    if (s->p.free) s->p.free(p, s->p.alloc_ctx);
    else (void)hipFree(p);
}

// Multiplier m and shift s with floor(v / d) = umulhi(v, m) >> s for every
// v < 2^31 (d >= 2): with l = ceil(log2 d), m = ceil(2^(31+l) / d) < 2^32
// and the rounding excess m d - 2^(31+l) < 2^l keeps v m / 2^(31+l) within
// 1/d of v/d.
void magic_divisor(uint32_t d, uint32_t &m, uint32_t &s)
{
    int l = 0;
    while ((uint64_t(1) << l) < d) ++l;
    const uint64_t S = 31 + uint64_t(l);
    m = uint32_t(((uint64_t(1) << S) + d - 1) / d);
    s = uint32_t(S - 32);
}

// Half-width of a body's box around the floor of its position.  The cells
// of a body lie within ceil(R) of that floor, its neighbour cells within
// ceil(R) + 1, and in one step (|v| < 1) every owner or flag change stays
// within ceil(R) + 2 of the old floor, inside the geometry box of half-width
// H + 1.  One cell of margin on top.
int body_half_width(double R) { return int(std::ceil(R)) + 2; }

double wrap_pos(double p, int n)
{
    p = std::fmod(p, double(n));
    if (p < 0.0) p += n;
    if (p >= n) p -= n;
    return p;
}

// Wait for the stream and turn device-side error flags into a status.
int sync_check(lb_sim *s)
{
    (void)hipSetDevice(s->device);
    if (hipStreamSynchronize(s->stream) != hipSuccess) return LB_EDEVICE;
    int err[NERR];
    if (hipMemcpy(err, s->d_err, sizeof(err), hipMemcpyDeviceToHost) != hipSuccess) return LB_EDEVICE;
    if (err[0] || err[1] || err[2]) {
        int zero[NERR] = {0, 0, 0, 0};
        (void)hipMemcpy(s->d_err, zero, sizeof(zero), hipMemcpyHostToDevice);
        if (err[1]) return LB_ENAN;
        return LB_EGEOM;
    }
    return LB_OK;
}

int upload_desc(lb_sim *s);

// The cells of a body's box that can be fluid cells next to the body for
// some position of the body within its floor cell: relative offsets r
// (|r_k| <= H), packed as three 10-bit fields biased by 512.  A cell
// qualifies when it is outside the sphere for some offset p of the centre in
// [0, 1]^3 (its farthest point of that cube lies beyond R) and one of its
// D3Q19 neighbours is inside for some p (the nearest point lies within R);
// the tolerance keeps the set a superset of what the exact fixed-point test
// can produce.
std::vector<uint32_t> shell_cells(const DevBody &B)
{
    const double R = double(B.Rq) / 1048576.0, R2 = R * R, tol = 1e-6 * (1.0 + R2);
    std::vector<uint32_t> out;
    for (int rz = -B.H; rz <= B.H; ++rz)
        for (int ry = -B.H; ry <= B.H; ++ry)
            for (int rx = -B.H; rx <= B.H; ++rx) {
                const int r[3] = {rx, ry, rz};
                double far2 = 0.0;
                for (int k = 0; k < 3; ++k) {
                    const double c = r[k] + 0.5;
                    far2 += std::max(c * c, (c - 1.0) * (c - 1.0));
                }
                if (far2 <= R2 - tol) continue;  // inside for every position
                bool near = false;
                for (int j = 1; j < Q && !near; ++j) {
                    const int cj[3] = {cx(j), cy(j), cz(j)};
                    double d2 = 0.0;
                    for (int k = 0; k < 3; ++k) {
                        const double c = r[k] + cj[k] + 0.5;
                        const double d = c < 0.0 ? -c : (c > 1.0 ? c - 1.0 : 0.0);
                        d2 += d * d;
                    }
                    near = d2 <= R2 + tol;
                }
                if (near)
                    out.push_back(uint32_t(rx + 512) | (uint32_t(ry + 512) << 10) | (uint32_t(rz + 512) << 20));
            }
    return out;
}

// Work lists: the moving bodies and the block ranges of their (grown) boxes
// for the geometry kernel; every body, the block ranges of its shell cells
// and where they sit in the shell array for the fluid kernel.
int rebuild_lists(lb_sim *s)
{
    const int nb = int(s->bodies.size());
    std::vector<int> mov_ids, mov_start(1, 0), all_ids, all_start(1, 0), all_base, all_count;
    std::vector<uint32_t> shell;
    for (int b = 0; b < nb; ++b) {
        const std::vector<uint32_t> sh = shell_cells(s->bodies[b]);
        all_ids.push_back(b);
        all_base.push_back(int(shell.size()));
        all_count.push_back(int(sh.size()));
        shell.insert(shell.end(), sh.begin(), sh.end());
        all_start.push_back(all_start.back() + int((sh.size() + CPB - 1) / CPB));
        if (s->bodies[b].mode == LB_FIXED) continue;
        // the geometry kernel walks the box grown by one cell on each side
        const int gside = 2 * s->bodies[b].H + 3;
        mov_ids.push_back(b);
        mov_start.push_back(mov_start.back() + int((uint64_t(gside) * gside * gside + CPB - 1) / CPB));
    }
    s->nmov = int(mov_ids.size());
    s->nblk_mov = mov_start.back();
    s->nblk_all = all_start.back();
    std::vector<int> packed(mov_ids);
    packed.insert(packed.end(), mov_start.begin(), mov_start.end());
    packed.insert(packed.end(), all_ids.begin(), all_ids.end());
    packed.insert(packed.end(), all_start.begin(), all_start.end());
    packed.insert(packed.end(), all_base.begin(), all_base.end());
    packed.insert(packed.end(), all_count.begin(), all_count.end());
    if (hipMemcpy(s->d_lists, packed.data(), packed.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
        return LB_EDEVICE;
    if (shell.size() > s->shell_cap) {
        dev_free(s, s->d_shell);
        s->d_shell = static_cast<uint32_t *>(dev_alloc(s, shell.size() * sizeof(uint32_t)));
        if (!s->d_shell) return LB_ENOMEM;
        s->shell_cap = shell.size();
    }
    if (!shell.empty() &&
        hipMemcpy(s->d_shell, shell.data(), shell.size() * sizeof(uint32_t), hipMemcpyHostToDevice) != hipSuccess)
        return LB_EDEVICE;
    // one record per boundary block: its body, its first shell cell, how
    // many cells it takes
    std::vector<int4> info;
    for (int m = 0; m < nb; ++m)
        for (int j = all_start[m]; j < all_start[m + 1]; ++j) {
            const int first = (j - all_start[m]) * CPB;
            info.push_back(make_int4(all_ids[m], all_base[m] + first, std::min(CPB, all_count[m] - first), m));
        }
    if (info.size() > s->blkinfo_cap) {
        dev_free(s, s->d_blkinfo);
        s->d_blkinfo = static_cast<int4 *>(dev_alloc(s, info.size() * sizeof(int4)));
        if (!s->d_blkinfo) return LB_ENOMEM;
        s->blkinfo_cap = info.size();
    }
    if (!info.empty() &&
        hipMemcpy(s->d_blkinfo, info.data(), info.size() * sizeof(int4), hipMemcpyHostToDevice) != hipSuccess)
        return LB_EDEVICE;
    // audit partials: one per streaming block and one per boundary block
    const size_t need = size_t(nblocks(s->args.box.n)) + size_t(s->nblk_all);
    if (need > s->audit_blocks) {
        dev_free(s, s->d_audit_part);
        s->d_audit_part = static_cast<double *>(dev_alloc(s, need * 5 * sizeof(double)));
        if (!s->d_audit_part) return LB_ENOMEM;
        s->audit_blocks = need;
    }
    return upload_desc(s);
}

}  // namespace

// The step kernels' descriptor of a simulation, for time levels t = t0 + k.
// Streaming blocks of the fluid launch: one per group of BLOCK cells, or
// with static walls one per group that holds a cell other than a wall.
static int stream_blocks(const lb_sim *s)
{
    return s->d_sgrp ? int(s->nsgrp) : int((uint64_t(s->args.box.n) + BLOCK - 1) / BLOCK);
}

void lbsq_fill_desc(const lb_sim *s, int64_t t0, int64_t t_end, SimDesc &d)
{
    std::memset(&d, 0, sizeof(d));
    d.a = s->args;
    d.f = s->f;
    d.f2 = s->f2;
    for (int k = 0; k < 2; ++k) {
        d.dens[k] = s->d_dens[k];
        d.own[k] = s->own[k];
        d.bodies[k] = s->d_bodies[k];
    }
    d.acc = s->d_acc;
    d.nbody = int(s->bodies.size());
    d.nmov = s->nmov;
    d.mov_ids = s->d_lists;
    d.mov_start = s->d_lists + s->nmov;
    d.all_ids = s->d_lists + 2 * s->nmov + 1;
    d.all_start = s->d_lists + 2 * s->nmov + 1 + d.nbody;
    d.all_base = s->d_lists + 2 * s->nmov + 2 + 2 * d.nbody;
    d.all_count = s->d_lists + 2 * s->nmov + 2 + 3 * d.nbody;
    d.shell = s->d_shell;
    d.wmask = s->d_wmask;
    d.blkinfo = s->d_blkinfo;
    d.audit_part = s->d_audit_part;
    d.err = s->d_err;
    // the last error word is the boundary blocks' arrival counter
    d.arrive = reinterpret_cast<unsigned int *>(s->d_err + (NERR - 1));
    d.wca_sigma = s->p.wca_sigma;
    d.wca_eps = s->p.wca_eps;
    d.t0 = t0;
    d.t_end = t_end;
    d.nblk_b = d.nbody > 0 ? s->nblk_all : 0;
    d.sgrp = s->d_sgrp;
    d.nblk_s = stream_blocks(s);
}

// Blocks of the fluid and geometry launches of a simulation.
void lbsq_sim_blocks(const lb_sim *s, uint32_t *fluid, uint32_t *geo)
{
    const int nbody = int(s->bodies.size());
    *fluid = uint32_t(stream_blocks(s)) + uint32_t(nbody > 0 ? s->nblk_all : 0);
    *geo = uint32_t(geo_blocks(nbody, s->nblk_mov));
}

namespace {

// the standalone descriptor: k counts the simulation's own steps
int upload_desc(lb_sim *s)
{
    SimDesc d;
    lbsq_fill_desc(s, 0, INT64_MAX, d);
    return hipMemcpy(s->d_desc, &d, sizeof(d), hipMemcpyHostToDevice) == hipSuccess ? LB_OK : LB_EDEVICE;
}

int pull_bodies(lb_sim *s)
{
    if (s->bodies.empty()) return LB_OK;
    if (hipMemcpy(s->bodies.data(), s->d_bodies[s->cur], s->bodies.size() * sizeof(DevBody),
                  hipMemcpyDeviceToHost) != hipSuccess)
        return LB_EDEVICE;
    return LB_OK;
}

// owners of the current buffer copied to the other one (set-up only)
int mirror_owner(lb_sim *s)
{
    if (hipMemcpyAsync(s->own[1 - s->cur], s->own[s->cur], s->args.box.n, hipMemcpyDeviceToDevice, s->stream) !=
        hipSuccess)
        return LB_EDEVICE;
    return LB_OK;
}

// whether the last completed step had an even index (the in-place layout)
bool after_even(const lb_sim *s) { return (s->steps & 1) == 1; }

// cells above which LB_LAYOUT_AUTO takes the two-buffer pull layout
constexpr uint64_t AUTO_PULL_CELLS = 5500000;

// The buffer holding the populations after the steps taken so far, and its
// layout: in place the one buffer, by the parity of the last step; in the
// pull layout the buffer the last step wrote (buffer steps & 1).
void *pop_buf(const lb_sim *s) { return s->f2 && (s->steps & 1) ? s->f2 : s->f; }
int pop_lay(const lb_sim *s) { return s->f2 ? LAY_AB : (after_even(s) ? LAY_AA_EVEN : LAY_AA_ODD); }

// Link densities of the cells next to a body, for the next step.
int refresh_dens(lb_sim *s)
{
    return launch_dens(s->p.storage, s->args, pop_buf(s), s->own[s->cur], pop_lay(s), s->d_dens[(s->steps + 1) & 1],
                       s->stream) == hipSuccess
               ? LB_OK
               : LB_EDEVICE;
}

// The groups of BLOCK cells the streaming blocks take: with static walls,
// only those holding a cell other than a wall (walls never turn fluid), so
// that all-wall regions cost the streaming launch no block.  own is the
// host copy of the owners (walls OWN_WALL).
int set_stream_groups(lb_sim *s, const uint8_t *own)
{
    const uint32_t n = s->args.box.n;
    std::vector<uint32_t> g;
    for (uint32_t b = 0; uint64_t(b) * BLOCK < n; ++b) {
        const uint32_t e = uint32_t(std::min<uint64_t>(n, (uint64_t(b) + 1) * BLOCK));
        for (uint32_t c = b * BLOCK; c < e; ++c)
            if (own[c] != OWN_WALL) {
                g.push_back(b);
                break;
            }
    }
    dev_free(s, s->d_sgrp);
    s->d_sgrp = nullptr;
    s->nsgrp = 0;
    if (!g.empty()) {
        s->d_sgrp = static_cast<uint32_t *>(dev_alloc(s, g.size() * sizeof(uint32_t)));
        if (!s->d_sgrp) return LB_ENOMEM;
        if (hipMemcpy(s->d_sgrp, g.data(), g.size() * sizeof(uint32_t), hipMemcpyHostToDevice) != hipSuccess)
            return LB_EDEVICE;
        s->nsgrp = uint32_t(g.size());
    }
    return upload_desc(s);
}

// Static walls of a simulation, from the host copy of its owners (walls
// OWN_WALL).  With walls: room for every cell's wall mask (the device fills
// it when it classifies the owners) and the list of streaming groups;
// without: neither, and every group streams.  Either way the descriptor is
// uploaded with the new pointers before anything is launched.
int set_walls(lb_sim *s, const uint8_t *own, bool *walls_out)
{
    const uint32_t n = s->args.box.n;
    bool walls = false;
    for (uint32_t c = 0; c < n && !walls; ++c) walls = own[c] == OWN_WALL;
    *walls_out = walls;
    if (!walls) {
        dev_free(s, s->d_sgrp);
        dev_free(s, s->d_wmask);
        s->d_sgrp = nullptr;
        s->d_wmask = nullptr;
        s->nsgrp = 0;
        return upload_desc(s);
    }
    if (!s->d_wmask) {
        s->d_wmask = static_cast<uint32_t *>(dev_alloc(s, size_t(n) * sizeof(uint32_t)));
        if (!s->d_wmask) return LB_ENOMEM;
    }
    return set_stream_groups(s, own);
}

int classify_now(lb_sim *s)
{
    if (!s->need_classify) return LB_OK;
    if (launch_classify(s->args.box, s->own[s->cur], s->d_wmask, 1, s->stream) != hipSuccess) return LB_EDEVICE;
    s->need_classify = false;
    const int rc = mirror_owner(s);
    return rc == LB_OK ? refresh_dens(s) : rc;
}

}  // namespace

void *lbsq_dev_alloc(lb_sim *s, size_t bytes) { return dev_alloc(s, bytes); }
int lbsq_sync_check(lb_sim *s) { return sync_check(s); }
const void *lbsq_pop_buf(const lb_sim *s) { return pop_buf(s); }
int lbsq_pop_lay(const lb_sim *s) { return pop_lay(s); }
void lbsq_dev_free(lb_sim *s, void *p) { dev_free(s, p); }

// Owner flags of the current buffer computed if pending; the handle counts
// as started from then on.
int lbsq_prepare(lb_sim *s)
{
    const int cl = classify_now(s);
    if (cl != LB_OK) return cl;
    s->started = true;
    return LB_OK;
}

extern "C" {

const char *lb_strerror(int code)
{
    switch (code) {
    case LB_OK: return "ok";
    case LB_EINVAL: return "invalid argument";
    case LB_ENOMEM: return "device allocation failed";
    case LB_EDEVICE: return "HIP runtime error";
    case LB_EGEOM: return "invalid geometry (overlap, body too large, or a body moved a cell or more in a step)";
    case LB_ESTATE: return "call not allowed in the current state";
    case LB_ENAN: return "non-finite populations detected";
    case LB_EBUDGET: return "memory budget exceeded";
    case LB_ECANCELED: return "request cancelled";
    default: return "unknown error";
    }
}

int lb_destroy(lb_sim *s)
{
    if (!s) return LB_EINVAL;
    (void)hipSetDevice(s->device);
    (void)hipStreamSynchronize(s->stream);
    for (auto &e : s->evs) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    dev_free(s, s->f);
    dev_free(s, s->f2);
    for (int k = 0; k < 2; ++k) {
        dev_free(s, s->d_dens[k]);
        dev_free(s, s->own[k]);
        dev_free(s, s->d_bodies[k]);
    }
    dev_free(s, s->d_lists);
    dev_free(s, s->d_shell);
    dev_free(s, s->d_wmask);
    dev_free(s, s->d_sgrp);
    dev_free(s, s->d_blkinfo);
    dev_free(s, s->d_desc);
    dev_free(s, s->d_batch_desc);
    dev_free(s, s->d_acc);
    dev_free(s, s->d_audit_part);
    dev_free(s, s->d_audit_out);
    dev_free(s, s->d_err);
    delete s;
    return LB_OK;
}

int lb_create(const lb_params *p, lb_sim **out)
{
    if (!p || !out) return LB_EINVAL;
    *out = nullptr;
    if (p->nx < 4 || p->ny < 4 || p->nz < 4) return LB_EINVAL;
    const uint64_t n = uint64_t(p->nx) * p->ny * p->nz;
    if (n >= (uint64_t(1) << 32)) return LB_EINVAL;
    if (!(p->nu > 0.0) || !(p->magic > 0.0) || !(p->rho0 > 0.0)) return LB_EINVAL;
    if (p->storage < 0 || p->storage > 2 || p->scale_log2 < 0 || p->scale_log2 > 20 || p->audit_every < 0)
        return LB_EINVAL;
    const double le = 1.0 / (3.0 * p->nu + 0.5);
    const double lo = 1.0 / (p->magic / (1.0 / le - 0.5) + 0.5);
    if (!(le > 0.0 && le < 2.0 && lo > 0.0 && lo < 2.0)) return LB_EINVAL;
    if (!(p->wca_sigma > 0.0) || p->wca_eps < 0.0) return LB_EINVAL;
    // one population plane must stay below 4 GiB (32-bit offsets in the kernels)
    if (plane_stride(n) * (p->storage == LB_STORAGE_F32 ? 4 : 2) > (uint64_t(1) << 32)) return LB_EINVAL;
    if ((p->alloc == nullptr) != (p->free == nullptr)) return LB_EINVAL;
    if (p->layout != LB_LAYOUT_INPLACE && p->layout != LB_LAYOUT_AB && p->layout != LB_LAYOUT_AUTO)
        return LB_EINVAL;

    lb_sim *s = new (std::nothrow) lb_sim();
    if (!s) return LB_ENOMEM;
    s->p = *p;
    // the pull layout above the measured crossover (in place wins at 160^3
    // and below, pull from 192^3 up, in FP32 and FP16 alike)
    if (s->p.layout == LB_LAYOUT_AUTO) s->p.layout = n > AUTO_PULL_CELLS ? LB_LAYOUT_AB : LB_LAYOUT_INPLACE;
    (void)hipGetDevice(&s->device);
    s->stream = static_cast<hipStream_t>(p->stream);
    Box &bx = s->args.box;
    bx.nx = p->nx;
    bx.ny = p->ny;
    bx.nz = p->nz;
    bx.n = uint32_t(n);
    bx.stride = plane_stride(n);
    // tiled populations wherever the step kernels' 32-bit byte offsets reach
    // the whole buffer (up to 56.5 million cells in FP32, 113 million in
    // the half-width forms); planes beyond
    const uint64_t esz = p->storage == LB_STORAGE_F32 ? 4 : 2;
    const bool tiled = (n + 255) / 256 * 256 * Q * esz <= (uint64_t(1) << 32);
    bx.dstride = tiled ? 256 : bx.stride;
    bx.tmul = tiled ? uint32_t(Q - 1) * 256 : 0;
    magic_divisor(uint32_t(p->nx), bx.mx, bx.sx);
    magic_divisor(uint32_t(p->ny), bx.my, bx.sy);
    s->args.lam_e = float(le);
    s->args.lam_o = float(lo);
    s->args.rho0 = float(p->rho0);
    s->args.rho0d = p->rho0;
    for (int k = 0; k < 3; ++k) s->args.g[k] = float(p->g[k]);
    s->args.scale = std::ldexp(1.0f, p->scale_log2);
    s->args.inv_scale = std::ldexp(1.0f, -p->scale_log2);
    {
        // bulk collision constants (FP32 stores unscaled deviations)
        const double sc = p->storage == LB_STORAGE_F32 ? 1.0 : std::ldexp(1.0, p->scale_log2);
        const double wk[3] = {1.0 / 3.0, 1.0 / 18.0, 1.0 / 36.0};
        for (int k = 0; k < 3; ++k) {
            s->args.c_lew[k] = float(le * wk[k]);
            s->args.c_lews[k] = float(le * wk[k] * sc);
            s->args.c_low3s[k] = float(3.0 * lo * wk[k] * sc);
        }
        s->args.c_k1 = float(0.5 * (1.0 - le));
        s->args.c_k2 = float(0.5 * (1.0 - lo));
        s->args.c_1mle = float(1.0 - le);
        s->args.c_s = float(sc);
        s->args.c_is = float(1.0 / sc);
    }
    s->esize = p->storage == LB_STORAGE_F32 ? 4 : 2;

    const size_t fbytes = size_t(Q) * bx.stride * s->esize;
    s->f = dev_alloc(s, fbytes);
    if (s->p.layout == LB_LAYOUT_AB) s->f2 = dev_alloc(s, fbytes);
    for (int k = 0; k < 2; ++k) {
        s->d_dens[k] = static_cast<float *>(dev_alloc(s, size_t(n) * sizeof(float)));
        s->own[k] = static_cast<uint8_t *>(dev_alloc(s, n));
        s->d_bodies[k] = static_cast<DevBody *>(dev_alloc(s, MAXB * sizeof(DevBody)));
    }
    s->d_lists = static_cast<int *>(dev_alloc(s, 6 * (MAXB + 1) * sizeof(int)));
    s->d_acc = static_cast<unsigned long long *>(dev_alloc(s, NACCSET * ACCSET_SIZE * sizeof(unsigned long long)));
    s->d_audit_part = static_cast<double *>(dev_alloc(s, size_t(nblocks(n)) * 5 * sizeof(double)));
    s->audit_blocks = size_t(nblocks(n));
    s->d_audit_out = static_cast<double *>(dev_alloc(s, 8 * sizeof(double)));
    s->d_err = static_cast<int *>(dev_alloc(s, NERR * sizeof(int)));
    s->d_desc = static_cast<SimDesc *>(dev_alloc(s, sizeof(SimDesc)));
    if (!s->f || (s->p.layout == LB_LAYOUT_AB && !s->f2) || !s->d_dens[0] || !s->d_dens[1] || !s->own[0] || !s->own[1] || !s->d_bodies[0] || !s->d_bodies[1] ||
        !s->d_lists || !s->d_acc || !s->d_audit_part || !s->d_audit_out || !s->d_err || !s->d_desc) {
        lb_destroy(s);
        return LB_ENOMEM;
    }
    hipError_t e = hipMemsetAsync(s->f, 0, fbytes, s->stream);
    if (e == hipSuccess && s->f2) e = hipMemsetAsync(s->f2, 0, fbytes, s->stream);
    if (e == hipSuccess) e = hipMemsetAsync(s->d_acc, 0, NACCSET * ACCSET_SIZE * sizeof(unsigned long long), s->stream);
    for (int k = 0; k < 2 && e == hipSuccess; ++k) e = hipMemsetAsync(s->d_dens[k], 0, size_t(n) * sizeof(float), s->stream);
    if (e == hipSuccess) e = hipMemsetAsync(s->own[0], 0, n, s->stream);
    if (e == hipSuccess) e = hipMemsetAsync(s->own[1], 0, n, s->stream);
    if (e == hipSuccess) e = hipMemsetAsync(s->d_err, 0, NERR * sizeof(int), s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess || upload_desc(s) != LB_OK || lbsq_noalloc_init(s->device) != LB_OK) {
        lb_destroy(s);
        return LB_EDEVICE;
    }
    *out = s;
    return LB_OK;
}

int lb_set_static_mask(lb_sim *s, const uint8_t *solid, size_t n)
{
    if (!s || !solid) return LB_EINVAL;
    if (n != s->args.box.n) return LB_EINVAL;
    if (s->started || !s->bodies.empty()) return LB_ESTATE;
    std::vector<uint8_t> h(n);
    for (size_t c = 0; c < n; ++c) h[c] = solid[c] ? OWN_WALL : OWN_FLUID;
    (void)hipSetDevice(s->device);
    bool walls = false;
    const int rc = set_walls(s, h.data(), &walls);
    if (rc != LB_OK) return rc;
    for (int k = 0; k < 2; ++k)
        if (hipMemcpy(s->own[k], h.data(), n, hipMemcpyHostToDevice) != hipSuccess) return LB_EDEVICE;
    s->need_classify = true;
    return LB_OK;
}

int lb_add_squirmer(lb_sim *s, const lb_squirmer *q, int *id)
{
    if (!s || !q) return LB_EINVAL;
    const TraceRange tr("lb_add_squirmer");
    if (s->started) return LB_ESTATE;
    if (int(s->bodies.size()) >= MAXB) return LB_EINVAL;
    if (q->mode < LB_FREE || q->mode > LB_PRESCRIBED) return LB_EINVAL;
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(q->pos[k]) || !std::isfinite(q->e[k]) || !std::isfinite(q->v[k]) ||
            !std::isfinite(q->w[k]))
            return LB_EINVAL;
    if (!(q->R > 0.5) || !std::isfinite(q->B1) || !std::isfinite(q->beta)) return LB_EINVAL;
    const double en = std::sqrt(q->e[0] * q->e[0] + q->e[1] * q->e[1] + q->e[2] * q->e[2]);
    if (!(en > 0.0)) return LB_EINVAL;
    for (int k = 0; k < 3; ++k)
        if (!(std::fabs(q->v[k]) < 1.0)) return LB_EINVAL;
    const Box &bx = s->args.box;
    DevBody B;
    std::memset(&B, 0, sizeof(B));
    if (!(q->R < 500.0)) return LB_EINVAL;  // shell offsets are packed in 10 bits
    B.H = body_half_width(q->R);
    const int side = 2 * B.H + 1;
    if (side + 2 > std::min(bx.nx, std::min(bx.ny, bx.nz))) return LB_EGEOM;
    const int n3[3] = {bx.nx, bx.ny, bx.nz};
    for (int k = 0; k < 3; ++k) {
        B.pos[k] = wrap_pos(q->pos[k], n3[k]);
        B.e[k] = q->e[k] / en;
        B.v[k] = q->v[k];
        B.w[k] = q->w[k];
    }
    B.R = q->R;
    B.B1 = q->B1;
    B.beta = q->beta;
    B.mode = q->mode;
    const double rho_p = q->rho_p > 0.0 ? q->rho_p : s->p.rho0;
    B.m = rho_p * 4.0 / 3.0 * M_PI * q->R * q->R * q->R;
    B.I = 0.4 * B.m * q->R * q->R;
    B.Rq = std::llrint(q->R * double(int64_t(1) << 20));
    const int b = int(s->bodies.size());
    (void)hipSetDevice(s->device);
    for (int k = 0; k < 2; ++k)
        if (hipMemcpy(s->d_bodies[k] + b, &B, sizeof(B), hipMemcpyHostToDevice) != hipSuccess) return LB_EDEVICE;
    if (launch_body_cells(bx, s->d_bodies[s->cur], b, side, s->own[s->cur], 1, s->d_err, s->stream) != hipSuccess)
        return LB_EDEVICE;
    const int st = sync_check(s);
    if (st == LB_EGEOM) return LB_EGEOM;
    if (st != LB_OK) return st;
    for (int k = 0; k < 2; ++k)
        if (launch_body_cells(bx, s->d_bodies[s->cur], b, side, s->own[k], 0, s->d_err, s->stream) != hipSuccess)
            return LB_EDEVICE;
    s->bodies.push_back(B);
    const int rc = rebuild_lists(s);
    if (rc != LB_OK) return rc;
    s->need_classify = true;
    if (id) *id = b;
    return sync_check(s);
}

int lb_step(lb_sim *s, int nsteps)
{
    if (!s || nsteps < 0) return LB_EINVAL;
    const TraceRange tr("lb_step");
    (void)hipSetDevice(s->device);
    const int cl = classify_now(s);
    if (cl != LB_OK) return cl;
    s->started = true;
    BatchLaunch L;
    std::memset(&L, 0, sizeof(L));
    L.desc = s->d_desc;
    L.map.nsim = 1;
    lbsq_sim_blocks(s, &L.map.fluid0[1], &L.map.geo0[1]);
    L.nbody_max = int(s->bodies.size());
    L.force = s->args.g[0] != 0.0f || s->args.g[1] != 0.0f || s->args.g[2] != 0.0f;
    L.audit_part = s->d_audit_part;
    L.audit_out = s->d_audit_out;
    L.npart = int(L.map.fluid0[1]);
    L.err = s->d_err;
    L.body_kernel = L.nbody_max > FUSE_MAX;
    L.stream = s->stream;
    for (int t = 0; t < nsteps; ++t) {
        L.k = s->steps;
        L.audit = s->p.audit_every > 0 && ((s->steps + 1) % s->p.audit_every == 0);
        L.ev_start = L.ev_stop = nullptr;
        if (s->timing) {
            hipEvent_t a, b;
            if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return LB_EDEVICE;
            s->evs.emplace_back(a, b);
            L.ev_start = a;
            L.ev_stop = b;
        }
        if (launch_batch_step(s->p.storage, L) != hipSuccess) return LB_EDEVICE;
        s->cur ^= 1;
        s->steps++;
    }
    return LB_OK;
}

int lb_sync(lb_sim *s)
{
    if (!s) return LB_EINVAL;
    return sync_check(s);
}

int lb_read_fields(lb_sim *s, double *rho, double *u, uint8_t *owner)
{
    if (!s || !rho || !u) return LB_EINVAL;
    const TraceRange tr("lb_read_fields");
    const int st = sync_check(s);
    if (st != LB_OK) return st;
    const uint32_t n = s->args.box.n;
    double *d_rho = static_cast<double *>(dev_alloc(s, size_t(n) * sizeof(double)));
    double *d_u = static_cast<double *>(dev_alloc(s, size_t(n) * 3 * sizeof(double)));
    uint8_t *d_o = static_cast<uint8_t *>(dev_alloc(s, n));
    int rc = LB_OK;
    if (!d_rho || !d_u || !d_o) rc = LB_ENOMEM;
    if (rc == LB_OK && launch_fields(s->p.storage, s->args, pop_buf(s), s->own[s->cur], pop_lay(s), 0, n, d_rho, d_u, d_o,
                                         s->stream) !=
                           hipSuccess)
        rc = LB_EDEVICE;
    if (rc == LB_OK && hipStreamSynchronize(s->stream) != hipSuccess) rc = LB_EDEVICE;
    if (rc == LB_OK && hipMemcpy(rho, d_rho, size_t(n) * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
        rc = LB_EDEVICE;
    if (rc == LB_OK && hipMemcpy(u, d_u, size_t(n) * 3 * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
        rc = LB_EDEVICE;
    if (rc == LB_OK && owner && hipMemcpy(owner, d_o, n, hipMemcpyDeviceToHost) != hipSuccess) rc = LB_EDEVICE;
    dev_free(s, d_rho);
    dev_free(s, d_u);
    dev_free(s, d_o);
    return rc;
}

int lb_force_parts(lb_sim *s, int id, double Fbb[3], double Tbb[3], double Fc[3], double Tc[3])
{
    if (!s || id < 0 || id >= int(s->bodies.size())) return LB_EINVAL;
    int st = sync_check(s);
    if (st != LB_OK) return st;
    st = pull_bodies(s);
    if (st != LB_OK) return st;
    const DevBody &B = s->bodies[id];
    for (int k = 0; k < 3; ++k) {
        if (Fbb) Fbb[k] = B.Fbb[k];
        if (Tbb) Tbb[k] = B.Tbb[k];
        if (Fc) Fc[k] = B.Fc[k];
        if (Tc) Tc[k] = B.Tc[k];
    }
    return LB_OK;
}

int lb_force_torque(lb_sim *s, int id, double F[3], double T[3])
{
    if (!F || !T) return LB_EINVAL;
    double fb[3], tb[3], fc[3], tc[3];
    const int st = lb_force_parts(s, id, fb, tb, fc, tc);
    if (st != LB_OK) return st;
    for (int k = 0; k < 3; ++k) {
        F[k] = fb[k] + fc[k];
        T[k] = tb[k] + tc[k];
    }
    return LB_OK;
}

int lb_body_state(lb_sim *s, int id, double pos[3], double e[3], double v[3], double w[3], double Fwca[3])
{
    if (!s || id < 0 || id >= int(s->bodies.size())) return LB_EINVAL;
    int st = sync_check(s);
    if (st != LB_OK) return st;
    st = pull_bodies(s);
    if (st != LB_OK) return st;
    const DevBody &B = s->bodies[id];
    for (int k = 0; k < 3; ++k) {
        if (pos) pos[k] = B.pos[k];
        if (e) e[k] = B.e[k];
        if (v) v[k] = B.v[k];
        if (w) w[k] = B.w[k];
        if (Fwca) Fwca[k] = B.Fwca[k];
    }
    return LB_OK;
}

int lb_links(lb_sim *s, uint32_t *cell, uint8_t *dir, uint8_t *owner, size_t cap, size_t *n)
{
    if (!s || !n) return LB_EINVAL;
    int st = sync_check(s);
    if (st != LB_OK) return st;
    const Box &bx = s->args.box;
    (void)hipSetDevice(s->device);
    st = classify_now(s);
    if (st != LB_OK) return st;
    uint32_t *d_mask = static_cast<uint32_t *>(dev_alloc(s, size_t(bx.n) * sizeof(uint32_t)));
    if (!d_mask) return LB_ENOMEM;
    std::vector<uint32_t> mask(bx.n);
    std::vector<uint8_t> own(bx.n);
    int rc = LB_OK;
    if (launch_link_mask(bx, s->own[s->cur], d_mask, s->stream) != hipSuccess ||
        hipStreamSynchronize(s->stream) != hipSuccess ||
        hipMemcpy(mask.data(), d_mask, size_t(bx.n) * sizeof(uint32_t), hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(own.data(), s->own[s->cur], bx.n, hipMemcpyDeviceToHost) != hipSuccess)
        rc = LB_EDEVICE;
    dev_free(s, d_mask);
    if (rc != LB_OK) return rc;
    size_t cnt = 0;
    for (uint32_t c = 0; c < bx.n; ++c) cnt += size_t(__builtin_popcount(mask[c]));
    *n = cnt;
    if (cnt > cap) return LB_EINVAL;
    if (cnt && (!cell || !dir || !owner)) return LB_EINVAL;
    size_t k = 0;
    for (uint32_t c = 0; c < bx.n; ++c) {
        const uint32_t m = mask[c];
        if (!m) continue;
        const int x = c % bx.nx, y = (c / bx.nx) % bx.ny, z = c / (uint32_t(bx.nx) * bx.ny);
        for (int i = 1; i < Q; ++i) {
            if (!(m & (1u << i))) continue;
            const int sx = (x - cx(i) + bx.nx) % bx.nx, sy = (y - cy(i) + bx.ny) % bx.ny,
                      sz = (z - cz(i) + bx.nz) % bx.nz;
            cell[k] = c;
            dir[k] = uint8_t(i);
            owner[k] = own[uint32_t(sx) + uint32_t(bx.nx) * (uint32_t(sy) + uint32_t(bx.ny) * uint32_t(sz))];
            ++k;
        }
    }
    return LB_OK;
}

int lb_read_populations(lb_sim *s, double *f)
{
    if (!s || !f) return LB_EINVAL;
    const int st = sync_check(s);
    if (st != LB_OK) return st;
    const uint32_t n = s->args.box.n;
    double *buf = static_cast<double *>(dev_alloc(s, size_t(n) * sizeof(double)));
    if (!buf) return LB_ENOMEM;
    int rc = LB_OK;
    for (int i = 0; i < Q && rc == LB_OK; ++i) {
        if (launch_plane(s->p.storage, s->args, pop_buf(s), s->own[s->cur], pop_lay(s), i, buf, 1, s->stream) !=
                hipSuccess ||
            hipStreamSynchronize(s->stream) != hipSuccess ||
            hipMemcpy(f + size_t(i) * n, buf, size_t(n) * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
            rc = LB_EDEVICE;
    }
    dev_free(s, buf);
    return rc;
}

int lb_write_populations(lb_sim *s, const double *f)
{
    if (!s || !f) return LB_EINVAL;
    const int st = sync_check(s);
    if (st != LB_OK) return st;
    const uint32_t n = s->args.box.n;
    double *buf = static_cast<double *>(dev_alloc(s, size_t(n) * sizeof(double)));
    if (!buf) return LB_ENOMEM;
    int rc = LB_OK;
    for (int i = 0; i < Q && rc == LB_OK; ++i) {
        if (hipMemcpy(buf, f + size_t(i) * n, size_t(n) * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
            launch_plane(s->p.storage, s->args, pop_buf(s), s->own[s->cur], pop_lay(s), i, buf, 0, s->stream) !=
                hipSuccess ||
            hipStreamSynchronize(s->stream) != hipSuccess)
            rc = LB_EDEVICE;
    }
    dev_free(s, buf);
    if (rc == LB_OK) rc = refresh_dens(s);
    return rc;
}

static int audit_now(lb_sim *s, double out[5])
{
    int st = sync_check(s);
    if (st != LB_OK) return st;
    if (launch_audit(s->p.storage, s->args, pop_buf(s), s->own[s->cur], pop_lay(s), s->d_audit_part, s->d_audit_out,
                     s->d_err, s->stream) != hipSuccess)
        return LB_EDEVICE;
    st = sync_check(s);
    if (st != LB_OK) return st;
    if (hipMemcpy(out, s->d_audit_out, 5 * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) return LB_EDEVICE;
    return LB_OK;
}

int lb_audit(lb_sim *s, double *mass, double P[3])
{
    if (!s || !mass || !P) return LB_EINVAL;
    const TraceRange tr("lb_audit");
    double a[5];
    const int st = audit_now(s, a);
    if (st != LB_OK) return st;
    *mass = s->p.rho0 * a[4] + a[0];
    for (int k = 0; k < 3; ++k) P[k] = a[1 + k];
    return LB_OK;
}

int lb_info(lb_sim *s, uint64_t *n_fluid, int64_t *steps)
{
    if (!s) return LB_EINVAL;
    if (n_fluid) {
        double a[5];
        const int st = audit_now(s, a);
        if (st != LB_OK) return st;
        *n_fluid = uint64_t(a[4]);
    }
    if (steps) *steps = s->steps;
    return LB_OK;
}

// ---------------------------------------------------------------------------
// checkpoint blob: header, populations (storage format), owners, bodies and
// both force-accumulator sets (they hold the conversion force still to be
// applied by the next integration)

struct StateHeader {
    uint64_t magic;
    int32_t nx, ny, nz, storage, scale_log2, nbody;
    int64_t steps;
    uint64_t pop_bytes;
    int32_t layout;  // the populations are saved in the handle's own layout
    int32_t pad;
};

// the saved-state format; the last byte is its version (3: populations in
// tiles of 256 cells where they fit 32-bit offsets, layout codes with
// LB_LAYOUT_AUTO = 0)
static constexpr uint64_t STATE_MAGIC = 0x34717362'6c03ull;
static constexpr size_t ACC_BYTES = NACCSET * ACCSET_SIZE * sizeof(unsigned long long);

int lb_state_size(lb_sim *s, size_t *bytes)
{
    if (!s || !bytes) return LB_EINVAL;
    *bytes = sizeof(StateHeader) + size_t(Q) * s->args.box.stride * s->esize + s->args.box.n +
             s->bodies.size() * sizeof(DevBody) + ACC_BYTES;
    return LB_OK;
}

int lb_save_state(lb_sim *s, void *buf, size_t bytes)
{
    size_t need = 0;
    if (!buf || lb_state_size(s, &need) != LB_OK || bytes < need) return LB_EINVAL;
    int st = sync_check(s);
    if (st != LB_OK) return st;
    st = pull_bodies(s);
    if (st != LB_OK) return st;
    st = classify_now(s);
    if (st != LB_OK) return st;
    if (hipStreamSynchronize(s->stream) != hipSuccess) return LB_EDEVICE;
    StateHeader h{STATE_MAGIC, s->p.nx, s->p.ny, s->p.nz, s->p.storage, s->p.scale_log2,
                  int32_t(s->bodies.size()), s->steps, uint64_t(Q) * s->args.box.stride * s->esize,
                  s->p.layout, 0};
    char *p = static_cast<char *>(buf);
    std::memcpy(p, &h, sizeof(h));
    p += sizeof(h);
    if (hipMemcpy(p, pop_buf(s), h.pop_bytes, hipMemcpyDeviceToHost) != hipSuccess) return LB_EDEVICE;
    p += h.pop_bytes;
    if (hipMemcpy(p, s->own[s->cur], s->args.box.n, hipMemcpyDeviceToHost) != hipSuccess) return LB_EDEVICE;
    p += s->args.box.n;
    if (!s->bodies.empty()) std::memcpy(p, s->bodies.data(), s->bodies.size() * sizeof(DevBody));
    p += s->bodies.size() * sizeof(DevBody);
    if (hipMemcpy(p, s->d_acc, ACC_BYTES, hipMemcpyDeviceToHost) != hipSuccess) return LB_EDEVICE;
    return LB_OK;
}

int lb_load_state(lb_sim *s, const void *buf, size_t bytes)
{
    if (!s || !buf || bytes < sizeof(StateHeader)) return LB_EINVAL;
    StateHeader h;
    std::memcpy(&h, buf, sizeof(h));
    if (h.magic != STATE_MAGIC || h.nx != s->p.nx || h.ny != s->p.ny || h.nz != s->p.nz ||
        h.storage != s->p.storage || h.scale_log2 != s->p.scale_log2 || h.nbody < 0 || h.nbody > MAXB ||
        h.pop_bytes != uint64_t(Q) * s->args.box.stride * s->esize || h.layout != s->p.layout)
        return LB_EINVAL;
    const size_t need = sizeof(h) + h.pop_bytes + s->args.box.n + size_t(h.nbody) * sizeof(DevBody) + ACC_BYTES;
    if (bytes < need) return LB_EINVAL;
    int st = sync_check(s);
    if (st != LB_OK) return st;
    const char *p = static_cast<const char *>(buf) + sizeof(h);
    s->cur = int(h.steps & 1);
    void *dst = s->f2 && (h.steps & 1) ? s->f2 : s->f;  // the buffer that holds step h.steps
    if (hipMemcpy(dst, p, h.pop_bytes, hipMemcpyHostToDevice) != hipSuccess) return LB_EDEVICE;
    p += h.pop_bytes;
    for (int k = 0; k < 2; ++k)
        if (hipMemcpy(s->own[k], p, s->args.box.n, hipMemcpyHostToDevice) != hipSuccess) return LB_EDEVICE;
    // static walls among the loaded owners (or none, replacing earlier
    // ones): their wall masks, as the first step would have computed them;
    // the loaded owner flags are kept
    bool walls = false;
    st = set_walls(s, reinterpret_cast<const uint8_t *>(p), &walls);
    if (st != LB_OK) return st;
    if (walls && launch_classify(s->args.box, s->own[s->cur], s->d_wmask, 0, s->stream) != hipSuccess)
        return LB_EDEVICE;
    p += s->args.box.n;
    s->bodies.assign(h.nbody, DevBody{});
    if (h.nbody) {
        std::memcpy(s->bodies.data(), p, size_t(h.nbody) * sizeof(DevBody));
        for (int k = 0; k < 2; ++k)
            if (hipMemcpy(s->d_bodies[k], s->bodies.data(), size_t(h.nbody) * sizeof(DevBody),
                          hipMemcpyHostToDevice) != hipSuccess)
                return LB_EDEVICE;
    }
    p += size_t(h.nbody) * sizeof(DevBody);
    if (hipMemcpy(s->d_acc, p, ACC_BYTES, hipMemcpyHostToDevice) != hipSuccess) return LB_EDEVICE;
    st = rebuild_lists(s);
    if (st != LB_OK) return st;
    s->steps = h.steps;
    s->started = true;
    s->need_classify = false;
    st = refresh_dens(s);
    if (st != LB_OK) return st;
    return sync_check(s);
}

int lb_kernel_timing(lb_sim *s, int enable)
{
    if (!s) return LB_EINVAL;
    const int st = sync_check(s);
    for (auto &e : s->evs) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    s->evs.clear();
    s->ms = 0.0;
    s->launches = 0;
    s->timing = enable != 0;
    return st;
}

int lb_kernel_time(lb_sim *s, double *ms, int64_t *launches)
{
    if (!s || !ms || !launches) return LB_EINVAL;
    const int st = sync_check(s);
    if (st != LB_OK) return st;
    int rc = LB_OK;
    for (auto &e : s->evs) {
        float t = 0.0f;
        if (rc == LB_OK && hipEventElapsedTime(&t, e.first, e.second) == hipSuccess) {
            s->ms += t;
            s->launches++;
        } else {
            rc = LB_EDEVICE;
        }
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    s->evs.clear();
    if (rc != LB_OK) return rc;
    *ms = s->ms;
    *launches = s->launches;
    return LB_OK;
}

}  // extern "C"
