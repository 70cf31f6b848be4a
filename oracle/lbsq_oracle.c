/*
 * lbsq_oracle.c -- plain FP64 CPU oracle for the lattice Boltzmann squirmer
 * method of Kuron, Staerk, Burkard, de Graaf and Holm, "A Lattice Boltzmann
 * Model for Squirmers" (arXiv:1903.04799).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the GPU path is checked against.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or helper with the HIP library.
 *
 * Everything is FP64 and written loop by loop in the order of the paper:
 *   - D3Q19 velocity set and the two-relaxation-time (TRT) collision,
 *     Sec. "Numerical Method", eq. (lb) and the equilibrium below it;
 *   - macroscopic moments rho = sum f, u = sum f c / rho (same section);
 *   - moving-wall bounce-back (the shifted reflection rule of the same
 *     section) with the Ladd surface velocity eq. (vb) plus the squirmer slip
 *     of eq. (squirmer), Sec. "The Squirmer Model";
 *   - momentum-exchange force and torque, eqs. (bbforce), (bbtorque), summed
 *     over boundary links, not averaged over two steps;
 *   - fluid <-> solid cell conversion with its compensating force,
 *     eq. (consforce);
 *   - WCA contact repulsion, eq. (wca);
 *   - symplectic Euler rigid-body integration (text after eq. (wca)).
 *
 * Readings taken where the printed text is garbled or silent (each with its
 * reason after it):
 *   - equilibrium coefficients 9/2 and 3/2 (the printed 1/6 cannot give the
 *     Navier-Stokes momentum flux);  u carries the 1/rho;
 *   - lambda_e, lambda_o are relaxation *rates*; nu = (1/lambda_e - 1/2)/3;
 *     the "magic" product Lambda = (1/lambda_e - 1/2)(1/lambda_o - 1/2);
 *   - the reflected population is the fluid node's own post-collision
 *     f_ibar(x_f) and rho in the wall term is the local density at x_f;
 *   - the wall velocity of a link is v + w x m + slip(m/|m|), evaluated at
 *     the link midpoint m = r_b + c_i/2 - r (minimum image), where the
 *     halfway bounce-back wall lies; the text names the boundary node r_b,
 *     but only the midpoint reproduces the swim speeds the paper plots in
 *     its resolution study (the solid node centre gives speeds 5-13% high,
 *     the fluid node 5-15% low, at R = 4..12);
 *   - force: sum over boundary links only of -c_i (f_ibar*(x) + f_i^in(x));
 *     torque with lever arm d to the solid node centre;
 *   - conversion: "+" for cells the body covers, "-" for cells it uncovers,
 *     with the matching torque d x (...); refill velocity v + w x d (no slip);
 *     refill density = mean density of D3Q19 neighbours fluid at both time
 *     levels, rho0 if none;
 *   - inside test in int64 fixed point with 2^-20 quanta, cell centres at
 *     i + 1/2, ties count as inside;
 *   - step order: stream + bounce-back + momentum exchange, collide,
 *     integrate, then geometry at the new positions and cell conversion;
 *     the conversion force enters the following integration (the same
 *     sequence of operations as converting at the start of the next step;
 *     the state between steps has cell owners that match the body
 *     positions);
 *   - symplectic Euler: v first, then r with the new v; w then e rotated by
 *     the exact rotation of angle |w| about w; m = rho_p 4/3 pi R^3,
 *     I = 2/5 m R^2;
 *   - WCA: F(r) = 24 eps / r [2 (s/r)^12 - (s/r)^6] along the centre line,
 *     r = surface-to-surface distance, cut off at 2^(1/6) s, r clamped at
 *     0.05 s (the printed trailing "+eps" belongs to the potential).
 *
 * Test-only hooks that are not part of the paper's method: a uniform body
 * force density g (Guo-type forcing split into TRT parts) used only for the
 * Poiseuille pin, and a per-cell velocity for static walls used only for the
 * Couette pin.
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define Q 19
#define OR_MAXB 253

enum { OR_FREE = 0, OR_FIXED = 1, OR_PRESCRIBED = 2 };
enum { OWN_FLUID = 0, OWN_WALL = 255 };

/* D3Q19: rest, 6 faces, 12 edges; pairs adjacent so that for odd i the
 * opposite direction is i+1. */
static const int CX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
static const int CY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
static const int CZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

static double weight(int i)
{
    int n = CX[i] * CX[i] + CY[i] * CY[i] + CZ[i] * CZ[i];
    if (n == 0) return 1.0 / 3.0;
    if (n == 1) return 1.0 / 18.0;
    return 1.0 / 36.0;
}

static int opposite(int i)
{
    if (i == 0) return 0;
    return (i % 2 == 1) ? i + 1 : i - 1;
}

typedef struct {
    double pos[3], e[3], v[3], w[3];
    double R, B1, beta, rho_p, m, I;
    int mode;
    double Fbb[3], Tbb[3], Fc[3], Tc[3], Fwca[3], F[3], T[3];
    double Fcn[3], Tcn[3]; /* conversion force/torque waiting for the next integration */
} or_body;

typedef struct {
    int nx, ny, nz;
    size_t n;
    double nu, magic, rho0, lam_e, lam_o;
    double g[3];
    double wca_sigma, wca_eps;
    double *f, *fnew;      /* [Q][n], post-collision populations */
    uint8_t *owner;        /* 0 fluid, 1..253 body id + 1, 255 wall */
    uint8_t *static_solid; /* 1 where a static wall is */
    double *wall_u;        /* optional [3][n] wall velocity (Couette hook) */
    uint8_t *uncovered;    /* per-step scratch */
    int nbody;
    or_body body[OR_MAXB];
    long step;
    /* per-step bookkeeping of the last step */
    double st_link_mass, st_covered_mass, st_uncovered_mass;
    long st_ncovered, st_nuncovered;
    /* link list of the last step */
    size_t nlinks, cap_links;
    uint32_t *lk_cell;
    uint8_t *lk_dir, *lk_body;
    /* covered / uncovered cells of the last step */
    size_t ncov, nunc, cap_conv;
    uint32_t *cov_cell, *unc_cell;
    uint8_t *cov_body, *unc_body;
    int geom_error;
    int runaway; /* a body moved a cell or more in one step: stepping stops */
} or_sim;

/* ------------------------------------------------------------------ */
/* small vector helpers                                                */

static void cross(const double a[3], const double b[3], double out[3])
{
    out[0] = a[1] * b[2] - a[2] * b[1];
    out[1] = a[2] * b[0] - a[0] * b[2];
    out[2] = a[0] * b[1] - a[1] * b[0];
}

static double dot(const double a[3], const double b[3])
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* Wrap a real-valued difference into the minimum image of a box of length L. */
static double minimg(double d, int L)
{
    while (d >= 0.5 * L) d -= L;
    while (d < -0.5 * L) d += L;
    return d;
}

static size_t cell_index(const or_sim *s, int x, int y, int z)
{
    return (size_t)x + (size_t)s->nx * ((size_t)y + (size_t)s->ny * (size_t)z);
}

static void cell_coords(const or_sim *s, size_t idx, int *x, int *y, int *z)
{
    *x = (int)(idx % (size_t)s->nx);
    *y = (int)((idx / (size_t)s->nx) % (size_t)s->ny);
    *z = (int)(idx / ((size_t)s->nx * (size_t)s->ny));
}

static int wrapi(int a, int n)
{
    a %= n;
    return a < 0 ? a + n : a;
}

/* Lever arm from a body centre to a cell centre (cell centres at i + 1/2). */
static void lever(const or_sim *s, const or_body *b, int x, int y, int z, double d[3])
{
    d[0] = minimg((x + 0.5) - b->pos[0], s->nx);
    d[1] = minimg((y + 0.5) - b->pos[1], s->ny);
    d[2] = minimg((z + 0.5) - b->pos[2], s->nz);
}

/* ------------------------------------------------------------------ */
/* model pieces exposed for the pins                                   */

/* D3Q19 velocities and weights. */
void or_lattice(int *c, double *w)
{
    for (int i = 0; i < Q; ++i) {
        c[3 * i + 0] = CX[i];
        c[3 * i + 1] = CY[i];
        c[3 * i + 2] = CZ[i];
        w[i] = weight(i);
    }
}

/* Second-order equilibrium, Sec. "Numerical Method" (coefficients 3, 9/2,
 * 3/2 for c_s^2 = 1/3). */
void or_feq(double rho, const double u[3], double *feq)
{
    double uu = dot(u, u);
    for (int i = 0; i < Q; ++i) {
        double cu = CX[i] * u[0] + CY[i] * u[1] + CZ[i] * u[2];
        feq[i] = weight(i) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
    }
}

/* Squirmer slip in the body's rest frame, eq. (squirmer):
 * u = B1 (1 + beta e.n)((e.n) n - e), n = d/|d|. */
void or_slip(const double d[3], const double e[3], double B1, double beta, double out[3])
{
    double r = sqrt(dot(d, d));
    double n[3] = {d[0] / r, d[1] / r, d[2] / r};
    double en = dot(e, n);
    double a = B1 * (1.0 + beta * en);
    for (int k = 0; k < 3; ++k) out[k] = a * (en * n[k] - e[k]);
}

/* WCA magnitude along the centre line as a function of the
 * surface-to-surface distance r, eq. (wca) without the stray constant. */
double or_wca(double r, double sigma, double eps)
{
    double rc = pow(2.0, 1.0 / 6.0) * sigma;
    if (r >= rc) return 0.0;
    if (r < 0.05 * sigma) r = 0.05 * sigma;
    double sr6 = pow(sigma / r, 6.0);
    return 24.0 * eps / r * (2.0 * sr6 * sr6 - sr6);
}

/* Rotate e about axis w by angle |w| (exact rotation, then renormalise). */
void or_rotate(double e[3], const double w[3])
{
    double th = sqrt(dot(w, w));
    if (th == 0.0) return;
    double k[3] = {w[0] / th, w[1] / th, w[2] / th};
    double kxe[3];
    cross(k, e, kxe);
    double ke = dot(k, e), c = cos(th), sn = sin(th);
    double out[3];
    for (int a = 0; a < 3; ++a) out[a] = e[a] * c + kxe[a] * sn + k[a] * ke * (1.0 - c);
    double nn = sqrt(dot(out, out));
    for (int a = 0; a < 3; ++a) e[a] = out[a] / nn;
}

/* Fixed-point inside test: cell (x,y,z) belongs to the sphere of radius R at
 * pos iff sum_k (X_k - P_k)^2 <= Rq^2 with X = (2i+1) 2^19, P = rint(pos 2^20),
 * Rq = rint(R 2^20), differences wrapped to the minimum image in quanta. */
int or_inside(int nx, int ny, int nz, int x, int y, int z, const double pos[3], double R)
{
    const int64_t ONE = (int64_t)1 << 20;
    int n[3] = {nx, ny, nz};
    int c[3] = {x, y, z};
    int64_t Rq = (int64_t)rint(R * (double)ONE);
    int64_t sum = 0;
    for (int k = 0; k < 3; ++k) {
        int64_t X = (2 * (int64_t)c[k] + 1) * (ONE / 2);
        int64_t P = (int64_t)rint(pos[k] * (double)ONE);
        int64_t L = (int64_t)n[k] * ONE;
        int64_t D = (X - P) % L;
        if (D < 0) D += L;
        if (D >= L / 2) D -= L;
        sum += D * D;
    }
    return sum <= Rq * Rq;
}

/* Symplectic Euler over one unit time step: velocities first, then the
 * position with the new velocity (wrapped into the periodic box), then the
 * orientation rotated by the new angular velocity.  FIXED bodies do not
 * move; PRESCRIBED bodies keep v and w and only advance r and e. */
void or_integrate(double pos[3], double e[3], double v[3], double w[3], const double F[3],
                  const double T[3], double m, double I, int mode, const int box[3])
{
    if (mode == OR_FREE) {
        for (int k = 0; k < 3; ++k) {
            v[k] += F[k] / m;
            w[k] += T[k] / I;
        }
    }
    if (mode == OR_FREE || mode == OR_PRESCRIBED) {
        for (int k = 0; k < 3; ++k) {
            double p = pos[k] + v[k];
            if (p >= box[k]) p -= box[k];
            if (p < 0.0) p += box[k];
            pos[k] = p;
        }
        or_rotate(e, w);
    }
}

/* ------------------------------------------------------------------ */
/* creation                                                            */

static double lam_e_of(double nu) { return 1.0 / (3.0 * nu + 0.5); }

or_sim *or_create(int nx, int ny, int nz, double nu, double magic, double rho0,
                  const double *g, double wca_sigma, double wca_eps)
{
    if (nx < 1 || ny < 1 || nz < 1 || nu <= 0.0 || magic <= 0.0) return NULL;
    or_sim *s = (or_sim *)calloc(1, sizeof(or_sim));
    s->nx = nx;
    s->ny = ny;
    s->nz = nz;
    s->n = (size_t)nx * ny * nz;
    s->nu = nu;
    s->magic = magic;
    s->rho0 = rho0;
    s->lam_e = lam_e_of(nu);
    /* Lambda = (1/lam_e - 1/2)(1/lam_o - 1/2) */
    s->lam_o = 1.0 / (magic / (1.0 / s->lam_e - 0.5) + 0.5);
    for (int k = 0; k < 3; ++k) s->g[k] = g ? g[k] : 0.0;
    s->wca_sigma = wca_sigma;
    s->wca_eps = wca_eps;
    s->f = (double *)calloc(Q * s->n, sizeof(double));
    s->fnew = (double *)calloc(Q * s->n, sizeof(double));
    s->owner = (uint8_t *)calloc(s->n, 1);
    s->static_solid = (uint8_t *)calloc(s->n, 1);
    s->uncovered = (uint8_t *)calloc(s->n, 1);
    for (int i = 0; i < Q; ++i)
        for (size_t x = 0; x < s->n; ++x) s->f[i * s->n + x] = weight(i) * rho0;
    return s;
}

void or_destroy(or_sim *s)
{
    if (!s) return;
    free(s->f);
    free(s->fnew);
    free(s->owner);
    free(s->static_solid);
    free(s->wall_u);
    free(s->uncovered);
    free(s->lk_cell);
    free(s->lk_dir);
    free(s->lk_body);
    free(s->cov_cell);
    free(s->unc_cell);
    free(s->cov_body);
    free(s->unc_body);
    free(s);
}

void or_relaxation_rates(const or_sim *s, double *lam_e, double *lam_o)
{
    *lam_e = s->lam_e;
    *lam_o = s->lam_o;
}

/* Geometry: owner of every cell from the walls and the body positions.
 * Returns 0, or -1 if two bodies claim the same cell. */
static int compute_owner(const or_sim *s, uint8_t *own)
{
    int err = 0;
    for (size_t idx = 0; idx < s->n; ++idx) {
        if (s->static_solid[idx]) {
            own[idx] = OWN_WALL;
            continue;
        }
        int x, y, z;
        cell_coords(s, idx, &x, &y, &z);
        uint8_t o = OWN_FLUID;
        for (int b = 0; b < s->nbody; ++b) {
            if (or_inside(s->nx, s->ny, s->nz, x, y, z, s->body[b].pos, s->body[b].R)) {
                if (o != OWN_FLUID) err = -1;
                else o = (uint8_t)(b + 1);
            }
        }
        own[idx] = o;
    }
    return err;
}

int or_set_static_mask(or_sim *s, const uint8_t *solid, const double *wall_u)
{
    if (s->step != 0) return -1;
    for (size_t x = 0; x < s->n; ++x) s->static_solid[x] = solid[x] ? 1 : 0;
    if (wall_u) {
        if (!s->wall_u) s->wall_u = (double *)calloc(3 * s->n, sizeof(double));
        memcpy(s->wall_u, wall_u, 3 * s->n * sizeof(double));
    }
    int err = compute_owner(s, s->owner);
    for (size_t x = 0; x < s->n; ++x)
        if (s->owner[x] != OWN_FLUID)
            for (int i = 0; i < Q; ++i) s->f[i * s->n + x] = 0.0;
    return err;
}

/* Add a body; returns its id (>= 0) or -1 on bad input (a free body needs
 * a positive density: its mass divides the force), -2 on overlap. */
int or_add_body(or_sim *s, const double pos[3], const double e[3], double R, double B1,
                double beta, int mode, const double v[3], const double w[3], double rho_p)
{
    if (s->step != 0 || s->nbody >= OR_MAXB || R <= 0.0) return -1;
    if (mode == OR_FREE && !(rho_p > 0.0)) return -1;
    double en = sqrt(dot(e, e));
    if (en == 0.0) return -1;
    or_body *b = &s->body[s->nbody];
    memset(b, 0, sizeof(*b));
    for (int k = 0; k < 3; ++k) {
        b->pos[k] = pos[k];
        b->e[k] = e[k] / en;
        b->v[k] = v ? v[k] : 0.0;
        b->w[k] = w ? w[k] : 0.0;
    }
    b->R = R;
    b->B1 = B1;
    b->beta = beta;
    b->mode = mode;
    b->rho_p = rho_p;
    b->m = rho_p * 4.0 / 3.0 * M_PI * R * R * R;
    b->I = 0.4 * b->m * R * R;
    s->nbody++;
    int err = compute_owner(s, s->owner);
    if (err) {
        s->nbody--;
        compute_owner(s, s->owner);
        return -2;
    }
    for (size_t x = 0; x < s->n; ++x)
        if (s->owner[x] != OWN_FLUID)
            for (int i = 0; i < Q; ++i) s->f[i * s->n + x] = 0.0;
    return s->nbody - 1;
}

/* ------------------------------------------------------------------ */
/* one time step                                                       */

static int is_fluid(uint8_t o) { return o == OWN_FLUID; }

static double cell_rho(const or_sim *s, const double *f, size_t idx)
{
    double r = 0.0;
    for (int i = 0; i < Q; ++i) r += f[i * s->n + idx];
    return r;
}

/* Wall velocity of the link in direction i whose source, the solid node
 * centred at cell (sx,sy,sz), has owner o.  For a body: eq. (vb) plus the
 * slip of eq. (squirmer), evaluated where the halfway bounce-back wall of the
 * link lies, at the link midpoint r_b + c_i/2; d receives the lever arm
 * r_b - r of eq. (bbtorque). */
static void boundary_velocity(const or_sim *s, uint8_t o, size_t sidx, int sx, int sy, int sz, int i,
                              double vb[3], double d[3])
{
    d[0] = d[1] = d[2] = 0.0;
    if (o == OWN_WALL) {
        for (int k = 0; k < 3; ++k) vb[k] = s->wall_u ? s->wall_u[k * s->n + sidx] : 0.0;
        return;
    }
    const or_body *b = &s->body[o - 1];
    lever(s, b, sx, sy, sz, d);
    double m[3] = {d[0] + 0.5 * CX[i], d[1] + 0.5 * CY[i], d[2] + 0.5 * CZ[i]};
    double wxm[3], slip[3] = {0.0, 0.0, 0.0};
    cross(b->w, m, wxm);
    if (b->B1 != 0.0) or_slip(m, b->e, b->B1, b->beta, slip);
    for (int k = 0; k < 3; ++k) vb[k] = b->v[k] + wxm[k] + slip[k];
}

/* Incoming population i at fluid cell x after streaming with bounce-back.
 * Returns 1 and fills the link data when the source node is solid. */
static double incoming(const or_sim *s, const double *f, size_t idx, int x, int y, int z, int i,
                       int *is_link, double vb[3], double d[3], double *rho_w)
{
    int sx = wrapi(x - CX[i], s->nx), sy = wrapi(y - CY[i], s->ny), sz = wrapi(z - CZ[i], s->nz);
    size_t sidx = cell_index(s, sx, sy, sz);
    uint8_t o = s->owner[sidx];
    if (is_fluid(o)) {
        *is_link = 0;
        return f[i * s->n + sidx];
    }
    *is_link = 1;
    boundary_velocity(s, o, sidx, sx, sy, sz, i, vb, d);
    double rw = cell_rho(s, f, idx);
    *rho_w = rw;
    double cv = CX[i] * vb[0] + CY[i] * vb[1] + CZ[i] * vb[2];
    return f[opposite(i) * s->n + idx] + 6.0 * weight(i) * rw * cv;
}

static void push_link(or_sim *s, size_t idx, int i, uint8_t o)
{
    if (s->nlinks == s->cap_links) {
        s->cap_links = s->cap_links ? 2 * s->cap_links : 1024;
        s->lk_cell = (uint32_t *)realloc(s->lk_cell, s->cap_links * sizeof(uint32_t));
        s->lk_dir = (uint8_t *)realloc(s->lk_dir, s->cap_links);
        s->lk_body = (uint8_t *)realloc(s->lk_body, s->cap_links);
    }
    s->lk_cell[s->nlinks] = (uint32_t)idx;
    s->lk_dir[s->nlinks] = (uint8_t)i;
    s->lk_body[s->nlinks] = o;
    s->nlinks++;
}

static void push_conv(or_sim *s, int covered, size_t idx, uint8_t o)
{
    if (s->ncov + s->nunc + 1 > s->cap_conv) {
        s->cap_conv = s->cap_conv ? 2 * s->cap_conv : 256;
        s->cov_cell = (uint32_t *)realloc(s->cov_cell, s->cap_conv * sizeof(uint32_t));
        s->unc_cell = (uint32_t *)realloc(s->unc_cell, s->cap_conv * sizeof(uint32_t));
        s->cov_body = (uint8_t *)realloc(s->cov_body, s->cap_conv);
        s->unc_body = (uint8_t *)realloc(s->unc_body, s->cap_conv);
    }
    if (covered) {
        s->cov_cell[s->ncov] = (uint32_t)idx;
        s->cov_body[s->ncov++] = o;
    } else {
        s->unc_cell[s->nunc] = (uint32_t)idx;
        s->unc_body[s->nunc++] = o;
    }
}

/* Cell conversion after the bodies have moved: covered cells hand their
 * momentum to the body, uncovered cells are refilled; the compensating force
 * and torque (eq. (consforce)) are kept for the next integration. */
static void convert_cells(or_sim *s)
{
    const size_t n = s->n;
    double *f = s->f;
    for (int b = 0; b < s->nbody; ++b)
        for (int k = 0; k < 3; ++k) s->body[b].Fcn[k] = s->body[b].Tcn[k] = 0.0;
    s->st_covered_mass = s->st_uncovered_mass = 0.0;
    s->st_ncovered = s->st_nuncovered = 0;
    s->ncov = s->nunc = 0;

    /* geometry at the new positions r(t+1) */
    uint8_t *own_new = (uint8_t *)malloc(n);
    if (compute_owner(s, own_new)) s->geom_error = 1;
    memset(s->uncovered, 0, n);

    /* covered cells: fluid before, body now; their momentum goes to the body */
    for (size_t idx = 0; idx < n; ++idx) {
        uint8_t o_old = s->owner[idx], o_new = own_new[idx];
        if (is_fluid(o_old) && o_new != OWN_FLUID && o_new != OWN_WALL) {
            or_body *B = &s->body[o_new - 1];
            int x, y, z;
            cell_coords(s, idx, &x, &y, &z);
            double p[3] = {0.0, 0.0, 0.0}, d[3], dxp[3];
            for (int i = 0; i < Q; ++i) {
                double fi = f[i * n + idx];
                p[0] += CX[i] * fi;
                p[1] += CY[i] * fi;
                p[2] += CZ[i] * fi;
            }
            lever(s, B, x, y, z, d);
            cross(d, p, dxp);
            for (int k = 0; k < 3; ++k) {
                B->Fcn[k] += p[k];
                B->Tcn[k] += dxp[k];
            }
            s->st_covered_mass += cell_rho(s, f, idx);
            s->st_ncovered++;
            push_conv(s, 1, idx, o_new);
        }
        if (o_old != OWN_FLUID && o_old != OWN_WALL && is_fluid(o_new)) s->uncovered[idx] = 1;
    }
    uint8_t *own_old = (uint8_t *)malloc(n);
    memcpy(own_old, s->owner, n);
    memcpy(s->owner, own_new, n);
    free(own_new);
    for (size_t idx = 0; idx < n; ++idx)
        if (!is_fluid(s->owner[idx]) && !s->uncovered[idx])
            for (int i = 0; i < Q; ++i) f[i * n + idx] = 0.0;

    /* uncovered cells: refill with f^eq(mean neighbour density, v + w x d).
     * The densities are taken before any refill is written. */
    double *refill_rho = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    for (size_t idx = 0; idx < n; ++idx) {
        if (!s->uncovered[idx]) continue;
        int x, y, z;
        cell_coords(s, idx, &x, &y, &z);
        double sum = 0.0;
        int cnt = 0;
        for (int i = 1; i < Q; ++i) {
            size_t nidx = cell_index(s, wrapi(x + CX[i], s->nx), wrapi(y + CY[i], s->ny),
                                     wrapi(z + CZ[i], s->nz));
            if (is_fluid(s->owner[nidx]) && !s->uncovered[nidx]) {
                sum += cell_rho(s, f, nidx);
                cnt++;
            }
        }
        refill_rho[idx] = cnt ? sum / cnt : s->rho0;
    }
    for (size_t idx = 0; idx < n; ++idx) {
        if (!s->uncovered[idx]) continue;
        int x, y, z;
        cell_coords(s, idx, &x, &y, &z);
        int bsel = own_old[idx] - 1; /* the body that left the cell */
        or_body *B = &s->body[bsel];
        double d[3], wxd[3], u[3], feq[Q], dxp[3];
        lever(s, B, x, y, z, d);
        cross(B->w, d, wxd);
        for (int k = 0; k < 3; ++k) u[k] = B->v[k] + wxd[k];
        double rb = refill_rho[idx];
        or_feq(rb, u, feq);
        for (int i = 0; i < Q; ++i) f[i * n + idx] = feq[i];
        double p[3] = {rb * u[0], rb * u[1], rb * u[2]};
        cross(d, p, dxp);
        for (int k = 0; k < 3; ++k) {
            B->Fcn[k] -= p[k];
            B->Tcn[k] -= dxp[k];
        }
        s->st_uncovered_mass += rb;
        s->st_nuncovered++;
        push_conv(s, 0, idx, (uint8_t)(bsel + 1));
    }
    free(refill_rho);
    free(own_old);
}

static void one_step(or_sim *s)
{
    const size_t n = s->n;
    double *f = s->f;

    for (int b = 0; b < s->nbody; ++b) {
        or_body *B = &s->body[b];
        for (int k = 0; k < 3; ++k) B->Fbb[k] = B->Tbb[k] = B->Fwca[k] = 0.0;
    }
    s->st_link_mass = 0.0;
    s->nlinks = 0;

    /* 4a. boundary links, momentum exchange and the wall mass term */
    for (size_t idx = 0; idx < n; ++idx) {
        if (!is_fluid(s->owner[idx])) continue;
        int x, y, z;
        cell_coords(s, idx, &x, &y, &z);
        for (int i = 1; i < Q; ++i) {
            int link;
            double vb[3], d[3], rw = 0.0;
            double fin = incoming(s, f, idx, x, y, z, i, &link, vb, d, &rw);
            if (!link) continue;
            int sx = wrapi(x - CX[i], s->nx), sy = wrapi(y - CY[i], s->ny),
                sz = wrapi(z - CZ[i], s->nz);
            uint8_t o = s->owner[cell_index(s, sx, sy, sz)];
            push_link(s, idx, i, o);
            double cv = CX[i] * vb[0] + CY[i] * vb[1] + CZ[i] * vb[2];
            s->st_link_mass += 6.0 * weight(i) * rw * cv;
            if (o == OWN_WALL) continue;
            or_body *B = &s->body[o - 1];
            double fout = f[opposite(i) * n + idx];
            double dp[3] = {-CX[i] * (fout + fin), -CY[i] * (fout + fin), -CZ[i] * (fout + fin)};
            double dxp[3];
            cross(d, dp, dxp);
            for (int k = 0; k < 3; ++k) {
                B->Fbb[k] += dp[k];
                B->Tbb[k] += dxp[k];
            }
        }
    }

    /* 4b + 5. stream with bounce-back, then TRT collision */
    double *fn = s->fnew;
    const double le = s->lam_e, lo = s->lam_o;
#pragma omp parallel for schedule(static)
    for (long long li = 0; li < (long long)n; ++li) {
        size_t idx = (size_t)li;
        if (!is_fluid(s->owner[idx])) {
            for (int i = 0; i < Q; ++i) fn[i * n + idx] = 0.0;
            continue;
        }
        int x, y, z;
        cell_coords(s, idx, &x, &y, &z);
        double fin[Q];
        fin[0] = f[idx];
        for (int i = 1; i < Q; ++i) {
            int link;
            double vb[3], d[3], rw;
            fin[i] = incoming(s, f, idx, x, y, z, i, &link, vb, d, &rw);
        }
        double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < Q; ++i) {
            rho += fin[i];
            j[0] += CX[i] * fin[i];
            j[1] += CY[i] * fin[i];
            j[2] += CZ[i] * fin[i];
        }
        double u[3];
        for (int k = 0; k < 3; ++k) u[k] = (j[k] + 0.5 * s->g[k]) / rho;
        double feq[Q];
        or_feq(rho, u, feq);
        double ug = dot(u, s->g);
        for (int i = 0; i < Q; ++i) {
            int ib = opposite(i);
            double fp = 0.5 * (fin[i] + fin[ib]), fm = 0.5 * (fin[i] - fin[ib]);
            double ep = 0.5 * (feq[i] + feq[ib]), em = 0.5 * (feq[i] - feq[ib]);
            double out = fin[i] - le * (fp - ep) - lo * (fm - em);
            /* test-only forcing (Guo terms split into even and odd parts) */
            double cg = CX[i] * s->g[0] + CY[i] * s->g[1] + CZ[i] * s->g[2];
            double cu = CX[i] * u[0] + CY[i] * u[1] + CZ[i] * u[2];
            double s_odd = 3.0 * weight(i) * cg;
            double s_even = weight(i) * (9.0 * cu * cg - 3.0 * ug);
            out += (1.0 - 0.5 * le) * s_even + (1.0 - 0.5 * lo) * s_odd;
            fn[i * n + idx] = out;
        }
    }
    s->f = fn;
    s->fnew = f;

    /* 6. WCA between bodies, then symplectic Euler */
    for (int a = 0; a < s->nbody; ++a)
        for (int b = a + 1; b < s->nbody; ++b) {
            or_body *A = &s->body[a], *B = &s->body[b];
            double dv[3] = {minimg(B->pos[0] - A->pos[0], s->nx), minimg(B->pos[1] - A->pos[1], s->ny),
                            minimg(B->pos[2] - A->pos[2], s->nz)};
            double dist = sqrt(dot(dv, dv));
            double fm = or_wca(dist - A->R - B->R, s->wca_sigma, s->wca_eps);
            if (fm == 0.0) continue;
            for (int k = 0; k < 3; ++k) {
                B->Fwca[k] += fm * dv[k] / dist;
                A->Fwca[k] -= fm * dv[k] / dist;
            }
        }
    int nn[3] = {s->nx, s->ny, s->nz};
    for (int b = 0; b < s->nbody; ++b) {
        or_body *B = &s->body[b];
        for (int k = 0; k < 3; ++k) {
            B->Fc[k] = B->Fcn[k];
            B->Tc[k] = B->Tcn[k];
            B->F[k] = B->Fbb[k] + B->Fc[k] + B->Fwca[k];
            B->T[k] = B->Tbb[k] + B->Tc[k];
        }
        or_integrate(B->pos, B->e, B->v, B->w, B->F, B->T, B->m, B->I, B->mode, nn);
        /* the cell conversion below compares owners one step apart, which
           takes a body moving less than one cell per step: a faster or
           non-finite velocity ends the run with a geometry error */
        for (int k = 0; k < 3; ++k)
            if (!(fabs(B->v[k]) < 1.0)) s->runaway = 1;
    }
    s->step++;
    if (s->runaway) {
        s->geom_error = 1;
        return;
    }
    convert_cells(s);
}

/* Test-only: the cell conversion of eq. (consforce) alone, on the state the
 * caller has written.  The owners still describe the bodies where they were
 * when the populations were set; the caller has moved the bodies since
 * (or_set_body_state).  Covered and uncovered cells are converted exactly
 * as at the end of a step, and the conversion force and torque are left in
 * Fc_next, Tc_next.  No streaming, collision or integration takes place. */
int or_convert_only(or_sim *s)
{
    s->geom_error = 0;
    convert_cells(s);
    return s->geom_error ? -2 : 0;
}

int or_step(or_sim *s, int nsteps)
{
    for (int t = 0; t < nsteps && !s->runaway; ++t) one_step(s);
    return s->geom_error ? -2 : 0;
}

/* ------------------------------------------------------------------ */
/* readout                                                             */

void or_get_fields(const or_sim *s, double *rho, double *u, uint8_t *owner)
{
    for (size_t idx = 0; idx < s->n; ++idx) {
        if (owner) owner[idx] = s->owner[idx];
        if (!is_fluid(s->owner[idx])) {
            rho[idx] = 0.0;
            u[idx] = u[s->n + idx] = u[2 * s->n + idx] = 0.0;
            continue;
        }
        double r = 0.0, j[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < Q; ++i) {
            double fi = s->f[i * s->n + idx];
            r += fi;
            j[0] += CX[i] * fi;
            j[1] += CY[i] * fi;
            j[2] += CZ[i] * fi;
        }
        rho[idx] = r;
        /* the stored populations are post-collision and already carry the
         * whole force impulse g; the half-step velocity takes back g/2 */
        for (int k = 0; k < 3; ++k) u[k * s->n + idx] = (j[k] - 0.5 * s->g[k]) / r;
    }
}

void or_get_populations(const or_sim *s, double *f)
{
    memcpy(f, s->f, Q * s->n * sizeof(double));
}

int or_set_populations(or_sim *s, const double *f)
{
    memcpy(s->f, f, Q * s->n * sizeof(double));
    for (size_t idx = 0; idx < s->n; ++idx)
        if (!is_fluid(s->owner[idx]))
            for (int i = 0; i < Q; ++i) s->f[i * s->n + idx] = 0.0;
    return 0;
}

/* out: pos e v w F T Fbb Tbb Fc Tc Fwca Fc_next Tc_next (13 x 3 doubles),
 * then m, I.  Fc, Tc entered the last integration; Fc_next, Tc_next come
 * from the conversion that followed it and enter the next one. */
int or_body_state(const or_sim *s, int id, double *out)
{
    if (id < 0 || id >= s->nbody) return -1;
    const or_body *B = &s->body[id];
    const double *src[13] = {B->pos, B->e, B->v, B->w, B->F, B->T, B->Fbb, B->Tbb,
                             B->Fc, B->Tc, B->Fwca, B->Fcn, B->Tcn};
    for (int a = 0; a < 13; ++a)
        for (int k = 0; k < 3; ++k) out[3 * a + k] = src[a][k];
    out[39] = B->m;
    out[40] = B->I;
    return 0;
}

/* Overwrite a body's kinematic state (checkpoint/resume and test set-ups). */
int or_set_body_state(or_sim *s, int id, const double pos[3], const double e[3], const double v[3],
                      const double w[3])
{
    if (id < 0 || id >= s->nbody) return -1;
    or_body *B = &s->body[id];
    for (int k = 0; k < 3; ++k) {
        B->pos[k] = pos[k];
        B->e[k] = e[k];
        B->v[k] = v[k];
        B->w[k] = w[k];
    }
    return 0;
}

/* The current link set: fluid cell, direction i (source x - c_i is solid),
 * owner of the solid node (body id + 1, or 255 for a wall).  Computed from
 * the current geometry, sorted by (cell, direction). Returns the count. */
size_t or_links(or_sim *s, uint32_t *cell, uint8_t *dir, uint8_t *body, size_t cap)
{
    size_t cnt = 0;
    for (size_t idx = 0; idx < s->n; ++idx) {
        if (!is_fluid(s->owner[idx])) continue;
        int x, y, z;
        cell_coords(s, idx, &x, &y, &z);
        for (int i = 1; i < Q; ++i) {
            size_t sidx = cell_index(s, wrapi(x - CX[i], s->nx), wrapi(y - CY[i], s->ny),
                                     wrapi(z - CZ[i], s->nz));
            uint8_t o = s->owner[sidx];
            if (is_fluid(o)) continue;
            if (cnt < cap) {
                cell[cnt] = (uint32_t)idx;
                dir[cnt] = (uint8_t)i;
                body[cnt] = o;
            }
            cnt++;
        }
    }
    return cnt;
}

/* Covered and uncovered cells of the last step (cells, owner id + 1). */
void or_conversions(const or_sim *s, uint32_t *cov, uint8_t *covb, size_t *ncov, uint32_t *unc,
                    uint8_t *uncb, size_t *nunc, size_t cap)
{
    for (size_t k = 0; k < s->ncov && k < cap; ++k) {
        cov[k] = s->cov_cell[k];
        covb[k] = s->cov_body[k];
    }
    for (size_t k = 0; k < s->nunc && k < cap; ++k) {
        unc[k] = s->unc_cell[k];
        uncb[k] = s->unc_body[k];
    }
    *ncov = s->ncov;
    *nunc = s->nunc;
}

/* Mass bookkeeping of the last step: link term, covered mass, uncovered mass. */
void or_step_stats(const or_sim *s, double *out)
{
    out[0] = s->st_link_mass;
    out[1] = s->st_covered_mass;
    out[2] = s->st_uncovered_mass;
    out[3] = (double)s->st_ncovered;
    out[4] = (double)s->st_nuncovered;
}

/* Neumaier compensated accumulation: sum += x, with the rounding error of
 * every addition kept in comp. */
static void acc(double *sum, double *comp, double x)
{
    double t = *sum + x;
    if (fabs(*sum) >= fabs(x)) *comp += (*sum - t) + x;
    else *comp += (x - t) + *sum;
    *sum = t;
}

/* Global FP64 mass and momentum of the fluid populations (compensated sums,
 * so that the audit itself adds no visible round-off). */
void or_audit(const or_sim *s, double *mass, double *P)
{
    double m = 0.0, mc = 0.0, p[3] = {0.0, 0.0, 0.0}, pc[3] = {0.0, 0.0, 0.0};
    for (size_t idx = 0; idx < s->n; ++idx) {
        if (!is_fluid(s->owner[idx])) continue;
        for (int i = 0; i < Q; ++i) {
            double fi = s->f[i * s->n + idx];
            acc(&m, &mc, fi);
            acc(&p[0], &pc[0], CX[i] * fi);
            acc(&p[1], &pc[1], CY[i] * fi);
            acc(&p[2], &pc[2], CZ[i] * fi);
        }
    }
    *mass = m + mc;
    for (int k = 0; k < 3; ++k) P[k] = p[k] + pc[k];
}

long or_get_step(const or_sim *s) { return s->step; }

/* OpenMP threads the stream/collide loop runs on, and a way to set them
 * (the CPU baseline times the oracle on all host threads and on one). */
int or_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void or_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
