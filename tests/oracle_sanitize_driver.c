/*
 * Drives every entry point of the FP64 oracle (oracle/lbsq_oracle.c) once
 * through a scene with static walls, a moving wall, a prescribed body that
 * converts cells every step and a free squirmer, so that the oracle can be
 * built and run under AddressSanitizer and UndefinedBehaviorSanitizer.  The
 * test that builds it checks for a clean exit and no sanitizer report.
 * Test infrastructure: it calls the oracle only.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct or_sim or_sim;
void or_lattice(int *c, double *w);
void or_feq(double rho, const double u[3], double *feq);
void or_slip(const double d[3], const double e[3], double B1, double beta, double out[3]);
double or_wca(double r, double sigma, double eps);
void or_rotate(double e[3], const double w[3]);
int or_inside(int nx, int ny, int nz, int x, int y, int z, const double pos[3], double R);
void or_integrate(double pos[3], double e[3], double v[3], double w[3], const double F[3], const double T[3],
                  double m, double I, int mode, const int box[3]);
or_sim *or_create(int nx, int ny, int nz, double nu, double magic, double rho0, const double *g, double wca_sigma,
                  double wca_eps);
void or_destroy(or_sim *s);
void or_relaxation_rates(const or_sim *s, double *lam_e, double *lam_o);
int or_set_static_mask(or_sim *s, const uint8_t *solid, const double *wall_u);
int or_add_body(or_sim *s, const double pos[3], const double e[3], double R, double B1, double beta, int mode,
                const double v[3], const double w[3], double rho_p);
int or_step(or_sim *s, int nsteps);
void or_get_fields(const or_sim *s, double *rho, double *u, uint8_t *owner);
void or_get_populations(const or_sim *s, double *f);
int or_set_populations(or_sim *s, const double *f);
int or_body_state(const or_sim *s, int id, double *out);
int or_set_body_state(or_sim *s, int id, const double pos[3], const double e[3], const double v[3],
                      const double w[3]);
size_t or_links(or_sim *s, uint32_t *cell, uint8_t *dir, uint8_t *body, size_t cap);
void or_conversions(const or_sim *s, uint32_t *cov, uint8_t *covb, size_t *ncov, uint32_t *unc, uint8_t *uncb,
                    size_t *nunc, size_t cap);
void or_step_stats(const or_sim *s, double *out);
void or_audit(const or_sim *s, double *mass, double *P);
long or_get_step(const or_sim *s);

#define CHECK(cond)                                                         \
    do {                                                                    \
        if (!(cond)) {                                                      \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            return 1;                                                       \
        }                                                                   \
    } while (0)

int main(void)
{
    /* model pieces */
    int c[57];
    double w[19], feq[19], out[3];
    or_lattice(c, w);
    const double u[3] = {0.01, -0.02, 0.005};
    or_feq(1.01, u, feq);
    const double d[3] = {3.0, 1.0, -2.0}, e0[3] = {1.0, 0.0, 0.0};
    or_slip(d, e0, 1e-3, 2.0, out);
    CHECK(or_wca(0.5, 1.0, 0.01) > 0.0 && or_wca(2.0, 1.0, 0.01) == 0.0);
    double e1[3] = {0.0, 1.0, 0.0};
    const double wr[3] = {0.01, 0.02, -0.03};
    or_rotate(e1, wr);
    const double p0[3] = {8.5, 8.5, 8.5};
    CHECK(or_inside(16, 16, 16, 8, 8, 8, p0, 3.0) == 1 && or_inside(16, 16, 16, 0, 0, 0, p0, 3.0) == 0);
    {
        double pos[3] = {15.9, 0.1, 7.0}, e[3] = {1.0, 0.0, 0.0}, v[3] = {0.3, -0.3, 0.0}, wv[3] = {0, 0, 0.01};
        const double F[3] = {1e-3, 0, 0}, T[3] = {0, 0, 1e-3};
        const int box[3] = {16, 16, 16};
        or_integrate(pos, e, v, wv, F, T, 100.0, 10.0, 0, box);
        CHECK(pos[0] >= 0.0 && pos[0] < 16.0 && pos[1] >= 0.0 && pos[1] < 16.0);
    }

    /* a scene */
    const int nx = 22, ny = 18, nz = 16;
    const size_t n = (size_t)nx * ny * nz;
    const double g[3] = {1e-6, 0.0, 0.0};
    or_sim *s = or_create(nx, ny, nz, 1.0 / 6.0, 3.0 / 16.0, 1.0, g, 1.0, 0.01);
    CHECK(s != NULL);
    double le, lo;
    or_relaxation_rates(s, &le, &lo);
    CHECK(le > 0.0 && lo > 0.0);
    uint8_t *solid = calloc(n, 1);
    double *wall_u = calloc(3 * n, sizeof(double));
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const size_t lo_cell = (size_t)x + (size_t)nx * (size_t)y;  /* z = 0 */
            const size_t hi_cell = lo_cell + (size_t)nx * ny * (nz - 1); /* z = nz-1, moving */
            solid[lo_cell] = 1;
            solid[hi_cell] = 1;
            wall_u[3 * hi_cell] = 1e-3;
        }
    CHECK(or_set_static_mask(s, solid, wall_u) == 0);
    /* a prescribed body moving 3.4 cells over the run, and a free squirmer
       that it never comes within contact range of */
    const double pa[3] = {6.3, 8.7, 7.9}, ea[3] = {1.0, 0.3, 0.0}, va[3] = {0.12, 0.05, 0.02}, wa[3] = {0, 0, 0.02};
    const double pb[3] = {17.5, 9.2, 8.1}, eb[3] = {-1.0, 0.2, 0.1}, zero[3] = {0, 0, 0};
    CHECK(or_add_body(s, pa, ea, 3.2, 0.0, 0.0, 2, va, wa, 0.0) == 0);  /* prescribed */
    CHECK(or_add_body(s, pb, eb, 3.0, 0.02, -3.0, 0, zero, zero, 0.0) == -1); /* free, no mass */
    CHECK(or_add_body(s, pb, eb, 3.0, 0.02, -3.0, 0, zero, zero, 1.0) == 1);  /* free */
    size_t conversions = 0;
    for (int t = 0; t < 25; ++t) {
        CHECK(or_step(s, 1) == 0);
        uint32_t cov[4096], unc[4096];
        uint8_t covb[4096], uncb[4096];
        size_t ncov = 0, nunc = 0;
        or_conversions(s, cov, covb, &ncov, unc, uncb, &nunc, 4096);
        conversions += ncov + nunc;
        double st[5];
        or_step_stats(s, st);
    }
    CHECK(or_get_step(s) == 25);
    CHECK(conversions > 0);
    const size_t nl = or_links(s, NULL, NULL, NULL, 0);
    CHECK(nl > 0);
    uint32_t *cell = malloc(nl * sizeof(uint32_t));
    uint8_t *dir = malloc(nl), *body = malloc(nl);
    CHECK(or_links(s, cell, dir, body, nl) == nl);
    double *rho = malloc(n * sizeof(double)), *uu = malloc(3 * n * sizeof(double));
    uint8_t *own = malloc(n);
    or_get_fields(s, rho, uu, own);
    double *f = malloc(19 * n * sizeof(double));
    or_get_populations(s, f);
    CHECK(or_set_populations(s, f) == 0);
    double bs[41];
    CHECK(or_body_state(s, 1, bs) == 0 && or_body_state(s, 2, bs) != 0);
    CHECK(or_set_body_state(s, 1, bs, bs + 3, bs + 6, bs + 9) == 0);
    CHECK(or_step(s, 3) == 0);
    double mass, P[3];
    or_audit(s, &mass, P);
    CHECK(mass > 0.0);
    or_destroy(s);

    /* a body faster than one cell per step ends the run with a geometry
       error instead of converting cells it jumped over */
    or_sim *r = or_create(16, 16, 16, 1.0 / 6.0, 3.0 / 16.0, 1.0, NULL, 1.0, 0.01);
    CHECK(r != NULL);
    const double pr[3] = {8.0, 8.0, 8.0}, vr[3] = {1.5, 0.0, 0.0};
    CHECK(or_add_body(r, pr, e0, 3.0, 0.0, 0.0, 2, vr, zero, 0.0) == 0);
    CHECK(or_step(r, 5) == -2);
    CHECK(or_get_step(r) == 1);
    or_destroy(r);

    free(solid);
    free(wall_u);
    free(cell);
    free(dir);
    free(body);
    free(rho);
    free(uu);
    free(own);
    free(f);
    printf("oracle driver: %zu conversions, %zu links, mass %.6f\n", conversions, nl, mass);
    return 0;
}
