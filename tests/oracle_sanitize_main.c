/* Test infrastructure: drives both CPU oracles (the LB oracle and the
 * finite-difference one) through every option on small, ragged and
 * degenerate domains, for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_oracle_sanitize.py).  A bad index,
 * an overflow, a leak or a non-finite field fails the run; the values
 * themselves are checked by the other oracle tests.
 *
 * The FD oracle has no header: its source is included here. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "lbpf_oracle.h"
#include "fd_oracle.c"

static int failures = 0;

#define CHECK(cond, what)                                              \
    do {                                                               \
        if (!(cond)) {                                                 \
            fprintf(stderr, "FAILED: %s (%s:%d)\n", what, __FILE__, __LINE__); \
            ++failures;                                                \
        }                                                              \
    } while (0)

/* A spherical seed of radius r at the domain centre, tanh profile. */
static void seed(int nx, int ny, int nz, double r, double* phi, double* U, double* th, double th0) {
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const size_t i = ((size_t)z * ny + y) * nx + x;
                const double dx = x - 0.5 * (nx - 1), dy = y - 0.5 * (ny - 1), dz = z - 0.5 * (nz - 1);
                const double d = sqrt(dx * dx + dy * dy + dz * dz) - r;
                phi[i] = -tanh(d / sqrt(2.0));
                U[i] = -0.3 + 0.01 * (double)((x + 2 * y + 3 * z) % 5);
                th[i] = th0;
            }
}

static int finite_all(const double* a, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!isfinite(a[i])) return 0;
    return 1;
}

static orc_params base(int nx, int ny, int nz, int q) {
    orc_params p;
    memset(&p, 0, sizeof(p));
    p.nx = nx; p.ny = ny; p.nz = nz;
    p.lattice = q;
    p.dx = 0.8; p.dt = 0.012;
    p.W0 = 1.0; p.tau0 = 1.0;
    p.lambda = 2.0; p.Mcinf = 0.4;
    p.k = 0.15; p.D = 1.0; p.kappa = 2.0;
    p.aniso = ORC_ANISO_CUBIC; p.eps = 0.05;
    return p;
}

static void run_lb(const char* name, const orc_params* p, int with_vfield) {
    const size_t n = (size_t)p->nx * p->ny * p->nz;
    double *phi = calloc(n, sizeof(double)), *U = calloc(n, sizeof(double)), *th = calloc(n, sizeof(double));
    orc_ctx* c = orc_create(p);
    CHECK(c != NULL, name);
    if (!c) { free(phi); free(U); free(th); return; }
    seed(p->nx, p->ny, p->nz, 2.5, phi, U, th, -0.4);
    CHECK(orc_init(c, phi, U, th) == 0, name);
    if (with_vfield) {
        double *vx = calloc(n, sizeof(double)), *vy = calloc(n, sizeof(double)), *vz = calloc(n, sizeof(double));
        for (size_t i = 0; i < n; ++i) { vx[i] = 0.01 * (double)(i % 7) / 7.0; vy[i] = -0.005; vz[i] = 0.002; }
        CHECK(orc_set_velocity_field(c, vx, vy, vz) == 0, name);
        free(vx); free(vy); free(vz);
    }
    CHECK(orc_step(c, 6) == 0, name);
    double rec[ORC_R_COUNT];
    const double centre[3] = {0.5 * (p->nx - 1), 0.5 * (p->ny - 1), 0.5 * (p->nz - 1)};
    orc_reduce(c, centre, rec);
    CHECK(rec[ORC_R_NONFINITE] == 0.0, name);
    orc_fields(c, phi, U, th);
    CHECK(finite_all(phi, n) && finite_all(U, n) && finite_all(th, n), name);
    const int qs[3] = {p->lattice, p->lattice_ut ? p->lattice_ut : p->lattice,
                       p->lattice_ut ? p->lattice_ut : p->lattice};
    for (int f = 0; f < 3; ++f) {
        double* pops = malloc((size_t)qs[f] * n * sizeof(double));
        orc_get_pops(c, f, pops);
        orc_set_pops(c, f, pops);
        free(pops);
    }
    CHECK(orc_stream_only(c, 3) == 0, name);
    CHECK(orc_step_count(c) == 6, name);
    orc_destroy(c);
    free(phi); free(U); free(th);
}

static void run_fd(const char* name, fdo_params p) {
    const size_t n = (size_t)p.nx * p.ny * p.nz;
    double *phi = calloc(n, sizeof(double)), *U = calloc(n, sizeof(double)), *th = calloc(n, sizeof(double));
    fdo_ctx* c = fdo_create(&p);
    CHECK(c != NULL, name);
    if (!c) { free(phi); free(U); free(th); return; }
    seed(p.nx, p.ny, p.nz, 2.5, phi, U, th, -0.4);
    fdo_set(c, phi, U, th);
    fdo_step(c, 0.01, 5);
    fdo_get(c, phi, U, th);
    CHECK(finite_all(phi, n) && finite_all(U, n) && finite_all(th, n), name);
    fdo_destroy(c);
    free(phi); free(U); free(th);
}

int main(void) {
    /* LB oracle: every lattice, wall kind, anisotropy and option */
    orc_params p = base(13, 11, 9, 19);
    p.wall[1] = ORC_WALL_SYMMETRY; p.wall[3] = ORC_WALL_SYMMETRY;
    run_lb("D3Q19 mixed walls", &p, 0);

    p = base(12, 7, 10, 15);
    p.lattice_ut = 7;
    p.aniso = ORC_ANISO_K41K61; p.eps = 0.0; p.delta = -0.02;
    p.vel[0] = 0.03; p.vel[1] = -0.01; p.vel[2] = 0.02;
    p.grad_stencil = 1;
    for (int f = 0; f < 6; ++f) p.wall[f] = ORC_WALL_SYMMETRY;
    run_lb("D3Q15 phi, D3Q7 U theta, K41/K61, advection, isotropic gradient", &p, 0);

    p = base(9, 9, 9, 7);
    p.skip_theta = 1;
    run_lb("D3Q7 isothermal", &p, 1);

    p = base(16, 14, 1, 19);
    p.Mcinf = 0.0; p.skip_U = 1;
    p.wall[4] = ORC_WALL_SYMMETRY; p.wall[5] = ORC_WALL_SYMMETRY;
    run_lb("one-node slab, pure substance", &p, 0);

    p = base(1, 1, 1, 19);
    run_lb("single node", &p, 0);

    p = base(2, 3, 1, 15);
    p.lattice_ut = 19;
    run_lb("2x3x1, D3Q15 phi with D3Q19 U theta", &p, 1);

    /* invalid parameters are refused, not run */
    p = base(4, 4, 4, 9);
    CHECK(orc_create(&p) == NULL, "lattice 9 refused");
    p = base(0, 4, 4, 19);
    CHECK(orc_create(&p) == NULL, "empty domain refused");

    /* FD oracle: both stencils, both anisotropies, the single-field modes */
    fdo_params f;
    memset(&f, 0, sizeof(f));
    f.nx = 11; f.ny = 9; f.nz = 7;
    f.dx = 0.8; f.W0 = 1.0; f.tau0 = 1.0; f.lambda = 2.0; f.Mcinf = 0.4; f.k = 0.15; f.D = 1.0; f.kappa = 2.0;
    f.aniso = 0; f.eps = 0.05; f.stencil = 6;
    run_fd("FD6 cubic", f);
    f.aniso = 1; f.eps = 0.0; f.delta = -0.02; f.skip_theta = 1;
    run_fd("FD6 K41/K61 isothermal", f);
    f.aniso = 0; f.eps = 0.0; f.delta = 0.0; f.skip_theta = 0; f.stencil = 18; f.Mcinf = 0.0; f.skip_U = 1;
    run_fd("FD18 pure substance", f);
    f.nx = 1; f.ny = 1; f.nz = 1;
    run_fd("FD single node", f);
    f.nx = 5; f.ny = 5; f.nz = 5; f.stencil = 18; f.eps = 0.05;
    CHECK(fdo_create(&f) == NULL, "FD18 with anisotropy refused");

    if (failures) {
        fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    printf("oracle sanitizer run: all cases clean\n");
    return 0;
}
