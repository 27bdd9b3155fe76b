/*
 * fd_oracle.c -- an independent finite-difference discretisation of the
 * phase-field model of Cartalade, Younsi & Plapp (arXiv:1602.07483), Sec. 2:
 * eq. (PhaseField_KarmaRappel) for phi, eq. (Concentration_Echebarria) for U
 * with the anti-trapping current of eq. (AntiTrapping_Current), and
 * eq. (Temp_Ramirez) for theta.  The paper checks its lattice-Boltzmann
 * schemes against finite-difference codes (Sec. 4); this file plays that
 * role for the LB oracle.
 *
 * TEST INFRASTRUCTURE ONLY, like the LB oracle next to it, with which it
 * shares nothing but the field layout ([nz][ny][nx], x fastest, FP64).
 *
 * Discretisation (explicit Euler, conservative flux form on a cell-centred
 * grid, walls half a cell outside the first and last node, zero flux through
 * every wall):
 *  - phi: tau0 a_s(n)^2 dphi/dt = W0^2 div F + phi - phi^3
 *         - lambda (Mc U + theta)(1 - phi^2)^2,
 *    with the face flux F = a_s^2 p + |p|^2 a_s da_s/dp, p the gradient on
 *    the face (normal component from the two adjacent nodes, transverse
 *    components averaged from the central differences at both nodes), and
 *    a_s at the node from central differences for tau.  da_s/dp is obtained
 *    from the gradient g of a_s with respect to the unit vector m = p/|p|,
 *    projected: da_s/dp = (g - m (g.m)) / |p|.
 *  - U:   zeta(phi) dU/dt = div(D q grad U - j_at) + (1 + (1-k)U) dphi/dt / 2
 *    with q and j_at on faces (q averaged, [1+(1-k)U] dphi/dt averaged, the
 *    unit normal from the face gradient of the new phi); zeta, q and dphi/dt
 *    use the phase field after the phi update of the same step.
 *  - theta: dtheta/dt = kappa lap theta + dphi/dt / 2, lap over the 6 face
 *    neighbours.
 * Two stencils for the Laplacian of the phase-field equation, as the paper's
 * FD6 and FD18 codes in its grid-anisotropy study (Sec. 4.1, isotropic case,
 * which names the stencil of that equation only):
 *  - stencil 6 (default): the flux form above; with a_s = 1 its div F uses
 *    the 6 face neighbours;
 *  - stencil 18: for an isotropic interface only (eps = 0, and delta = 0
 *    for K41/K61, so that a_s = 1 and the anisotropic flux vanishes), the
 *    phi Laplacian uses the 6 face and 12 edge neighbours,
 *    lap f = [2 sum_faces f + sum_edges f - 24 f] / (6 dx^2), whose O(dx^2)
 *    error does not depend on direction.  theta and U keep their face forms.
 * skip_U (pure substances, M c_inf = 0, where U does not act on phi or
 * theta): U is held at its initial value and its equation is not solved.
 * Where |grad phi|^2 dx^2 <= 1e-12 the normal is undefined: a_s = 1 and the
 * anisotropic and anti-trapping terms vanish.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t nx, ny, nz;
    double dx, W0, tau0, lambda, Mcinf, k, D, kappa;
    int32_t aniso;          /* 0: cubic, 1: K41/K61 */
    double eps, delta;
    int32_t skip_theta;     /* 1: isothermal (Sec. 4.2 benchmark): theta held */
    int32_t stencil;        /* phi Laplacian: 0 or 6 face neighbours; 18: faces and edges */
    int32_t skip_U;         /* 1: pure substance (M c_inf = 0): U held */
} fdo_params;

typedef struct {
    fdo_params p;
    size_t n;
    double *phi, *U, *th, *phin, *Un, *thn, *fx, *fy, *fz;
} fdo_ctx;

#define FD_SMIN 1e-12

/* a_s(m) and g = d a_s / d m (m a unit vector, components treated as free) */
static void as_and_grad(const fdo_params* p, const double m[3], double* a, double g[3]) {
    const double x2 = m[0] * m[0], y2 = m[1] * m[1], z2 = m[2] * m[2];
    const double s4 = x2 * x2 + y2 * y2 + z2 * z2;
    double ds4[3] = {4.0 * m[0] * x2, 4.0 * m[1] * y2, 4.0 * m[2] * z2};
    if (p->aniso == 0) {
        /* eq. (Anisotropic-Function_As) */
        *a = 1.0 - 3.0 * p->eps + 4.0 * p->eps * s4;
        for (int i = 0; i < 3; ++i) g[i] = 4.0 * p->eps * ds4[i];
    } else {
        /* eq. (As_K41-K61): K41 = S4 - 3/5, K61 = 3 S4 + 66 x2 y2 z2 - 17/7 */
        const double p6 = x2 * y2 * z2;
        *a = 1.0 + p->eps * (s4 - 0.6) + p->delta * (3.0 * s4 + 66.0 * p6 - 17.0 / 7.0);
        const double dp6[3] = {2.0 * m[0] * y2 * z2, 2.0 * m[1] * x2 * z2, 2.0 * m[2] * x2 * y2};
        for (int i = 0; i < 3; ++i)
            g[i] = p->eps * ds4[i] + p->delta * (3.0 * ds4[i] + 66.0 * dp6[i]);
    }
}

/* face flux vector F = a^2 p + |p|^2 a da/dp; returns component `axis` */
static double aniso_flux(const fdo_params* p, const double pg[3], int axis) {
    const double s = pg[0] * pg[0] + pg[1] * pg[1] + pg[2] * pg[2];
    if (s * p->dx * p->dx <= FD_SMIN) return pg[axis];
    const double mag = sqrt(s);
    const double m[3] = {pg[0] / mag, pg[1] / mag, pg[2] / mag};
    double a, g[3];
    as_and_grad(p, m, &a, g);
    const double gm = g[0] * m[0] + g[1] * m[1] + g[2] * m[2];
    const double dadp = (g[axis] - m[axis] * gm) / mag;
    return a * a * pg[axis] + s * a * dadp;
}

static double node_as(const fdo_params* p, const double pg[3]) {
    const double s = pg[0] * pg[0] + pg[1] * pg[1] + pg[2] * pg[2];
    if (s * p->dx * p->dx <= FD_SMIN) return 1.0;
    const double mag = sqrt(s);
    const double m[3] = {pg[0] / mag, pg[1] / mag, pg[2] / mag};
    double a, g[3];
    as_and_grad(p, m, &a, g);
    return a;
}

static inline int clampi(int v, int n) { return v < 0 ? 0 : (v >= n ? n - 1 : v); }

#define IDX(x, y, z) (((size_t)(z) * ny + (size_t)(y)) * nx + (size_t)(x))

/* central-difference gradient at node (x,y,z) with mirror ghosts */
static void grad_node(const double* f, int x, int y, int z, int nx, int ny, int nz, double dx,
                      double out[3]) {
    out[0] = (f[IDX(clampi(x + 1, nx), y, z)] - f[IDX(clampi(x - 1, nx), y, z)]) / (2.0 * dx);
    out[1] = (f[IDX(x, clampi(y + 1, ny), z)] - f[IDX(x, clampi(y - 1, ny), z)]) / (2.0 * dx);
    out[2] = (f[IDX(x, y, clampi(z + 1, nz))] - f[IDX(x, y, clampi(z - 1, nz))]) / (2.0 * dx);
}

/* gradient on the face between node (x,y,z) and its +axis neighbour */
static void grad_face(const double* f, int x, int y, int z, int axis, int nx, int ny, int nz, double dx,
                      double out[3]) {
    const int x1 = x + (axis == 0), y1 = y + (axis == 1), z1 = z + (axis == 2);
    double g0[3], g1[3];
    grad_node(f, x, y, z, nx, ny, nz, dx, g0);
    grad_node(f, x1, y1, z1, nx, ny, nz, dx, g1);
    for (int i = 0; i < 3; ++i) out[i] = 0.5 * (g0[i] + g1[i]);
    out[axis] = (f[IDX(x1, y1, z1)] - f[IDX(x, y, z)]) / dx;
}

/* Laplacian times dx^2 at node (x,y,z) with mirror ghosts: the 6 face
 * neighbours, or the isotropic form over the 6 face and 12 edge neighbours */
static double lap_dx2(const double* f, int x, int y, int z, int nx, int ny, int nz, int stencil) {
    const double f0 = f[IDX(x, y, z)];
    double faces = 0.0;
    for (int d = -1; d <= 1; d += 2)
        faces += f[IDX(clampi(x + d, nx), y, z)] + f[IDX(x, clampi(y + d, ny), z)] +
                 f[IDX(x, y, clampi(z + d, nz))];
    if (stencil != 18) return faces - 6.0 * f0;
    double edges = 0.0;
    for (int a = -1; a <= 1; a += 2)
        for (int b = -1; b <= 1; b += 2)
            edges += f[IDX(clampi(x + a, nx), clampi(y + b, ny), z)] +
                     f[IDX(clampi(x + a, nx), y, clampi(z + b, nz))] +
                     f[IDX(x, clampi(y + a, ny), clampi(z + b, nz))];
    return (2.0 * faces + edges - 24.0 * f0) / 6.0;
}

void fdo_destroy(fdo_ctx* c);

fdo_ctx* fdo_create(const fdo_params* p) {
    if (!p || p->nx < 1 || p->ny < 1 || p->nz < 1 || !(p->dx > 0)) return NULL;
    if (p->stencil != 0 && p->stencil != 6 && p->stencil != 18) return NULL;
    if (p->stencil == 18 && (p->eps != 0.0 || (p->aniso == 1 && p->delta != 0.0))) return NULL;
    fdo_ctx* c = (fdo_ctx*)calloc(1, sizeof(fdo_ctx));
    if (!c) return NULL;
    c->p = *p;
    c->n = (size_t)p->nx * p->ny * p->nz;
    double** arrs[] = {&c->phi, &c->U, &c->th, &c->phin, &c->Un, &c->thn, &c->fx, &c->fy, &c->fz};
    for (size_t i = 0; i < sizeof(arrs) / sizeof(arrs[0]); ++i) {
        *arrs[i] = (double*)calloc(c->n, sizeof(double));
        if (!*arrs[i]) {
            fdo_destroy(c);   /* frees the arrays already allocated (the rest are NULL) */
            return NULL;
        }
    }
    return c;
}

void fdo_destroy(fdo_ctx* c) {
    if (!c) return;
    free(c->phi); free(c->U); free(c->th); free(c->phin); free(c->Un); free(c->thn);
    free(c->fx); free(c->fy); free(c->fz);
    free(c);
}

void fdo_set(fdo_ctx* c, const double* phi, const double* U, const double* th) {
    memcpy(c->phi, phi, c->n * sizeof(double));
    memcpy(c->U, U, c->n * sizeof(double));
    memcpy(c->th, th, c->n * sizeof(double));
}

void fdo_get(const fdo_ctx* c, double* phi, double* U, double* th) {
    memcpy(phi, c->phi, c->n * sizeof(double));
    memcpy(U, c->U, c->n * sizeof(double));
    memcpy(th, c->th, c->n * sizeof(double));
}

/* nsteps explicit Euler steps of size dt */
void fdo_step(fdo_ctx* c, double dt, int64_t nsteps) {
    const fdo_params* p = &c->p;
    const int nx = p->nx, ny = p->ny, nz = p->nz;
    const double dx = p->dx, W2 = p->W0 * p->W0, k = p->k;
    const double jat_c = p->W0 / (2.0 * sqrt(2.0));
    double* fl[3] = {c->fx, c->fy, c->fz};
    for (int64_t s = 0; s < nsteps; ++s) {
        /* phi: face fluxes, then the node update */
        for (int axis = 0; axis < 3; ++axis) {
            const int lim[3] = {nx - 1, ny - 1, nz - 1};
#pragma omp parallel for collapse(2) schedule(static)
            for (int z = 0; z < nz; ++z)
                for (int y = 0; y < ny; ++y)
                    for (int x = 0; x < nx; ++x) {
                        const int pos[3] = {x, y, z};
                        double v = 0.0;   /* the wall face carries no flux */
                        if (pos[axis] < lim[axis]) {
                            double pg[3];
                            grad_face(c->phi, x, y, z, axis, nx, ny, nz, dx, pg);
                            v = aniso_flux(p, pg, axis);
                        }
                        fl[axis][IDX(x, y, z)] = v;
                    }
        }
#pragma omp parallel for collapse(2) schedule(static)
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    const size_t i = IDX(x, y, z);
                    double div = (c->fx[i] - (x > 0 ? c->fx[IDX(x - 1, y, z)] : 0.0)) +
                                 (c->fy[i] - (y > 0 ? c->fy[IDX(x, y - 1, z)] : 0.0)) +
                                 (c->fz[i] - (z > 0 ? c->fz[IDX(x, y, z - 1)] : 0.0));
                    div /= dx;
                    if (p->stencil == 18) div = lap_dx2(c->phi, x, y, z, nx, ny, nz, 18) / (dx * dx);
                    double pg[3];
                    grad_node(c->phi, x, y, z, nx, ny, nz, dx, pg);
                    const double a = node_as(p, pg);
                    const double ph = c->phi[i];
                    const double om = 1.0 - ph * ph;
                    const double rhs = W2 * div + ph - ph * ph * ph -
                                       p->lambda * (p->Mcinf * c->U[i] + c->th[i]) * om * om;
                    c->phin[i] = ph + dt * rhs / (p->tau0 * a * a);
                }
        /* U: face fluxes with the new phi */
        for (int axis = 0; axis < 3 && !p->skip_U; ++axis) {
            const int lim[3] = {nx - 1, ny - 1, nz - 1};
#pragma omp parallel for collapse(2) schedule(static)
            for (int z = 0; z < nz; ++z)
                for (int y = 0; y < ny; ++y)
                    for (int x = 0; x < nx; ++x) {
                        const int pos[3] = {x, y, z};
                        double v = 0.0;
                        if (pos[axis] < lim[axis]) {
                            const size_t i0 = IDX(x, y, z);
                            const size_t i1 = IDX(x + (axis == 0), y + (axis == 1), z + (axis == 2));
                            const double qf = 0.25 * ((1.0 - c->phin[i0]) + (1.0 - c->phin[i1]));
                            v = p->D * qf * (c->U[i1] - c->U[i0]) / dx;
                            double pg[3];
                            grad_face(c->phin, x, y, z, axis, nx, ny, nz, dx, pg);
                            const double s2 = pg[0] * pg[0] + pg[1] * pg[1] + pg[2] * pg[2];
                            if (s2 * dx * dx > FD_SMIN) {
                                const double A0 = (1.0 + (1.0 - k) * c->U[i0]) * (c->phin[i0] - c->phi[i0]) / dt;
                                const double A1 = (1.0 + (1.0 - k) * c->U[i1]) * (c->phin[i1] - c->phi[i1]) / dt;
                                const double jat = -jat_c * 0.5 * (A0 + A1) * pg[axis] / sqrt(s2);
                                v -= jat;
                            }
                        }
                        fl[axis][IDX(x, y, z)] = v;
                    }
        }
#pragma omp parallel for collapse(2) schedule(static)
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    const size_t i = IDX(x, y, z);
                    double div = (c->fx[i] - (x > 0 ? c->fx[IDX(x - 1, y, z)] : 0.0)) +
                                 (c->fy[i] - (y > 0 ? c->fy[IDX(x, y - 1, z)] : 0.0)) +
                                 (c->fz[i] - (z > 0 ? c->fz[IDX(x, y, z - 1)] : 0.0));
                    div /= dx;
                    const double dphi = c->phin[i] - c->phi[i];
                    const double zeta = 0.5 * (1.0 + k) - 0.5 * (1.0 - k) * c->phin[i];
                    c->Un[i] = p->skip_U ? c->U[i]
                                         : c->U[i] + (dt * div + 0.5 * (1.0 + (1.0 - k) * c->U[i]) * dphi) / zeta;
                    /* theta: face Laplacian with mirror ghosts */
                    const double t0 = c->th[i];
                    const double lap = lap_dx2(c->th, x, y, z, nx, ny, nz, 6);
                    c->thn[i] = p->skip_theta ? t0 : t0 + dt * p->kappa * lap / (dx * dx) + 0.5 * dphi;
                }
        double* t;
        t = c->phi; c->phi = c->phin; c->phin = t;
        t = c->U; c->U = c->Un; c->Un = t;
        t = c->th; c->th = c->thn; c->thn = t;
    }
}
