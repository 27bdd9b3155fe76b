/*
 * lbpf_oracle.c -- plain FP64 CPU oracle for the lattice-Boltzmann (LB)
 * phase-field scheme of Cartalade, Younsi & Plapp (arXiv:1602.07483).
 *
 * TEST INFRASTRUCTURE ONLY: used by the test-suite, the smoke check and the CPU
 * baseline of the benchmark.  The GPU library never includes or links it.
 *
 * The time step follows the paper's algorithm in the paper's order
 * (Sec. 3.4, "Algorithm implementation"): for the phase field, node terms ->
 * collision (eq. Collision_Stage) -> streaming (eq. Deplacement_STD) with the
 * bounce-back rule -> phi as the zeroth moment; then, with the new phi, the
 * supersaturation (Sec. 3.3) and heat (Sec. 3.1) schemes: collision ->
 * streaming -> zeroth moments.  Collision and streaming are separate passes
 * over separate arrays, exactly as written in the paper; nothing is fused,
 * blocked or reordered.
 *
 * Readings where the paper is silent or ambiguous (each one is also listed in
 * the design notes of the repository):
 *  R1  U and theta use the new phase field: dphi/dt = (phi^{n+1}-phi^n)/dt
 *      (explicit Euler), q, zeta, grad phi and j_at from phi^{n+1}; U^n and
 *      theta^n elsewhere.  Q_phi uses U^n and theta^n.
 *  R2  The non-local population g_i(x+e_i,t) of eq. (Collision_Stage) is the
 *      post-streaming population i of the neighbour at the same time level.
 *  R3  "Boundary node" = node having at least one link that crosses a no-flux
 *      wall; there a_s^2 is replaced by 1 in the prefactor and in the
 *      non-local term, while eta_phi and N keep a_s(n).  Across a symmetry
 *      wall the non-local value is the mirror image population.
 *  R4  Bounce-back is the half-way (link-wise) rule, the wall lying half a
 *      link outside the last node.  A symmetry wall reflects specularly.  A
 *      link that crosses both kinds of wall bounces back.
 *  R5  Gradients: second-order central differences along the three axes,
 *      with mirror ghosts psi(-1)=psi(0), psi(n)=psi(n-1).
 *  R6  grad(q/zeta) and F = grad(1/zeta) are central differences of the nodal
 *      fields q/zeta and 1/zeta; div(q F) uses the compact face-averaged form
 *      sum_a [ (q_x+q_{x+a})/2 (w_{x+a}-w_x) - (q_x+q_{x-a})/2 (w_x-w_{x-a}) ] / dx^2.
 *  R7  When |grad phi|^2 dx^2 <= 1e-12 the normal is undefined: a_s = 1,
 *      N = 0, j_at = 0.
 *  R8  The derivative of a_s printed in Sec. 3.4 (eq. Derivees_As) has a typo
 *      in its index list for the second component; the indices used here are
 *      (alpha,beta,gamma) = (x,y,z), (y,x,z), (z,x,y).
 *  R20 Advection (end of Sec. 3.1): only theta is advected, by the uniform
 *      velocity of the parameters or by a per-node field that replaces it;
 *      the equilibrium at node x takes v(x).  Walls bounce back the whole
 *      population, the advective part included.
 *  R21 Isothermal runs (the alloy benchmark of Sec. 4.2 sets theta = 0):
 *      with skip_theta the heat equation is not solved and theta keeps its
 *      initial value everywhere.
 *  R23 Options for studies, off by default: skip_U holds U (pure
 *      substances, M c_inf = 0, where U acts on nothing); grad_stencil = 1
 *      takes the gradients of phi from the isotropic lattice form
 *      (e^2 dx)^-1 sum_i w_i e_i phi(x + e_i) instead of R5.
 *  R22 Separate lattices (lattice_ut): the U and theta schemes may run on
 *      another lattice than the phase field, as the 2D validation of Sec.
 *      4.1 uses D2Q9 for phi and D2Q5 for theta; each scheme takes the e^2,
 *      weights and A_i, B_i of its own lattice.
 */
#include "lbpf_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXQ 19
#define SMIN 1e-12

/* One lattice: vectors, weights, A_i, B_i, e^2, opposite and reflected links. */
typedef struct {
    int q;
    int e[MAXQ][3];
    double w[MAXQ], A[MAXQ], B[MAXQ], e2;
    int opp[MAXQ];
    int refl[8][MAXQ];   /* refl[mask][i]: e_i with the components in mask flipped */
} orc_lat;

struct orc_ctx {
    orc_params p;
    orc_lat lg;          /* lattice of g (phase field) */
    orc_lat lt;          /* lattice of h and f (U, theta): lg unless lattice_ut is set */
    size_t n;
    double *pop[3];      /* g, h, f: post-streaming populations */
    double *star[3];     /* post-collision populations */
    double *phi, *U, *th, *phi_old;
    /* phase-field node terms */
    double *as2, *eta, *Nvec, *Qphi;
    int *bnode;
    /* supersaturation / heat node terms */
    double *r, *wz, *qf, *J, *srcU, *Qth;
    double *vfield;      /* NULL, or per-node advective velocity [3][n] */
    int64_t steps;
};

/* ------------------------------------------------------------------------- */
/* Lattices: Tables 1 and 2 of Sec. 3.4 (vectors e_i, weights w_i, A_i, B_i,  */
/* and e^2), typed in from the tables.                                        */
/* ------------------------------------------------------------------------- */
static const int E7[7][3] = {
    {0,0,0},{1,0,0},{0,1,0},{-1,0,0},{0,-1,0},{0,0,1},{0,0,-1}};
static const int E15x[8][3] = {
    {1,1,1},{-1,1,1},{-1,-1,1},{1,-1,1},{1,1,-1},{-1,1,-1},{-1,-1,-1},{1,-1,-1}};
static const int E19x[12][3] = {
    {1,1,0},{-1,1,0},{1,-1,0},{-1,-1,0},{1,0,1},{-1,0,1},
    {1,0,-1},{-1,0,-1},{0,1,1},{0,-1,1},{0,1,-1},{0,-1,-1}};

int orc_lattice(int q, int32_t* e, double* w, double* A, double* B, double* e2)
{
    int i;
    if (q != 7 && q != 15 && q != 19) return -1;
    for (i = 0; i < 7; ++i) {
        e[3*i+0] = E7[i][0]; e[3*i+1] = E7[i][1]; e[3*i+2] = E7[i][2];
    }
    for (i = 7; i < q; ++i) {
        const int* v = (q == 15) ? E15x[i-7] : E19x[i-7];
        e[3*i+0] = v[0]; e[3*i+1] = v[1]; e[3*i+2] = v[2];
    }
    if (q == 7) {
        *e2 = 1.0/4.0;
        w[0] = 1.0/4.0; A[0] = 1.0; B[0] = -3.0/4.0;
        for (i = 1; i < 7; ++i) { w[i] = 1.0/8.0; A[i] = 0.0; B[i] = 1.0/8.0; }
    } else if (q == 15) {
        *e2 = 1.0/3.0;
        w[0] = 2.0/9.0; A[0] = 1.0; B[0] = -7.0/9.0;
        for (i = 1; i < 7; ++i)  { w[i] = 1.0/9.0;  A[i] = 0.0; B[i] = 1.0/9.0; }
        for (i = 7; i < 15; ++i) { w[i] = 1.0/72.0; A[i] = 0.0; B[i] = 1.0/72.0; }
    } else {
        *e2 = 1.0/3.0;
        w[0] = 1.0/3.0; A[0] = 1.0; B[0] = -2.0/3.0;
        for (i = 1; i < 7; ++i)  { w[i] = 1.0/18.0; A[i] = 0.0; B[i] = 1.0/18.0; }
        for (i = 7; i < 19; ++i) { w[i] = 1.0/36.0; A[i] = 0.0; B[i] = 1.0/36.0; }
    }
    return 0;
}

/* Index of the direction whose vector equals (x,y,z); -1 if none. */
static int find_dir(const orc_lat* L, int x, int y, int z)
{
    int i;
    for (i = 0; i < L->q; ++i)
        if (L->e[i][0] == x && L->e[i][1] == y && L->e[i][2] == z) return i;
    return -1;
}

/* The lattice table of q (7, 15 or 19) with its opposite and reflected links. */
static void lat_init(orc_lat* L, int q)
{
    int32_t e[3*MAXQ];
    int i, mask;
    L->q = q;
    orc_lattice(q, e, L->w, L->A, L->B, &L->e2);
    for (i = 0; i < q; ++i) {
        L->e[i][0] = e[3*i]; L->e[i][1] = e[3*i+1]; L->e[i][2] = e[3*i+2];
    }
    for (i = 0; i < q; ++i) {
        L->opp[i] = find_dir(L, -L->e[i][0], -L->e[i][1], -L->e[i][2]);
        for (mask = 0; mask < 8; ++mask)
            L->refl[mask][i] = find_dir(L,
                (mask & 1) ? -L->e[i][0] : L->e[i][0],
                (mask & 2) ? -L->e[i][1] : L->e[i][1],
                (mask & 4) ? -L->e[i][2] : L->e[i][2]);
    }
}

/* ------------------------------------------------------------------------- */
/* Anisotropy: a_s(n) and the vector N of Sec. 2, eq. (TermesAnisotropes).     */
/* ------------------------------------------------------------------------- */
void orc_anisotropy(int aniso, double eps, double delta, const double p[3],
                    double* a_out, double N[3])
{
    const double s = p[0]*p[0] + p[1]*p[1] + p[2]*p[2];
    double dadp[3];
    double a;
    int al;
    if (aniso == ORC_ANISO_CUBIC) {
        /* eq. (Anisotropic-Function_As): a_s = 1 - 3 eps + 4 eps sum n^4,
         * n = -grad phi/|grad phi| (even in n, so p = grad phi is used). */
        const double s2 = s * s;
        const double sum4 = (p[0]*p[0]*p[0]*p[0] + p[1]*p[1]*p[1]*p[1]
                             + p[2]*p[2]*p[2]*p[2]) / s2;
        a = 1.0 - 3.0*eps + 4.0*eps*sum4;
        /* eq. (Derivees_As), with the index triples of reading R8. */
        for (al = 0; al < 3; ++al) {
            const int be = (al == 0) ? 1 : 0;
            const int ga = (al == 2) ? 1 : 2;
            const double pa = p[al], pb = p[be], pg = p[ga];
            const double br = pb*pb*pb*pb - pa*pa*pb*pb - pa*pa*pg*pg + pg*pg*pg*pg;
            dadp[al] = -16.0*eps / (s2*s) * pa * br;
        }
    } else {
        /* eq. (As_K41-K61): a_s = 1 + eps (sum n^4 - 3/5)
         *                     + delta (3 sum n^4 + 66 nx^2 ny^2 nz^2 - 17/7).
         * The paper prints no derivative: it is taken by the chain rule,
         * d a/d p_al = sum_be (d a/d m_be) (delta_{al be} - m_al m_be)/|p|,
         * with m = p/|p| and d a/d m the plain polynomial derivative. */
        const double ps = sqrt(s);
        const double m[3] = {p[0]/ps, p[1]/ps, p[2]/ps};
        const double sum4 = m[0]*m[0]*m[0]*m[0] + m[1]*m[1]*m[1]*m[1] + m[2]*m[2]*m[2]*m[2];
        const double prod = m[0]*m[0]*m[1]*m[1]*m[2]*m[2];
        double dadm[3], proj = 0.0;
        a = 1.0 + eps*(sum4 - 3.0/5.0) + delta*(3.0*sum4 + 66.0*prod - 17.0/7.0);
        for (al = 0; al < 3; ++al) {
            const int be = (al + 1) % 3, ga = (al + 2) % 3;
            dadm[al] = 4.0*eps*m[al]*m[al]*m[al]
                     + delta*(12.0*m[al]*m[al]*m[al] + 132.0*m[al]*m[be]*m[be]*m[ga]*m[ga]);
        }
        for (al = 0; al < 3; ++al) proj += m[al]*dadm[al];
        for (al = 0; al < 3; ++al) dadp[al] = (dadm[al] - m[al]*proj) / ps;
    }
    *a_out = a;
    /* eq. (TermesAnisotropes): N = |grad phi|^2 a_s d a_s / d(grad phi). */
    for (al = 0; al < 3; ++al) N[al] = s * a * dadp[al];
}

/* Equilibrium of the phase field, Sec. 3.2 eq. (Feq_Phase):
 * g_i^(0) = w_i (phi - e_i.N cphi / e^2), cphi = dt W0^2 / (dx tau0). */
void orc_geq(int q, double phi, const double N[3], double cphi, double* out)
{
    int32_t e[3*MAXQ]; double w[MAXQ], A[MAXQ], B[MAXQ], e2;
    int i;
    if (orc_lattice(q, e, w, A, B, &e2)) return;
    for (i = 0; i < q; ++i) {
        const double eN = e[3*i]*N[0] + e[3*i+1]*N[1] + e[3*i+2]*N[2];
        out[i] = w[i] * (phi - eN * cphi / e2);
    }
}

/* Equilibrium of the supersaturation, Sec. 3.3 eq. (Feq_Transport):
 * h_i^(0) = A_i U + B_i (r U + e_i.J (dt/dx) / e^2), r = q(phi)/zeta(phi). */
void orc_heq(int q, double U, double r, const double J[3], double dt_over_dx, double* out)
{
    int32_t e[3*MAXQ]; double w[MAXQ], A[MAXQ], B[MAXQ], e2;
    int i;
    if (orc_lattice(q, e, w, A, B, &e2)) return;
    for (i = 0; i < q; ++i) {
        const double eJ = e[3*i]*J[0] + e[3*i+1]*J[1] + e[3*i+2]*J[2];
        out[i] = A[i]*U + B[i]*(r*U + eJ*dt_over_dx/e2);
    }
}

/* ------------------------------------------------------------------------- */
/* Grid helpers                                                               */
/* ------------------------------------------------------------------------- */
static size_t nidx(const orc_ctx* c, int x, int y, int z)
{
    return ((size_t)z * (size_t)c->p.ny + (size_t)y) * (size_t)c->p.nx + (size_t)x;
}

static int clampi(int v, int n) { return v < 0 ? 0 : (v >= n ? n - 1 : v); }

/* Field value with mirror ghosts (reading R5). */
static double fget(const orc_ctx* c, const double* f, int x, int y, int z)
{
    return f[nidx(c, clampi(x, c->p.nx), clampi(y, c->p.ny), clampi(z, c->p.nz))];
}

/* Bit mask of the axes along which (x,y,z) lies outside the domain, and
 * whether any of the crossed walls is a no-flux wall. */
static int crossed(const orc_ctx* c, const int t[3], int* noflux)
{
    const int nn[3] = {c->p.nx, c->p.ny, c->p.nz};
    int al, mask = 0;
    *noflux = 0;
    for (al = 0; al < 3; ++al) {
        if (t[al] < 0) {
            mask |= 1 << al;
            if (c->p.wall[2*al] == ORC_WALL_NOFLUX) *noflux = 1;
        } else if (t[al] >= nn[al]) {
            mask |= 1 << al;
            if (c->p.wall[2*al+1] == ORC_WALL_NOFLUX) *noflux = 1;
        }
    }
    return mask;
}

/* Central-difference gradient with mirror ghosts (reading R5). */
static void grad(const orc_ctx* c, const double* f, int x, int y, int z, double g[3])
{
    const double h = 1.0 / (2.0 * c->p.dx);
    g[0] = (fget(c, f, x+1, y, z) - fget(c, f, x-1, y, z)) * h;
    g[1] = (fget(c, f, x, y+1, z) - fget(c, f, x, y-1, z)) * h;
    g[2] = (fget(c, f, x, y, z+1) - fget(c, f, x, y, z-1)) * h;
}

/* Gradient of phi: R5, or with grad_stencil = 1 the isotropic lattice form
 * (e^2 dx)^-1 sum_i w_i e_i phi(x + e_i) over the phase field's lattice,
 * with the same mirror ghosts. */
static void grad_phi(const orc_ctx* c, const double* f, int x, int y, int z, double g[3])
{
    if (c->p.grad_stencil != 1) {
        grad(c, f, x, y, z, g);
        return;
    }
    const orc_lat* L = &c->lg;
    g[0] = g[1] = g[2] = 0.0;
    for (int i = 1; i < L->q; ++i) {
        const double v = L->w[i] * fget(c, f, x + L->e[i][0], y + L->e[i][1], z + L->e[i][2]);
        for (int al = 0; al < 3; ++al) g[al] += v * L->e[i][al];
    }
    for (int al = 0; al < 3; ++al) g[al] /= L->e2 * c->p.dx;
}

/* ------------------------------------------------------------------------- */
/* Creation                                                                   */
/* ------------------------------------------------------------------------- */
void orc_destroy(orc_ctx* c)
{
    int k;
    if (!c) return;
    for (k = 0; k < 3; ++k) { free(c->pop[k]); free(c->star[k]); }
    free(c->phi); free(c->U); free(c->th); free(c->phi_old);
    free(c->as2); free(c->eta); free(c->Nvec); free(c->Qphi); free(c->bnode);
    free(c->r); free(c->wz); free(c->qf); free(c->J); free(c->srcU); free(c->Qth);
    free(c->vfield);
    free(c);
}

orc_ctx* orc_create(const orc_params* p)
{
    orc_ctx* c;
    int i, k;
    if (!p || p->nx < 1 || p->ny < 1 || p->nz < 1) return NULL;
    if (p->lattice != 7 && p->lattice != 15 && p->lattice != 19) return NULL;
    if (p->lattice_ut != 0 && p->lattice_ut != 7 && p->lattice_ut != 15 && p->lattice_ut != 19)
        return NULL;
    if (!(p->dx > 0) || !(p->dt > 0) || !(p->tau0 > 0) || !(p->W0 > 0)) return NULL;
    if (!(p->k > 0 && p->k < 1)) return NULL;
    if (p->grad_stencil != 0 && p->grad_stencil != 1) return NULL;
    c = (orc_ctx*)calloc(1, sizeof(orc_ctx));
    if (!c) return NULL;
    c->p = *p;
    lat_init(&c->lg, p->lattice);
    lat_init(&c->lt, p->lattice_ut ? p->lattice_ut : p->lattice);
    c->n = (size_t)p->nx * (size_t)p->ny * (size_t)p->nz;
    for (k = 0; k < 3; ++k) {
        const int qk = k == 0 ? c->lg.q : c->lt.q;
        c->pop[k]  = (double*)calloc((size_t)qk * c->n, sizeof(double));
        c->star[k] = (double*)calloc((size_t)qk * c->n, sizeof(double));
        if (!c->pop[k] || !c->star[k]) { orc_destroy(c); return NULL; }
    }
#define ALLOC(ptr, cnt, type) do { ptr = (type*)calloc((cnt), sizeof(type)); \
        if (!ptr) { orc_destroy(c); return NULL; } } while (0)
    ALLOC(c->phi, c->n, double); ALLOC(c->U, c->n, double); ALLOC(c->th, c->n, double);
    ALLOC(c->phi_old, c->n, double);
    ALLOC(c->as2, c->n, double); ALLOC(c->eta, c->n, double); ALLOC(c->Nvec, 3*c->n, double);
    ALLOC(c->Qphi, c->n, double); ALLOC(c->bnode, c->n, int);
    ALLOC(c->r, c->n, double); ALLOC(c->wz, c->n, double); ALLOC(c->qf, c->n, double);
    ALLOC(c->J, 3*c->n, double); ALLOC(c->srcU, c->n, double); ALLOC(c->Qth, c->n, double);
#undef ALLOC
    /* Boundary nodes (reading R3): any link crossing a no-flux wall. */
    {
        int x, y, z;
        for (z = 0; z < p->nz; ++z)
        for (y = 0; y < p->ny; ++y)
        for (x = 0; x < p->nx; ++x) {
            int b = 0;
            for (i = 1; i < c->lg.q; ++i) {
                int t[3] = {x + c->lg.e[i][0], y + c->lg.e[i][1], z + c->lg.e[i][2]};
                int nf;
                if (crossed(c, t, &nf) && nf) b = 1;
            }
            c->bnode[nidx(c, x, y, z)] = b;
        }
    }
    return c;
}

int64_t orc_step_count(const orc_ctx* c) { return c->steps; }

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------- */
/* Streaming, Sec. 3.4 eq. (Deplacement_STD), with the walls of reading R4.   */
/* Push form: population i leaving x goes to x+e_i.                           */
/* ------------------------------------------------------------------------- */
static void stream(const orc_ctx* c, const orc_lat* L, const double* src, double* dst)
{
    const int nx = c->p.nx, ny = c->p.ny, nz = c->p.nz;
    const size_t n = c->n;
    int z;
#pragma omp parallel for collapse(2) schedule(static)
    for (z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
        const size_t s = nidx(c, x, y, z);
        for (int i = 0; i < L->q; ++i) {
            int t[3] = {x + L->e[i][0], y + L->e[i][1], z + L->e[i][2]};
            int nf;
            const int mask = crossed(c, t, &nf);
            if (!mask) {
                dst[(size_t)i*n + nidx(c, t[0], t[1], t[2])] = src[(size_t)i*n + s];
            } else if (nf) {
                /* half-way bounce-back: back into x along the opposite link */
                dst[(size_t)L->opp[i]*n + s] = src[(size_t)i*n + s];
            } else {
                /* specular reflection on symmetry walls */
                const int j = L->refl[mask][i];
                dst[(size_t)j*n + nidx(c, clampi(t[0], nx), clampi(t[1], ny), clampi(t[2], nz))]
                    = src[(size_t)i*n + s];
            }
        }
    }
}

static void moment0(const orc_ctx* c, const orc_lat* L, const double* pop, double* fld)
{
    const size_t n = c->n;
    long long s;
#pragma omp parallel for schedule(static)
    for (s = 0; s < (long long)n; ++s) {
        double acc = 0.0;
        for (int i = 0; i < L->q; ++i) acc += pop[(size_t)i*n + (size_t)s];
        fld[s] = acc;
    }
}

/* ------------------------------------------------------------------------- */
/* Phase-field node terms: a_s^2, N (eq. TermesAnisotropes), eta_phi          */
/* (eq. LBE_RelaxationTime) and Q_phi (eq. LBE_SourceTerm).                   */
/* ------------------------------------------------------------------------- */
static void phi_terms(orc_ctx* c, const double* phi, const double* U, const double* th)
{
    const orc_params* p = &c->p;
    int z;
#pragma omp parallel for collapse(2) schedule(static)
    for (z = 0; z < p->nz; ++z)
    for (int y = 0; y < p->ny; ++y)
    for (int x = 0; x < p->nx; ++x) {
        const size_t s = nidx(c, x, y, z);
        double g[3], a = 1.0, N[3] = {0.0, 0.0, 0.0};
        grad_phi(c, phi, x, y, z, g);
        if ((g[0]*g[0] + g[1]*g[1] + g[2]*g[2]) * p->dx * p->dx > SMIN)
            orc_anisotropy(p->aniso, p->eps, p->delta, g, &a, N);
        c->as2[s] = a * a;
        c->Nvec[3*s+0] = N[0]; c->Nvec[3*s+1] = N[1]; c->Nvec[3*s+2] = N[2];
        c->eta[s] = a*a * p->W0*p->W0 * p->dt / (c->lg.e2 * p->tau0 * p->dx*p->dx) + 0.5;
        {
            const double f = phi[s];
            const double om = 1.0 - f*f;
            c->Qphi[s] = (f - p->lambda * (p->Mcinf * U[s] + th[s]) * om) * om;
        }
    }
}

/* Phase-field collision, Sec. 3.4 eq. (Collision_Stage), for every node and
 * direction; the result goes to star[0]. */
static void phi_collide(orc_ctx* c)
{
    const orc_params* p = &c->p;
    const size_t n = c->n;
    const double* g = c->pop[0];
    double* gs = c->star[0];
    const double cphi = p->dt * p->W0 * p->W0 / (p->dx * p->tau0);
    int z;
#pragma omp parallel for collapse(2) schedule(static)
    for (z = 0; z < p->nz; ++z)
    for (int y = 0; y < p->ny; ++y)
    for (int x = 0; x < p->nx; ++x) {
        const size_t s = nidx(c, x, y, z);
        const double a2 = c->bnode[s] ? 1.0 : c->as2[s];
        const double* N = &c->Nvec[3*s];
        const orc_lat* L = &c->lg;
        for (int i = 0; i < L->q; ++i) {
            int t[3] = {x + L->e[i][0], y + L->e[i][1], z + L->e[i][2]};
            int nf;
            const int mask = crossed(c, t, &nf);
            double nl;
            if (!mask)
                nl = g[(size_t)i*n + nidx(c, t[0], t[1], t[2])];
            else if (nf)
                nl = 0.0;   /* boundary node: coefficient (1 - a2) is zero */
            else
                nl = g[(size_t)L->refl[mask][i]*n
                       + nidx(c, clampi(t[0], p->nx), clampi(t[1], p->ny), clampi(t[2], p->nz))];
            {
                const double eN = L->e[i][0]*N[0] + L->e[i][1]*N[1] + L->e[i][2]*N[2];
                const double geq = L->w[i] * (c->phi[s] - eN * cphi / L->e2);
                const double gi = g[(size_t)i*n + s];
                gs[(size_t)i*n + s] = (gi - (1.0 - a2) * nl - (gi - geq) / c->eta[s]
                                       + L->w[i] * c->Qphi[s] * p->dt / p->tau0) / a2;
            }
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Supersaturation and heat node terms, Sec. 3.3 eqs. (Def_Jtot), (Def_S),    */
/* (Def_Qu), Sec. 2 eq. (AntiTrapping_Current), Sec. 3.1 eq. (Source_Tempr).   */
/* phin = phi^{n+1} (reading R1).                                             */
/* ------------------------------------------------------------------------- */
static void ut_terms(orc_ctx* c, const double* phin, const double* phio,
                     const double* U, const double* th)
{
    const orc_params* p = &c->p;
    const double k = p->k;
    const size_t n = c->n;
    long long s0;
    int z;
    (void)th;
    /* nodal zeta, q, r = q/zeta and w = 1/zeta */
#pragma omp parallel for schedule(static)
    for (s0 = 0; s0 < (long long)n; ++s0) {
        const double f = phin[s0];
        const double zeta = 0.5*(1.0 + k) - 0.5*(1.0 - k)*f;
        const double q = 0.5*(1.0 - f);
        c->qf[s0] = q;
        c->r[s0] = q / zeta;
        c->wz[s0] = 1.0 / zeta;
    }
#pragma omp parallel for collapse(2) schedule(static)
    for (z = 0; z < p->nz; ++z)
    for (int y = 0; y < p->ny; ++y)
    for (int x = 0; x < p->nx; ++x) {
        const size_t s = nidx(c, x, y, z);
        const double f = phin[s];
        const double zeta = 0.5*(1.0 + k) - 0.5*(1.0 - k)*f;
        const double q = c->qf[s];
        const double u = U[s];
        const double dtphi = (phin[s] - phio[s]) / p->dt;
        double G[3], F[3], pg[3], jat[3] = {0.0, 0.0, 0.0};
        double divq = 0.0;
        grad(c, c->r, x, y, z, G);
        grad(c, c->wz, x, y, z, F);
        grad_phi(c, phin, x, y, z, pg);
        {
            const double s2 = pg[0]*pg[0] + pg[1]*pg[1] + pg[2]*pg[2];
            if (s2 * p->dx * p->dx > SMIN) {
                const double mag = sqrt(s2);
                const double pre = -p->W0 / (2.0 * sqrt(2.0)) * (1.0 + (1.0 - k)*u) * dtphi;
                for (int al = 0; al < 3; ++al) jat[al] = pre * pg[al] / mag;
            }
        }
        /* compact div(q grad w), reading R6 */
        {
            const int d[3][3] = {{1,0,0},{0,1,0},{0,0,1}};
            const double wc = c->wz[s];
            for (int al = 0; al < 3; ++al) {
                const double qp = fget(c, c->qf, x+d[al][0], y+d[al][1], z+d[al][2]);
                const double qm = fget(c, c->qf, x-d[al][0], y-d[al][1], z-d[al][2]);
                const double wp = fget(c, c->wz, x+d[al][0], y+d[al][1], z+d[al][2]);
                const double wm = fget(c, c->wz, x-d[al][0], y-d[al][1], z-d[al][2]);
                divq += 0.5*(q + qp)*(wp - wc) - 0.5*(q + qm)*(wc - wm);
            }
            divq /= p->dx * p->dx;
        }
        {
            double S = u * p->D * divq;
            for (int al = 0; al < 3; ++al) {
                c->J[3*s+al] = p->D * (G[al] + q * F[al]) * u + jat[al] / zeta;
                S += jat[al] * F[al];
            }
            /* source of eq. (LBE_Eq_Transport): S + Q_U / zeta */
            c->srcU[s] = S + (1.0 + (1.0 - k)*u) * 0.5 * dtphi / zeta;
        }
        c->Qth[s] = 0.5 * dtphi;
    }
}

/* Heat equilibrium at node s, eq. (EqFunction_Tempr); with an advective
 * velocity v the advection-diffusion form of Sec. 3.1:
 * w_i theta [1 + e^-2 (e_i . v) dt/dx].  v is the node's entry of the
 * velocity field when one is set, else the uniform p->vel. */
static double theta_eq(const orc_ctx* c, int i, size_t s, double t)
{
    const orc_params* p = &c->p;
    double v[3] = {p->vel[0], p->vel[1], p->vel[2]};
    if (c->vfield)
        for (int a = 0; a < 3; ++a) v[a] = c->vfield[(size_t)a * c->n + s];
    const orc_lat* L = &c->lt;
    const double ev = L->e[i][0]*v[0] + L->e[i][1]*v[1] + L->e[i][2]*v[2];
    return L->w[i] * t * (1.0 + ev * p->dt / (L->e2 * p->dx));
}

int orc_set_velocity_field(orc_ctx* c, const double* vx, const double* vy, const double* vz)
{
    const size_t n = c->n;
    if (!vx && !vy && !vz) {
        free(c->vfield);
        c->vfield = NULL;
        return 0;
    }
    if (!vx || !vy || !vz) return -1;
    if (!c->vfield) c->vfield = (double*)malloc(3 * n * sizeof(double));
    if (!c->vfield) return -1;
    memcpy(c->vfield, vx, n * sizeof(double));
    memcpy(c->vfield + n, vy, n * sizeof(double));
    memcpy(c->vfield + 2 * n, vz, n * sizeof(double));
    return 0;
}

/* Supersaturation and heat collisions, eqs. (LBE_Eq_Transport), (LBE_Eq_Temp). */
static void ut_collide(orc_ctx* c)
{
    const orc_params* p = &c->p;
    const size_t n = c->n;
    const orc_lat* L = &c->lt;
    const double etaU = p->D * p->dt / (L->e2 * p->dx * p->dx) + 0.5;
    const double etaT = p->kappa * p->dt / (L->e2 * p->dx * p->dx) + 0.5;
    long long s;
#pragma omp parallel for schedule(static)
    for (s = 0; s < (long long)n; ++s) {
        const double u = c->U[s], t = c->th[s];
        const double* J = &c->J[3*s];
        for (int i = 0; i < L->q; ++i) {
            const size_t o = (size_t)i*n + (size_t)s;
            const double eJ = L->e[i][0]*J[0] + L->e[i][1]*J[1] + L->e[i][2]*J[2];
            const double heq = L->A[i]*u + L->B[i]*(c->r[s]*u + eJ * p->dt / (L->e2 * p->dx));
            const double feq = theta_eq(c, i, (size_t)s, t);
            const double hi = c->pop[1][o], fi = c->pop[2][o];
            if (!p->skip_U) c->star[1][o] = hi - (hi - heq) / etaU + L->w[i] * c->srcU[s] * p->dt;
            c->star[2][o] = fi - (fi - feq) / etaT + L->w[i] * c->Qth[s] * p->dt;
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Initial state: equilibria of the initial fields.                          */
/* ------------------------------------------------------------------------- */
int orc_init(orc_ctx* c, const double* phi, const double* U, const double* theta)
{
    const orc_params* p = &c->p;
    const size_t n = c->n;
    const double cphi = p->dt * p->W0 * p->W0 / (p->dx * p->tau0);
    memcpy(c->phi, phi, n * sizeof(double));
    memcpy(c->U, U, n * sizeof(double));
    memcpy(c->th, theta, n * sizeof(double));
    phi_terms(c, c->phi, c->U, c->th);
    /* h: J without the anti-trapping part (no time derivative is known) */
    ut_terms(c, c->phi, c->phi, c->U, c->th);
    for (size_t s = 0; s < n; ++s) {
        double geq[MAXQ], heq[MAXQ];
        orc_geq(c->lg.q, c->phi[s], &c->Nvec[3*s], cphi, geq);
        orc_heq(c->lt.q, c->U[s], c->r[s], &c->J[3*s], p->dt / p->dx, heq);
        for (int i = 0; i < c->lg.q; ++i)
            c->pop[0][(size_t)i*n + s] = geq[i];
        for (int i = 0; i < c->lt.q; ++i) {
            c->pop[1][(size_t)i*n + s] = heq[i];
            c->pop[2][(size_t)i*n + s] = theta_eq(c, i, s, c->th[s]);
        }
    }
    c->steps = 0;
    return 0;
}

int orc_step(orc_ctx* c, int64_t nsteps)
{
    for (int64_t it = 0; it < nsteps; ++it) {
        /* 1. phase field at time n */
        phi_terms(c, c->phi, c->U, c->th);
        phi_collide(c);
        stream(c, &c->lg, c->star[0], c->pop[0]);
        memcpy(c->phi_old, c->phi, c->n * sizeof(double));
        moment0(c, &c->lg, c->pop[0], c->phi);
        /* 2. supersaturation and temperature with the new phase field */
        ut_terms(c, c->phi, c->phi_old, c->U, c->th);
        ut_collide(c);
        if (!c->p.skip_U) {       /* pure substances hold U */
            stream(c, &c->lt, c->star[1], c->pop[1]);
            moment0(c, &c->lt, c->pop[1], c->U);
        }
        if (!c->p.skip_theta) {   /* isothermal runs hold theta */
            stream(c, &c->lt, c->star[2], c->pop[2]);
            moment0(c, &c->lt, c->pop[2], c->th);
        }
        c->steps++;
    }
    return 0;
}

int orc_stream_only(orc_ctx* c, int64_t nsteps)
{
    for (int64_t it = 0; it < nsteps; ++it) {
        for (int k = 0; k < 3; ++k) {
            double* tmp;
            stream(c, k == 0 ? &c->lg : &c->lt, c->pop[k], c->star[k]);
            tmp = c->pop[k]; c->pop[k] = c->star[k]; c->star[k] = tmp;
        }
    }
    return 0;
}

void orc_fields(const orc_ctx* c, double* phi, double* U, double* theta)
{
    if (phi) memcpy(phi, c->phi, c->n * sizeof(double));
    if (U) memcpy(U, c->U, c->n * sizeof(double));
    if (theta) memcpy(theta, c->th, c->n * sizeof(double));
}

void orc_get_pops(const orc_ctx* c, int field, double* out)
{
    memcpy(out, c->pop[field], (size_t)(field == 0 ? c->lg.q : c->lt.q) * c->n * sizeof(double));
}

void orc_set_pops(orc_ctx* c, int field, const double* in)
{
    double* fld = field == 0 ? c->phi : (field == 1 ? c->U : c->th);
    const orc_lat* L = field == 0 ? &c->lg : &c->lt;
    memcpy(c->pop[field], in, (size_t)L->q * c->n * sizeof(double));
    moment0(c, L, c->pop[field], fld);
}

/* ------------------------------------------------------------------------- */
/* Diagnostics.  The paper defines only the tip velocity (Sec. 4.1); the      */
/* solute content follows from the definition of U in Sec. 2 (c/c_inf =       */
/* zeta(phi)(1+(1-k)U)), the enthalpy from the heat equation's source.        */
/* Plain serial sums in x-fastest order.                                      */
/* ------------------------------------------------------------------------- */
void orc_reduce(const orc_ctx* c, const double centre[3], double* out)
{
    const orc_params* p = &c->p;
    const double k = p->k, dv = p->dx * p->dx * p->dx;
    const int nn[3] = {p->nx, p->ny, p->nz};
    double solid = 0, mass = 0, enth = 0, sumu = 0, sumphi = 0;
    double tip[3] = {-INFINITY, -INFINITY, -INFINITY};
    double pmin = INFINITY, pmax = -INFINITY, bad = 0;
    for (int z = 0; z < p->nz; ++z)
    for (int y = 0; y < p->ny; ++y)
    for (int x = 0; x < p->nx; ++x) {
        const size_t s = nidx(c, x, y, z);
        const double f = c->phi[s], u = c->U[s], t = c->th[s];
        const int pos[3] = {x, y, z};
        if (!isfinite(f) || !isfinite(u) || !isfinite(t)) { bad += 1; continue; }
        solid += 0.5 * (1.0 + f);
        mass += (0.5*(1.0 + k) - 0.5*(1.0 - k)*f) * (1.0 + (1.0 - k)*u) * dv;
        enth += (t - 0.5 * f) * dv;
        sumu += u * dv;
        sumphi += f * dv;
        if (f < pmin) pmin = f;
        if (f > pmax) pmax = f;
        for (int al = 0; al < 3; ++al) {
            int q[3] = {x, y, z};
            double fn;
            q[al] += 1;
            if (q[al] >= nn[al]) continue;
            fn = c->phi[nidx(c, q[0], q[1], q[2])];
            if (f > 0.0 && fn <= 0.0) {
                const double xc = pos[al] + f / (f - fn);
                if (xc > tip[al]) tip[al] = xc;
            }
        }
    }
    out[ORC_R_SOLID] = solid / (double)c->n;
    out[ORC_R_MASS] = mass;
    out[ORC_R_ENTHALPY] = enth;
    for (int al = 0; al < 3; ++al)
        out[ORC_R_TIPX + al] = isfinite(tip[al]) ? tip[al] - centre[al] : NAN;
    out[ORC_R_PHIMIN] = pmin;
    out[ORC_R_PHIMAX] = pmax;
    out[ORC_R_NONFINITE] = bad;
    out[ORC_R_SUMU] = sumu;
    out[ORC_R_SUMPHI] = sumphi;
}
