/*
 * pf_oracle.c -- plain, slow, FP64 CPU reference of the phase-field FEM step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant with
 * the HIP library: every quantity below is recomputed from its definition.
 *
 * What it computes (paper section / equation in brackets):
 *   - Allen-Cahn       d eta/dt = -L dF/d eta                         [Sec. 2.1, Eq. 1]
 *   - Cahn-Hilliard    split form dc/dt = div(M grad mu),
 *                      mu = f'(c) - kappa lap c                       [Sec. 2.2, Eqs. 9-10]
 *   - free energy      F = int f(c) + kappa/2 |grad c|^2              [Eqs. 5-6]
 *   - semi-discrete    M dU/dt + r(U, theta) = 0                      [Eq. 11]
 *   - explicit step    U <- U - dt M^-1 r(U)                          [Eq. 12]
 *   - implicit step    R = M (U - U_old)/dt + r(U) = 0, Newton        [Eqs. 13-14, Sec. 2.3]
 *   - sensitivities    chain rule / adjoint                           [Eq. 18, Supp. Note 2]
 *
 * Discretisation (the paper fixes "standard Lagrange" elements on a mesh; the
 * readings below are the ones this project adopts):
 *   - Q1 (bi/tri-linear) elements on a uniform grid of spacing h,
 *   - 2-point Gauss-Legendre quadrature per axis for every integral, or (quad = 1)
 *     the 2-point Gauss-Lobatto rule per axis, whose points are the element's
 *     nodes (nodal quadrature: every integral, the energy and the mass included),
 *   - row-sum lumped mass everywhere M appears, or (mass = 1, implicit path only)
 *     the consistent mass M_ab = sum_e sum_q detJ phi_a(q) phi_b(q) in the time
 *     term and the Cahn-Hilliard mu-row (every term Gauss-integrated),
 *   - periodic (n elements per axis) or no-flux (n-1 elements, natural BC).
 * Node index = i + n0*(j + n1*k) (x fastest).  Cahn-Hilliard states are laid
 * out as [c (N values) ; mu (N values)].
 *
 * Everything is an explicit element loop: gather the element's nodal values,
 * evaluate at each quadrature point, add each node's share.  No blocking, no
 * fusion, no precomputed stencils.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PERIODIC 0
#define ORC_NOFLUX 1
#define ORC_AC 0
#define ORC_CH 1
#define ORC_FSYM 0 /* f = W (c^2 - 1)^2 / 4 */
#define ORC_F01 1  /* f = W c^2 (1 - c)^2   */

typedef struct {
    int32_t dim;   /* 2 or 3 */
    int32_t bc;    /* ORC_PERIODIC / ORC_NOFLUX */
    int32_t model; /* ORC_AC / ORC_CH */
    int32_t fe;    /* ORC_FSYM / ORC_F01 */
    int64_t n[3];  /* nodes per axis; n[2] = 1 in 2-D */
    double h;      /* grid spacing */
    double W;      /* barrier height */
    double kappa;  /* gradient-energy coefficient */
    double mob;    /* mobility: L (Allen-Cahn) or M (Cahn-Hilliard) */
    int32_t mass;  /* 0: lumped mass; 1: consistent mass (implicit path only) */
    int32_t quad;  /* 0: 2-point Gauss-Legendre per axis; 1: 2-point Gauss-Lobatto */
} orc_problem;

/* ------------------------------------------------------------------------ */
/* reference element                                                         */
/* ------------------------------------------------------------------------ */
typedef struct {
    int d, nv;            /* dimension; vertices per element = quad points = 2^d */
    double detJ;          /* (h/2)^d; Gauss weights are 1 */
    double phi[8][8];     /* phi[q][a]: shape function a at quadrature point q */
    double grad[8][8][3]; /* grad[q][a][k]: d phi_a / d x_k at q (physical) */
} orc_ref;

/* Quadrature points xi_k = +-g per axis, weight 1 each: g = 1/sqrt(3) for
 * Gauss-Legendre, g = 1 for Gauss-Lobatto (the points are the nodes). */
static void ref_build(orc_ref* R, const orc_problem* pr)
{
    const int d = pr->dim;
    const double h = pr->h;
    const double g = pr->quad ? 1.0 : 1.0 / sqrt(3.0);
    R->d = d;
    R->nv = 1 << d;
    R->detJ = pow(0.5 * h, d);
    for (int q = 0; q < R->nv; ++q) {
        double xi[3];
        for (int k = 0; k < d; ++k) xi[k] = ((q >> k) & 1) ? g : -g;
        for (int a = 0; a < R->nv; ++a) {
            double s[3], f[3];
            for (int k = 0; k < d; ++k) {
                s[k] = ((a >> k) & 1) ? 1.0 : -1.0;
                f[k] = 0.5 * (1.0 + s[k] * xi[k]);
            }
            double p = 1.0;
            for (int k = 0; k < d; ++k) p *= f[k];
            R->phi[q][a] = p;
            for (int k = 0; k < d; ++k) {
                /* d/dx = (2/h) d/dxi; d/dxi_k of (1 + s xi)/2 = s/2 */
                double gk = 0.5 * s[k] * (2.0 / h);
                for (int l = 0; l < d; ++l)
                    if (l != k) gk *= f[l];
                R->grad[q][a][k] = gk;
            }
        }
    }
}

static int64_t orc_nnodes(const orc_problem* p)
{
    int64_t N = 1;
    for (int k = 0; k < p->dim; ++k) N *= p->n[k];
    return N;
}

static int64_t elems_on_axis(const orc_problem* p, int k)
{
    if (k >= p->dim) return 1;
    return p->bc == ORC_PERIODIC ? p->n[k] : p->n[k] - 1;
}

static void elem_nodes(const orc_problem* p, const int64_t e[3], int nv, int64_t* idx)
{
    for (int a = 0; a < nv; ++a) {
        int64_t ijk[3] = {0, 0, 0};
        for (int k = 0; k < p->dim; ++k) {
            ijk[k] = e[k] + ((a >> k) & 1);
            if (p->bc == ORC_PERIODIC) ijk[k] %= p->n[k];
        }
        idx[a] = ijk[0] + p->n[0] * (ijk[1] + p->n[1] * ijk[2]);
    }
}

/* iterate over all elements: E holds the current element's lower corner */
#define FOR_EACH_ELEMENT(p, E)                                   \
    for (E[2] = 0; E[2] < elems_on_axis(p, 2); ++E[2])           \
        for (E[1] = 0; E[1] < elems_on_axis(p, 1); ++E[1])       \
            for (E[0] = 0; E[0] < elems_on_axis(p, 0); ++E[0])

/* ------------------------------------------------------------------------ */
/* local free energy and its derivatives                                      */
/* ------------------------------------------------------------------------ */
static double fe_f(int fe, double W, double c)
{
    if (fe == ORC_FSYM) return 0.25 * W * (c * c - 1.0) * (c * c - 1.0);
    return W * c * c * (1.0 - c) * (1.0 - c);
}
static double fe_df(int fe, double W, double c)
{
    if (fe == ORC_FSYM) return W * (c * c * c - c);
    return 2.0 * W * c * (1.0 - c) * (1.0 - 2.0 * c);
}
static double fe_d2f(int fe, double W, double c)
{
    if (fe == ORC_FSYM) return W * (3.0 * c * c - 1.0);
    return 2.0 * W * (1.0 - 6.0 * c + 6.0 * c * c);
}

/* ------------------------------------------------------------------------ */
/* element-loop assemblies                                                    */
/* ------------------------------------------------------------------------ */

/* element E's share of assemble_first (below), added into out */
static void assemble_first_elem(const orc_problem* p, const orc_ref* R, double W, const double* u,
                                double cf, double ck, const int64_t E[3], double* out)
{
    int64_t idx[8];
    elem_nodes(p, E, R->nv, idx);
    for (int q = 0; q < R->nv; ++q) {
        double uq = 0.0, gq[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < R->nv; ++a) {
            uq += R->phi[q][a] * u[idx[a]];
            for (int k = 0; k < R->d; ++k) gq[k] += R->grad[q][a][k] * u[idx[a]];
        }
        double fq = (cf != 0.0) ? cf * fe_df(p->fe, W, uq) : 0.0;
        for (int a = 0; a < R->nv; ++a) {
            double gg = 0.0;
            for (int k = 0; k < R->d; ++k) gg += gq[k] * R->grad[q][a][k];
            out[idx[a]] += R->detJ * (fq * R->phi[q][a] + ck * gg);
        }
    }
}

#ifdef ORC_OMP
/* Timing build only (compiled with -fopenmp -DORC_OMP; the test-suite's oracle is the
 * serial build).  Elements whose lower-corner indices have the same parity on every
 * axis share no node when every periodic axis has an even node count (no-flux grids
 * have no wrap), so the 2^d colours run one after another, each colour's elements in
 * parallel.  Each node then sums its element shares in colour order, not element
 * order: results differ from the serial build in the last bits only. */
static int colourable(const orc_problem* p)
{
    if (p->bc != ORC_PERIODIC) return 1;
    for (int k = 0; k < p->dim; ++k)
        if (p->n[k] % 2) return 0;
    return 1;
}
#endif

/* out_a += sum_e sum_q detJ * ( cf * f'(u_q) phi_a(q) + ck * grad u_q . grad phi_a(q) )
 * The first variation of  int cf*f(u) + ck/2 |grad u|^2  (Eqs. 5-6). */
static void assemble_first(const orc_problem* p, double W, const double* u, double cf,
                           double ck, double* out)
{
    orc_ref R;
    ref_build(&R, p);
#ifdef ORC_OMP
    if (colourable(p)) {
        const int64_t ne[3] = {elems_on_axis(p, 0), elems_on_axis(p, 1), elems_on_axis(p, 2)};
        for (int col = 0; col < (1 << p->dim); ++col) {
            const int64_t o[3] = {col & 1, (col >> 1) & 1, (col >> 2) & 1};
            const int64_t m[3] = {(ne[0] - o[0] + 1) / 2, (ne[1] - o[1] + 1) / 2,
                                  p->dim == 3 ? (ne[2] - o[2] + 1) / 2 : 1};
#pragma omp parallel for schedule(static)
            for (int64_t t = 0; t < m[0] * m[1] * m[2]; ++t) {
                const int64_t E[3] = {o[0] + 2 * (t % m[0]), o[1] + 2 * ((t / m[0]) % m[1]),
                                      p->dim == 3 ? o[2] + 2 * (t / (m[0] * m[1])) : 0};
                assemble_first_elem(p, &R, W, u, cf, ck, E, out);
            }
        }
        return;
    }
#endif
    int64_t E[3];
    FOR_EACH_ELEMENT(p, E)
    assemble_first_elem(p, &R, W, u, cf, ck, E, out);
}

/* out_a += sum_e sum_q detJ * ( cf * f''(u_q) v_q phi_a(q) + ck * grad v_q . grad phi_a(q) )
 * The derivative of assemble_first with respect to u, applied to v.  The
 * underlying matrix is symmetric, so this is also its transpose product. */
static void assemble_second(const orc_problem* p, double W, const double* u, const double* v,
                            double cf, double ck, double* out)
{
    orc_ref R;
    ref_build(&R, p);
    int64_t E[3], idx[8];
    FOR_EACH_ELEMENT(p, E)
    {
        elem_nodes(p, E, R.nv, idx);
        for (int q = 0; q < R.nv; ++q) {
            double uq = 0.0, vq = 0.0, gq[3] = {0.0, 0.0, 0.0};
            for (int a = 0; a < R.nv; ++a) {
                uq += R.phi[q][a] * u[idx[a]];
                vq += R.phi[q][a] * v[idx[a]];
                for (int k = 0; k < R.d; ++k) gq[k] += R.grad[q][a][k] * v[idx[a]];
            }
            double fq = (cf != 0.0) ? cf * fe_d2f(p->fe, W, uq) * vq : 0.0;
            for (int a = 0; a < R.nv; ++a) {
                double gg = 0.0;
                for (int k = 0; k < R.d; ++k) gg += gq[k] * R.grad[q][a][k];
                out[idx[a]] += R.detJ * (fq * R.phi[q][a] + ck * gg);
            }
        }
    }
}

/* out_a += diagonal entry a of the matrix behind assemble_second */
static void assemble_second_diag(const orc_problem* p, const double* u, double cf, double ck,
                                 double* out)
{
    orc_ref R;
    ref_build(&R, p);
    int64_t E[3], idx[8];
    FOR_EACH_ELEMENT(p, E)
    {
        elem_nodes(p, E, R.nv, idx);
        for (int q = 0; q < R.nv; ++q) {
            double uq = 0.0;
            for (int a = 0; a < R.nv; ++a) uq += R.phi[q][a] * u[idx[a]];
            double fq = (cf != 0.0) ? cf * fe_d2f(p->fe, p->W, uq) : 0.0;
            for (int a = 0; a < R.nv; ++a) {
                double gg = 0.0;
                for (int k = 0; k < R.d; ++k) gg += R.grad[q][a][k] * R.grad[q][a][k];
                out[idx[a]] += R.detJ * (fq * R.phi[q][a] * R.phi[q][a] + ck * gg);
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* exported: mass, energy, residual                                           */
/* ------------------------------------------------------------------------ */

/* threads the timing build's parallel loops use (1 in the serial build) */
#ifdef ORC_OMP
#include <omp.h>
int orc_threads(void) { return omp_get_max_threads(); }
#else
int orc_threads(void) { return 1; }
#endif

int64_t orc_ndof(const orc_problem* p)
{
    return (p->model == ORC_CH ? 2 : 1) * orc_nnodes(p);
}

/* lumped (row-sum) mass: m_a = sum_e sum_q detJ phi_a(q)   [Eq. 11, M lumped] */
int orc_lumped_mass(const orc_problem* p, double* m)
{
    orc_ref R;
    ref_build(&R, p);
    int64_t N = orc_nnodes(p), E[3], idx[8];
    memset(m, 0, (size_t)N * sizeof(double));
    FOR_EACH_ELEMENT(p, E)
    {
        elem_nodes(p, E, R.nv, idx);
        for (int q = 0; q < R.nv; ++q)
            for (int a = 0; a < R.nv; ++a) m[idx[a]] += R.detJ * R.phi[q][a];
    }
    return 0;
}

/* out = M v on one field: the lumped mass m_a v_a (mass == 0), or the consistent
 * mass (mass == 1), sum_e sum_q detJ phi_a(q) phi_b(q) v_b, the Gauss-integrated
 * int phi_a v_h. */
static void apply_mass(const orc_problem* p, const double* v, double* out)
{
    int64_t N = orc_nnodes(p);
    if (p->mass == 0) {
        double* m = (double*)malloc((size_t)N * sizeof(double));
        orc_lumped_mass(p, m);
        for (int64_t i = 0; i < N; ++i) out[i] = m[i] * v[i];
        free(m);
        return;
    }
    orc_ref R;
    ref_build(&R, p);
    int64_t E[3], idx[8];
    memset(out, 0, (size_t)N * sizeof(double));
    FOR_EACH_ELEMENT(p, E)
    {
        elem_nodes(p, E, R.nv, idx);
        for (int q = 0; q < R.nv; ++q) {
            double vq = 0.0;
            for (int b = 0; b < R.nv; ++b) vq += R.phi[q][b] * v[idx[b]];
            for (int a = 0; a < R.nv; ++a) out[idx[a]] += R.detJ * R.phi[q][a] * vq;
        }
    }
}

/* discrete free energy E_h = sum_e sum_q detJ [ f(c_q) + kappa/2 |grad c_q|^2 ]  [Eqs. 5-6] */
double orc_energy(const orc_problem* p, const double* U)
{
    orc_ref R;
    ref_build(&R, p);
    int64_t E[3], idx[8];
    double sum = 0.0;
    FOR_EACH_ELEMENT(p, E)
    {
        elem_nodes(p, E, R.nv, idx);
        for (int q = 0; q < R.nv; ++q) {
            double cq = 0.0, gq[3] = {0.0, 0.0, 0.0};
            for (int a = 0; a < R.nv; ++a) {
                cq += R.phi[q][a] * U[idx[a]];
                for (int k = 0; k < R.d; ++k) gq[k] += R.grad[q][a][k] * U[idx[a]];
            }
            double g2 = 0.0;
            for (int k = 0; k < R.d; ++k) g2 += gq[k] * gq[k];
            sum += R.detJ * (fe_f(p->fe, p->W, cq) + 0.5 * p->kappa * g2);
        }
    }
    return sum;
}

/* total conserved quantity sum_a m_a c_a */
double orc_total_mass(const orc_problem* p, const double* U)
{
    int64_t N = orc_nnodes(p);
    double* m = (double*)malloc((size_t)N * sizeof(double));
    orc_lumped_mass(p, m);
    double s = 0.0;
    for (int64_t i = 0; i < N; ++i) s += m[i] * U[i];
    free(m);
    return s;
}

/* r(U, theta) of Eq. 11.
 *   Allen-Cahn:   r = L * [ N(eta) + kappa K eta ]
 *   Cahn-Hilliard (mass matrix diag(m, 0), Eqs. 9-10 in weak form):
 *       r_c  = M * K mu
 *       r_mu = m mu - [ N(c) + kappa K c ]
 * with N(u)_a = sum_e sum_q detJ f'(u_q) phi_a(q) and K the Q1 stiffness. */
int orc_residual(const orc_problem* p, const double* U, double* r)
{
    int64_t N = orc_nnodes(p);
    if (p->model == ORC_AC) {
        memset(r, 0, (size_t)N * sizeof(double));
        assemble_first(p, p->W, U, p->mob, p->mob * p->kappa, r);
        return 0;
    }
    const double* c = U;
    const double* mu = U + N;
    double* rc = r;
    double* rm = r + N;
    memset(r, 0, (size_t)(2 * N) * sizeof(double));
    assemble_first(p, p->W, mu, 0.0, p->mob, rc);
    double* g = (double*)calloc((size_t)N, sizeof(double));
    assemble_first(p, p->W, c, 1.0, p->kappa, g);
    apply_mass(p, mu, rm);
    for (int64_t i = 0; i < N; ++i) rm[i] -= g[i];
    free(g);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* explicit time stepping   [Eq. 12]                                          */
/* ------------------------------------------------------------------------ */

/* nsteps of forward Euler with the lumped mass, in place.
 *   Allen-Cahn:    eta <- eta - dt * r(eta) / m
 *   Cahn-Hilliard: mu  <- [N(c) + kappa K c] / m      (algebraic row solved)
 *                  c   <- c - dt * M K mu / m
 * On return the Cahn-Hilliard mu plane holds [N(c)+kappa K c]/m of the final c. */
int orc_explicit(const orc_problem* p, double dt, int64_t nsteps, double* U)
{
    if (p->mass != 0) return -2; /* a consistent mass needs a solve: implicit path only */
    int64_t N = orc_nnodes(p);
    double* m = (double*)malloc((size_t)N * sizeof(double));
    double* t = (double*)malloc((size_t)N * sizeof(double));
    orc_lumped_mass(p, m);
    if (p->model == ORC_AC) {
        for (int64_t s = 0; s < nsteps; ++s) {
            memset(t, 0, (size_t)N * sizeof(double));
            assemble_first(p, p->W, U, p->mob, p->mob * p->kappa, t);
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < N; ++i) U[i] -= dt * t[i] / m[i];
        }
    } else {
        double* c = U;
        double* mu = U + N;
        for (int64_t s = 0; s <= nsteps; ++s) {
            memset(t, 0, (size_t)N * sizeof(double));
            assemble_first(p, p->W, c, 1.0, p->kappa, t);
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < N; ++i) mu[i] = t[i] / m[i];
            if (s == nsteps) break;
            memset(t, 0, (size_t)N * sizeof(double));
            assemble_first(p, p->W, mu, 0.0, p->mob, t);
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < N; ++i) c[i] -= dt * t[i] / m[i];
        }
    }
    free(t);
    free(m);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* implicit (backward Euler) residual, Jacobian products   [Eqs. 13-14]       */
/* ------------------------------------------------------------------------ */

/* R = M (U - U_old)/dt + r(U); for Cahn-Hilliard the mass block is diag(M, 0). */
int orc_be_residual(const orc_problem* p, double dt, const double* Uold, const double* U,
                    double* R)
{
    int64_t N = orc_nnodes(p);
    orc_residual(p, U, R);
    double* d = (double*)malloc((size_t)N * sizeof(double));
    double* t = (double*)malloc((size_t)N * sizeof(double));
    for (int64_t i = 0; i < N; ++i) d[i] = U[i] - Uold[i];
    apply_mass(p, d, t);
    for (int64_t i = 0; i < N; ++i) R[i] += t[i] / dt;
    free(t);
    free(d);
    return 0;
}

/* Jv = (dR/dU) v with R = inv_dt * M (U - U_old) + r(U).  inv_dt = 0 gives dr/dU.
 *   Allen-Cahn:     Jv = inv_dt m v + L [ N'(eta) v + kappa K v ]
 *   Cahn-Hilliard:  Jv_c  = inv_dt m v_c + M K v_mu
 *                   Jv_mu = m v_mu - [ N'(c) v_c + kappa K v_c ]      */
int orc_jvp(const orc_problem* p, double inv_dt, const double* U, const double* v, double* Jv)
{
    int64_t N = orc_nnodes(p);
    double* mv = (double*)malloc((size_t)N * sizeof(double));
    apply_mass(p, v, mv); /* M v (first field) */
    if (p->model == ORC_AC) {
        memset(Jv, 0, (size_t)N * sizeof(double));
        assemble_second(p, p->W, U, v, p->mob, p->mob * p->kappa, Jv);
        for (int64_t i = 0; i < N; ++i) Jv[i] += inv_dt * mv[i];
    } else {
        memset(Jv, 0, (size_t)(2 * N) * sizeof(double));
        double* a = (double*)calloc((size_t)N, sizeof(double));
        double* mw = (double*)malloc((size_t)N * sizeof(double));
        apply_mass(p, v + N, mw);
        assemble_second(p, p->W, U, v + N, 0.0, p->mob, Jv); /* M K v_mu */
        assemble_second(p, p->W, U, v, 1.0, p->kappa, a);    /* N'(c) v_c + kappa K v_c */
        for (int64_t i = 0; i < N; ++i) {
            Jv[i] += inv_dt * mv[i];
            Jv[N + i] = mw[i] - a[i];
        }
        free(mw);
        free(a);
    }
    free(mv);
    return 0;
}

/* w^T (dR/dU): the transpose product of orc_jvp.
 *   Allen-Cahn: the matrix is symmetric, same as orc_jvp.
 *   Cahn-Hilliard: [ inv_dt m w_c - (N'(c) + kappa K) w_mu ;  M K w_c + m w_mu ] */
int orc_jvp_t(const orc_problem* p, double inv_dt, const double* U, const double* w, double* Jtw)
{
    if (p->model == ORC_AC) return orc_jvp(p, inv_dt, U, w, Jtw);
    int64_t N = orc_nnodes(p);
    double* mc = (double*)malloc((size_t)N * sizeof(double));
    double* mw = (double*)malloc((size_t)N * sizeof(double));
    apply_mass(p, w, mc);     /* the mass is symmetric: M^T w = M w */
    apply_mass(p, w + N, mw);
    memset(Jtw, 0, (size_t)(2 * N) * sizeof(double));
    double* a = (double*)calloc((size_t)N, sizeof(double));
    assemble_second(p, p->W, U, w + N, 1.0, p->kappa, a);      /* A w_mu */
    assemble_second(p, p->W, U, w, 0.0, p->mob, Jtw + N);       /* M K w_c */
    for (int64_t i = 0; i < N; ++i) {
        Jtw[i] = inv_dt * mc[i] - a[i];
        Jtw[N + i] += mw[i];
    }
    free(a);
    free(mw);
    free(mc);
    return 0;
}

/* g[3] = w^T dr/dtheta at U for theta = (mobility, kappa, W). */
int orc_dr_dtheta(const orc_problem* p, const double* U, const double* w, double* g)
{
    int64_t N = orc_nnodes(p);
    double* t = (double*)malloc((size_t)N * sizeof(double));
    g[0] = g[1] = g[2] = 0.0;
    if (p->model == ORC_AC) {
        /* r = L [N_W(eta) + kappa K eta], N_W linear in W */
        memset(t, 0, (size_t)N * sizeof(double));
        assemble_first(p, p->W, U, 1.0, p->kappa, t); /* r / L */
        for (int64_t i = 0; i < N; ++i) g[0] += w[i] * t[i];
        memset(t, 0, (size_t)N * sizeof(double));
        assemble_first(p, p->W, U, 0.0, p->mob, t); /* dr/dkappa = L K eta */
        for (int64_t i = 0; i < N; ++i) g[1] += w[i] * t[i];
        memset(t, 0, (size_t)N * sizeof(double));
        assemble_first(p, 1.0, U, p->mob, 0.0, t); /* dr/dW = L N_1(eta) */
        for (int64_t i = 0; i < N; ++i) g[2] += w[i] * t[i];
    } else {
        const double* c = U;
        const double* mu = U + N;
        memset(t, 0, (size_t)N * sizeof(double));
        assemble_first(p, p->W, mu, 0.0, 1.0, t); /* dr_c/dM = K mu */
        for (int64_t i = 0; i < N; ++i) g[0] += w[i] * t[i];
        memset(t, 0, (size_t)N * sizeof(double));
        assemble_first(p, p->W, c, 0.0, 1.0, t); /* dr_mu/dkappa = -K c */
        for (int64_t i = 0; i < N; ++i) g[1] -= w[N + i] * t[i];
        memset(t, 0, (size_t)N * sizeof(double));
        assemble_first(p, 1.0, c, 1.0, 0.0, t); /* dr_mu/dW = -N_1(c) */
        for (int64_t i = 0; i < N; ++i) g[2] -= w[N + i] * t[i];
    }
    free(t);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* linear solvers for the Newton correction                                   */
/* ------------------------------------------------------------------------ */

static double dot(int64_t n, const double* a, const double* b)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* Gaussian elimination with partial pivoting on a dense n x n row-major A;
 * solves A x = b in place (b becomes x).  Returns -1 if singular. */
static int dense_solve(int64_t n, double* A, double* b)
{
    for (int64_t k = 0; k < n; ++k) {
        int64_t piv = k;
        for (int64_t i = k + 1; i < n; ++i)
            if (fabs(A[i * n + k]) > fabs(A[piv * n + k])) piv = i;
        if (A[piv * n + k] == 0.0) return -1;
        if (piv != k) {
            for (int64_t j = 0; j < n; ++j) {
                double t = A[k * n + j];
                A[k * n + j] = A[piv * n + j];
                A[piv * n + j] = t;
            }
            double t = b[k];
            b[k] = b[piv];
            b[piv] = t;
        }
        for (int64_t i = k + 1; i < n; ++i) {
            double l = A[i * n + k] / A[k * n + k];
            if (l == 0.0) continue;
            for (int64_t j = k; j < n; ++j) A[i * n + j] -= l * A[k * n + j];
            b[i] -= l * b[k];
        }
    }
    for (int64_t i = n - 1; i >= 0; --i) {
        double s = b[i];
        for (int64_t j = i + 1; j < n; ++j) s -= A[i * n + j] * b[j];
        b[i] = s / A[i * n + i];
    }
    return 0;
}

/* dense dR/dU (or its transpose), column by column from unit vectors */
static void dense_jacobian(const orc_problem* p, double inv_dt, const double* U, int transpose,
                           double* A)
{
    int64_t n = orc_ndof(p);
    double* e = (double*)calloc((size_t)n, sizeof(double));
    double* col = (double*)malloc((size_t)n * sizeof(double));
    for (int64_t j = 0; j < n; ++j) {
        e[j] = 1.0;
        if (transpose)
            orc_jvp_t(p, inv_dt, U, e, col);
        else
            orc_jvp(p, inv_dt, U, e, col);
        e[j] = 0.0;
        for (int64_t i = 0; i < n; ++i) A[i * n + j] = col[i];
    }
    free(col);
    free(e);
}

/* Point (Allen-Cahn) or per-node 2x2 block (Cahn-Hilliard) Jacobi preconditioner:
 * z = P^-1 y, with P the (block) diagonal of dR/dU. */
typedef struct {
    const orc_problem* p;
    int64_t N;
    double *m, *dk, *dn; /* lumped mass, diag K, diag N'(u) */
    double inv_dt;
} orc_prec;

static void prec_build(orc_prec* P, const orc_problem* p, double inv_dt, const double* U)
{
    P->p = p;
    P->N = orc_nnodes(p);
    P->inv_dt = inv_dt;
    P->m = (double*)malloc((size_t)P->N * sizeof(double));
    P->dk = (double*)calloc((size_t)P->N, sizeof(double));
    P->dn = (double*)calloc((size_t)P->N, sizeof(double));
    orc_lumped_mass(p, P->m);
    assemble_second_diag(p, U, 0.0, 1.0, P->dk);
    assemble_second_diag(p, U, 1.0, 0.0, P->dn);
}
static void prec_free(orc_prec* P)
{
    free(P->m);
    free(P->dk);
    free(P->dn);
}
static void prec_apply(const orc_prec* P, const double* y, double* z)
{
    const orc_problem* p = P->p;
    int64_t N = P->N;
    if (p->model == ORC_AC) {
        for (int64_t i = 0; i < N; ++i) {
            double d = P->inv_dt * P->m[i] + p->mob * (P->dn[i] + p->kappa * P->dk[i]);
            z[i] = y[i] / d;
        }
        return;
    }
    for (int64_t i = 0; i < N; ++i) {
        /* [[a, b], [c, d]] = [[inv_dt m, M K_ii], [-(N'_ii + kappa K_ii), m]] */
        double a = P->inv_dt * P->m[i], b = p->mob * P->dk[i];
        double c = -(P->dn[i] + p->kappa * P->dk[i]), d = P->m[i];
        double det = a * d - b * c;
        double y0 = y[i], y1 = y[N + i];
        z[i] = (d * y0 - b * y1) / det;
        z[N + i] = (-c * y0 + a * y1) / det;
    }
}

/* Restarted GMRES(restart) with right preconditioning, modified Gram-Schmidt
 * Arnoldi and Givens rotations (textbook form).  Solves J x = b (or J^T x = b)
 * starting from x = 0, until ||b - J x|| <= rtol ||b||.  Returns iterations. */
static int gmres(const orc_problem* p, double inv_dt, const double* U, int transpose,
                 const double* b, double* x, int restart, int maxit, double rtol)
{
    int64_t n = orc_ndof(p);
    int mr = restart;
    double* V = (double*)malloc((size_t)(mr + 1) * (size_t)n * sizeof(double));
    double* Z = (double*)malloc((size_t)mr * (size_t)n * sizeof(double));
    double* H = (double*)calloc((size_t)(mr + 1) * (size_t)mr, sizeof(double));
    double* cs = (double*)malloc((size_t)mr * sizeof(double));
    double* sn = (double*)malloc((size_t)mr * sizeof(double));
    double* gvec = (double*)malloc((size_t)(mr + 1) * sizeof(double));
    double* y = (double*)malloc((size_t)mr * sizeof(double));
    double* w = (double*)malloc((size_t)n * sizeof(double));
    orc_prec P;
    prec_build(&P, p, inv_dt, U);
    /* the transpose of a block-diagonal preconditioned system is preconditioned
     * by the transposed blocks; swapping the off-diagonal entries does that */
    double bnorm = sqrt(dot(n, b, b));
    memset(x, 0, (size_t)n * sizeof(double));
    int total = 0;
    if (bnorm == 0.0) goto done;
    for (;;) {
        /* r = b - J x */
        if (transpose)
            orc_jvp_t(p, inv_dt, U, x, w);
        else
            orc_jvp(p, inv_dt, U, x, w);
        for (int64_t i = 0; i < n; ++i) w[i] = b[i] - w[i];
        double beta = sqrt(dot(n, w, w));
        if (beta <= rtol * bnorm || total >= maxit) break;
        for (int64_t i = 0; i < n; ++i) V[i] = w[i] / beta;
        memset(gvec, 0, (size_t)(mr + 1) * sizeof(double));
        gvec[0] = beta;
        int j;
        for (j = 0; j < mr && total < maxit; ++j, ++total) {
            double* zj = Z + (size_t)j * n;
            if (!transpose) {
                prec_apply(&P, V + (size_t)j * n, zj);
            } else {
                /* transposed 2x2 blocks for Cahn-Hilliard */
                if (p->model == ORC_AC) {
                    prec_apply(&P, V + (size_t)j * n, zj);
                } else {
                    int64_t N = P.N;
                    const double* vj = V + (size_t)j * n;
                    for (int64_t i = 0; i < N; ++i) {
                        double a = P.inv_dt * P.m[i], bb = p->mob * P.dk[i];
                        double c = -(P.dn[i] + p->kappa * P.dk[i]), d = P.m[i];
                        double det = a * d - bb * c; /* transpose: [[a, c],[bb, d]] */
                        zj[i] = (d * vj[i] - c * vj[N + i]) / det;
                        zj[N + i] = (-bb * vj[i] + a * vj[N + i]) / det;
                    }
                }
            }
            if (transpose)
                orc_jvp_t(p, inv_dt, U, zj, w);
            else
                orc_jvp(p, inv_dt, U, zj, w);
            for (int i = 0; i <= j; ++i) {
                double hij = dot(n, w, V + (size_t)i * n);
                H[i * mr + j] = hij;
                for (int64_t k = 0; k < n; ++k) w[k] -= hij * V[(size_t)i * n + k];
            }
            double hn = sqrt(dot(n, w, w));
            H[(j + 1) * mr + j] = hn;
            if (hn > 0.0)
                for (int64_t k = 0; k < n; ++k) V[(size_t)(j + 1) * n + k] = w[k] / hn;
            for (int i = 0; i < j; ++i) {
                double t = cs[i] * H[i * mr + j] + sn[i] * H[(i + 1) * mr + j];
                H[(i + 1) * mr + j] = -sn[i] * H[i * mr + j] + cs[i] * H[(i + 1) * mr + j];
                H[i * mr + j] = t;
            }
            double a = H[j * mr + j], bb = H[(j + 1) * mr + j];
            double rr = sqrt(a * a + bb * bb);
            cs[j] = a / rr;
            sn[j] = bb / rr;
            H[j * mr + j] = rr;
            H[(j + 1) * mr + j] = 0.0;
            gvec[j + 1] = -sn[j] * gvec[j];
            gvec[j] = cs[j] * gvec[j];
            if (fabs(gvec[j + 1]) <= rtol * bnorm || hn == 0.0) {
                ++j;
                ++total;
                break;
            }
        }
        /* back substitution H y = g, x += Z y */
        for (int i = j - 1; i >= 0; --i) {
            double s = gvec[i];
            for (int k = i + 1; k < j; ++k) s -= H[i * mr + k] * y[k];
            y[i] = s / H[i * mr + i];
        }
        for (int i = 0; i < j; ++i)
            for (int64_t k = 0; k < n; ++k) x[k] += y[i] * Z[(size_t)i * n + k];
    }
done:
    prec_free(&P);
    free(w);
    free(y);
    free(gvec);
    free(sn);
    free(cs);
    free(H);
    free(Z);
    free(V);
    return total;
}

/* Solve (dR/dU) x = b (transpose = 0) or (dR/dU)^T x = b (transpose = 1).
 * solver 0: dense LU, solver 1: GMRES(30) to lin_rtol.  Returns iterations. */
int orc_linear_solve(const orc_problem* p, double inv_dt, const double* U, int transpose,
                     const double* b, double* x, int solver, double lin_rtol)
{
    int64_t n = orc_ndof(p);
    if (solver == 0) {
        double* A = (double*)malloc((size_t)n * (size_t)n * sizeof(double));
        dense_jacobian(p, inv_dt, U, transpose, A);
        memcpy(x, b, (size_t)n * sizeof(double));
        int rc = dense_solve(n, A, x);
        free(A);
        return rc;
    }
    return gmres(p, inv_dt, U, transpose, b, x, 30, 100000, lin_rtol);
}

/* Backward-Euler step by Newton-Raphson   [Eqs. 13-14, Sec. 2.3].
 * U holds the initial guess on entry and the iterate on exit.  Stops when
 * ||R||_2 <= rtol * ||R(initial guess)||_2 or after maxit corrections.
 * hist[0..its] receives ||R|| per iterate.  Returns 0 if converged, 1 if not. */
int orc_newton_be(const orc_problem* p, double dt, const double* Uold, double* U, double rtol,
                  int maxit, int solver, double lin_rtol, int* its, double* hist)
{
    int64_t n = orc_ndof(p);
    double* R = (double*)malloc((size_t)n * sizeof(double));
    double* d = (double*)malloc((size_t)n * sizeof(double));
    orc_be_residual(p, dt, Uold, U, R);
    double r0 = sqrt(dot(n, R, R)), rk = r0;
    hist[0] = r0;
    int k = 0, conv = (r0 == 0.0);
    while (!conv && k < maxit) {
        for (int64_t i = 0; i < n; ++i) R[i] = -R[i];
        orc_linear_solve(p, 1.0 / dt, U, 0, R, d, solver, lin_rtol);
        for (int64_t i = 0; i < n; ++i) U[i] += d[i];
        orc_be_residual(p, dt, Uold, U, R);
        rk = sqrt(dot(n, R, R));
        ++k;
        hist[k] = rk;
        conv = rk <= rtol * r0;
    }
    *its = k;
    free(d);
    free(R);
    return conv ? 0 : 1;
}

/* ------------------------------------------------------------------------ */
/* sensitivities   [Eq. 18, Supp. Note 2, Eqs. II.1-II.6]                     */
/* ------------------------------------------------------------------------ */

/* Discrete adjoint of orc_explicit.  Given gU = dO/dU at the final state (for
 * Cahn-Hilliard only its c plane is used: the final mu is a derived output),
 * returns dO/dtheta in theta_bar[3] (mobility, kappa, W) and dO/dU0 in U0_bar
 * (c plane for Cahn-Hilliard).  Each step U_{n+1} = S(U_n, theta) is one
 * constraint; the reverse sweep applies lambda_n = (dS/dU_n)^T lambda_{n+1}
 * and theta_bar += (dS/dtheta)^T lambda_{n+1} (II.5-II.6 step by step).
 * The forward trajectory is stored whole. */
int orc_explicit_adjoint(const orc_problem* p, double dt, int64_t nsteps, const double* U0,
                         const double* gU, double* theta_bar, double* U0_bar)
{
    if (p->mass != 0) return -2; /* explicit path: lumped mass only */
    int64_t N = orc_nnodes(p);
    double* traj = (double*)malloc((size_t)(nsteps + 1) * (size_t)N * sizeof(double));
    double* m = (double*)malloc((size_t)N * sizeof(double));
    double* lam = (double*)malloc((size_t)N * sizeof(double));
    double* t1 = (double*)malloc((size_t)N * sizeof(double));
    double* t2 = (double*)malloc((size_t)N * sizeof(double));
    double* st = (double*)malloc((size_t)orc_ndof(p) * sizeof(double));
    orc_lumped_mass(p, m);
    memcpy(st, U0, (size_t)orc_ndof(p) * sizeof(double));
    memcpy(traj, st, (size_t)N * sizeof(double));
    for (int64_t s = 0; s < nsteps; ++s) {
        orc_explicit(p, dt, 1, st);
        memcpy(traj + (size_t)(s + 1) * N, st, (size_t)N * sizeof(double));
    }
    memcpy(lam, gU, (size_t)N * sizeof(double));
    theta_bar[0] = theta_bar[1] = theta_bar[2] = 0.0;
    for (int64_t s = nsteps - 1; s >= 0; --s) {
        const double* u = traj + (size_t)s * N;
        if (p->model == ORC_AC) {
            /* S(u) = u - dt r(u)/m */
            for (int64_t i = 0; i < N; ++i) t1[i] = dt * lam[i] / m[i];
            double g[3];
            orc_dr_dtheta(p, u, t1, g);
            for (int k = 0; k < 3; ++k) theta_bar[k] -= g[k];
            memset(t2, 0, (size_t)N * sizeof(double));
            assemble_second(p, p->W, u, t1, p->mob, p->mob * p->kappa, t2);
            for (int64_t i = 0; i < N; ++i) lam[i] -= t2[i];
        } else {
            /* S(c) = c - dt M^-1 [mob K] M^-1 A(c), A(c) = N(c) + kappa K c */
            for (int64_t i = 0; i < N; ++i) t1[i] = dt * lam[i] / m[i];
            memset(t2, 0, (size_t)N * sizeof(double));
            assemble_second(p, p->W, u, t1, 0.0, 1.0, t2); /* K t1 */
            /* theta: dS/dmob = -dt M^-1 K mu */
            double* mu = (double*)calloc((size_t)N, sizeof(double));
            assemble_first(p, p->W, u, 1.0, p->kappa, mu);
            for (int64_t i = 0; i < N; ++i) mu[i] /= m[i];
            double* kmu = (double*)calloc((size_t)N, sizeof(double));
            assemble_first(p, p->W, mu, 0.0, 1.0, kmu);
            double* kc = (double*)calloc((size_t)N, sizeof(double));
            assemble_first(p, p->W, u, 0.0, 1.0, kc);
            double* n1 = (double*)calloc((size_t)N, sizeof(double));
            assemble_first(p, 1.0, u, 1.0, 0.0, n1);
            for (int64_t i = 0; i < N; ++i) {
                /* lam^T dS/dtheta, with v = M^-1 mob K (dt M^-1 lam) = mob t2 / m */
                theta_bar[0] -= t1[i] * kmu[i];
                theta_bar[1] -= p->mob * t2[i] / m[i] * kc[i];
                theta_bar[2] -= p->mob * t2[i] / m[i] * n1[i];
            }
            free(n1);
            free(kc);
            free(kmu);
            free(mu);
            /* lam -= A'(c)^T (mob K dt M^-1 lam / m) */
            for (int64_t i = 0; i < N; ++i) t1[i] = p->mob * t2[i] / m[i];
            memset(t2, 0, (size_t)N * sizeof(double));
            assemble_second(p, p->W, u, t1, 1.0, p->kappa, t2);
            for (int64_t i = 0; i < N; ++i) lam[i] -= t2[i];
        }
    }
    memcpy(U0_bar, lam, (size_t)N * sizeof(double));
    free(st);
    free(t2);
    free(t1);
    free(lam);
    free(m);
    free(traj);
    return 0;
}

/* Adjoint of one backward-Euler step U = Newton(U_old, theta), R(U, U_old) = 0:
 * solve (dR/dU)^T lambda = gU, then U_old_bar = (M/dt) lambda and
 * theta_bar = -(dr/dtheta)^T lambda at U   (II.5-II.6).  solver as in
 * orc_linear_solve. */
int orc_newton_adjoint(const orc_problem* p, double dt, const double* U, const double* gU,
                       double* Uold_bar, double* theta_bar, int solver)
{
    int64_t n = orc_ndof(p), N = orc_nnodes(p);
    double* lam = (double*)malloc((size_t)n * sizeof(double));
    double* m = (double*)malloc((size_t)N * sizeof(double));
    orc_linear_solve(p, 1.0 / dt, U, 1, gU, lam, solver, 1e-13);
    memset(Uold_bar, 0, (size_t)n * sizeof(double));
    apply_mass(p, lam, m); /* (M/dt)^T lam on the mass rows; M is symmetric */
    for (int64_t i = 0; i < N; ++i) Uold_bar[i] = m[i] / dt;
    double g[3];
    orc_dr_dtheta(p, U, lam, g);
    for (int k = 0; k < 3; ++k) theta_bar[k] = -g[k];
    free(m);
    free(lam);
    return 0;
}
