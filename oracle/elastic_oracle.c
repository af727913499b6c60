/*
 * elastic_oracle.c -- plain, slow, FP64 CPU reference of the Eshelby-inclusion
 * benchmark: small-strain linear elasticity with an eigenstrain.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite may.  It shares no code, header, table
 * or constant with the HIP library.
 *
 * What it computes (paper passage in brackets):
 *   - equilibrium  div sigma = 0                                            [Eq. 3]
 *   - stress       sigma = C : (eps(u) - eps0), C isotropic (E, nu)         [Eq. 4]
 *   - eigenstrain  eps0_ij = delta_ij m s(r),  s(r) = 1/2 - 1/2 tanh(l (r - a)),
 *                  r = distance from the origin corner (the inclusion sits at
 *                  the corner; the printed "+" before the tanh would put the
 *                  misfit outside the inclusion and is read as "-")      [Supp. Note 3, III.1]
 * Discretisation: vector Q1 elements on the grid [0, (n-1) h]^dim (n - 1
 * elements per axis), 2-point Gauss-Legendre quadrature per axis (exact for the
 * Q1 stiffness), eps0 evaluated at the quadrature points.  dim = 2 is plane
 * strain.  Boundary conditions: symmetry on the faces through the origin
 * (u_x = 0 on x = 0, u_y = 0 on y = 0, u_z = 0 on z = 0), traction-free on the
 * others (natural).  Displacements are laid out component-major:
 * u = [u_x (N values) ; u_y ; (u_z)], node index i + n0 (j + n1 k).
 *
 *   K u = f,  K_ab = sum_e sum_q |J| B_a^T C B_b,  f_a = sum_e sum_q |J| B_a^T C eps0(x_q)
 * with the constrained rows and columns replaced by the identity (u = 0 there).
 * The objective is the volume change  O(u) = int div u dV = sum_e sum_q |J| div u(x_q).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t dim;   /* 2 (plane strain) or 3 */
    int32_t sym;   /* 1: symmetry planes through the origin (the benchmark); 0: every face
                    * traction-free (K then has the rigid-body null space; for checks only) */
    int64_t n[3];  /* nodes per axis; n[2] = 1 in 2-D */
    double h;      /* grid spacing */
    double E, nu;  /* Young's modulus, Poisson's ratio */
    double m, a, l; /* eigenstrain magnitude, inclusion radius, interface sharpness */
} orc_el_problem;

static int64_t el_nnodes(const orc_el_problem* p)
{
    int64_t N = 1;
    for (int k = 0; k < p->dim; ++k) N *= p->n[k];
    return N;
}

static void el_lame(const orc_el_problem* p, double* lam, double* mu)
{
    *lam = p->E * p->nu / ((1.0 + p->nu) * (1.0 - 2.0 * p->nu));
    *mu = p->E / (2.0 * (1.0 + p->nu));
}

/* reference element: Gauss points, shape values and physical gradients */
typedef struct {
    int d, nv;
    double detJ;
    double xi[8][3];      /* quadrature point offsets in [0, h] per axis */
    double phi[8][8];     /* phi[q][a] */
    double grad[8][8][3]; /* grad[q][a][k] */
} el_ref;

static void el_ref_build(el_ref* R, int d, double h)
{
    const double g = 1.0 / sqrt(3.0);
    R->d = d;
    R->nv = 1 << d;
    R->detJ = pow(0.5 * h, d);
    for (int q = 0; q < R->nv; ++q) {
        for (int k = 0; k < d; ++k) R->xi[q][k] = 0.5 * h * (1.0 + (((q >> k) & 1) ? g : -g));
        for (int a = 0; a < R->nv; ++a) {
            double f[3], s[3];
            for (int k = 0; k < d; ++k) {
                const double x = ((q >> k) & 1) ? g : -g;
                s[k] = ((a >> k) & 1) ? 1.0 : -1.0;
                f[k] = 0.5 * (1.0 + s[k] * x);
            }
            double v = 1.0;
            for (int k = 0; k < d; ++k) v *= f[k];
            R->phi[q][a] = v;
            for (int k = 0; k < d; ++k) {
                double gk = s[k] / h;
                for (int l2 = 0; l2 < d; ++l2)
                    if (l2 != k) gk *= f[l2];
                R->grad[q][a][k] = gk;
            }
        }
    }
}

static void el_elem_nodes(const orc_el_problem* p, const int64_t e[3], int nv, int64_t* idx)
{
    for (int a = 0; a < nv; ++a) {
        int64_t ijk[3] = {0, 0, 0};
        for (int k = 0; k < p->dim; ++k) ijk[k] = e[k] + ((a >> k) & 1);
        idx[a] = ijk[0] + p->n[0] * (ijk[1] + p->n[1] * ijk[2]);
    }
}

#define EL_FOR_EACH_ELEMENT(p, E)                                           \
    for (E[2] = 0; E[2] < ((p)->dim == 3 ? (p)->n[2] - 1 : 1); ++E[2])     \
        for (E[1] = 0; E[1] < (p)->n[1] - 1; ++E[1])                       \
            for (E[0] = 0; E[0] < (p)->n[0] - 1; ++E[0])

double orc_el_eigen(const orc_el_problem* p, double r)
{
    return p->m * (0.5 - 0.5 * tanh(p->l * (r - p->a)));
}

/* 1 if displacement component c of node i is free, 0 if constrained */
int orc_el_free(const orc_el_problem* p, int64_t i, int c)
{
    if (!p->sym) return 1;
    int64_t ijk[3];
    ijk[0] = i % p->n[0];
    ijk[1] = (i / p->n[0]) % p->n[1];
    ijk[2] = i / (p->n[0] * p->n[1]);
    return ijk[c] != 0;
}

/* y = K_{lam,mu} u restricted to free degrees of freedom (constrained rows get u) */
static void el_apply_lame(const orc_el_problem* p, double lam, double mu, const double* u, double* y,
                          int identity_rows)
{
    el_ref R;
    el_ref_build(&R, p->dim, p->h);
    const int64_t N = el_nnodes(p);
    const int d = p->dim;
    memset(y, 0, (size_t)(d * N) * sizeof(double));
    int64_t E[3], idx[8];
    EL_FOR_EACH_ELEMENT(p, E)
    {
        el_elem_nodes(p, E, R.nv, idx);
        for (int q = 0; q < R.nv; ++q) {
            double G[3][3] = {{0}};  /* G[i][k] = d u_i / d x_k (constrained dofs taken as 0) */
            for (int a = 0; a < R.nv; ++a)
                for (int i = 0; i < d; ++i) {
                    const double ui = orc_el_free(p, idx[a], i) ? u[i * N + idx[a]] : 0.0;
                    for (int k = 0; k < d; ++k) G[i][k] += R.grad[q][a][k] * ui;
                }
            double tr = 0.0;
            for (int i = 0; i < d; ++i) tr += G[i][i];
            double S[3][3];
            for (int i = 0; i < d; ++i)
                for (int k = 0; k < d; ++k) S[i][k] = mu * (G[i][k] + G[k][i]) + (i == k ? lam * tr : 0.0);
            for (int a = 0; a < R.nv; ++a)
                for (int i = 0; i < d; ++i) {
                    if (!orc_el_free(p, idx[a], i)) continue;
                    double s = 0.0;
                    for (int k = 0; k < d; ++k) s += S[i][k] * R.grad[q][a][k];
                    y[i * N + idx[a]] += R.detJ * s;
                }
        }
    }
    if (identity_rows)
        for (int i = 0; i < d; ++i)
            for (int64_t a = 0; a < N; ++a)
                if (!orc_el_free(p, a, i)) y[i * N + a] = u[i * N + a];
}

/* f_a = sum_e sum_q |J| B_a^T C_{lam,mu} eps0(x_q) on free dofs (0 on constrained) */
static void el_rhs_lame(const orc_el_problem* p, double lam, double mu, double* f)
{
    el_ref R;
    el_ref_build(&R, p->dim, p->h);
    const int64_t N = el_nnodes(p);
    const int d = p->dim;
    memset(f, 0, (size_t)(d * N) * sizeof(double));
    int64_t E[3], idx[8];
    EL_FOR_EACH_ELEMENT(p, E)
    {
        el_elem_nodes(p, E, R.nv, idx);
        for (int q = 0; q < R.nv; ++q) {
            double r2 = 0.0;
            for (int k = 0; k < d; ++k) {
                const double x = (double)E[k] * p->h + R.xi[q][k];
                r2 += x * x;
            }
            const double e0 = orc_el_eigen(p, sqrt(r2));
            /* sigma0 = C eps0 = (d lam + 2 mu) e0 I */
            const double s0 = ((double)d * lam + 2.0 * mu) * e0;
            for (int a = 0; a < R.nv; ++a)
                for (int i = 0; i < d; ++i)
                    if (orc_el_free(p, idx[a], i)) f[i * N + idx[a]] += R.detJ * s0 * R.grad[q][a][i];
        }
    }
}

int orc_el_apply(const orc_el_problem* p, const double* u, double* y)
{
    double lam, mu;
    el_lame(p, &lam, &mu);
    el_apply_lame(p, lam, mu, u, y, 1);
    return 0;
}

int orc_el_rhs(const orc_el_problem* p, double* f)
{
    double lam, mu;
    el_lame(p, &lam, &mu);
    el_rhs_lame(p, lam, mu, f);
    return 0;
}

/* g with O(u) = g . u = sum_e sum_q |J| div u(x_q) (constrained dofs contribute 0) */
int orc_el_volume_weights(const orc_el_problem* p, double* g)
{
    el_ref R;
    el_ref_build(&R, p->dim, p->h);
    const int64_t N = el_nnodes(p);
    const int d = p->dim;
    memset(g, 0, (size_t)(d * N) * sizeof(double));
    int64_t E[3], idx[8];
    EL_FOR_EACH_ELEMENT(p, E)
    {
        el_elem_nodes(p, E, R.nv, idx);
        for (int q = 0; q < R.nv; ++q)
            for (int a = 0; a < R.nv; ++a)
                for (int i = 0; i < d; ++i)
                    if (orc_el_free(p, idx[a], i)) g[i * N + idx[a]] += R.detJ * R.grad[q][a][i];
    }
    return 0;
}

static double el_dot(int64_t n, const double* a, const double* b)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* conjugate gradients on K u = b (K symmetric positive definite), u = 0 start,
 * to ||r|| <= rtol ||b||.  Returns iterations, -1 without convergence. */
static int el_cg(const orc_el_problem* p, const double* b, double* u, double rtol, int maxit)
{
    const int64_t n = p->dim * el_nnodes(p);
    double* r = (double*)malloc((size_t)n * sizeof(double));
    double* s = (double*)malloc((size_t)n * sizeof(double));
    double* q = (double*)malloc((size_t)n * sizeof(double));
    memset(u, 0, (size_t)n * sizeof(double));
    memcpy(r, b, (size_t)n * sizeof(double));
    memcpy(s, b, (size_t)n * sizeof(double));
    const double bn = sqrt(el_dot(n, b, b));
    double rr = el_dot(n, r, r);
    int it = 0, ok = bn == 0.0;
    for (; !ok && it < maxit; ++it) {
        orc_el_apply(p, s, q);
        const double alpha = rr / el_dot(n, s, q);
        for (int64_t i = 0; i < n; ++i) {
            u[i] += alpha * s[i];
            r[i] -= alpha * q[i];
        }
        const double rr2 = el_dot(n, r, r);
        if (sqrt(rr2) <= rtol * bn) {
            ok = 1;
            ++it;
            break;
        }
        const double beta = rr2 / rr;
        rr = rr2;
        for (int64_t i = 0; i < n; ++i) s[i] = r[i] + beta * s[i];
    }
    free(q);
    free(s);
    free(r);
    return ok ? it : -1;
}

/* the equilibrium displacement; returns CG iterations or -1 */
int orc_el_solve(const orc_el_problem* p, double* u, double rtol, int maxit)
{
    const int64_t n = p->dim * el_nnodes(p);
    double* f = (double*)malloc((size_t)n * sizeof(double));
    orc_el_rhs(p, f);
    const int it = el_cg(p, f, u, rtol, maxit);
    free(f);
    return it;
}

/* Sensitivities of O(u) = g . u with respect to theta = (E, nu) at the
 * equilibrium K(theta) u = f(theta), by the adjoint method of Eq. 18 applied to
 * the static residual R(u, theta) = K u - f:  solve K^T lam = g (K is
 * symmetric), then dO/dtheta = -lam . dR/dtheta = lam . (df/dtheta - dK/dtheta u).
 * K and f are linear in the Lame constants (lambda, mu), so the derivatives are
 * taken in (lambda, mu) and mapped to (E, nu) by the chain rule.
 * g = NULL selects the volume-change weights.  out = {O, dO/dE, dO/dnu}.
 * u (optional, may be NULL) receives the displacement.  Returns 0, or -1 if a
 * CG solve did not converge. */
int orc_el_sensitivity(const orc_el_problem* p, const double* g_in, double rtol, int maxit,
                       double* out, double* u_out)
{
    const int64_t n = p->dim * el_nnodes(p);
    double* g = (double*)malloc((size_t)n * sizeof(double));
    double* u = (double*)malloc((size_t)n * sizeof(double));
    double* la = (double*)malloc((size_t)n * sizeof(double));
    double* t = (double*)malloc((size_t)n * sizeof(double));
    double* k = (double*)malloc((size_t)n * sizeof(double));
    if (g_in) {
        memcpy(g, g_in, (size_t)n * sizeof(double));
        for (int c = 0; c < p->dim; ++c)
            for (int64_t a = 0; a < n / p->dim; ++a)
                if (!orc_el_free(p, a, c)) g[c * (n / p->dim) + a] = 0.0;
    } else {
        orc_el_volume_weights(p, g);
    }
    int rc = 0;
    if (orc_el_solve(p, u, rtol, maxit) < 0) rc = -1;
    if (el_cg(p, g, la, rtol, maxit) < 0) rc = -1;
    out[0] = el_dot(n, g, u);
    /* d/dlambda and d/dmu of (f - K u), dotted with the adjoint */
    el_rhs_lame(p, 1.0, 0.0, t);
    el_apply_lame(p, 1.0, 0.0, u, k, 0);
    double d_lam = 0.0, d_mu = 0.0;
    for (int64_t i = 0; i < n; ++i) d_lam += la[i] * (t[i] - k[i]);
    el_rhs_lame(p, 0.0, 1.0, t);
    el_apply_lame(p, 0.0, 1.0, u, k, 0);
    for (int64_t i = 0; i < n; ++i) d_mu += la[i] * (t[i] - k[i]);
    const double E = p->E, nu = p->nu;
    const double D = (1.0 + nu) * (1.0 - 2.0 * nu);
    const double dlam_dE = nu / D, dmu_dE = 1.0 / (2.0 * (1.0 + nu));
    const double dlam_dnu = E * (1.0 + 2.0 * nu * nu) / (D * D);
    const double dmu_dnu = -E / (2.0 * (1.0 + nu) * (1.0 + nu));
    out[1] = d_lam * dlam_dE + d_mu * dmu_dE;
    out[2] = d_lam * dlam_dnu + d_mu * dmu_dnu;
    if (u_out) memcpy(u_out, u, (size_t)n * sizeof(double));
    free(k);
    free(t);
    free(la);
    free(u);
    free(g);
    return rc;
}

/* Objective value O(u) = g . u for given u and g (g = NULL: the volume change). */
double orc_el_objective(const orc_el_problem* p, const double* g_in, const double* u)
{
    const int64_t n = p->dim * el_nnodes(p);
    if (g_in) return el_dot(n, g_in, u);
    double* g = (double*)malloc((size_t)n * sizeof(double));
    orc_el_volume_weights(p, g);
    const double v = el_dot(n, g, u);
    free(g);
    return v;
}

/* sum over quadrature points of |J| eps0(x_q): the volume integral of one diagonal
 * eigenstrain component under the same quadrature as the stiffness */
double orc_el_eigen_integral(const orc_el_problem* p)
{
    el_ref R;
    el_ref_build(&R, p->dim, p->h);
    double s = 0.0;
    int64_t E[3];
    EL_FOR_EACH_ELEMENT(p, E)
    {
        for (int q = 0; q < R.nv; ++q) {
            double r2 = 0.0;
            for (int k = 0; k < p->dim; ++k) {
                const double x = (double)E[k] * p->h + R.xi[q][k];
                r2 += x * x;
            }
            s += R.detJ * orc_el_eigen(p, sqrt(r2));
        }
    }
    return s;
}
