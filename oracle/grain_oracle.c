/*
 * grain_oracle.c -- plain, slow, FP64 CPU reference of multi-order-parameter
 * Allen-Cahn (grain growth).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite does.  It shares no code, header, table
 * or constant with the HIP library.
 *
 * What it computes: p non-conserved order parameters eta_1..eta_p, one per
 * grain, each following the Allen-Cahn equation of Eq. 1 with the same
 * mobility L and gradient coefficient kappa (Sec. 2.4: one formulation applied
 * to every grain's order parameter).  The paper takes the grain-growth energy
 * from the literature it cites and does not print it; this oracle uses the
 * standard multi-order-parameter form
 *     f(eta) = sum_i (eta_i^4/4 - eta_i^2/2) + gamma sum_{i<j} eta_i^2 eta_j^2 + 1/4
 *     df/deta_i = eta_i^3 - eta_i + 2 gamma eta_i sum_{j != i} eta_j^2
 * and F = int f + kappa/2 sum_i |grad eta_i|^2.
 * Discretisation as for the single order parameter: Q1 elements, 2-point
 * Gauss-Legendre per axis, row-sum lumped mass, periodic (n elements per axis)
 * or no-flux (n - 1 elements).  States hold p planes [eta_1 (N) ; ... ; eta_p].
 *   r_i = L [ N_i(eta) + kappa K eta_i ],  N_i(eta)_a = sum_e sum_q detJ df/deta_i(eta(q)) phi_a(q)
 *   explicit step: eta_i <- eta_i - dt r_i / m
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t dim;  /* 2 or 3 */
    int32_t bc;   /* 0 periodic, 1 no-flux */
    int64_t n[3]; /* nodes per axis; n[2] = 1 in 2-D */
    double h;
    double L, kappa, gamma;
    int32_t p; /* order parameters */
    int32_t pad;
} orc_gg_problem;

typedef struct {
    int d, nv;
    double detJ;
    double phi[8][8];
    double grad[8][8][3];
} gg_ref;

static void gg_ref_build(gg_ref* R, int d, double h)
{
    const double g = 1.0 / sqrt(3.0);
    R->d = d;
    R->nv = 1 << d;
    R->detJ = pow(0.5 * h, d);
    for (int q = 0; q < R->nv; ++q)
        for (int a = 0; a < R->nv; ++a) {
            double f[3], s[3];
            for (int k = 0; k < d; ++k) {
                const double xi = ((q >> k) & 1) ? g : -g;
                s[k] = ((a >> k) & 1) ? 1.0 : -1.0;
                f[k] = 0.5 * (1.0 + s[k] * xi);
            }
            double v = 1.0;
            for (int k = 0; k < d; ++k) v *= f[k];
            R->phi[q][a] = v;
            for (int k = 0; k < d; ++k) {
                double gk = s[k] / h;
                for (int l = 0; l < d; ++l)
                    if (l != k) gk *= f[l];
                R->grad[q][a][k] = gk;
            }
        }
}

static int64_t gg_nnodes(const orc_gg_problem* p)
{
    int64_t N = 1;
    for (int k = 0; k < p->dim; ++k) N *= p->n[k];
    return N;
}

static int64_t gg_elems(const orc_gg_problem* p, int k)
{
    if (k >= p->dim) return 1;
    return p->bc == 0 ? p->n[k] : p->n[k] - 1;
}

static void gg_elem_nodes(const orc_gg_problem* p, const int64_t e[3], int nv, int64_t* idx)
{
    for (int a = 0; a < nv; ++a) {
        int64_t ijk[3] = {0, 0, 0};
        for (int k = 0; k < p->dim; ++k) {
            ijk[k] = e[k] + ((a >> k) & 1);
            if (p->bc == 0) ijk[k] %= p->n[k];
        }
        idx[a] = ijk[0] + p->n[0] * (ijk[1] + p->n[1] * ijk[2]);
    }
}

#define GG_FOR_EACH_ELEMENT(p, E)                       \
    for (E[2] = 0; E[2] < gg_elems(p, 2); ++E[2])       \
        for (E[1] = 0; E[1] < gg_elems(p, 1); ++E[1])   \
            for (E[0] = 0; E[0] < gg_elems(p, 0); ++E[0])

/* local free energy and its gradient at one point (eta holds p values) */
double orc_gg_f(const orc_gg_problem* p, const double* eta)
{
    double f = 0.25;
    for (int i = 0; i < p->p; ++i) {
        const double e2 = eta[i] * eta[i];
        f += 0.25 * e2 * e2 - 0.5 * e2;
        for (int j = i + 1; j < p->p; ++j) f += p->gamma * e2 * eta[j] * eta[j];
    }
    return f;
}

void orc_gg_df(const orc_gg_problem* p, const double* eta, double* df)
{
    for (int i = 0; i < p->p; ++i) {
        double others = 0.0;
        for (int j = 0; j < p->p; ++j)
            if (j != i) others += eta[j] * eta[j];
        df[i] = eta[i] * eta[i] * eta[i] - eta[i] + 2.0 * p->gamma * eta[i] * others;
    }
}

int orc_gg_lumped_mass(const orc_gg_problem* p, double* m)
{
    gg_ref R;
    gg_ref_build(&R, p->dim, p->h);
    const int64_t N = gg_nnodes(p);
    int64_t E[3], idx[8];
    memset(m, 0, (size_t)N * sizeof(double));
    GG_FOR_EACH_ELEMENT(p, E)
    {
        gg_elem_nodes(p, E, R.nv, idx);
        for (int q = 0; q < R.nv; ++q)
            for (int a = 0; a < R.nv; ++a) m[idx[a]] += R.detJ * R.phi[q][a];
    }
    return 0;
}

/* r_i = L [ N_i(eta) + kappa K eta_i ] for every order parameter */
int orc_gg_residual(const orc_gg_problem* p, const double* U, double* r)
{
    gg_ref R;
    gg_ref_build(&R, p->dim, p->h);
    const int64_t N = gg_nnodes(p);
    const int P = p->p;
    if (P < 1 || P > 64) return -1;
    double eq[64], gq[64][3], df[64];
    int64_t E[3], idx[8];
    memset(r, 0, (size_t)(P * N) * sizeof(double));
    GG_FOR_EACH_ELEMENT(p, E)
    {
        gg_elem_nodes(p, E, R.nv, idx);
        for (int q = 0; q < R.nv; ++q) {
            for (int i = 0; i < P; ++i) {
                eq[i] = 0.0;
                gq[i][0] = gq[i][1] = gq[i][2] = 0.0;
                for (int a = 0; a < R.nv; ++a) {
                    const double u = U[i * N + idx[a]];
                    eq[i] += R.phi[q][a] * u;
                    for (int k = 0; k < R.d; ++k) gq[i][k] += R.grad[q][a][k] * u;
                }
            }
            orc_gg_df(p, eq, df);
            for (int i = 0; i < P; ++i)
                for (int a = 0; a < R.nv; ++a) {
                    double gg = 0.0;
                    for (int k = 0; k < R.d; ++k) gg += gq[i][k] * R.grad[q][a][k];
                    r[i * N + idx[a]] += p->L * R.detJ * (df[i] * R.phi[q][a] + p->kappa * gg);
                }
        }
    }
    return 0;
}

/* nsteps of lumped-mass forward Euler, in place */
int orc_gg_explicit(const orc_gg_problem* p, double dt, int64_t nsteps, double* U)
{
    const int64_t N = gg_nnodes(p);
    const int64_t n = p->p * N;
    double* m = (double*)malloc((size_t)N * sizeof(double));
    double* r = (double*)malloc((size_t)n * sizeof(double));
    orc_gg_lumped_mass(p, m);
    int rc = 0;
    for (int64_t s = 0; s < nsteps && rc == 0; ++s) {
        rc = orc_gg_residual(p, U, r);
        for (int64_t k = 0; k < n; ++k) U[k] -= dt * r[k] / m[k % N];
    }
    free(r);
    free(m);
    return rc;
}

/* E_h = sum_e sum_q detJ [ f(eta_q) + kappa/2 sum_i |grad eta_i,q|^2 ] */
double orc_gg_energy(const orc_gg_problem* p, const double* U)
{
    gg_ref R;
    gg_ref_build(&R, p->dim, p->h);
    const int64_t N = gg_nnodes(p);
    const int P = p->p;
    double eq[64];
    int64_t E[3], idx[8];
    double sum = 0.0;
    GG_FOR_EACH_ELEMENT(p, E)
    {
        gg_elem_nodes(p, E, R.nv, idx);
        for (int q = 0; q < R.nv; ++q) {
            double g2 = 0.0;
            for (int i = 0; i < P; ++i) {
                double gq[3] = {0.0, 0.0, 0.0};
                eq[i] = 0.0;
                for (int a = 0; a < R.nv; ++a) {
                    const double u = U[i * N + idx[a]];
                    eq[i] += R.phi[q][a] * u;
                    for (int k = 0; k < R.d; ++k) gq[k] += R.grad[q][a][k] * u;
                }
                for (int k = 0; k < R.d; ++k) g2 += gq[k] * gq[k];
            }
            sum += R.detJ * (orc_gg_f(p, eq) + 0.5 * p->kappa * g2);
        }
    }
    return sum;
}

/* ------------------------------------------------------------------------ */
/* backward Euler   [Eqs. 13-14]                                             */
/* ------------------------------------------------------------------------ */

/* second derivatives of f: H_ii = 3 eta_i^2 - 1 + 2 gamma sum_{j != i} eta_j^2,
 * H_ij = 4 gamma eta_i eta_j (i != j); hv = H v */
static void gg_hess_apply(const orc_gg_problem* p, const double* eta, const double* v, double* hv)
{
    for (int i = 0; i < p->p; ++i) {
        double s = 0.0;
        for (int j = 0; j < p->p; ++j) {
            if (j == i) {
                double others = 0.0;
                for (int k = 0; k < p->p; ++k)
                    if (k != i) others += eta[k] * eta[k];
                s += (3.0 * eta[i] * eta[i] - 1.0 + 2.0 * p->gamma * others) * v[i];
            } else {
                s += 4.0 * p->gamma * eta[i] * eta[j] * v[j];
            }
        }
        hv[i] = s;
    }
}

/* R = m (U - Uold)/dt + r(U) for every order parameter */
int orc_gg_be_residual(const orc_gg_problem* p, double dt, const double* Uold, const double* U, double* R)
{
    const int64_t N = gg_nnodes(p);
    double* m = (double*)malloc((size_t)N * sizeof(double));
    orc_gg_lumped_mass(p, m);
    int rc = orc_gg_residual(p, U, R);
    for (int64_t k = 0; k < p->p * N; ++k) R[k] += m[k % N] * (U[k] - Uold[k]) / dt;
    free(m);
    return rc;
}

/* Jv = inv_dt m v + L [ sum_e sum_q detJ (H(eta_q) v_q)_i phi_a(q) + kappa K v_i ] */
int orc_gg_jvp(const orc_gg_problem* p, double inv_dt, const double* U, const double* v, double* Jv)
{
    gg_ref R;
    gg_ref_build(&R, p->dim, p->h);
    const int64_t N = gg_nnodes(p);
    const int P = p->p;
    if (P < 1 || P > 64) return -1;
    double eq[64], vq[64], gv[64][3], hv[64];
    int64_t E[3], idx[8];
    double* m = (double*)malloc((size_t)N * sizeof(double));
    orc_gg_lumped_mass(p, m);
    for (int64_t k = 0; k < P * N; ++k) Jv[k] = inv_dt * m[k % N] * v[k];
    free(m);
    GG_FOR_EACH_ELEMENT(p, E)
    {
        gg_elem_nodes(p, E, R.nv, idx);
        for (int q = 0; q < R.nv; ++q) {
            for (int i = 0; i < P; ++i) {
                eq[i] = vq[i] = 0.0;
                gv[i][0] = gv[i][1] = gv[i][2] = 0.0;
                for (int a = 0; a < R.nv; ++a) {
                    eq[i] += R.phi[q][a] * U[i * N + idx[a]];
                    vq[i] += R.phi[q][a] * v[i * N + idx[a]];
                    for (int k = 0; k < R.d; ++k) gv[i][k] += R.grad[q][a][k] * v[i * N + idx[a]];
                }
            }
            gg_hess_apply(p, eq, vq, hv);
            for (int i = 0; i < P; ++i)
                for (int a = 0; a < R.nv; ++a) {
                    double gg = 0.0;
                    for (int k = 0; k < R.d; ++k) gg += gv[i][k] * R.grad[q][a][k];
                    Jv[i * N + idx[a]] += p->L * R.detJ * (hv[i] * R.phi[q][a] + p->kappa * gg);
                }
        }
    }
    return 0;
}

/* one backward-Euler step by Newton with a dense Jacobian (columns from
 * orc_gg_jvp) and Gaussian elimination with partial pivoting; small grids only.
 * U holds the initial guess on entry.  Returns 0 on ||R|| <= rtol ||R_0||. */
int orc_gg_newton_be(const orc_gg_problem* p, double dt, const double* Uold, double* U, double rtol,
                     int maxit, int* its)
{
    const int64_t n = p->p * gg_nnodes(p);
    double* A = (double*)malloc((size_t)(n * n) * sizeof(double));
    double* Rv = (double*)malloc((size_t)n * sizeof(double));
    double* e = (double*)calloc((size_t)n, sizeof(double));
    double* col = (double*)malloc((size_t)n * sizeof(double));
    double r0 = -1.0;
    int k = 0, ok = 0;
    for (;; ++k) {
        orc_gg_be_residual(p, dt, Uold, U, Rv);
        double rn = 0.0;
        for (int64_t i = 0; i < n; ++i) rn += Rv[i] * Rv[i];
        rn = sqrt(rn);
        if (r0 < 0.0) r0 = rn;
        if (rn <= rtol * r0 || rn == 0.0) {
            ok = 1;
            break;
        }
        if (k >= maxit) break;
        for (int64_t j = 0; j < n; ++j) {
            e[j] = 1.0;
            orc_gg_jvp(p, 1.0 / dt, U, e, col);
            e[j] = 0.0;
            for (int64_t i = 0; i < n; ++i) A[i * n + j] = col[i];
        }
        /* solve A d = -R by elimination with partial pivoting */
        for (int64_t i = 0; i < n; ++i) Rv[i] = -Rv[i];
        for (int64_t c = 0; c < n; ++c) {
            int64_t piv = c;
            for (int64_t i = c + 1; i < n; ++i)
                if (fabs(A[i * n + c]) > fabs(A[piv * n + c])) piv = i;
            if (piv != c) {
                for (int64_t j = 0; j < n; ++j) {
                    const double t = A[c * n + j];
                    A[c * n + j] = A[piv * n + j];
                    A[piv * n + j] = t;
                }
                const double t = Rv[c];
                Rv[c] = Rv[piv];
                Rv[piv] = t;
            }
            for (int64_t i = c + 1; i < n; ++i) {
                const double l = A[i * n + c] / A[c * n + c];
                for (int64_t j = c; j < n; ++j) A[i * n + j] -= l * A[c * n + j];
                Rv[i] -= l * Rv[c];
            }
        }
        for (int64_t i = n - 1; i >= 0; --i) {
            double s = Rv[i];
            for (int64_t j = i + 1; j < n; ++j) s -= A[i * n + j] * Rv[j];
            Rv[i] = s / A[i * n + i];
        }
        for (int64_t i = 0; i < n; ++i) U[i] += Rv[i];
    }
    if (its) *its = k;
    free(col);
    free(e);
    free(Rv);
    free(A);
    return ok ? 0 : -1;
}
