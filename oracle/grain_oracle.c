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
