/*
 * coupled_oracle.c -- plain, slow, FP64 CPU reference of the coupled
 * Allen-Cahn / Cahn-Hilliard model.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite may.  It shares no code, header, table
 * or constant with the HIP library.
 *
 * Model (paper section / equation in brackets):
 *   - free energy  F = int f_a(c) (1 - h(eta)) + f_b(c) h(eta) + kappa_eta/2 |grad eta|^2
 *                  (composition gradients neglected)                        [Sec. 2.1, Eq. 7]
 *   - benchmark polynomials, mobilities and kappa_eta                       [Supp. Note 3]
 *       f_a(c) = -1.6704 - 4.776 c + 5.1622 c^2 - 2.7375 c^3 + 1.3687 c^4
 *       f_b(c) = 5.0 c^2 - 5.9746 c - 1.5924
 *       h(eta) = 10 eta^3 - 15 eta^4 + 6 eta^5
 *   - order parameter (Allen-Cahn)    d eta/dt = -M_eta dF/d eta            [Eq. 1]
 *   - composition (Cahn-Hilliard)     dc/dt = div(M_c grad mu), mu = dF/dc  [Eqs. 2, 9-10]
 *   - lumped-mass semi-discrete form and forward-Euler step                 [Eqs. 11-12]
 *
 * Discretisation as in pf_oracle.c: Q1 elements on a uniform grid, 2-point
 * Gauss-Legendre quadrature per axis, row-sum lumped mass, periodic or no-flux
 * (natural) boundaries.  States are laid out as [c ; mu ; eta] (N values each).
 *
 *   r_c   = M_c sum_e sum_q |J| grad mu_q . grad phi_a
 *   r_mu  = m_a mu_a - sum_e sum_q |J| [f_a'(c_q)(1 - h(eta_q)) + f_b'(c_q) h(eta_q)] phi_a(q)
 *   r_eta = M_eta sum_e sum_q |J| [(f_b(c_q) - f_a(c_q)) h'(eta_q) phi_a(q)
 *                                  + kappa_eta grad eta_q . grad phi_a(q)]
 * Explicit step: mu <- g(c, eta)/m from the old state, then c <- c - dt r_c(mu)/m and
 * eta <- eta - dt r_eta(c_old, eta_old)/m; mu is recomputed from the new state at
 * the end of the call.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t dim;   /* 2 or 3 */
    int32_t bc;    /* 0 periodic, 1 no-flux */
    int64_t n[3];  /* nodes per axis; n[2] = 1 in 2-D */
    double h;      /* grid spacing */
    double Mc;     /* composition mobility */
    double Meta;   /* order-parameter mobility */
    double kappa;  /* kappa_eta */
} orc_cp_problem;

/* ---- the benchmark's local free energies and interpolation function ------- */
double orc_cp_fa(double c)
{
    return -1.6704 - 4.776 * c + 5.1622 * c * c - 2.7375 * c * c * c + 1.3687 * c * c * c * c;
}
double orc_cp_dfa(double c)
{
    return -4.776 + 2.0 * 5.1622 * c - 3.0 * 2.7375 * c * c + 4.0 * 1.3687 * c * c * c;
}
double orc_cp_fb(double c) { return 5.0 * c * c - 5.9746 * c - 1.5924; }
double orc_cp_dfb(double c) { return 10.0 * c - 5.9746; }
double orc_cp_h(double e) { return 10.0 * e * e * e - 15.0 * e * e * e * e + 6.0 * e * e * e * e * e; }
double orc_cp_dh(double e) { return 30.0 * e * e - 60.0 * e * e * e + 30.0 * e * e * e * e; }

/* ---- grid and reference element ------------------------------------------- */
static int64_t cp_nnodes(const orc_cp_problem* p)
{
    int64_t N = 1;
    for (int k = 0; k < p->dim; ++k) N *= p->n[k];
    return N;
}

static int64_t cp_elems(const orc_cp_problem* p, int k)
{
    if (k >= p->dim) return 1;
    return p->bc == 0 ? p->n[k] : p->n[k] - 1;
}

typedef struct {
    int d, nv;
    double detJ;
    double phi[8][8];     /* phi[q][a] */
    double grad[8][8][3]; /* grad[q][a][k] */
} cp_ref;

static void cp_ref_build(cp_ref* R, int d, double h)
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
                double gk = s[k] / h; /* d/dx of (1 + s xi)/2 with dxi/dx = 2/h */
                for (int l = 0; l < d; ++l)
                    if (l != k) gk *= f[l];
                R->grad[q][a][k] = gk;
            }
        }
}

static void cp_elem_nodes(const orc_cp_problem* p, const int64_t e[3], int nv, int64_t* idx)
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

#define CP_FOR_EACH_ELEMENT(p, E)                       \
    for (E[2] = 0; E[2] < cp_elems(p, 2); ++E[2])       \
        for (E[1] = 0; E[1] < cp_elems(p, 1); ++E[1])   \
            for (E[0] = 0; E[0] < cp_elems(p, 0); ++E[0])

int orc_cp_lumped_mass(const orc_cp_problem* p, double* m)
{
    cp_ref R;
    cp_ref_build(&R, p->dim, p->h);
    int64_t E[3], idx[8];
    memset(m, 0, (size_t)cp_nnodes(p) * sizeof(double));
    CP_FOR_EACH_ELEMENT(p, E)
    {
        cp_elem_nodes(p, E, R.nv, idx);
        for (int q = 0; q < R.nv; ++q)
            for (int a = 0; a < R.nv; ++a) m[idx[a]] += R.detJ * R.phi[q][a];
    }
    return 0;
}

/* g_a = sum_e sum_q |J| [f_a'(c_q)(1 - h(eta_q)) + f_b'(c_q) h(eta_q)] phi_a     (dF/dc)
 * s_a = sum_e sum_q |J| [(f_b - f_a)(c_q) h'(eta_q) phi_a + kappa grad eta_q . grad phi_a]
 *                                                                          (dF/d eta) */
static void cp_assemble_g_s(const orc_cp_problem* p, const double* c, const double* eta,
                            double* g, double* s)
{
    cp_ref R;
    cp_ref_build(&R, p->dim, p->h);
    const int64_t N = cp_nnodes(p);
    if (g) memset(g, 0, (size_t)N * sizeof(double));
    if (s) memset(s, 0, (size_t)N * sizeof(double));
    int64_t E[3], idx[8];
    CP_FOR_EACH_ELEMENT(p, E)
    {
        cp_elem_nodes(p, E, R.nv, idx);
        for (int q = 0; q < R.nv; ++q) {
            double cq = 0.0, eq = 0.0, ge[3] = {0.0, 0.0, 0.0};
            for (int a = 0; a < R.nv; ++a) {
                cq += R.phi[q][a] * c[idx[a]];
                eq += R.phi[q][a] * eta[idx[a]];
                for (int k = 0; k < R.d; ++k) ge[k] += R.grad[q][a][k] * eta[idx[a]];
            }
            const double hq = orc_cp_h(eq);
            const double gq = orc_cp_dfa(cq) * (1.0 - hq) + orc_cp_dfb(cq) * hq;
            const double sq = (orc_cp_fb(cq) - orc_cp_fa(cq)) * orc_cp_dh(eq);
            for (int a = 0; a < R.nv; ++a) {
                if (g) g[idx[a]] += R.detJ * gq * R.phi[q][a];
                if (s) {
                    double gg = 0.0;
                    for (int k = 0; k < R.d; ++k) gg += ge[k] * R.grad[q][a][k];
                    s[idx[a]] += R.detJ * (sq * R.phi[q][a] + p->kappa * gg);
                }
            }
        }
    }
}

/* out_a = sum_e sum_q |J| grad u_q . grad phi_a  (the Q1 stiffness applied to u) */
static void cp_stiffness(const orc_cp_problem* p, const double* u, double* out)
{
    cp_ref R;
    cp_ref_build(&R, p->dim, p->h);
    memset(out, 0, (size_t)cp_nnodes(p) * sizeof(double));
    int64_t E[3], idx[8];
    CP_FOR_EACH_ELEMENT(p, E)
    {
        cp_elem_nodes(p, E, R.nv, idx);
        for (int q = 0; q < R.nv; ++q) {
            double gu[3] = {0.0, 0.0, 0.0};
            for (int a = 0; a < R.nv; ++a)
                for (int k = 0; k < R.d; ++k) gu[k] += R.grad[q][a][k] * u[idx[a]];
            for (int a = 0; a < R.nv; ++a) {
                double gg = 0.0;
                for (int k = 0; k < R.d; ++k) gg += gu[k] * R.grad[q][a][k];
                out[idx[a]] += R.detJ * gg;
            }
        }
    }
}

int orc_cp_residual(const orc_cp_problem* p, const double* U, double* r)
{
    const int64_t N = cp_nnodes(p);
    const double *c = U, *mu = U + N, *eta = U + 2 * N;
    double* m = (double*)malloc((size_t)N * sizeof(double));
    double* g = (double*)malloc((size_t)N * sizeof(double));
    orc_cp_lumped_mass(p, m);
    cp_stiffness(p, mu, r);
    cp_assemble_g_s(p, c, eta, g, r + 2 * N);
    for (int64_t i = 0; i < N; ++i) {
        r[i] *= p->Mc;
        r[N + i] = m[i] * mu[i] - g[i];
        r[2 * N + i] *= p->Meta;
    }
    free(g);
    free(m);
    return 0;
}

int orc_cp_explicit(const orc_cp_problem* p, double dt, int64_t nsteps, double* U)
{
    const int64_t N = cp_nnodes(p);
    double *c = U, *mu = U + N, *eta = U + 2 * N;
    double* m = (double*)malloc((size_t)N * sizeof(double));
    double* g = (double*)malloc((size_t)N * sizeof(double));
    double* s = (double*)malloc((size_t)N * sizeof(double));
    double* kmu = (double*)malloc((size_t)N * sizeof(double));
    orc_cp_lumped_mass(p, m);
    for (int64_t st = 0; st <= nsteps; ++st) {
        cp_assemble_g_s(p, c, eta, g, st < nsteps ? s : NULL);
        for (int64_t i = 0; i < N; ++i) mu[i] = g[i] / m[i];
        if (st == nsteps) break;
        cp_stiffness(p, mu, kmu);
        for (int64_t i = 0; i < N; ++i) {
            c[i] -= dt * p->Mc * kmu[i] / m[i];
            eta[i] -= dt * p->Meta * s[i] / m[i];
        }
    }
    free(kmu);
    free(s);
    free(g);
    free(m);
    return 0;
}

/* E_h = sum_e sum_q |J| [f_a(c_q)(1 - h(eta_q)) + f_b(c_q) h(eta_q) + kappa/2 |grad eta_q|^2] */
double orc_cp_energy(const orc_cp_problem* p, const double* U)
{
    const int64_t N = cp_nnodes(p);
    const double *c = U, *eta = U + 2 * N;
    cp_ref R;
    cp_ref_build(&R, p->dim, p->h);
    double sum = 0.0;
    int64_t E[3], idx[8];
    CP_FOR_EACH_ELEMENT(p, E)
    {
        cp_elem_nodes(p, E, R.nv, idx);
        for (int q = 0; q < R.nv; ++q) {
            double cq = 0.0, eq = 0.0, ge[3] = {0.0, 0.0, 0.0};
            for (int a = 0; a < R.nv; ++a) {
                cq += R.phi[q][a] * c[idx[a]];
                eq += R.phi[q][a] * eta[idx[a]];
                for (int k = 0; k < R.d; ++k) ge[k] += R.grad[q][a][k] * eta[idx[a]];
            }
            double g2 = 0.0;
            for (int k = 0; k < R.d; ++k) g2 += ge[k] * ge[k];
            const double hq = orc_cp_h(eq);
            sum += R.detJ * (orc_cp_fa(cq) * (1.0 - hq) + orc_cp_fb(cq) * hq + 0.5 * p->kappa * g2);
        }
    }
    return sum;
}

/* sum_a m_a c_a (the conserved composition) */
double orc_cp_total_mass(const orc_cp_problem* p, const double* U)
{
    const int64_t N = cp_nnodes(p);
    double* m = (double*)malloc((size_t)N * sizeof(double));
    orc_cp_lumped_mass(p, m);
    double s = 0.0;
    for (int64_t i = 0; i < N; ++i) s += m[i] * U[i];
    free(m);
    return s;
}

/* ------------------------------------------------------------------------ */
/* backward Euler (Eqs. 13-14) for the coupled model                         */
/* ------------------------------------------------------------------------ */
/* second derivatives of the benchmark polynomials */
double orc_cp_d2fa(double c) { return 2.0 * 5.1622 - 6.0 * 2.7375 * c + 12.0 * 1.3687 * c * c; }
double orc_cp_d2fb(double c) { (void)c; return 10.0; }
double orc_cp_d2h(double e) { return 60.0 * e - 180.0 * e * e + 120.0 * e * e * e; }

/* R = M (U - U_old)/dt + r(U), mass on the c and eta rows */
int orc_cp_be_residual(const orc_cp_problem* p, double dt, const double* Uold, const double* U,
                       double* R)
{
    const int64_t N = cp_nnodes(p);
    double* m = (double*)malloc((size_t)N * sizeof(double));
    orc_cp_lumped_mass(p, m);
    orc_cp_residual(p, U, R);
    for (int64_t i = 0; i < N; ++i) {
        R[i] += m[i] * (U[i] - Uold[i]) / dt;
        R[2 * N + i] += m[i] * (U[2 * N + i] - Uold[2 * N + i]) / dt;
    }
    free(m);
    return 0;
}

/* Jv = (dR/dU) v, R = inv_dt M (U - U_old) + r(U):
 *   Jv_c   = inv_dt m v_c + M_c K v_mu
 *   Jv_mu  = m v_mu - sum_q |J| [g_cc v_c,q + g_ce v_eta,q] phi_a
 *   Jv_eta = inv_dt m v_eta + M_eta [ sum_q |J| (g_ce v_c,q + s_ee v_eta,q) phi_a + kappa K v_eta ]
 * with g_cc = f_a''(1 - h) + f_b'' h, g_ce = (f_b' - f_a') h', s_ee = (f_b - f_a) h''. */
int orc_cp_jvp(const orc_cp_problem* p, double inv_dt, const double* U, const double* v, double* Jv)
{
    const int64_t N = cp_nnodes(p);
    const double *c = U, *eta = U + 2 * N;
    const double *vc = v, *vm = v + N, *ve = v + 2 * N;
    cp_ref R;
    cp_ref_build(&R, p->dim, p->h);
    double* m = (double*)malloc((size_t)N * sizeof(double));
    orc_cp_lumped_mass(p, m);
    memset(Jv, 0, (size_t)(3 * N) * sizeof(double));
    cp_stiffness(p, vm, Jv); /* K v_mu into the c rows */
    int64_t E[3], idx[8];
    CP_FOR_EACH_ELEMENT(p, E)
    {
        cp_elem_nodes(p, E, R.nv, idx);
        for (int q = 0; q < R.nv; ++q) {
            double cq = 0.0, eq = 0.0, vcq = 0.0, veq = 0.0, gv[3] = {0.0, 0.0, 0.0};
            for (int a = 0; a < R.nv; ++a) {
                cq += R.phi[q][a] * c[idx[a]];
                eq += R.phi[q][a] * eta[idx[a]];
                vcq += R.phi[q][a] * vc[idx[a]];
                veq += R.phi[q][a] * ve[idx[a]];
                for (int k = 0; k < R.d; ++k) gv[k] += R.grad[q][a][k] * ve[idx[a]];
            }
            const double h = orc_cp_h(eq), dh = orc_cp_dh(eq), d2h = orc_cp_d2h(eq);
            const double gcc = orc_cp_d2fa(cq) * (1.0 - h) + orc_cp_d2fb(cq) * h;
            const double gce = (orc_cp_dfb(cq) - orc_cp_dfa(cq)) * dh;
            const double see = (orc_cp_fb(cq) - orc_cp_fa(cq)) * d2h;
            for (int a = 0; a < R.nv; ++a) {
                double gg = 0.0;
                for (int k = 0; k < R.d; ++k) gg += gv[k] * R.grad[q][a][k];
                Jv[N + idx[a]] -= R.detJ * (gcc * vcq + gce * veq) * R.phi[q][a];
                Jv[2 * N + idx[a]] +=
                    p->Meta * R.detJ * ((gce * vcq + see * veq) * R.phi[q][a] + p->kappa * gg);
            }
        }
    }
    for (int64_t i = 0; i < N; ++i) {
        Jv[i] = p->Mc * Jv[i] + inv_dt * m[i] * vc[i];
        Jv[N + i] += m[i] * vm[i];
        Jv[2 * N + i] += inv_dt * m[i] * ve[i];
    }
    free(m);
    return 0;
}

/* dense LU with partial pivoting, in place; x <- A^-1 b.  Returns 0 or -1 (singular). */
static int cp_dense_solve(int64_t n, double* A, double* b)
{
    int64_t* piv = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    for (int64_t k = 0; k < n; ++k) {
        int64_t pr = k;
        for (int64_t i = k + 1; i < n; ++i)
            if (fabs(A[i * n + k]) > fabs(A[pr * n + k])) pr = i;
        if (A[pr * n + k] == 0.0) {
            free(piv);
            return -1;
        }
        piv[k] = pr;
        if (pr != k) {
            for (int64_t j = 0; j < n; ++j) {
                const double t = A[k * n + j];
                A[k * n + j] = A[pr * n + j];
                A[pr * n + j] = t;
            }
            const double t = b[k];
            b[k] = b[pr];
            b[pr] = t;
        }
        for (int64_t i = k + 1; i < n; ++i) {
            const double l = A[i * n + k] / A[k * n + k];
            A[i * n + k] = l;
            for (int64_t j = k + 1; j < n; ++j) A[i * n + j] -= l * A[k * n + j];
            b[i] -= l * b[k];
        }
    }
    for (int64_t i = n - 1; i >= 0; --i) {
        double s = b[i];
        for (int64_t j = i + 1; j < n; ++j) s -= A[i * n + j] * b[j];
        b[i] = s / A[i * n + i];
    }
    free(piv);
    return 0;
}

/* One backward-Euler step by Newton from U (initial guess, in place), dense LU of
 * the assembled Jacobian (columns from orc_cp_jvp on unit vectors): small grids
 * only.  Stops at ||R|| <= rtol ||R(U_start)||.  Returns 0 when converged. */
int orc_cp_newton_be(const orc_cp_problem* p, double dt, const double* Uold, double* U, double rtol,
                     int maxit, int* its)
{
    const int64_t n = 3 * cp_nnodes(p);
    double* R = (double*)malloc((size_t)n * sizeof(double));
    double* A = (double*)malloc((size_t)(n * n) * sizeof(double));
    double* e = (double*)calloc((size_t)n, sizeof(double));
    double* col = (double*)malloc((size_t)n * sizeof(double));
    int k = 0, rc = -1;
    orc_cp_be_residual(p, dt, Uold, U, R);
    double r0 = 0.0;
    for (int64_t i = 0; i < n; ++i) r0 += R[i] * R[i];
    r0 = sqrt(r0);
    double rk = r0;
    for (; k <= maxit; ++k) {
        if (rk <= rtol * r0 || rk == 0.0) {
            rc = 0;
            break;
        }
        if (k == maxit) break;
        for (int64_t j = 0; j < n; ++j) {
            e[j] = 1.0;
            orc_cp_jvp(p, 1.0 / dt, U, e, col);
            e[j] = 0.0;
            for (int64_t i = 0; i < n; ++i) A[i * n + j] = col[i];
        }
        for (int64_t i = 0; i < n; ++i) R[i] = -R[i];
        if (cp_dense_solve(n, A, R)) break;
        for (int64_t i = 0; i < n; ++i) U[i] += R[i];
        orc_cp_be_residual(p, dt, Uold, U, R);
        rk = 0.0;
        for (int64_t i = 0; i < n; ++i) rk += R[i] * R[i];
        rk = sqrt(rk);
    }
    if (its) *its = k;
    free(col);
    free(e);
    free(A);
    free(R);
    return rc;
}
