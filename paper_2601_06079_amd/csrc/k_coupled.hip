// k_coupled.hip -- the coupled Allen-Cahn / Cahn-Hilliard model (Eq. 7) with the
// benchmark's free energies (Supp. Note 3), on 2-D and 3-D grids, periodic or
// no-flux.  States are [c ; mu ; eta].
//
//   F = int f_a(c) (1 - h(eta)) + f_b(c) h(eta) + kappa/2 |grad eta|^2   (no grad c term)
//   mu  = dF/dc:        m mu_a = sum_e sum_q |J| [f_a'(c_q)(1 - h) + f_b'(c_q) h] phi_a
//   eta (Allen-Cahn):   m d eta_a/dt = -M_eta sum_e sum_q |J| [(f_b - f_a)(c_q) h'(eta_q) phi_a
//                                                            + kappa grad eta_q . grad phi_a]
//   c (Cahn-Hilliard):  m dc_a/dt = -M_c (K mu)_a
//
// Node-centric like k_node.hip: one thread per node, 3^d neighbourhood, the 4^d
// quadrature values of its 2^d elements by sum factorisation; on no-flux grids
// reflected neighbours and rows divided by 2^b (see reflect in device.hpp).
#include <cmath>

#include "node_common.hpp"

namespace pfk {
namespace {

// the benchmark polynomials (Supp. Note 3), Horner form
template <typename T>
__device__ __forceinline__ T fa(T c)
{
    return fmaT(fmaT(fmaT(fmaT((T)1.3687, c, (T)-2.7375), c, (T)5.1622), c, (T)-4.776), c, (T)-1.6704);
}
template <typename T>
__device__ __forceinline__ T dfa(T c)
{
    return fmaT(fmaT(fmaT((T)(4 * 1.3687), c, (T)(-3 * 2.7375)), c, (T)(2 * 5.1622)), c, (T)-4.776);
}
template <typename T>
__device__ __forceinline__ T fb(T c)
{
    return fmaT(fmaT((T)5.0, c, (T)-5.9746), c, (T)-1.5924);
}
template <typename T>
__device__ __forceinline__ T dfb(T c)
{
    return fmaT((T)10.0, c, (T)-5.9746);
}
// h = eta^3 (10 - 15 eta + 6 eta^2), h' = 30 eta^2 (1 - eta)^2
template <typename T>
__device__ __forceinline__ T hfun(T e)
{
    return e * e * e * fmaT(fmaT((T)6, e, (T)-15), e, (T)10);
}
template <typename T>
__device__ __forceinline__ T dhfun(T e)
{
    const T t = e * ((T)1 - e);
    return (T)30 * t * t;
}

template <typename T>
struct MuSrc {  // f_a'(c)(1 - h(eta)) + f_b'(c) h(eta)
    __device__ T operator()(T c, T e) const
    {
        const T d = dfa(c);
        return fmaT(dfb(c) - d, hfun(e), d);
    }
};
template <typename T>
struct EtaSrc {  // (f_b(c) - f_a(c)) h'(eta)
    __device__ T operator()(T c, T e) const { return (fb(c) - fa(c)) * dhfun(e); }
};

// mu = g(c, eta) / m; with eta_out also the forward-Euler update
// eta_out = eta - dt M_eta [s(c, eta) + kappa K eta] / m.  Both are ratios of a row
// to the lumped mass, which need no boundary factor on no-flux grids.
template <typename T, int D>
__global__ __launch_bounds__(256) void k_cp_mu_eta(const T* __restrict__ c, const T* __restrict__ eta,
                                                   T* __restrict__ mu, T* __restrict__ eta_out, Geom g,
                                                   T detJ, T inv_m, T kappa, T dtMeta)
{
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int i, j, k;
    if (!node_of<D>(g, idx, i, j, k)) return;
    T u[NB<D>::K], e[NB<D>::K];
    gather<T, D>(c, g, i, j, k, u);
    gather<T, D>(eta, g, i, j, k, e);
    mu[idx] = detJ * quad_sum<T, D, true>(u, e, MuSrc<T>{}) * inv_m;
    if (eta_out) {
        const T s = detJ * quad_sum<T, D, true>(u, e, EtaSrc<T>{});
        const T ke = stiff<T, D>(e, (T)g.h);
        eta_out[idx] = e[NB<D>::K / 2] - dtMeta * inv_m * (s + kappa * ke);
    }
}

// r = [M_c K mu ;  m mu - g(c, eta) ;  M_eta (s(c, eta) + kappa K eta)], rows / 2^b on
// no-flux grids; with Uold the backward-Euler time term inv_dt m (U - Uold) is added
// to the c and eta rows (Eq. 14)
template <typename T, int D>
__global__ __launch_bounds__(256) void k_cp_residual(const T* __restrict__ U, const T* __restrict__ Uold,
                                                     T* __restrict__ r, Geom g, T detJ, T m, T kappa,
                                                     T Mc, T Meta, T inv_dt)
{
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int i, j, k;
    if (!node_of<D>(g, idx, i, j, k)) return;
    T u[NB<D>::K], w[NB<D>::K], e[NB<D>::K];
    gather<T, D>(U, g, i, j, k, u);
    gather<T, D>(U + g.N, g, i, j, k, w);
    gather<T, D>(U + 2 * g.N, g, i, j, k, e);
    const T h = (T)g.h;
    const T ib = (T)1 / (T)bfactor<D>(g, i, j, k);
    const T gsrc = detJ * quad_sum<T, D, true>(u, e, MuSrc<T>{});
    const T s = detJ * quad_sum<T, D, true>(u, e, EtaSrc<T>{});
    const T tc = Uold ? inv_dt * m * (u[NB<D>::K / 2] - Uold[idx]) : (T)0;
    const T te = Uold ? inv_dt * m * (e[NB<D>::K / 2] - Uold[2 * g.N + idx]) : (T)0;
    r[idx] = (Mc * stiff<T, D>(w, h) + tc) * ib;
    r[g.N + idx] = (m * w[NB<D>::K / 2] - gsrc) * ib;
    r[2 * g.N + idx] = (Meta * (s + kappa * stiff<T, D>(e, h)) + te) * ib;
}

// second derivatives of the local energy density f_a(c)(1 - h) + f_b(c) h
template <typename T>
__device__ __forceinline__ void hessian(T c, T e, T& gcc, T& gce, T& see)
{
    const T h = hfun(e), dh = dhfun(e);
    const T d2h = (T)60 * e * fmaT(fmaT((T)2, e, (T)-3), e, (T)1);  // 60e - 180e^2 + 120e^3
    const T d2fa = fmaT(fmaT((T)(12 * 1.3687), c, (T)(-6 * 2.7375)), c, (T)(2 * 5.1622));
    gcc = fmaT((T)10 - d2fa, h, d2fa);
    gce = (dfb(c) - dfa(c)) * dh;
    see = (fb(c) - fa(c)) * d2h;
}

// sum over the 4^D quadrature points around the centre node (weights as quad_sum)
// of the two Hessian-direction products
//   S1 = g_cc vc + g_ce ve  (mu row),  S2 = g_ce vc + s_ee ve  (eta row)
template <typename T, int D>
__device__ __forceinline__ void hess_sums(const T* c, const T* e, const T* vc, const T* ve, T& S1, T& S2)
{
    auto pt = [](T cq, T eq, T vcq, T veq, T& a, T& b) {
        T gcc, gce, see;
        hessian(cq, eq, gcc, gce, see);
        a = fmaT(gcc, vcq, gce * veq);
        b = fmaT(gce, vcq, see * veq);
    };
    if constexpr (D == 2) {
        T X[4][3][4];  // [field][row][qx]
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            interp3to4(c[3 * b], c[3 * b + 1], c[3 * b + 2], X[0][b]);
            interp3to4(e[3 * b], e[3 * b + 1], e[3 * b + 2], X[1][b]);
            interp3to4(vc[3 * b], vc[3 * b + 1], vc[3 * b + 2], X[2][b]);
            interp3to4(ve[3 * b], ve[3 * b + 1], ve[3 * b + 2], X[3][b]);
        }
        T col1[4], col2[4];
#pragma unroll
        for (int qx = 0; qx < 4; ++qx) {
            T q[4][4];
#pragma unroll
            for (int f = 0; f < 4; ++f) interp3to4(X[f][0][qx], X[f][1][qx], X[f][2][qx], q[f]);
            T a[4], bb[4];
#pragma unroll
            for (int qy = 0; qy < 4; ++qy) pt(q[0][qy], q[1][qy], q[2][qy], q[3][qy], a[qy], bb[qy]);
            col1[qx] = wsum4(a);
            col2[qx] = wsum4(bb);
        }
        S1 = wsum4(col1);
        S2 = wsum4(col2);
    } else {
        T X[4][9][4];  // [field][row (y,z)][qx]
#pragma unroll
        for (int r = 0; r < 9; ++r) {
            interp3to4(c[3 * r], c[3 * r + 1], c[3 * r + 2], X[0][r]);
            interp3to4(e[3 * r], e[3 * r + 1], e[3 * r + 2], X[1][r]);
            interp3to4(vc[3 * r], vc[3 * r + 1], vc[3 * r + 2], X[2][r]);
            interp3to4(ve[3 * r], ve[3 * r + 1], ve[3 * r + 2], X[3][r]);
        }
        T pl1[4], pl2[4];
#pragma unroll
        for (int qx = 0; qx < 4; ++qx) {
            T Y[4][3][4];  // [field][z][qy]
#pragma unroll
            for (int f = 0; f < 4; ++f)
#pragma unroll
                for (int zc = 0; zc < 3; ++zc)
                    interp3to4(X[f][3 * zc][qx], X[f][3 * zc + 1][qx], X[f][3 * zc + 2][qx], Y[f][zc]);
            T row1[4], row2[4];
#pragma unroll
            for (int qy = 0; qy < 4; ++qy) {
                T q[4][4];
#pragma unroll
                for (int f = 0; f < 4; ++f) interp3to4(Y[f][0][qy], Y[f][1][qy], Y[f][2][qy], q[f]);
                T a[4], bb[4];
#pragma unroll
                for (int qz = 0; qz < 4; ++qz) pt(q[0][qz], q[1][qz], q[2][qz], q[3][qz], a[qz], bb[qz]);
                row1[qy] = wsum4(a);
                row2[qy] = wsum4(bb);
            }
            pl1[qx] = wsum4(row1);
            pl2[qx] = wsum4(row2);
        }
        S1 = wsum4(pl1);
        S2 = wsum4(pl2);
    }
}

// Jv of R = inv_dt M (U - Uold) + r(U) at U, rows / 2^b on no-flux grids:
//   Jv_c   = inv_dt m v_c + M_c K v_mu
//   Jv_mu  = m v_mu - |J| S1
//   Jv_eta = inv_dt m v_eta + M_eta (|J| S2 + kappa K v_eta)
template <typename T, int D>
__global__ __launch_bounds__(256) void k_cp_jvp(const T* __restrict__ U, const T* __restrict__ V,
                                                T* __restrict__ Jv, Geom g, T detJ, T m, T kappa, T Mc,
                                                T Meta, T inv_dt)
{
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int i, j, k;
    if (!node_of<D>(g, idx, i, j, k)) return;
    T u[NB<D>::K], e[NB<D>::K], vc[NB<D>::K], vm[NB<D>::K], ve[NB<D>::K];
    gather<T, D>(U, g, i, j, k, u);
    gather<T, D>(U + 2 * g.N, g, i, j, k, e);
    gather<T, D>(V, g, i, j, k, vc);
    gather<T, D>(V + g.N, g, i, j, k, vm);
    gather<T, D>(V + 2 * g.N, g, i, j, k, ve);
    const T h = (T)g.h;
    const T ib = (T)1 / (T)bfactor<D>(g, i, j, k);
    T S1, S2;
    hess_sums<T, D>(u, e, vc, ve, S1, S2);
    constexpr int C = NB<D>::K / 2;
    Jv[idx] = (inv_dt * m * vc[C] + Mc * stiff<T, D>(vm, h)) * ib;
    Jv[g.N + idx] = (m * vm[C] - detJ * S1) * ib;
    Jv[2 * g.N + idx] = (inv_dt * m * ve[C] + Meta * (detJ * S2 + kappa * stiff<T, D>(ve, h))) * ib;
}

// 3x3 block-Jacobi inverse of dR/dU at each node (row-major, 9 values per node):
//   [[inv_dt m, M_c K_aa, 0], [-|J| Dcc, m, -|J| Dce], [M_eta |J| Dce, 0, inv_dt m + M_eta (|J| Dee + kappa K_aa)]]
// with D.. = sum_q (second derivative at q) phi_a(q)^2; rows / 2^b on no-flux grids.
template <typename T, int D>
__global__ __launch_bounds__(256) void k_cp_prec(const T* __restrict__ U, T* __restrict__ pinv, Geom g,
                                                 T detJ, T m, T kappa, T Mc, T Meta, T inv_dt)
{
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int i, j, k;
    if (!node_of<D>(g, idx, i, j, k)) return;
    T u[NB<D>::K], e[NB<D>::K];
    gather<T, D>(U, g, i, j, k, u);
    gather<T, D>(U + 2 * g.N, g, i, j, k, e);
    struct Gcc { __device__ T operator()(T c, T ee) const { T a, b, d; hessian(c, ee, a, b, d); return a; } };
    struct Gce { __device__ T operator()(T c, T ee) const { T a, b, d; hessian(c, ee, a, b, d); return b; } };
    struct See { __device__ T operator()(T c, T ee) const { T a, b, d; hessian(c, ee, a, b, d); return d; } };
    // quad_sum_sq evaluates F(u_q, 1); the second field is needed here, so the
    // squared-weight sums are formed with a two-field quadrature of F(c, eta) * 1
    const double dcc = (double)detJ * (double)quad_sum_sq2<T, D>(u, e, Gcc{});
    const double dce = (double)detJ * (double)quad_sum_sq2<T, D>(u, e, Gce{});
    const double dee = (double)detJ * (double)quad_sum_sq2<T, D>(u, e, See{});
    const double kd = (double)stiff_diag<T, D>((T)g.h);
    const double ib = 1.0 / bfactor<D>(g, i, j, k);
    double A[3][3] = {{(double)inv_dt * m, (double)Mc * kd, 0.0},
                      {-dcc, (double)m, -dce},
                      {(double)Meta * dce, 0.0, (double)inv_dt * m + (double)Meta * (dee + (double)kappa * kd)}};
    for (int r = 0; r < 3; ++r)
        for (int cc = 0; cc < 3; ++cc) A[r][cc] *= ib;
    // inverse by cofactors
    const double c00 = A[1][1] * A[2][2] - A[1][2] * A[2][1];
    const double c01 = A[1][2] * A[2][0] - A[1][0] * A[2][2];
    const double c02 = A[1][0] * A[2][1] - A[1][1] * A[2][0];
    const double det = A[0][0] * c00 + A[0][1] * c01 + A[0][2] * c02;
    const double id = 1.0 / det;
    T* P = pinv + 9 * idx;
    P[0] = (T)(c00 * id);
    P[1] = (T)((A[0][2] * A[2][1] - A[0][1] * A[2][2]) * id);
    P[2] = (T)((A[0][1] * A[1][2] - A[0][2] * A[1][1]) * id);
    P[3] = (T)(c01 * id);
    P[4] = (T)((A[0][0] * A[2][2] - A[0][2] * A[2][0]) * id);
    P[5] = (T)((A[0][2] * A[1][0] - A[0][0] * A[1][2]) * id);
    P[6] = (T)(c02 * id);
    P[7] = (T)((A[0][1] * A[2][0] - A[0][0] * A[2][1]) * id);
    P[8] = (T)((A[0][0] * A[1][1] - A[0][1] * A[1][0]) * id);
}

// ---- energy and mass (FP64): each thread owns the element whose lower corner is
// its node (none past the upper boundary of a no-flux grid) and its node's mass.
__device__ __forceinline__ double cp_density(double c, double e)
{
    const double h = hfun(e);
    return fa(c) * (1.0 - h) + fb(c) * h;
}

constexpr int EB = 256;

template <typename T, int D>
__global__ __launch_bounds__(EB) void k_cp_energy(const T* __restrict__ U, double* __restrict__ part,
                                                  Geom g, double kappa)
{
    const long long idx = (long long)blockIdx.x * EB + threadIdx.x;
    double en = 0.0, ms = 0.0;
    int i, j, k;
    if (node_of<D>(g, idx, i, j, k)) {
        const T* c = U;
        const T* eta = U + 2 * g.N;
        const double h = g.h;
        const double B[2][2] = {{GP, GM}, {GM, GP}};
        const int xs[2] = {i, wrap(i + 1, g.n[0])}, ys[2] = {j, wrap(j + 1, g.n[1])};
        const int zs[2] = {k, D == 3 ? wrap(k + 1, g.n[2]) : k};
        constexpr int NZ = D == 3 ? 2 : 1;
        double cv[2][2][2], ev[2][2][2];  // [az][ay][ax]
        for (int az = 0; az < NZ; ++az)
            for (int ay = 0; ay < 2; ++ay)
                for (int ax = 0; ax < 2; ++ax) {
                    const long long o = ((long long)zs[az] * g.n[1] + ys[ay]) * g.n[0] + xs[ax];
                    cv[az][ay][ax] = c[o];
                    ev[az][ay][ax] = eta[o];
                }
        const double detJ = D == 2 ? 0.25 * h * h : 0.125 * h * h * h;
        for (int qz = 0; qz < NZ; ++qz)
            for (int qy = 0; qy < 2; ++qy)
                for (int qx = 0; qx < 2; ++qx) {
                    double cq = 0.0, eq = 0.0, gr[3] = {0.0, 0.0, 0.0};
                    for (int az = 0; az < NZ; ++az)
                        for (int ay = 0; ay < 2; ++ay)
                            for (int ax = 0; ax < 2; ++ax) {
                                const double bz = D == 3 ? B[qz][az] : 1.0;
                                const double sx = ax ? 1.0 : -1.0, sy = ay ? 1.0 : -1.0,
                                             sz = az ? 1.0 : -1.0;
                                const double wv = B[qx][ax] * B[qy][ay] * bz;
                                cq += wv * cv[az][ay][ax];
                                eq += wv * ev[az][ay][ax];
                                gr[0] += sx / h * B[qy][ay] * bz * ev[az][ay][ax];
                                gr[1] += sy / h * B[qx][ax] * bz * ev[az][ay][ax];
                                if (D == 3) gr[2] += sz / h * B[qx][ax] * B[qy][ay] * ev[az][ay][ax];
                            }
                    en += detJ * (cp_density(cq, eq) +
                                  0.5 * kappa * (gr[0] * gr[0] + gr[1] * gr[1] + gr[2] * gr[2]));
                }
        const double mnode = D == 2 ? h * h : h * h * h;
        ms = mnode * (double)cv[0][0][0];
        if (g.bc) {
            const bool elem = i + 1 < g.n[0] && j + 1 < g.n[1] && (D == 2 || k + 1 < g.n[2]);
            if (!elem) en = 0.0;
            ms /= bfactor<D>(g, i, j, k);
        }
    }
    // block reduction in a fixed order
    __shared__ double se[EB / WAVE], sm[EB / WAVE];
    for (int off = WAVE / 2; off > 0; off >>= 1) {
        en += __shfl_down(en, off, WAVE);
        ms += __shfl_down(ms, off, WAVE);
    }
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    if (lane == 0) {
        se[wv] = en;
        sm[wv] = ms;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int w = 0; w < EB / WAVE; ++w) {
            a += se[w];
            b += sm[w];
        }
        part[2 * blockIdx.x] = a;
        part[2 * blockIdx.x + 1] = b;
    }
}

inline unsigned blocks_for(const Geom& g) { return (unsigned)((g.N + 255) / 256); }

#define CP_DIM(g, ...)           \
    if ((g).dim == 2) {          \
        constexpr int D = 2;     \
        __VA_ARGS__;             \
    } else {                     \
        constexpr int D = 3;     \
        __VA_ARGS__;             \
    }

}  // namespace

template <typename T>
void launch_cp_mu_eta(const Geom& g, double kappa, double dt_Meta, const T* c, const T* eta, T* mu,
                      T* eta_out, hipStream_t s)
{
    const double detJ = std::pow(0.5 * g.h, g.dim), m = std::pow(g.h, g.dim);
    CP_DIM(g, {
        k_cp_mu_eta<T, D><<<blocks_for(g), 256, 0, s>>>(c, eta, mu, eta_out, g, (T)detJ, (T)(1.0 / m),
                                                         (T)kappa, (T)dt_Meta);
    });
}

template <typename T>
void launch_cp_residual(const Geom& g, double kappa, double Mc, double Meta, const T* U, T* r,
                        hipStream_t s, const T* Uold, double inv_dt)
{
    const double detJ = std::pow(0.5 * g.h, g.dim), m = std::pow(g.h, g.dim);
    CP_DIM(g, {
        k_cp_residual<T, D><<<blocks_for(g), 256, 0, s>>>(U, Uold, r, g, (T)detJ, (T)m, (T)kappa, (T)Mc,
                                                           (T)Meta, (T)inv_dt);
    });
}

template <typename T>
void launch_cp_jvp(const Geom& g, double kappa, double Mc, double Meta, double inv_dt, const T* U,
                   const T* v, T* Jv, hipStream_t s)
{
    const double detJ = std::pow(0.5 * g.h, g.dim), m = std::pow(g.h, g.dim);
    CP_DIM(g, {
        k_cp_jvp<T, D><<<blocks_for(g), 256, 0, s>>>(U, v, Jv, g, (T)detJ, (T)m, (T)kappa, (T)Mc,
                                                      (T)Meta, (T)inv_dt);
    });
}

template <typename T>
void launch_cp_prec(const Geom& g, double kappa, double Mc, double Meta, double inv_dt, const T* U,
                    T* pinv, hipStream_t s)
{
    const double detJ = std::pow(0.5 * g.h, g.dim), m = std::pow(g.h, g.dim);
    CP_DIM(g, {
        k_cp_prec<T, D><<<blocks_for(g), 256, 0, s>>>(U, pinv, g, (T)detJ, (T)m, (T)kappa, (T)Mc,
                                                       (T)Meta, (T)inv_dt);
    });
}

template <typename T>
void launch_cp_energy(const Geom& g, double kappa, const T* U, double* partials, double* out,
                      hipStream_t s)
{
    const int nb = (int)((g.N + EB - 1) / EB);
    CP_DIM(g, { k_cp_energy<T, D><<<nb, EB, 0, s>>>(U, partials, g, kappa); });
    launch_reduce_pairs(partials, nb, out, s);
}

#define INST_CP(T)                                                                                 \
    template void launch_cp_mu_eta<T>(const Geom&, double, double, const T*, const T*, T*, T*,     \
                                      hipStream_t);                                                \
    template void launch_cp_residual<T>(const Geom&, double, double, double, const T*, T*,         \
                                        hipStream_t, const T*, double);                            \
    template void launch_cp_jvp<T>(const Geom&, double, double, double, double, const T*, const T*, \
                                   T*, hipStream_t);                                               \
    template void launch_cp_prec<T>(const Geom&, double, double, double, double, const T*, T*,     \
                                    hipStream_t);                                                  \
    template void launch_cp_energy<T>(const Geom&, double, const T*, double*, double*, hipStream_t);
INST_CP(float)
INST_CP(double)

}  // namespace pfk
