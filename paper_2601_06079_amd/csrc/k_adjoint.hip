// k_adjoint.hip -- vector-Jacobian products for sensitivities (Eq. 18,
// Supp. Note 2 Eqs. II.1-II.6).
//
// Parameter derivatives of r(U, theta), theta = (mobility, kappa, W); both
// free energies are linear in W, so N_W(u) = W N_1(u):
//   Allen-Cahn    r = L [W N_1(eta) + kappa K eta]
//                   dr/dL = W N_1 + kappa K eta,  dr/dkappa = L K eta,  dr/dW = L N_1
//   Cahn-Hilliard r_c = M K mu, r_mu = m mu - [W N_1(c) + kappa K c]
//                   dr_c/dM = K mu,  dr_mu/dkappa = -K c,  dr_mu/dW = -N_1(c)
// theta_bar accumulates w^T dr/dtheta in FP64: per-block partials, then one
// fixed-order reduction per parameter (bitwise reproducible).
#include <cmath>

#include "node_common.hpp"

namespace pfk {
namespace {

constexpr int AB = 256;

// block sum of 3 doubles, written as part[i * gridDim.x + blockIdx.x]
__device__ __forceinline__ void block_partials3(double a0, double a1, double a2, double* part)
{
    __shared__ double sh[AB / WAVE][3];
    double v[3] = {a0, a1, a2};
#pragma unroll
    for (int i = 0; i < 3; ++i)
        for (int off = WAVE / 2; off > 0; off >>= 1) v[i] += __shfl_down(v[i], off, WAVE);
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    if (lane == 0)
        for (int i = 0; i < 3; ++i) sh[wv][i] = v[i];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int i = 0; i < 3; ++i) {
            double s = 0.0;
            for (int w = 0; w < AB / WAVE; ++w) s += sh[w][i];
            part[(long long)i * gridDim.x + blockIdx.x] = s;
        }
}

__global__ __launch_bounds__(AB) void k_reduce3(const double* __restrict__ part, int nb,
                                                double* __restrict__ out)
{
    __shared__ double sh[AB];
    for (int i = 0; i < 3; ++i) {
        double a = 0.0;
        for (int b = threadIdx.x; b < nb; b += AB) a += part[(long long)i * nb + b];
        sh[threadIdx.x] = a;
        __syncthreads();
        for (int s = AB / 2; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[i] += sh[0];
        __syncthreads();
    }
}

// theta partials of scale * w^T dr/dtheta at U
template <typename T, int D, int MODEL>
__global__ __launch_bounds__(AB) void k_dtheta(const T* __restrict__ U, const T* __restrict__ w,
                                               Geom g, Cub<T> F1, T detJ, T W, T kappa, T mob,
                                               double scale, double* __restrict__ part)
{
    const long long idx = (long long)blockIdx.x * AB + threadIdx.x;
    double t0 = 0.0, t1 = 0.0, t2 = 0.0;
    int i, j, k;
    if (node_of<D>(g, idx, i, j, k)) {
        T u[NB<D>::K];
        gather<T, D>(U, g, i, j, k, u);
        const T h = (T)g.h;
        const double n1 = (double)(detJ * quad_sum<T, D, false>(u, u, F1));
        const double ku = (double)stiff<T, D>(u, h);
        scale /= bfactor<D>(g, i, j, k);  // no-flux rows (1 on periodic grids)
        if constexpr (MODEL == 0) {
            const double wi = scale * (double)w[idx];
            t0 = wi * ((double)W * n1 + (double)kappa * ku);
            t1 = wi * (double)mob * ku;
            t2 = wi * (double)mob * n1;
        } else {
            T mu[NB<D>::K];
            gather<T, D>(U + g.N, g, i, j, k, mu);
            const double wc = scale * (double)w[idx], wm = scale * (double)w[g.N + idx];
            t0 = wc * (double)stiff<T, D>(mu, h);
            t1 = -wm * ku;
            t2 = -wm * n1;
        }
    }
    block_partials3(t0, t1, t2, part);
}

// Ubar[a] += inv_dt (M lambda)[a] on the first N entries (the rows with mass);
// c = inv_dt h^d, lumped m_a = h^d / 2^b on a no-flux grid; g.cm: the consistent
// mass (symmetric, so M^T lambda = M lambda), inv_dt passed as cdt
template <typename T, int D>
__global__ __launch_bounds__(AB) void k_mass_axpy(const T* __restrict__ lam, T* __restrict__ ub,
                                                  Geom g, T c, T cdt)
{
    const long long idx = (long long)blockIdx.x * AB + threadIdx.x;
    int i, j, k;
    if (!node_of<D>(g, idx, i, j, k)) return;
    if (g.cm) {
        T l[NB<D>::K];
        gather<T, D>(lam, g, i, j, k, l);
        ub[idx] += cdt * cmass<T, D>(l, (T)g.h) / (T)bfactor<D>(g, i, j, k);
    } else {
        ub[idx] += c / (T)bfactor<D>(g, i, j, k) * lam[idx];
    }
}

// Allen-Cahn explicit step S(eta) = eta - dt r(eta)/m:
//   Ubar += vbar - (dt/m) J_r(eta) vbar   (J_r symmetric)
//   theta partials of -(dt/m) vbar^T dr/dtheta
// On a no-flux grid (m_a = h^d / 2^b, rows = reflected rows / 2^b) the first line
// is vbar - (dt/h^d) [J_reflected (2^b vbar)] / 2^b and the theta partials use the
// reflected rows unscaled.
template <typename T, int D>
__global__ __launch_bounds__(AB) void k_vjp_ac_step(const T* __restrict__ eta,
                                                    const T* __restrict__ vb, T* __restrict__ ub,
                                                    Geom g, Cub<T> F1, Lin<T> F2, T detJ, T W,
                                                    T kappa, T mob, T dt_over_m,
                                                    double* __restrict__ part)
{
    const long long idx = (long long)blockIdx.x * AB + threadIdx.x;
    double t0 = 0.0, t1 = 0.0, t2 = 0.0;
    int i, j, k;
    if (node_of<D>(g, idx, i, j, k)) {
        T u[NB<D>::K], v[NB<D>::K];
        gather<T, D>(eta, g, i, j, k, u);
        gather<T, D, true>(vb, g, i, j, k, v);
        const T h = (T)g.h;
        const T Nv = detJ * quad_sum<T, D, true>(u, v, F2);
        const T Kv = stiff<T, D>(v, h);
        const T vc = vb[idx];
        const T ib = (T)1 / (T)bfactor<D>(g, i, j, k);
        ub[idx] += vc - dt_over_m * mob * (Nv + kappa * Kv) * ib;
        const double n1 = (double)(detJ * quad_sum<T, D, false>(u, u, F1));
        const double ku = (double)stiff<T, D>(u, h);
        const double wi = -(double)dt_over_m * (double)vc;
        t0 = wi * ((double)W * n1 + (double)kappa * ku);
        t1 = wi * (double)mob * ku;
        t2 = wi * (double)mob * n1;
    }
    block_partials3(t0, t1, t2, part);
}

// Cahn-Hilliard split step S(c) = c - dt M^-1 [M_mob K] M^-1 A(c), A = W N_1 + kappa K.
// On a no-flux grid pass a applies K to 2^b vbar and pass b divides its rows by 2^b
// (t itself is (M dt / h^2d) K_reflected(2^b vbar), with no further factor).
// Pass a: t = mob K (dt vbar / m) / m ; theta_M partial -sum (dt vbar/m) (K mu), mu = A(c)/m
template <typename T, int D>
__global__ __launch_bounds__(AB) void k_vjp_ch_a(const T* __restrict__ mu, const T* __restrict__ vb,
                                                 T* __restrict__ t, Geom g, T dt_over_m, T mob,
                                                 T inv_m, double* __restrict__ part)
{
    const long long idx = (long long)blockIdx.x * AB + threadIdx.x;
    double t0 = 0.0;
    int i, j, k;
    if (node_of<D>(g, idx, i, j, k)) {
        T v[NB<D>::K], w[NB<D>::K];
        gather<T, D, true>(vb, g, i, j, k, v);  // 2^b vbar on no-flux grids
        gather<T, D>(mu, g, i, j, k, w);
        const T h = (T)g.h;
        t[idx] = mob * dt_over_m * stiff<T, D>(v, h) * inv_m;
        t0 = -(double)dt_over_m * (double)vb[idx] * (double)stiff<T, D>(w, h);
    }
    block_partials3(t0, 0.0, 0.0, part);
}

// Pass b: Ubar += vbar - A'(c) t ; theta_kappa, theta_W partials -t (K c), -t N_1(c)
template <typename T, int D>
__global__ __launch_bounds__(AB) void k_vjp_ch_b(const T* __restrict__ c, const T* __restrict__ t,
                                                 const T* __restrict__ vb, T* __restrict__ ub,
                                                 Geom g, Cub<T> F1, Lin<T> F2, T detJ, T kappa,
                                                 double* __restrict__ part)
{
    const long long idx = (long long)blockIdx.x * AB + threadIdx.x;
    double t1 = 0.0, t2 = 0.0;
    int i, j, k;
    if (node_of<D>(g, idx, i, j, k)) {
        T u[NB<D>::K], v[NB<D>::K];
        gather<T, D>(c, g, i, j, k, u);
        gather<T, D>(t, g, i, j, k, v);
        const T h = (T)g.h;
        const T ib = (T)1 / (T)bfactor<D>(g, i, j, k);  // no-flux rows (1 on periodic grids)
        const T At = (detJ * quad_sum<T, D, true>(u, v, F2) + kappa * stiff<T, D>(v, h)) * ib;
        ub[idx] += vb[idx] - At;
        const double ti = (double)v[NB<D>::K / 2] * (double)ib;
        t1 = -ti * (double)stiff<T, D>(u, h);
        t2 = -ti * (double)(detJ * quad_sum<T, D, false>(u, u, F1));
    }
    block_partials3(0.0, t1, t2, part);
}



inline unsigned nblk(const Geom& g) { return (unsigned)((g.N + AB - 1) / AB); }

#define DIM_SWITCH(g, ...)   \
    if ((g).dim == 2) {      \
        constexpr int D = 2; \
        __VA_ARGS__;         \
    } else {                 \
        constexpr int D = 3; \
        __VA_ARGS__;         \
    }

// f' at W = 1 (N_1 in the header comment)
template <typename T>
Cub<T> unit_cubic(const FreeEnergy& f)
{
    const FreeEnergy one = make_free_energy(f.fe, 1.0);
    return Cub<T>{(T)one.a1, (T)one.a2, (T)one.a3};
}

}  // namespace

template <typename T>
void launch_dtheta(const Geom& g, int model, const FreeEnergy& f, double kappa, double mob,
                   const T* U, const T* w, double scale, double* part, double* theta_bar,
                   hipStream_t s)
{
    const double detJ = std::pow(0.5 * g.h, g.dim);
    const unsigned nb = nblk(g);
    DIM_SWITCH(g, {
        if (model == 0)
            k_dtheta<T, D, 0><<<nb, AB, 0, s>>>(U, w, g, unit_cubic<T>(f), (T)detJ, (T)f.W,
                                                 (T)kappa, (T)mob, scale, part);
        else
            k_dtheta<T, D, 1><<<nb, AB, 0, s>>>(U, w, g, unit_cubic<T>(f), (T)detJ, (T)f.W,
                                                 (T)kappa, (T)mob, scale, part);
    });
    k_reduce3<<<1, AB, 0, s>>>(part, (int)nb, theta_bar);
}

template <typename T>
void launch_mass_axpy(const Geom& g, double inv_dt, const T* lam, T* ub, hipStream_t s)
{
    const double m = std::pow(g.h, g.dim);
    DIM_SWITCH(g, { k_mass_axpy<T, D><<<nblk(g), AB, 0, s>>>(lam, ub, g, (T)(inv_dt * m), (T)inv_dt); });
}

template <typename T>
void launch_vjp_explicit(const Geom& g, int model, const FreeEnergy& f, double kappa, double mob,
                         double dt, const T* U, const T* vbar, T* ubar, T* scratch, double* part,
                         double* theta_bar, hipStream_t s)
{
    const double detJ = std::pow(0.5 * g.h, g.dim), m = std::pow(g.h, g.dim);
    const unsigned nb = nblk(g);
    const Lin<T> F2{(T)f.b0, (T)f.b1, (T)f.b2};
    if (model == 0) {
        DIM_SWITCH(g, {
            k_vjp_ac_step<T, D><<<nb, AB, 0, s>>>(U, vbar, ubar, g, unit_cubic<T>(f), F2, (T)detJ,
                                                   (T)f.W, (T)kappa, (T)mob, (T)(dt / m), part);
        });
        k_reduce3<<<1, AB, 0, s>>>(part, (int)nb, theta_bar);
        return;
    }
    T* mu = scratch;
    T* t = scratch + g.N;
    launch_chem<T>(g, f, kappa, U, mu, s);
    DIM_SWITCH(g, {
        k_vjp_ch_a<T, D><<<nb, AB, 0, s>>>(mu, vbar, t, g, (T)(dt / m), (T)mob, (T)(1.0 / m), part);
    });
    k_reduce3<<<1, AB, 0, s>>>(part, (int)nb, theta_bar);
    DIM_SWITCH(g, {
        k_vjp_ch_b<T, D><<<nb, AB, 0, s>>>(U, t, vbar, ubar, g, unit_cubic<T>(f), F2, (T)detJ,
                                            (T)kappa, part);
    });
    k_reduce3<<<1, AB, 0, s>>>(part, (int)nb, theta_bar);
}


#define INST_ADJ(T)                                                                              \
    template void launch_dtheta<T>(const Geom&, int, const FreeEnergy&, double, double, const T*, \
                                   const T*, double, double*, double*, hipStream_t);            \
    template void launch_mass_axpy<T>(const Geom&, double, const T*, T*, hipStream_t);           \
    template void launch_vjp_explicit<T>(const Geom&, int, const FreeEnergy&, double, double,    \
                                         double, const T*, const T*, T*, T*, double*, double*,   \
                                         hipStream_t);
INST_ADJ(float)
INST_ADJ(double)

}  // namespace pfk
