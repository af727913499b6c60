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
// no-flux grids
template <typename T, int D>
__global__ __launch_bounds__(256) void k_cp_residual(const T* __restrict__ U, T* __restrict__ r, Geom g,
                                                     T detJ, T m, T kappa, T Mc, T Meta)
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
    r[idx] = Mc * stiff<T, D>(w, h) * ib;
    r[g.N + idx] = (m * w[NB<D>::K / 2] - gsrc) * ib;
    r[2 * g.N + idx] = Meta * (s + kappa * stiff<T, D>(e, h)) * ib;
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
                        hipStream_t s)
{
    const double detJ = std::pow(0.5 * g.h, g.dim), m = std::pow(g.h, g.dim);
    CP_DIM(g, {
        k_cp_residual<T, D><<<blocks_for(g), 256, 0, s>>>(U, r, g, (T)detJ, (T)m, (T)kappa, (T)Mc,
                                                           (T)Meta);
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
                                        hipStream_t);                                              \
    template void launch_cp_energy<T>(const Geom&, double, const T*, double*, double*, hipStream_t);
INST_CP(float)
INST_CP(double)

}  // namespace pfk
