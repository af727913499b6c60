// k_node.hip -- node-centric kernels for 2-D and 3-D periodic Q1 grids:
// residual (Eq. 11) and backward-Euler residual (Eq. 14), Jacobian products,
// preconditioner, chemical potential, node-centric explicit updates, energy.
// The shared device helpers and the quadrature scheme are in node_common.hpp.
// g.quad selects Gauss-Lobatto (nodal) quadrature: N(u)_a = m f'(u_a), the 5/7-point
// stiffness stencil and the lumped mass (the branch is uniform over the grid).
#include <cmath>

#include "node_common.hpp"

namespace pfk {

namespace {

// r(U): Allen-Cahn  r = L [N + kappa K u];  Cahn-Hilliard r_c = M K mu, r_mu = m mu - [N(c) + kappa K c]
// With Uold != nullptr the time term inv_dt m (U - Uold) of Eq. 14 is added to
// the rows that carry mass (Allen-Cahn eta, Cahn-Hilliard c).  g.cm: the
// consistent mass (3^d stencil) replaces m in the time term and the mu-row.
template <typename T, int D, int MODEL>
__global__ __launch_bounds__(256) void k_residual(const T* __restrict__ U, const T* __restrict__ Uold,
                                                  T* __restrict__ r, Geom g, Cub<T> F, T detJ,
                                                  T kappa, T mob, T m, T inv_dt)
{
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int i, j, k;
    if (!node_of<D>(g, idx, i, j, k)) return;
    T u[NB<D>::K];
    gather<T, D>(U, g, i, j, k, u);
    const T h = (T)g.h;
    const T Nn = g.quad ? m * F(u[NB<D>::K / 2], (T)0) : detJ * quad_sum<T, D, false>(u, u, F);
    const T Ku = stiff_q<T, D>(g, u, h);
    T tt = (T)0;
    if (Uold) {
        if (g.cm) {
            T uo[NB<D>::K];
            gather<T, D>(Uold, g, i, j, k, uo);
#pragma unroll
            for (int q = 0; q < NB<D>::K; ++q) uo[q] = u[q] - uo[q];
            tt = inv_dt * cmass<T, D>(uo, h);
        } else {
            tt = inv_dt * m * (u[NB<D>::K / 2] - Uold[idx]);
        }
    }
    const T ib = (T)1 / (T)bfactor<D>(g, i, j, k);  // no-flux rows (1 on periodic grids)
    if constexpr (MODEL == 0) {
        r[idx] = (mob * (Nn + kappa * Ku) + tt) * ib;
    } else {
        T w[NB<D>::K];
        gather<T, D>(U + g.N, g, i, j, k, w);
        r[idx] = (mob * stiff_q<T, D>(g, w, h) + tt) * ib;
        const T mw = g.cm ? cmass<T, D>(w, h) : m * w[NB<D>::K / 2];
        r[g.N + idx] = (mw - (Nn + kappa * Ku)) * ib;
    }
}

// (Block-)Jacobi preconditioner of dR/dU at U:
//   Allen-Cahn:    pinv[a] = 1 / (inv_dt m + L (N'_aa + kappa K_aa))
//   Cahn-Hilliard: pinv[4a..4a+3] = inverse of [[inv_dt m, M K_aa], [-(N'_aa + kappa K_aa), m]]
// (row-major), with N'_aa = sum_e sum_q |J| f''(u_q) phi_a(q)^2.
template <typename T, int D, int MODEL>
__global__ __launch_bounds__(256) void k_prec(const T* __restrict__ U, T* __restrict__ pinv, Geom g,
                                              Lin<T> F, T detJ, T kappa, T mob, T m, T inv_dt)
{
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int i, j, k;
    if (!node_of<D>(g, idx, i, j, k)) return;
    T u[NB<D>::K];
    gather<T, D>(U, g, i, j, k, u);
    const double nd = g.quad ? (double)(m * F(u[NB<D>::K / 2], (T)1)) : (double)(detJ * quad_sum_sq<T, D>(u, F));
    const double kd = g.quad ? (double)stiff_lob_diag<T, D>((T)g.h) : (double)stiff_diag<T, D>((T)g.h);
    const double ib = 1.0 / bfactor<D>(g, i, j, k);  // no-flux rows (1 on periodic grids)
    if constexpr (MODEL == 0) {
        pinv[idx] = (T)(1.0 / (ib * ((double)inv_dt * m + (double)mob * (nd + (double)kappa * kd))));
    } else {
        const double a = ib * (double)inv_dt * m, b = ib * (double)mob * kd;
        const double c = -ib * (nd + (double)kappa * kd), d = ib * (double)m;
        const double det = a * d - b * c;
        T* P = pinv + 4 * idx;
        P[0] = (T)(d / det);
        P[1] = (T)(-b / det);
        P[2] = (T)(-c / det);
        P[3] = (T)(a / det);
    }
}

// Jv for R = inv_dt M (U - U_old) + r(U)
// TRANS = 1 gives the transpose product w^T dR/dU (differs from J only for
// Cahn-Hilliard):  [inv_dt m w_c - (N'(c) + kappa K) w_mu ;  M K w_c + m w_mu].
// ACC = 1 adds the result into Jv instead of overwriting it.  g.cm: the
// (symmetric) consistent mass replaces m.  The preconditioner keeps the lumped
// mass as its approximation of the mass blocks.
template <typename T, int D, int MODEL, int TRANS, int ACC>
__global__ __launch_bounds__(256) void k_jvp(const T* __restrict__ U, const T* __restrict__ V,
                                             T* __restrict__ Jv, Geom g, Lin<T> F, T detJ, T kappa,
                                             T mob, T m, T inv_dt)
{
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int i, j, k;
    if (!node_of<D>(g, idx, i, j, k)) return;
    T u[NB<D>::K], v[NB<D>::K];
    gather<T, D>(U, g, i, j, k, u);
    const T h = (T)g.h;
    const T ib = (T)1 / (T)bfactor<D>(g, i, j, k);  // no-flux rows (1 on periodic grids)
    if constexpr (MODEL == 0) {
        gather<T, D>(V, g, i, j, k, v);
        const T Nv = g.quad ? m * F(u[NB<D>::K / 2], v[NB<D>::K / 2]) : detJ * quad_sum<T, D, true>(u, v, F);
        const T Kv = stiff_q<T, D>(g, v, h);
        const T mv = g.cm ? cmass<T, D>(v, h) : m * v[NB<D>::K / 2];
        const T out = (inv_dt * mv + mob * (Nv + kappa * Kv)) * ib;
        Jv[idx] = ACC ? Jv[idx] + out : out;
    } else {
        T w[NB<D>::K];
        gather<T, D>(V, g, i, j, k, v);         // c-plane of the direction
        gather<T, D>(V + g.N, g, i, j, k, w);   // mu-plane of the direction
        T oc, om;
        const T mv = g.cm ? cmass<T, D>(v, h) : m * v[NB<D>::K / 2];
        const T mw = g.cm ? cmass<T, D>(w, h) : m * w[NB<D>::K / 2];
        const T uc = u[NB<D>::K / 2];
        if constexpr (TRANS == 0) {
            const T Nv = g.quad ? m * F(uc, v[NB<D>::K / 2]) : detJ * quad_sum<T, D, true>(u, v, F);
            oc = inv_dt * mv + mob * stiff_q<T, D>(g, w, h);
            om = mw - (Nv + kappa * stiff_q<T, D>(g, v, h));
        } else {
            const T Nw = g.quad ? m * F(uc, w[NB<D>::K / 2]) : detJ * quad_sum<T, D, true>(u, w, F);
            oc = inv_dt * mv - (Nw + kappa * stiff_q<T, D>(g, w, h));
            om = mob * stiff_q<T, D>(g, v, h) + mw;
        }
        oc *= ib;
        om *= ib;
        Jv[idx] = ACC ? Jv[idx] + oc : oc;
        Jv[g.N + idx] = ACC ? Jv[g.N + idx] + om : om;
    }
}

template <typename T, int D>
__global__ __launch_bounds__(256) void k_chem(const T* __restrict__ c, T* __restrict__ mu, Geom g,
                                              Cub<T> F, T detJ, T kappa, T inv_m)
{
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int i, j, k;
    if (!node_of<D>(g, idx, i, j, k)) return;
    T u[NB<D>::K];
    gather<T, D>(c, g, i, j, k, u);
    const T h = (T)g.h, m = D == 2 ? h * h : h * h * h;  // interior nodal mass h^D
    const T Nn = g.quad ? m * F(u[NB<D>::K / 2], (T)0) : detJ * quad_sum<T, D, false>(u, u, F);
    mu[idx] = (Nn + kappa * stiff_q<T, D>(g, u, h)) * inv_m;
}

template <typename T, int D>
__global__ __launch_bounds__(256) void k_ch_update(const T* __restrict__ c, const T* __restrict__ mu,
                                                   T* __restrict__ cout, Geom g, T dtM_over_m)
{
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int i, j, k;
    if (!node_of<D>(g, idx, i, j, k)) return;
    T w[NB<D>::K];
    gather<T, D>(mu, g, i, j, k, w);
    cout[idx] = c[idx] - dtM_over_m * stiff_q<T, D>(g, w, (T)g.h);
}

template <typename T, int D>
__global__ __launch_bounds__(256) void k_ac_step(const T* __restrict__ eta, T* __restrict__ out,
                                                 Geom g, Cub<T> F, T detJ, T kappa, T dtL_over_m)
{
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int i, j, k;
    if (!node_of<D>(g, idx, i, j, k)) return;
    T u[NB<D>::K];
    gather<T, D>(eta, g, i, j, k, u);
    const T h = (T)g.h, m = D == 2 ? h * h : h * h * h;  // interior nodal mass h^D
    const T Nn = g.quad ? m * F(u[NB<D>::K / 2], (T)0) : detJ * quad_sum<T, D, false>(u, u, F);
    const T r = Nn + kappa * stiff_q<T, D>(g, u, h);
    out[idx] = u[NB<D>::K / 2] - dtL_over_m * r;
}

// ---- energy and mass ---------------------------------------------------------
// Each thread owns the element whose lower corner is its node (none past the upper
// boundary of a no-flux grid) and the mass term of its node.
__device__ __forceinline__ double f_local(int fe, double W, double q)
{
    if (fe == 0) {
        const double t = q * q - 1.0;
        return 0.25 * W * t * t;
    }
    const double t = q * (1.0 - q);
    return W * t * t;
}

constexpr int EBLK = 256;

template <typename T, int D>
__global__ __launch_bounds__(EBLK) void k_energy(const T* __restrict__ c, double* __restrict__ part,
                                                 Geom g, int fe, double W, double kappa)
{
    const long long idx = (long long)blockIdx.x * EBLK + threadIdx.x;
    double e = 0.0, ms = 0.0;
    int i, j, k;
    if (node_of<D>(g, idx, i, j, k)) {
        const double h = g.h;
        // 1-D shape functions at the quadrature points: Gauss (GP, GM), or
        // Gauss-Lobatto (the points are the nodes: the identity)
        const double bp = g.quad ? 1.0 : GP, bm = g.quad ? 0.0 : GM;
        const double B[2][2] = {{bp, bm}, {bm, bp}};
        const int i1 = wrap(i + 1, g.n[0]), j1 = wrap(j + 1, g.n[1]);
        if constexpr (D == 2) {
            double u[2][2];  // [ay][ax]
            u[0][0] = c[(long long)j * g.n[0] + i];
            u[0][1] = c[(long long)j * g.n[0] + i1];
            u[1][0] = c[(long long)j1 * g.n[0] + i];
            u[1][1] = c[(long long)j1 * g.n[0] + i1];
            const double detJ = 0.25 * h * h;
            for (int qy = 0; qy < 2; ++qy)
                for (int qx = 0; qx < 2; ++qx) {
                    double cq = 0.0, gx = 0.0, gy = 0.0;
                    for (int ay = 0; ay < 2; ++ay)
                        for (int ax = 0; ax < 2; ++ax) {
                            const double sx = ax ? 1.0 : -1.0, sy = ay ? 1.0 : -1.0;
                            cq += B[qx][ax] * B[qy][ay] * u[ay][ax];
                            gx += sx / h * B[qy][ay] * u[ay][ax];
                            gy += sy / h * B[qx][ax] * u[ay][ax];
                        }
                    e += detJ * (f_local(fe, W, cq) + 0.5 * kappa * (gx * gx + gy * gy));
                }
            ms = h * h * u[0][0];
        } else {
            const int k1 = wrap(k + 1, g.n[2]);
            double u[2][2][2];  // [az][ay][ax]
            const int zz[2] = {k, k1}, yy[2] = {j, j1}, xx[2] = {i, i1};
            for (int az = 0; az < 2; ++az)
                for (int ay = 0; ay < 2; ++ay)
                    for (int ax = 0; ax < 2; ++ax)
                        u[az][ay][ax] = c[((long long)zz[az] * g.n[1] + yy[ay]) * g.n[0] + xx[ax]];
            const double detJ = 0.125 * h * h * h;
            for (int qz = 0; qz < 2; ++qz)
                for (int qy = 0; qy < 2; ++qy)
                    for (int qx = 0; qx < 2; ++qx) {
                        double cq = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
                        for (int az = 0; az < 2; ++az)
                            for (int ay = 0; ay < 2; ++ay)
                                for (int ax = 0; ax < 2; ++ax) {
                                    const double sx = ax ? 1.0 : -1.0, sy = ay ? 1.0 : -1.0,
                                                 sz = az ? 1.0 : -1.0;
                                    const double v = u[az][ay][ax];
                                    cq += B[qx][ax] * B[qy][ay] * B[qz][az] * v;
                                    gx += sx / h * B[qy][ay] * B[qz][az] * v;
                                    gy += sy / h * B[qx][ax] * B[qz][az] * v;
                                    gz += sz / h * B[qx][ax] * B[qy][ay] * v;
                                }
                        e += detJ * (f_local(fe, W, cq) +
                                     0.5 * kappa * (gx * gx + gy * gy + gz * gz));
                    }
            ms = h * h * h * u[0][0][0];
        }
        // no-flux: the element exists only below the upper boundary; lumped mass h^d / 2^b
        if (g.bc) {
            const bool elem = i + 1 < g.n[0] && j + 1 < g.n[1] && (D == 2 || k + 1 < g.n[2]);
            if (!elem) e = 0.0;
            ms /= bfactor<D>(g, i, j, k);
        }
    }
    // block reduction, fixed order: wave shuffle tree, then waves in order
    __shared__ double se[EBLK / WAVE], sm[EBLK / WAVE];
    for (int off = WAVE / 2; off > 0; off >>= 1) {
        e += __shfl_down(e, off, WAVE);
        ms += __shfl_down(ms, off, WAVE);
    }
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    if (lane == 0) {
        se[wv] = e;
        sm[wv] = ms;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int w = 0; w < EBLK / WAVE; ++w) {
            a += se[w];
            b += sm[w];
        }
        part[2 * blockIdx.x] = a;
        part[2 * blockIdx.x + 1] = b;
    }
}

// single block sums the per-block partials in a fixed order
__global__ __launch_bounds__(256) void k_reduce_pairs(const double* __restrict__ part, int nb,
                                                      double* __restrict__ out)
{
    __shared__ double se[256], sm[256];
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) {
        a += part[2 * i];
        b += part[2 * i + 1];
    }
    se[threadIdx.x] = a;
    sm[threadIdx.x] = b;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            se[threadIdx.x] += se[threadIdx.x + s];
            sm[threadIdx.x] += sm[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = se[0];
        out[1] = sm[0];
    }
}

inline dim3 grid_for(const Geom& g) { return dim3((unsigned)((g.N + 255) / 256)); }

template <typename T>
Cub<T> cub_of(const FreeEnergy& f, double scale)
{
    return Cub<T>{(T)(scale * f.a1), (T)(scale * f.a2), (T)(scale * f.a3)};
}

}  // namespace

int energy_blocks(const Geom& g) { return (int)((g.N + EBLK - 1) / EBLK); }

void launch_reduce_pairs(const double* part, int nb, double* out, hipStream_t s)
{
    k_reduce_pairs<<<1, 256, 0, s>>>(part, nb, out);
}

#define DIM_SWITCH(g, ...)         \
    if ((g).dim == 2) {            \
        constexpr int D = 2;       \
        __VA_ARGS__;               \
    } else {                       \
        constexpr int D = 3;       \
        __VA_ARGS__;               \
    }

template <typename T>
void launch_residual(const Geom& g, int model, const FreeEnergy& f, double kappa, double mob,
                     const T* U, T* r, hipStream_t s, const T* Uold, double inv_dt)
{
    const double detJ = std::pow(0.5 * g.h, g.dim), m = std::pow(g.h, g.dim);
    DIM_SWITCH(g, {
        if (model == 0)
            k_residual<T, D, 0><<<grid_for(g), 256, 0, s>>>(U, Uold, r, g, cub_of<T>(f, 1.0),
                                                             (T)detJ, (T)kappa, (T)mob, (T)m,
                                                             (T)inv_dt);
        else
            k_residual<T, D, 1><<<grid_for(g), 256, 0, s>>>(U, Uold, r, g, cub_of<T>(f, 1.0),
                                                             (T)detJ, (T)kappa, (T)mob, (T)m,
                                                             (T)inv_dt);
    });
}

template <typename T>
void launch_jvp(const Geom& g, int model, const FreeEnergy& f, double kappa, double mob,
                double inv_dt, const T* U, const T* v, T* Jv, hipStream_t s, int trans, int acc)
{
    if (g.dim == 3 && !acc && !g.cm && !g.quad) {
        launch_jvp3d<T>(g, model, f, kappa, mob, inv_dt, U, v, Jv, s, trans);
        return;
    }
    // Allen-Cahn's Jacobian is symmetric, so its transpose product is the product
    if (!acc && (model == 0 || !trans) && launch_jvp2d_stream<T>(g, model, f, kappa, mob, inv_dt, U, v, Jv, s))
        return;
    const double detJ = std::pow(0.5 * g.h, g.dim), m = std::pow(g.h, g.dim);
    Lin<T> F{(T)f.b0, (T)f.b1, (T)f.b2};
#define JVP_L(MODEL, TR, AC)                                                                    \
    k_jvp<T, D, MODEL, TR, AC><<<grid_for(g), 256, 0, s>>>(U, v, Jv, g, F, (T)detJ, (T)kappa,  \
                                                           (T)mob, (T)m, (T)inv_dt)
    DIM_SWITCH(g, {
        if (model == 0) {
            if (acc) JVP_L(0, 0, 1); else JVP_L(0, 0, 0);
        } else if (!trans) {
            if (acc) JVP_L(1, 0, 1); else JVP_L(1, 0, 0);
        } else {
            if (acc) JVP_L(1, 1, 1); else JVP_L(1, 1, 0);
        }
    });
#undef JVP_L
}

template <typename T>
void launch_prec(const Geom& g, int model, const FreeEnergy& f, double kappa, double mob,
                 double inv_dt, const T* U, T* pinv, hipStream_t s)
{
    const double detJ = std::pow(0.5 * g.h, g.dim), m = std::pow(g.h, g.dim);
    Lin<T> F{(T)f.b0, (T)f.b1, (T)f.b2};
    DIM_SWITCH(g, {
        if (model == 0)
            k_prec<T, D, 0><<<grid_for(g), 256, 0, s>>>(U, pinv, g, F, (T)detJ, (T)kappa, (T)mob,
                                                         (T)m, (T)inv_dt);
        else
            k_prec<T, D, 1><<<grid_for(g), 256, 0, s>>>(U, pinv, g, F, (T)detJ, (T)kappa, (T)mob,
                                                         (T)m, (T)inv_dt);
    });
}

template <typename T>
void launch_chem(const Geom& g, const FreeEnergy& f, double kappa, const T* c, T* mu,
                 hipStream_t s)
{
    const double detJ = std::pow(0.5 * g.h, g.dim), m = std::pow(g.h, g.dim);
    DIM_SWITCH(g, {
        k_chem<T, D><<<grid_for(g), 256, 0, s>>>(c, mu, g, cub_of<T>(f, 1.0), (T)detJ, (T)kappa,
                                                  (T)(1.0 / m));
    });
}

template <typename T>
void launch_ch_update(const Geom& g, double dtM, const T* c, const T* mu, T* c_out, hipStream_t s)
{
    const double m = std::pow(g.h, g.dim);
    DIM_SWITCH(g, { k_ch_update<T, D><<<grid_for(g), 256, 0, s>>>(c, mu, c_out, g, (T)(dtM / m)); });
}

template <typename T>
void launch_ac_step(const Geom& g, const FreeEnergy& f, double kappa, double dtL, const T* eta,
                    T* eta_out, hipStream_t s)
{
    const double detJ = std::pow(0.5 * g.h, g.dim), m = std::pow(g.h, g.dim);
    DIM_SWITCH(g, {
        k_ac_step<T, D><<<grid_for(g), 256, 0, s>>>(eta, eta_out, g, cub_of<T>(f, 1.0), (T)detJ,
                                                     (T)kappa, (T)(dtL / m));
    });
}

template <typename T>
void launch_energy(const Geom& g, const FreeEnergy& f, double kappa, const T* c, double* partials,
                   double* out, hipStream_t s)
{
    const int nb = energy_blocks(g);
    DIM_SWITCH(g, { k_energy<T, D><<<nb, EBLK, 0, s>>>(c, partials, g, f.fe, f.W, kappa); });
    k_reduce_pairs<<<1, 256, 0, s>>>(partials, nb, out);
}

#define INST(T)                                                                                   \
    template void launch_residual<T>(const Geom&, int, const FreeEnergy&, double, double, const T*, \
                                     T*, hipStream_t, const T*, double);                          \
    template void launch_jvp<T>(const Geom&, int, const FreeEnergy&, double, double, double,       \
                                const T*, const T*, T*, hipStream_t, int, int);                   \
    template void launch_prec<T>(const Geom&, int, const FreeEnergy&, double, double, double,      \
                                 const T*, T*, hipStream_t);                                      \
    template void launch_chem<T>(const Geom&, const FreeEnergy&, double, const T*, T*, hipStream_t); \
    template void launch_ch_update<T>(const Geom&, double, const T*, const T*, T*, hipStream_t);   \
    template void launch_ac_step<T>(const Geom&, const FreeEnergy&, double, double, const T*, T*,  \
                                    hipStream_t);                                                 \
    template void launch_energy<T>(const Geom&, const FreeEnergy&, double, const T*, double*,      \
                                   double*, hipStream_t);
INST(float)
INST(double)

}  // namespace pfk
