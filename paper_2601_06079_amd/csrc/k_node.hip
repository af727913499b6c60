// k_node.hip -- node-centric kernels for 2-D and 3-D periodic Q1 grids.
//
// One thread owns one node.  It reads the 3^d neighbourhood of the node and
// evaluates the node's row of the weak form directly, summing over the 2^d
// elements that share the node (no atomics, fixed summation order):
//   nonlinear term  N(u)_a = sum_e sum_q |J| f'(u_q) phi_a(q)        (Eqs. 5-6, 10)
//   gradient term   (K u)_a = sum_e sum_q |J| grad u_q . grad phi_a   (exact: a closed
//                   tensor stencil, K = sum_k Khat_k (x) Mhat_others, Khat = [-1 2 -1]/h,
//                   Mhat = h [1 4 1] / 6)
// The 4^d quadrature values of the 2^d elements are produced by sum
// factorisation: interp3to4 along x, then y (then z).
#include <cmath>

#include "device.hpp"
#include "kernels.hpp"

namespace pfk {

FreeEnergy make_free_energy(int fe, double W)
{
    FreeEnergy f{};
    f.W = W;
    f.fe = fe;
    if (fe == 0) {  // W (q^2 - 1)^2 / 4
        f.a1 = -W; f.a2 = 0.0; f.a3 = W;
        f.b0 = -W; f.b1 = 0.0; f.b2 = 3.0 * W;
    } else {        // W q^2 (1 - q)^2
        f.a1 = 2.0 * W; f.a2 = -6.0 * W; f.a3 = 4.0 * W;
        f.b0 = 2.0 * W; f.b1 = -12.0 * W; f.b2 = 12.0 * W;
    }
    return f;
}

namespace {

template <int D>
struct NB {
    static constexpr int K = D == 2 ? 9 : 27;
};

// Neighbourhood index: (dx+1) + 3 (dy+1) + 9 (dz+1)
template <typename T, int D>
__device__ __forceinline__ void gather(const T* __restrict__ u, const Geom& g, int i, int j, int k,
                                       T out[NB<D>::K])
{
    const int xs[3] = {wrap(i - 1, g.n[0]), i, wrap(i + 1, g.n[0])};
    const int ys[3] = {wrap(j - 1, g.n[1]), j, wrap(j + 1, g.n[1])};
    if constexpr (D == 2) {
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int a = 0; a < 3; ++a) out[a + 3 * b] = u[(long long)ys[b] * g.n[0] + xs[a]];
    } else {
        const int zs[3] = {wrap(k - 1, g.n[2]), k, wrap(k + 1, g.n[2])};
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int b = 0; b < 3; ++b)
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    out[a + 3 * b + 9 * c] =
                        u[((long long)zs[c] * g.n[1] + ys[b]) * g.n[0] + xs[a]];
    }
}

// Unit-coefficient Q1 stiffness row at the centre node (2-D: h-free; 3-D: times h).
template <typename T, int D>
__device__ __forceinline__ T stiff(const T* u, T h)
{
    if constexpr (D == 2) {
        T kx[3], mx[3];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            kx[b] = (T)2 * u[1 + 3 * b] - u[3 * b] - u[2 + 3 * b];
            mx[b] = (T)4 * u[1 + 3 * b] + u[3 * b] + u[2 + 3 * b];
        }
        const T km = kx[0] + (T)4 * kx[1] + kx[2];  // Khat_x (x) Mhat_y
        const T mk = (T)2 * mx[1] - mx[0] - mx[2];  // Mhat_x (x) Khat_y
        return (km + mk) * (T)(1.0 / 6.0);
    } else {
        T km[3], mk[3], mm[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            T kx[3], mx[3];
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const T* r = u + 3 * b + 9 * c;
                kx[b] = (T)2 * r[1] - r[0] - r[2];
                mx[b] = (T)4 * r[1] + r[0] + r[2];
            }
            km[c] = kx[0] + (T)4 * kx[1] + kx[2];
            mk[c] = (T)2 * mx[1] - mx[0] - mx[2];
            mm[c] = mx[0] + (T)4 * mx[1] + mx[2];
        }
        const T a = (km[0] + mk[0]) + (T)4 * (km[1] + mk[1]) + (km[2] + mk[2]);  // (..) (x) Mhat_z
        const T b = (T)2 * mm[1] - mm[0] - mm[2];                              // Mhat Mhat Khat_z
        return (a + b) * h * (T)(1.0 / 36.0);
    }
}

// sum_q w_q F(u_q[, v_q]) over the 4^D quadrature points around the centre node;
// w = tensor product of (GM, GP, GP, GM).  |J| is applied by the caller.
template <typename T, int D, bool WITHV, typename Fn>
__device__ __forceinline__ T quad_sum(const T* u, const T* v, Fn F)
{
    if constexpr (D == 2) {
        T Xu[3][4], Xv[3][4];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            interp3to4(u[3 * b], u[3 * b + 1], u[3 * b + 2], Xu[b]);
            if constexpr (WITHV) interp3to4(v[3 * b], v[3 * b + 1], v[3 * b + 2], Xv[b]);
        }
        T col[4];
#pragma unroll
        for (int qx = 0; qx < 4; ++qx) {
            T qu[4], qv[4], fv[4];
            interp3to4(Xu[0][qx], Xu[1][qx], Xu[2][qx], qu);
            if constexpr (WITHV) interp3to4(Xv[0][qx], Xv[1][qx], Xv[2][qx], qv);
#pragma unroll
            for (int qy = 0; qy < 4; ++qy) fv[qy] = F(qu[qy], WITHV ? qv[qy] : (T)0);
            col[qx] = wsum4(fv);
        }
        return wsum4(col);
    } else {
        T Xu[9][4], Xv[9][4];
#pragma unroll
        for (int r = 0; r < 9; ++r) {
            interp3to4(u[3 * r], u[3 * r + 1], u[3 * r + 2], Xu[r]);
            if constexpr (WITHV) interp3to4(v[3 * r], v[3 * r + 1], v[3 * r + 2], Xv[r]);
        }
        T plane[4];
#pragma unroll
        for (int qx = 0; qx < 4; ++qx) {
            T Yu[3][4], Yv[3][4];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                interp3to4(Xu[3 * c][qx], Xu[3 * c + 1][qx], Xu[3 * c + 2][qx], Yu[c]);
                if constexpr (WITHV)
                    interp3to4(Xv[3 * c][qx], Xv[3 * c + 1][qx], Xv[3 * c + 2][qx], Yv[c]);
            }
            T row[4];
#pragma unroll
            for (int qy = 0; qy < 4; ++qy) {
                T qu[4], qv[4], fv[4];
                interp3to4(Yu[0][qy], Yu[1][qy], Yu[2][qy], qu);
                if constexpr (WITHV) interp3to4(Yv[0][qy], Yv[1][qy], Yv[2][qy], qv);
#pragma unroll
                for (int qz = 0; qz < 4; ++qz) fv[qz] = F(qu[qz], WITHV ? qv[qz] : (T)0);
                row[qy] = wsum4(fv);
            }
            plane[qx] = wsum4(row);
        }
        return wsum4(plane);
    }
}

template <int D>
__device__ __forceinline__ bool node_of(const Geom& g, long long idx, int& i, int& j, int& k)
{
    if (idx >= g.N) return false;
    i = (int)(idx % g.n[0]);
    long long r = idx / g.n[0];
    j = (int)(r % g.n[1]);
    k = D == 3 ? (int)(r / g.n[1]) : 0;
    return true;
}

template <typename T>
struct Cub {
    T a1, a2, a3;
    __device__ T operator()(T q, T) const { return cubic(q, a1, a2, a3); }
};
template <typename T>
struct Lin {  // f''(q) v
    T b0, b1, b2;
    __device__ T operator()(T q, T v) const { return fmaT(fmaT(b2, q, b1), q, b0) * v; }
};

// r(U): Allen-Cahn  r = L [N + kappa K u];  Cahn-Hilliard r_c = M K mu, r_mu = m mu - [N(c) + kappa K c]
template <typename T, int D, int MODEL>
__global__ __launch_bounds__(256) void k_residual(const T* __restrict__ U, T* __restrict__ r,
                                                  Geom g, Cub<T> F, T detJ, T kappa, T mob, T m)
{
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int i, j, k;
    if (!node_of<D>(g, idx, i, j, k)) return;
    T u[NB<D>::K];
    gather<T, D>(U, g, i, j, k, u);
    const T h = (T)g.h;
    const T Nn = detJ * quad_sum<T, D, false>(u, u, F);
    const T Ku = stiff<T, D>(u, h);
    if constexpr (MODEL == 0) {
        r[idx] = mob * (Nn + kappa * Ku);
    } else {
        T w[NB<D>::K];
        gather<T, D>(U + g.N, g, i, j, k, w);
        r[idx] = mob * stiff<T, D>(w, h);
        r[g.N + idx] = m * w[NB<D>::K / 2] - (Nn + kappa * Ku);
    }
}

// Jv for R = inv_dt M (U - U_old) + r(U)
template <typename T, int D, int MODEL>
__global__ __launch_bounds__(256) void k_jvp(const T* __restrict__ U, const T* __restrict__ V,
                                             T* __restrict__ Jv, Geom g, Lin<T> F, T detJ, T kappa,
                                             T mob, T m, T inv_dt)
{
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int i, j, k;
    if (!node_of<D>(g, idx, i, j, k)) return;
    T u[NB<D>::K], v[NB<D>::K];
    gather<T, D>(U, g, i, j, k, u);
    gather<T, D>(V, g, i, j, k, v);
    const T h = (T)g.h;
    const T Nv = detJ * quad_sum<T, D, true>(u, v, F);
    const T Kv = stiff<T, D>(v, h);
    const T vc = v[NB<D>::K / 2];
    if constexpr (MODEL == 0) {
        Jv[idx] = inv_dt * m * vc + mob * (Nv + kappa * Kv);
    } else {
        T w[NB<D>::K];
        gather<T, D>(V + g.N, g, i, j, k, w);
        Jv[idx] = inv_dt * m * vc + mob * stiff<T, D>(w, h);
        Jv[g.N + idx] = m * w[NB<D>::K / 2] - (Nv + kappa * Kv);
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
    mu[idx] = (detJ * quad_sum<T, D, false>(u, u, F) + kappa * stiff<T, D>(u, (T)g.h)) * inv_m;
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
    cout[idx] = c[idx] - dtM_over_m * stiff<T, D>(w, (T)g.h);
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
    const T r = detJ * quad_sum<T, D, false>(u, u, F) + kappa * stiff<T, D>(u, (T)g.h);
    out[idx] = u[NB<D>::K / 2] - dtL_over_m * r;
}

// ---- energy and mass ---------------------------------------------------------
// Each thread owns the element whose lower corner is its node.
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
        const double B[2][2] = {{GP, GM}, {GM, GP}};
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
                     const T* U, T* r, hipStream_t s)
{
    const double detJ = std::pow(0.5 * g.h, g.dim), m = std::pow(g.h, g.dim);
    DIM_SWITCH(g, {
        if (model == 0)
            k_residual<T, D, 0><<<grid_for(g), 256, 0, s>>>(U, r, g, cub_of<T>(f, 1.0), (T)detJ,
                                                             (T)kappa, (T)mob, (T)m);
        else
            k_residual<T, D, 1><<<grid_for(g), 256, 0, s>>>(U, r, g, cub_of<T>(f, 1.0), (T)detJ,
                                                             (T)kappa, (T)mob, (T)m);
    });
}

template <typename T>
void launch_jvp(const Geom& g, int model, const FreeEnergy& f, double kappa, double mob,
                double inv_dt, const T* U, const T* v, T* Jv, hipStream_t s)
{
    const double detJ = std::pow(0.5 * g.h, g.dim), m = std::pow(g.h, g.dim);
    Lin<T> F{(T)f.b0, (T)f.b1, (T)f.b2};
    DIM_SWITCH(g, {
        if (model == 0)
            k_jvp<T, D, 0><<<grid_for(g), 256, 0, s>>>(U, v, Jv, g, F, (T)detJ, (T)kappa, (T)mob,
                                                        (T)m, (T)inv_dt);
        else
            k_jvp<T, D, 1><<<grid_for(g), 256, 0, s>>>(U, v, Jv, g, F, (T)detJ, (T)kappa, (T)mob,
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
                                     T*, hipStream_t);                                            \
    template void launch_jvp<T>(const Geom&, int, const FreeEnergy&, double, double, double,       \
                                const T*, const T*, T*, hipStream_t);                             \
    template void launch_chem<T>(const Geom&, const FreeEnergy&, double, const T*, T*, hipStream_t); \
    template void launch_ch_update<T>(const Geom&, double, const T*, const T*, T*, hipStream_t);   \
    template void launch_ac_step<T>(const Geom&, const FreeEnergy&, double, double, const T*, T*,  \
                                    hipStream_t);                                                 \
    template void launch_energy<T>(const Geom&, const FreeEnergy&, double, const T*, double*,      \
                                   double*, hipStream_t);
INST(float)
INST(double)

}  // namespace pfk
