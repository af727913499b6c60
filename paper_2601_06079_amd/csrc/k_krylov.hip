// k_krylov.hip -- vector kernels of the Newton/GMRES solver (Sec. 2.3; the
// paper leaves the linear solver open, this library uses restarted GMRES).
//
// Vectors are FP32 or FP64 device arrays; every dot product and norm
// accumulates in FP64.  Reductions are two-stage with a fixed shape (a fixed
// number of blocks, each writing one partial per output, then one block per
// output summing the partials in index order), so results are bitwise
// reproducible run to run.
//
// Classical Gram-Schmidt with one re-orthogonalisation (CGS2) is fused into
// three sweeps over the Krylov basis V (k vectors, leading dimension ld):
//   k_mdot        h1 = V^T w
//   k_axpy_mdot   w <- w - V h1 and, in the same sweep, h2 = V^T w
//   k_axpy_norm   w <- w - V h2 and ||w||^2
#include <cmath>

#include "device.hpp"
#include "kernels.hpp"
#include "krylov.hpp"

namespace pfk {
namespace {

constexpr int KB = 256;  // threads per block of the reduction kernels

// block-wide sum of NV doubles held per thread; result valid in thread 0
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV])
{
    __shared__ double sh[KB / WAVE][NV];
#pragma unroll
    for (int i = 0; i < NV; ++i)
        for (int off = WAVE / 2; off > 0; off >>= 1) v[i] += __shfl_down(v[i], off, WAVE);
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < NV; ++i) sh[wv][i] = v[i];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            double s = 0.0;
            for (int w = 0; w < KB / WAVE; ++w) s += sh[w][i];
            v[i] = s;
        }
}

// h[i] partials: part[i * nb + block] = sum over this block's entries of V_i . w
template <typename T>
__global__ __launch_bounds__(KB) void k_mdot(const T* __restrict__ V, long long ld, int k,
                                             const T* __restrict__ w, long long n,
                                             double* __restrict__ part)
{
    const int nb = gridDim.x;
    for (int c0 = 0; c0 < k; c0 += 8) {
        double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (long long e = (long long)blockIdx.x * KB + threadIdx.x; e < n; e += (long long)nb * KB) {
            const double we = (double)w[e];
#pragma unroll
            for (int i = 0; i < 8; ++i)
                if (c0 + i < k) acc[i] = fma((double)V[(c0 + i) * ld + e], we, acc[i]);
        }
        block_sum<8>(acc);
        if (threadIdx.x == 0)
            for (int i = 0; i < 8 && c0 + i < k; ++i) part[(long long)(c0 + i) * nb + blockIdx.x] = acc[i];
        __syncthreads();
    }
}

// w <- w - sum_i h[i] V_i ; then part[i] = V_i . w  (KMAX >= k)
template <typename T, int KMAX>
__global__ __launch_bounds__(KB) void k_axpy_mdot(const T* __restrict__ V, long long ld, int k,
                                                  const double* __restrict__ h, T* __restrict__ w,
                                                  long long n, double* __restrict__ part)
{
    const int nb = gridDim.x;
    double acc[KMAX];
#pragma unroll
    for (int i = 0; i < KMAX; ++i) acc[i] = 0.0;
    for (long long e = (long long)blockIdx.x * KB + threadIdx.x; e < n; e += (long long)nb * KB) {
        T v[KMAX];
        double s = (double)w[e];
#pragma unroll
        for (int i = 0; i < KMAX; ++i)
            if (i < k) {
                v[i] = V[i * ld + e];
                s = fma(-h[i], (double)v[i], s);
            }
        const T wn = (T)s;
        w[e] = wn;
#pragma unroll
        for (int i = 0; i < KMAX; ++i)
            if (i < k) acc[i] = fma((double)v[i], (double)wn, acc[i]);
    }
    // reduce in groups of 8 to bound shared memory
#pragma unroll
    for (int c0 = 0; c0 < KMAX; c0 += 8) {
        double a[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) a[i] = acc[c0 + i];
        block_sum<8>(a);
        if (threadIdx.x == 0)
            for (int i = 0; i < 8 && c0 + i < k; ++i) part[(long long)(c0 + i) * nb + blockIdx.x] = a[i];
        __syncthreads();
    }
}

// w <- w - sum_i h[i] V_i ; part[0] = ||w||^2
template <typename T>
__global__ __launch_bounds__(KB) void k_axpy_norm(const T* __restrict__ V, long long ld, int k,
                                                  const double* __restrict__ h, T* __restrict__ w,
                                                  long long n, double* __restrict__ part)
{
    double acc[1] = {0.0};
    for (long long e = (long long)blockIdx.x * KB + threadIdx.x; e < n; e += (long long)gridDim.x * KB) {
        double s = (double)w[e];
        for (int i = 0; i < k; ++i) s = fma(-h[i], (double)V[i * ld + e], s);
        const T wn = (T)s;
        w[e] = wn;
        acc[0] = fma((double)wn, (double)wn, acc[0]);
    }
    block_sum<1>(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = acc[0];
}

// part[block] = partial ||x||^2 (x = a - b when b != nullptr)
template <typename T>
__global__ __launch_bounds__(KB) void k_norm2(const T* __restrict__ a, const T* __restrict__ b,
                                              long long n, double* __restrict__ part)
{
    double acc[1] = {0.0};
    for (long long e = (long long)blockIdx.x * KB + threadIdx.x; e < n; e += (long long)gridDim.x * KB) {
        const double x = b ? (double)a[e] - (double)b[e] : (double)a[e];
        acc[0] = fma(x, x, acc[0]);
    }
    block_sum<1>(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = acc[0];
}

// out[i] (op)= sum_b part[i * nb + b], one block per i, fixed order
__global__ __launch_bounds__(KB) void k_reduce_cols(const double* __restrict__ part, int nb, int k,
                                                    double* __restrict__ out, int accumulate)
{
    const int i = blockIdx.x;
    if (i >= k) return;
    double a[1] = {0.0};
    for (int b = threadIdx.x; b < nb; b += KB) a[0] += part[(long long)i * nb + b];
    block_sum<1>(a);
    if (threadIdx.x == 0) out[i] = accumulate ? out[i] + a[0] : a[0];
}

// v = w / sqrt(nrm2[0]) (0 when the norm is 0);  z = P^-1 v
// (for Cahn-Hilliard, tr = 1 applies the transposed 2x2 blocks)
template <typename T, int MODEL>
__global__ __launch_bounds__(KB) void k_normalize_prec(const T* __restrict__ w,
                                                       const double* __restrict__ nrm2,
                                                       T* __restrict__ v, T* __restrict__ z,
                                                       const T* __restrict__ pinv, long long N,
                                                       double sign, int tr)
{
    const long long i = (long long)blockIdx.x * KB + threadIdx.x;
    if (i >= N) return;
    const double nn = nrm2[0];
    const double inv = nn > 0.0 ? sign / sqrt(nn) : 0.0;
    if constexpr (MODEL == 0) {
        const T vi = (T)((double)w[i] * inv);
        v[i] = vi;
        if (z) z[i] = pinv ? vi * pinv[i] : vi;
    } else {
        const T vc = (T)((double)w[i] * inv), vm = (T)((double)w[N + i] * inv);
        v[i] = vc;
        v[N + i] = vm;
        if (z) {
            if (pinv) {
                const T* P = pinv + 4 * i;
                const T p01 = tr ? P[2] : P[1], p10 = tr ? P[1] : P[2];
                z[i] = P[0] * vc + p01 * vm;
                z[N + i] = p10 * vc + P[3] * vm;
            } else {
                z[i] = vc;
                z[N + i] = vm;
            }
        }
    }
}

// x += P^-1 (sum_i y[i] V_i)
template <typename T, int MODEL>
__global__ __launch_bounds__(KB) void k_update(const T* __restrict__ V, long long ld, int k,
                                               const double* __restrict__ y,
                                               const T* __restrict__ pinv, T* __restrict__ x,
                                               long long N, int tr)
{
    const long long i = (long long)blockIdx.x * KB + threadIdx.x;
    if (i >= N) return;
    if constexpr (MODEL == 0) {
        double s = 0.0;
        for (int j = 0; j < k; ++j) s = fma(y[j], (double)V[j * ld + i], s);
        const T t = (T)s;
        x[i] += pinv ? t * pinv[i] : t;
    } else {
        double sc = 0.0, sm = 0.0;
        for (int j = 0; j < k; ++j) {
            sc = fma(y[j], (double)V[j * ld + i], sc);
            sm = fma(y[j], (double)V[j * ld + N + i], sm);
        }
        const T tc = (T)sc, tm = (T)sm;
        if (pinv) {
            const T* P = pinv + 4 * i;
            const T p01 = tr ? P[2] : P[1], p10 = tr ? P[1] : P[2];
            x[i] += P[0] * tc + p01 * tm;
            x[N + i] += p10 * tc + P[3] * tm;
        } else {
            x[i] += tc;
            x[N + i] += tm;
        }
    }
}

// w = b - w   (turns J x into the residual b - J x), elementwise
template <typename T>
__global__ __launch_bounds__(KB) void k_rsub(const T* __restrict__ b, T* __restrict__ w, long long n)
{
    const long long i = (long long)blockIdx.x * KB + threadIdx.x;
    if (i < n) w[i] = b[i] - w[i];
}

// y = alpha * x (elementwise copy with scale)
template <typename T>
__global__ __launch_bounds__(KB) void k_scale(const T* __restrict__ x, T* __restrict__ y, double alpha,
                                              long long n)
{
    const long long i = (long long)blockIdx.x * KB + threadIdx.x;
    if (i < n) y[i] = (T)(alpha * (double)x[i]);
}

// x += y ; part[0] = max |y| partial, part[1] = max |x| partial  (for the rounding-floor test)
template <typename T>
__global__ __launch_bounds__(KB) void k_add_maxabs(T* __restrict__ x, const T* __restrict__ y,
                                                   long long n, double* __restrict__ part)
{
    double my = 0.0, mx = 0.0;
    for (long long e = (long long)blockIdx.x * KB + threadIdx.x; e < n; e += (long long)gridDim.x * KB) {
        const T v = x[e] + y[e];
        x[e] = v;
        my = fmax(my, fabs((double)y[e]));
        mx = fmax(mx, fabs((double)v));
    }
    __shared__ double s0[KB], s1[KB];
    s0[threadIdx.x] = my;
    s1[threadIdx.x] = mx;
    __syncthreads();
    for (int s = KB / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            s0[threadIdx.x] = fmax(s0[threadIdx.x], s0[threadIdx.x + s]);
            s1[threadIdx.x] = fmax(s1[threadIdx.x], s1[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s0[0];
        part[2 * blockIdx.x + 1] = s1[0];
    }
}

inline unsigned grid1(long long n) { return (unsigned)((n + KB - 1) / KB); }

}  // namespace

int krylov_blocks(long long n)
{
    // up to 4096 partial-sum blocks (16 waves per SIMD requested at 4 M entries)
    long long b = (n + KB - 1) / KB;
    return (int)(b < 4096 ? (b < 1 ? 1 : b) : 4096);
}

template <typename T>
void kr_mdot(const T* V, long long ld, int k, const T* w, long long n, double* part, double* out,
             int accumulate, hipStream_t s)
{
    const int nb = krylov_blocks(n);
    k_mdot<T><<<nb, KB, 0, s>>>(V, ld, k, w, n, part);
    k_reduce_cols<<<k, KB, 0, s>>>(part, nb, k, out, accumulate);
}

template <typename T>
void kr_axpy_mdot(const T* V, long long ld, int k, const double* h, T* w, long long n, double* part,
                  double* out, hipStream_t s)
{
    const int nb = krylov_blocks(n);
    if (k <= 8)
        k_axpy_mdot<T, 8><<<nb, KB, 0, s>>>(V, ld, k, h, w, n, part);
    else if (k <= 16)
        k_axpy_mdot<T, 16><<<nb, KB, 0, s>>>(V, ld, k, h, w, n, part);
    else if (k <= 32)
        k_axpy_mdot<T, 32><<<nb, KB, 0, s>>>(V, ld, k, h, w, n, part);
    else
        k_axpy_mdot<T, 72><<<nb, KB, 0, s>>>(V, ld, k, h, w, n, part);
    k_reduce_cols<<<k, KB, 0, s>>>(part, nb, k, out, 0);
}

template <typename T>
void kr_axpy_norm(const T* V, long long ld, int k, const double* h, T* w, long long n, double* part,
                  double* out, hipStream_t s)
{
    const int nb = krylov_blocks(n);
    k_axpy_norm<T><<<nb, KB, 0, s>>>(V, ld, k, h, w, n, part);
    k_reduce_cols<<<1, KB, 0, s>>>(part, nb, 1, out, 0);
}

template <typename T>
void kr_norm2(const T* a, const T* b, long long n, double* part, double* out, hipStream_t s)
{
    const int nb = krylov_blocks(n);
    k_norm2<T><<<nb, KB, 0, s>>>(a, b, n, part);
    k_reduce_cols<<<1, KB, 0, s>>>(part, nb, 1, out, 0);
}

template <typename T>
void kr_normalize_prec(int model, const T* w, const double* nrm2, T* v, T* z, const T* pinv,
                       long long N, double sign, hipStream_t s, int tr)
{
    if (model == 0)
        k_normalize_prec<T, 0><<<grid1(N), KB, 0, s>>>(w, nrm2, v, z, pinv, N, sign, tr);
    else
        k_normalize_prec<T, 1><<<grid1(N), KB, 0, s>>>(w, nrm2, v, z, pinv, N, sign, tr);
}

template <typename T>
void kr_update(int model, const T* V, long long ld, int k, const double* y, const T* pinv, T* x,
               long long N, hipStream_t s, int tr)
{
    if (model == 0)
        k_update<T, 0><<<grid1(N), KB, 0, s>>>(V, ld, k, y, pinv, x, N, tr);
    else
        k_update<T, 1><<<grid1(N), KB, 0, s>>>(V, ld, k, y, pinv, x, N, tr);
}

template <typename T>
void kr_rsub(const T* b, T* w, long long n, hipStream_t s)
{
    k_rsub<T><<<grid1(n), KB, 0, s>>>(b, w, n);
}

template <typename T>
void kr_scale(const T* x, T* y, double alpha, long long n, hipStream_t s)
{
    k_scale<T><<<grid1(n), KB, 0, s>>>(x, y, alpha, n);
}

template <typename T>
void kr_add_maxabs(T* x, const T* y, long long n, double* part, hipStream_t s)
{
    k_add_maxabs<T><<<krylov_blocks(n), KB, 0, s>>>(x, y, n, part);
}

#define INST_KR(T)                                                                              \
    template void kr_mdot<T>(const T*, long long, int, const T*, long long, double*, double*, int, \
                             hipStream_t);                                                      \
    template void kr_axpy_mdot<T>(const T*, long long, int, const double*, T*, long long, double*, \
                                  double*, hipStream_t);                                        \
    template void kr_axpy_norm<T>(const T*, long long, int, const double*, T*, long long, double*, \
                                  double*, hipStream_t);                                        \
    template void kr_norm2<T>(const T*, const T*, long long, double*, double*, hipStream_t);     \
    template void kr_normalize_prec<T>(int, const T*, const double*, T*, T*, const T*, long long, \
                                       double, hipStream_t, int);                               \
    template void kr_update<T>(int, const T*, long long, int, const double*, const T*, T*,       \
                               long long, hipStream_t, int);                                    \
    template void kr_rsub<T>(const T*, T*, long long, hipStream_t);                              \
    template void kr_scale<T>(const T*, T*, double, long long, hipStream_t);                     \
    template void kr_add_maxabs<T>(T*, const T*, long long, double*, hipStream_t);
INST_KR(float)
INST_KR(double)

}  // namespace pfk
