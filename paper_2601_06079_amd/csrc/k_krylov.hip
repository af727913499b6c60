// k_krylov.hip -- vector kernels of the Newton/GMRES solver (Sec. 2.3; the
// paper leaves the linear solver open, this library uses restarted GMRES).
//
// Vectors are FP32 or FP64 device arrays; every dot product and norm
// accumulates in FP64.  Reductions are two-stage with a fixed shape (a fixed
// number of blocks, each writing one partial per output, then one block per
// output summing the partials in index order), so results are bitwise
// reproducible run to run.
//
// Classical Gram-Schmidt with selective re-orthogonalisation is fused into two or
// three sweeps over the Krylov basis V (k vectors, leading dimension ld):
//   k_dots            h1 = V^T w and ||w||^2
//   k_axpy_dots       w <- w - V h1 and, in the same sweep, h2 = V^T w, ||w||^2
//   k_axpy_normalize  w <- w - V h2, whose norm is sqrt(||w||^2 - ||h2||^2)
//                     without another pass; the normalised vector is stored
//                     as the next basis vector and the preconditioner applied.
// When the first projection keeps at least a tenth of ||w||^2 (||w - V h1||^2 =
// ||w||^2 - ||h1||^2 >= ||w||^2 / 10), one projection is enough (selective
// re-orthogonalisation in the manner of Daniel, Gragg, Kaufman and Stewart: the
// orthogonality a projection loses grows with ||w|| / ||w - V h1||, here at most
// sqrt(10)): k_axpy_dots and the reduction after it return at once and
// k_axpy_normalize projects w with h1.  Every kernel takes that decision from the same
// reduced values in the same order, so all agree; the host sees h2 = 0.
#include <algorithm>
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

// ---- Gram-Schmidt sweeps ----------------------------------------------------
// Each lane streams VW consecutive entries per load (16 bytes: 4 floats or 2
// doubles) of w and of every basis vector; the column loop is unrolled to KMAX
// (>= k) so that all loads of one chunk are in flight together.  Columns
// i >= k re-load column k - 1 (a cache hit) and are masked out, which keeps
// the unrolled loop free of branches.

template <typename T, int VW>
struct alignas(VW * sizeof(T)) Pack {
    T v[VW];
};

template <typename T, int VW>
__device__ __forceinline__ Pack<T, VW> ldp(const T* p)
{
    return *reinterpret_cast<const Pack<T, VW>*>(p);
}

template <typename T, int VW>
__device__ __forceinline__ void stp(T* p, const Pack<T, VW>& x)
{
    *reinterpret_cast<Pack<T, VW>*>(p) = x;
}

// write the block sums of acc[0..cnt) to part[i * nb + block]
template <int NV>
__device__ __forceinline__ void store_partials(double (&acc)[NV], int cnt, double* __restrict__ part)
{
    const int nb = gridDim.x;
#pragma unroll
    for (int c0 = 0; c0 < NV; c0 += 8) {
        double a[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) a[i] = c0 + i < NV ? acc[c0 + i] : 0.0;
        block_sum<8>(a);
        if (threadIdx.x == 0)
            for (int i = 0; i < 8 && c0 + i < cnt; ++i) part[(long long)(c0 + i) * nb + blockIdx.x] = a[i];
        __syncthreads();
    }
}

// The re-orthogonalisation test on the first pass's reduced values h1[0..k)
// (= V^T w) and h1[k] (= ||w||^2): true when one projection is enough.  nn
// receives ||w - V h1||^2 = ||w||^2 - ||h1||^2.
// thr: the share of ||w||^2 one projection must keep (default 0.1)
__device__ __forceinline__ bool cgs_one_pass(const double* __restrict__ h1, int k, double thr, double& nn)
{
    double hsq = 0.0;
    for (int i = 0; i < k; ++i) hsq = fma(h1[i], h1[i], hsq);
    nn = h1[k] - hsq;
    return nn >= thr * h1[k];
}

// part[i * nb + block] = this block's share of V_i . w  (i < k <= KMAX),
// part[k * nb + block] = its share of ||w||^2
template <typename T, int KMAX, int VW>
__global__ __launch_bounds__(KB) void k_dots(const T* __restrict__ V, long long ld, int k,
                                             const T* __restrict__ w, long long n,
                                             double* __restrict__ part)
{
    double acc[KMAX + 1];
#pragma unroll
    for (int i = 0; i <= KMAX; ++i) acc[i] = 0.0;
    const long long nv = n / VW;
    for (long long e = (long long)blockIdx.x * KB + threadIdx.x; e < nv; e += (long long)gridDim.x * KB) {
        const Pack<T, VW> wv = ldp<T, VW>(w + e * VW);
        Pack<T, VW> vv[KMAX];
#pragma unroll
        for (int i = 0; i < KMAX; ++i) vv[i] = ldp<T, VW>(V + (i < k ? i : k - 1) * ld + e * VW);
#pragma unroll
        for (int i = 0; i < KMAX; ++i)
#pragma unroll
            for (int l = 0; l < VW; ++l) acc[i] = fma((double)vv[i].v[l], (double)wv.v[l], acc[i]);
#pragma unroll
        for (int l = 0; l < VW; ++l) acc[KMAX] = fma((double)wv.v[l], (double)wv.v[l], acc[KMAX]);
    }
    // ||w||^2 to slot k so that the partial columns are contiguous
    double out[KMAX + 1];
#pragma unroll
    for (int i = 0; i <= KMAX; ++i) out[i] = i < k ? acc[i] : (i == k ? acc[KMAX] : 0.0);
    store_partials<KMAX + 1>(out, k + 1, part);
}

// w <- w - V h ; part[i * nb + block] = share of V_i . w (i < k), part[k * nb + block] = share of ||w||^2
// (returns at once when one projection is enough: see cgs_one_pass)
template <typename T, int KMAX, int VW>
__global__ __launch_bounds__(KB) void k_axpy_dots(const T* __restrict__ V, long long ld, int k,
                                                  const double* __restrict__ h, T* __restrict__ w,
                                                  long long n, double* __restrict__ part, double thr)
{
    double nn1;
    if (cgs_one_pass(h, k, thr, nn1)) return;  // uniform over the grid
    double hh[KMAX], acc[KMAX + 1];
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
        hh[i] = i < k ? h[i] : 0.0;
        acc[i] = 0.0;
    }
    acc[KMAX] = 0.0;
    const long long nv = n / VW;
    for (long long e = (long long)blockIdx.x * KB + threadIdx.x; e < nv; e += (long long)gridDim.x * KB) {
        Pack<T, VW> wv = ldp<T, VW>(w + e * VW);
        Pack<T, VW> vv[KMAX];
#pragma unroll
        for (int i = 0; i < KMAX; ++i) vv[i] = ldp<T, VW>(V + (i < k ? i : k - 1) * ld + e * VW);
#pragma unroll
        for (int l = 0; l < VW; ++l) {
            double s = (double)wv.v[l];
#pragma unroll
            for (int i = 0; i < KMAX; ++i) s = fma(-hh[i], (double)vv[i].v[l], s);
            wv.v[l] = (T)s;
        }
        stp<T, VW>(w + e * VW, wv);
#pragma unroll
        for (int l = 0; l < VW; ++l) {
            const double wn = (double)wv.v[l];
#pragma unroll
            for (int i = 0; i < KMAX; ++i) acc[i] = fma((double)vv[i].v[l], wn, acc[i]);
            acc[KMAX] = fma(wn, wn, acc[KMAX]);
        }
    }
    // move ||w||^2 to slot k so that the partial columns are contiguous
    double out[KMAX + 1];
#pragma unroll
    for (int i = 0; i <= KMAX; ++i) out[i] = i < k ? acc[i] : (i == k ? acc[KMAX] : 0.0);
    store_partials<KMAX + 1>(out, k + 1, part);
}

// x[0..VW) -= V h over one chunk of one plane (columns masked as above)
template <typename T, int KMAX, int VW>
__device__ __forceinline__ void axpy_chunk(const T* __restrict__ V, long long ld, int k,
                                           const double (&hh)[KMAX], long long off, double (&x)[VW])
{
    Pack<T, VW> vv[KMAX];
#pragma unroll
    for (int i = 0; i < KMAX; ++i) vv[i] = ldp<T, VW>(V + (i < k ? i : k - 1) * ld + off);
#pragma unroll
    for (int l = 0; l < VW; ++l)
#pragma unroll
        for (int i = 0; i < KMAX; ++i) x[l] = fma(-hh[i], (double)vv[i].v[l], x[l]);
}

// Last Gram-Schmidt sweep fused with the normalisation and the preconditioner:
//   w'' = w - V h  (h: the second-pass coefficients h2, sums2[k] = ||w||^2 after
//   the first pass; or, when one projection is enough, h1 on the untouched w),
//   ||w''||^2 = ||w||^2 - ||h||^2  (h is the projection of w on V),
//   v = w'' / ||w''||  -> vnext,   z = P^-1 v.
// nrm2[0] receives ||w''||^2.  With one projection the second-pass outputs h2 are
// set to 0 (device and host copies) for the Hessenberg column.  Node-indexed: VW
// nodes per lane, planes at offset N (MODEL 1: the c and mu planes with per-node
// 2x2 blocks; MODEL 2: the three planes of the coupled model with 3x3 blocks).
template <typename T, int KMAX, int VW, int MODEL>
__global__ __launch_bounds__(KB) void k_axpy_normalize(const T* __restrict__ V, long long ld, int k,
                                                       const double* __restrict__ sums1,
                                                       double* __restrict__ sums2,
                                                       double* __restrict__ sums2_host,
                                                       const T* __restrict__ w, T* __restrict__ vnext,
                                                       T* __restrict__ z, const T* __restrict__ pinv,
                                                       long long N, int tr, double* __restrict__ nrm2,
                                                       double* __restrict__ nrm2_host, double thr)
{
    double nn;
    const bool one = cgs_one_pass(sums1, k, thr, nn);
    const double* sums = one ? sums1 : sums2;
    double hh[KMAX];
    double hsq = 0.0;
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
        hh[i] = i < k ? sums[i] : 0.0;
        hsq = fma(hh[i], hh[i], hsq);
    }
    if (!one) nn = sums[k] - hsq;
    const double inv = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        nrm2[0] = nn > 0.0 ? nn : 0.0;
        if (nrm2_host) __hip_atomic_store(nrm2_host, nn > 0.0 ? nn : 0.0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        if (one)
            for (int i = 0; i <= k; ++i) {
                sums2[i] = 0.0;
                if (sums2_host) __hip_atomic_store(sums2_host + i, 0.0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            }
    }
    const long long nv = N / VW;
    for (long long e = (long long)blockIdx.x * KB + threadIdx.x; e < nv; e += (long long)gridDim.x * KB) {
        const long long o = e * VW;
        double xc[VW];
        {
            const Pack<T, VW> wv = ldp<T, VW>(w + o);
#pragma unroll
            for (int l = 0; l < VW; ++l) xc[l] = (double)wv.v[l];
        }
        axpy_chunk<T, KMAX, VW>(V, ld, k, hh, o, xc);
        Pack<T, VW> vc;
#pragma unroll
        for (int l = 0; l < VW; ++l) vc.v[l] = (T)((T)xc[l] * inv);
        stp<T, VW>(vnext + o, vc);
        if constexpr (MODEL == 0) {
            Pack<T, VW> zc;
            if (pinv) {
                const Pack<T, VW> pv = ldp<T, VW>(pinv + o);
#pragma unroll
                for (int l = 0; l < VW; ++l) zc.v[l] = vc.v[l] * pv.v[l];
            } else {
                zc = vc;
            }
            stp<T, VW>(z + o, zc);
        } else if constexpr (MODEL == 2) {
            // three planes (coupled model), 3x3 blocks
            Pack<T, VW> vv[3];
            vv[0] = vc;
#pragma unroll
            for (int f = 1; f < 3; ++f) {
                double xf[VW];
                const Pack<T, VW> wv = ldp<T, VW>(w + f * N + o);
#pragma unroll
                for (int l = 0; l < VW; ++l) xf[l] = (double)wv.v[l];
                axpy_chunk<T, KMAX, VW>(V, ld, k, hh, f * N + o, xf);
#pragma unroll
                for (int l = 0; l < VW; ++l) vv[f].v[l] = (T)((T)xf[l] * inv);
                stp<T, VW>(vnext + f * N + o, vv[f]);
            }
            Pack<T, VW> zz[3];
#pragma unroll
            for (int l = 0; l < VW; ++l) {
                if (pinv) {
                    const T* P = pinv + 9 * (o + l);
#pragma unroll
                    for (int r = 0; r < 3; ++r) {
                        T acc = (T)0;
#pragma unroll
                        for (int cc = 0; cc < 3; ++cc) acc += (tr ? P[3 * cc + r] : P[3 * r + cc]) * vv[cc].v[l];
                        zz[r].v[l] = acc;
                    }
                } else {
#pragma unroll
                    for (int r = 0; r < 3; ++r) zz[r].v[l] = vv[r].v[l];
                }
            }
#pragma unroll
            for (int f = 0; f < 3; ++f) stp<T, VW>(z + f * N + o, zz[f]);
        } else {
            double xm[VW];
            {
                const Pack<T, VW> wv = ldp<T, VW>(w + N + o);
#pragma unroll
                for (int l = 0; l < VW; ++l) xm[l] = (double)wv.v[l];
            }
            axpy_chunk<T, KMAX, VW>(V, ld, k, hh, N + o, xm);
            Pack<T, VW> vm;
#pragma unroll
            for (int l = 0; l < VW; ++l) vm.v[l] = (T)((T)xm[l] * inv);
            stp<T, VW>(vnext + N + o, vm);
            Pack<T, VW> zc, zm;
            if (pinv) {
#pragma unroll
                for (int l = 0; l < VW; ++l) {
                    const T* P = pinv + 4 * (o + l);
                    const T p01 = tr ? P[2] : P[1], p10 = tr ? P[1] : P[2];
                    zc.v[l] = P[0] * vc.v[l] + p01 * vm.v[l];
                    zm.v[l] = p10 * vc.v[l] + P[3] * vm.v[l];
                }
            } else {
                zc = vc;
                zm = vm;
            }
            stp<T, VW>(z + o, zc);
            stp<T, VW>(z + N + o, zm);
        }
    }
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
// (host: optional host-mapped copy of out, written with system-scope stores so
// that the host reads it once the kernel has completed)
// (skip_h1: the first-pass values of a Gram-Schmidt step; when one projection is
// enough there -- see cgs_one_pass -- there is nothing to reduce)
__global__ __launch_bounds__(KB) void k_reduce_cols(const double* __restrict__ part, int nb, int k,
                                                    double* __restrict__ out, int accumulate,
                                                    double* __restrict__ host = nullptr,
                                                    const double* __restrict__ skip_h1 = nullptr, int skip_k = 0,
                                                    double skip_thr = 0.0)
{
    const int i = blockIdx.x;
    if (i >= k) return;
    if (skip_h1) {
        double nn;
        if (cgs_one_pass(skip_h1, skip_k, skip_thr, nn)) return;  // uniform over the grid
    }
    double a[1] = {0.0};
    for (int b = threadIdx.x; b < nb; b += KB) a[0] += part[(long long)i * nb + b];
    block_sum<1>(a);
    if (threadIdx.x == 0) {
        const double r = accumulate ? out[i] + a[0] : a[0];
        out[i] = r;
        if (host) __hip_atomic_store(host + i, r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
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
    } else if constexpr (MODEL == 2) {
        T vv[3];
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            vv[f] = (T)((double)w[f * N + i] * inv);
            v[f * N + i] = vv[f];
        }
        if (z) {
            const T* P = pinv ? pinv + 9 * i : nullptr;
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                T acc = (T)0;
                if (P) {
#pragma unroll
                    for (int cc = 0; cc < 3; ++cc) acc += (tr ? P[3 * cc + r] : P[3 * r + cc]) * vv[cc];
                } else {
                    acc = vv[r];
                }
                z[r * N + i] = acc;
            }
        }
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
    } else if constexpr (MODEL == 2) {
        T t[3];
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            double sf = 0.0;
            for (int j = 0; j < k; ++j) sf = fma(y[j], (double)V[j * ld + f * N + i], sf);
            t[f] = (T)sf;
        }
        const T* P = pinv ? pinv + 9 * i : nullptr;
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            T acc = (T)0;
            if (P) {
#pragma unroll
                for (int cc = 0; cc < 3; ++cc) acc += (tr ? P[3 * cc + r] : P[3 * r + cc]) * t[cc];
            } else {
                acc = t[r];
            }
            x[r * N + i] += acc;
        }
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

// out[0] = max_b part[2b], out[1] = max_b part[2b+1]; one block (host: optional
// host-mapped copy, system-scope stores)
__global__ __launch_bounds__(KB) void k_max_pairs(const double* __restrict__ part, int nb,
                                                  double* __restrict__ out, double* __restrict__ host)
{
    __shared__ double s0[KB], s1[KB];
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < nb; i += KB) {
        a = fmax(a, part[2 * i]);
        b = fmax(b, part[2 * i + 1]);
    }
    s0[threadIdx.x] = a;
    s1[threadIdx.x] = b;
    __syncthreads();
    for (int st = KB / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            s0[threadIdx.x] = fmax(s0[threadIdx.x], s0[threadIdx.x + st]);
            s1[threadIdx.x] = fmax(s1[threadIdx.x], s1[threadIdx.x + st]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = s0[0];
        out[1] = s1[0];
        if (host) {
            __hip_atomic_store(host, s0[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            __hip_atomic_store(host + 1, s1[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
}

// ---- preconditioned conjugate gradients ---------------------------------------

// sums of nb (a, b) pairs in a fixed order, the same in every block
__device__ __forceinline__ void cg_reduce_pairs(const double* __restrict__ part, int nb, double& a, double& b)
{
    __shared__ double res[2];
    double v[2] = {0.0, 0.0};
    for (int i = threadIdx.x; i < nb; i += KB) {
        v[0] += part[2 * i];
        v[1] += part[2 * i + 1];
    }
    block_sum<2>(v);
    if (threadIdx.x == 0) {
        res[0] = v[0];
        res[1] = v[1];
    }
    __syncthreads();
    a = res[0];
    b = res[1];
}

// The done flag as one block-wide decision: block 0 of a step kernel may set it
// while other blocks start, and a block whose waves disagreed would split at
// its barriers.
__device__ __forceinline__ bool cg_block_done(const double* st)
{
    __shared__ int flag;
    if (threadIdx.x == 0) flag = st[CG_DONE] != 0.0;
    __syncthreads();
    return flag != 0;
}

__device__ __forceinline__ void cg_host_store(double* host, int i, double v)
{
    __hip_atomic_store(&host[i], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

template <typename T>
__global__ __launch_bounds__(KB) void k_cg_start(const T* __restrict__ b, const T* __restrict__ pinv,
                                                 T* __restrict__ r, T* __restrict__ z, T* __restrict__ p,
                                                 T* __restrict__ x, long long n, double* __restrict__ part,
                                                 double* __restrict__ st, double* __restrict__ host,
                                                 double tol2, double maxit)
{
    double v[2] = {0.0, 0.0};
    for (long long e = (long long)blockIdx.x * KB + threadIdx.x; e < n; e += (long long)gridDim.x * KB) {
        const T bv = b[e];
        const T zv = pinv ? pinv[e] * bv : bv;
        r[e] = bv;
        z[e] = zv;
        p[e] = T(0);
        x[e] = T(0);
        v[0] += (double)bv * (double)zv;
        v[1] += (double)bv * (double)bv;
    }
    block_sum<2>(v);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = v[0];
        part[2 * blockIdx.x + 1] = v[1];
        if (blockIdx.x == 0) {
            for (int i = 0; i < CG_NSTATE; ++i) st[i] = 0.0;
            st[CG_TOL2] = tol2;
            st[CG_MAXIT] = maxit;
            for (int i = 0; i < 3; ++i) cg_host_store(host, i, 0.0);
        }
    }
}

template <typename T>
__global__ __launch_bounds__(KB) void k_cg_dir(const T* __restrict__ z, T* __restrict__ p, long long n,
                                               const double* __restrict__ part, int nb, double* st,
                                               double* __restrict__ host)
{
    __shared__ double sc[2];
    if (cg_block_done(st)) return;
    double rz, rr;
    cg_reduce_pairs(part, nb, rz, rr);
    if (threadIdx.x == 0) {
        const double its = st[CG_ITS];
        double done = 0.0;
        if (!(std::isfinite(rz) && std::isfinite(rr))) done = CG_NONFINITE;
        else if (rr <= st[CG_TOL2]) done = CG_CONVERGED;
        else if (its >= st[CG_MAXIT]) done = CG_MAXITS;
        else if (!(rz > 0.0)) done = CG_BREAKDOWN;
        sc[0] = done;
        sc[1] = (done == 0.0 && its > 0.0) ? rz / st[CG_RZOLD] : 0.0;
        if (blockIdx.x == 0) {
            st[CG_RZ] = rz;
            st[CG_RR] = rr;
            cg_host_store(host, CG_H_RR, rr);
            cg_host_store(host, CG_H_ITS, its);
            if (done != 0.0) {
                st[CG_DONE] = done;
                cg_host_store(host, CG_H_DONE, done);
            }
        }
    }
    __syncthreads();
    if (sc[0] != 0.0) return;
    const T beta = (T)sc[1];
    for (long long e = (long long)blockIdx.x * KB + threadIdx.x; e < n; e += (long long)gridDim.x * KB)
        p[e] = fmaT(beta, p[e], z[e]);
}

template <typename T>
__global__ __launch_bounds__(KB) void k_cg_pq(const T* __restrict__ p, const T* __restrict__ q, long long n,
                                              double* __restrict__ part2, const double* __restrict__ st)
{
    if (cg_block_done(st)) return;
    double v[1] = {0.0};
    for (long long e = (long long)blockIdx.x * KB + threadIdx.x; e < n; e += (long long)gridDim.x * KB)
        v[0] += (double)p[e] * (double)q[e];
    block_sum<1>(v);
    if (threadIdx.x == 0) part2[blockIdx.x] = v[0];
}

template <typename T>
__global__ __launch_bounds__(KB) void k_cg_alpha(T* __restrict__ x, T* __restrict__ r, T* __restrict__ z,
                                                 const T* __restrict__ p, const T* __restrict__ q,
                                                 const T* __restrict__ pinv, long long n,
                                                 const double* __restrict__ part2, int nb2,
                                                 double* __restrict__ part, double* st, double* __restrict__ host)
{
    __shared__ double sc[1];
    __shared__ double red[1];
    if (cg_block_done(st)) return;
    double v1[1] = {0.0};
    for (int i = threadIdx.x; i < nb2; i += KB) v1[0] += part2[i];
    block_sum<1>(v1);
    if (threadIdx.x == 0) red[0] = v1[0];
    __syncthreads();
    const double pq = red[0];
    if (threadIdx.x == 0) {
        const bool ok = pq > 0.0 && std::isfinite(pq);
        sc[0] = ok ? st[CG_RZ] / pq : 0.0;
        if (blockIdx.x == 0) {
            if (ok) {
                st[CG_RZOLD] = st[CG_RZ];
                st[CG_ITS] = st[CG_ITS] + 1.0;
                cg_host_store(host, CG_H_ITS, st[CG_ITS]);
            } else {
                // p.q <= 0: the operator is not positive definite along p
                st[CG_DONE] = std::isfinite(pq) ? (double)CG_BREAKDOWN : (double)CG_NONFINITE;
                cg_host_store(host, CG_H_DONE, st[CG_DONE]);
            }
        }
    }
    __syncthreads();
    if (sc[0] == 0.0) return;
    const T alpha = (T)sc[0];
    double v[2] = {0.0, 0.0};
    for (long long e = (long long)blockIdx.x * KB + threadIdx.x; e < n; e += (long long)gridDim.x * KB) {
        x[e] = fmaT(alpha, p[e], x[e]);
        const T rv = fmaT(-alpha, q[e], r[e]);
        const T zv = pinv ? pinv[e] * rv : rv;
        r[e] = rv;
        z[e] = zv;
        v[0] += (double)rv * (double)zv;
        v[1] += (double)rv * (double)rv;
    }
    block_sum<2>(v);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = v[0];
        part[2 * blockIdx.x + 1] = v[1];
    }
}

inline unsigned grid1(long long n) { return (unsigned)((n + KB - 1) / KB); }

}  // namespace

int krylov_blocks(long long n)
{
    // at least 16 entries per thread, at most 1024 partial-sum blocks (4 per CU)
    long long b = (n + 16 * KB - 1) / (16 * KB);
    return (int)(b < 1024 ? (b < 1 ? 1 : b) : 1024);
}

namespace {

// 16-byte lanes when every plane offset keeps that alignment, else scalar lanes
template <typename T>
bool wide_ok(long long N)
{
    return N % (long long)(16 / sizeof(T)) == 0;
}

// Blocks of `kernel` that fit on the device at once (its occupancy times the CU
// count), queried once per kernel.  A sweep launched on more blocks than that
// runs a partial second round; fewer, longer-running blocks stream the same bytes.
template <typename K>
int resident_blocks(K kernel)
{
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, KB, 0) != hipSuccess ||
        hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        return 1 << 30;  // no cap
    }
    return (per_cu < 1 ? 1 : per_cu) * (cus < 1 ? 1 : cus);
}

template <typename T, int KMAX, int VW>
void cgs2_k(int model, const T* V, long long ld, int k, T* w, T* vnext, T* z, const T* pinv,
            long long N, long long n, double* part, const KrOut& o, int tr, hipStream_t s)
{
    static const int cap_dots = resident_blocks(k_dots<T, KMAX, VW>);
    static const int cap_axpy = resident_blocks(k_axpy_dots<T, KMAX, VW>);
    static const int cap_norm0 = resident_blocks(k_axpy_normalize<T, KMAX, VW, 0>);
    static const int cap_norm1 = resident_blocks(k_axpy_normalize<T, KMAX, VW, 1>);
    static const int cap_norm2 = resident_blocks(k_axpy_normalize<T, KMAX, VW, 2>);
    const int cap_norm = model == 0 ? cap_norm0 : (model == 1 ? cap_norm1 : cap_norm2);
    const int nb = krylov_blocks(n);
    const int nb1 = std::min(nb, cap_dots), nb2 = std::min(nb, cap_axpy);
    k_dots<T, KMAX, VW><<<nb1, KB, 0, s>>>(V, ld, k, w, n, part);
    k_reduce_cols<<<k + 1, KB, 0, s>>>(part, nb1, k + 1, o.h1, 0, o.host_h1);
    const int tv = tune_gs_reorth();
    const double thr = tv == 0 ? 0.1 : (tv - 1) / 1000.0;
    k_axpy_dots<T, KMAX, VW><<<nb2, KB, 0, s>>>(V, ld, k, o.h1, w, n, part, thr);
    k_reduce_cols<<<k + 1, KB, 0, s>>>(part, nb2, k + 1, o.h2, 0, o.host_h2, o.h1, k, thr);
    const long long chunks = (N / VW + KB - 1) / KB;
    const int nbn = (int)std::max<long long>(1, std::min<long long>(chunks, cap_norm));
    if (model == 0)
        k_axpy_normalize<T, KMAX, VW, 0><<<nbn, KB, 0, s>>>(V, ld, k, o.h1, o.h2, o.host_h2, w, vnext, z, pinv, N, tr,
                                                            o.nrm2, o.host_nrm2, thr);
    else if (model == 1)
        k_axpy_normalize<T, KMAX, VW, 1><<<nbn, KB, 0, s>>>(V, ld, k, o.h1, o.h2, o.host_h2, w, vnext, z, pinv, N, tr,
                                                            o.nrm2, o.host_nrm2, thr);
    else
        k_axpy_normalize<T, KMAX, VW, 2><<<nbn, KB, 0, s>>>(V, ld, k, o.h1, o.h2, o.host_h2, w, vnext, z, pinv, N, tr,
                                                            o.nrm2, o.host_nrm2, thr);
}

template <typename T, int VW>
void cgs2_v(int model, const T* V, long long ld, int k, T* w, T* vnext, T* z, const T* pinv,
            long long N, long long n, double* part, const KrOut& o, int tr, hipStream_t s)
{
#define PF_CGS2(KM) cgs2_k<T, KM, VW>(model, V, ld, k, w, vnext, z, pinv, N, n, part, o, tr, s)
    if (k <= 4) PF_CGS2(4);
    else if (k <= 8) PF_CGS2(8);
    else if (k <= 12) PF_CGS2(12);
    else if (k <= 16) PF_CGS2(16);
    else if (k <= 24) PF_CGS2(24);
    else PF_CGS2(32);
#undef PF_CGS2
}

}  // namespace

template <typename T>
int kr_cgs2(int model, const T* V, long long ld, int k, T* w, T* vnext, T* z, const T* pinv,
            long long N, double* part, const KrOut& o, hipStream_t s, int tr)
{
    if (k < 1 || k > KR_MAXK) return -1;
    const long long n = (model == 0 ? 1 : model == 1 ? 2 : 3) * N;
    constexpr int VW = 16 / sizeof(T);
    if (wide_ok<T>(N))
        cgs2_v<T, VW>(model, V, ld, k, w, vnext, z, pinv, N, n, part, o, tr, s);
    else
        cgs2_v<T, 1>(model, V, ld, k, w, vnext, z, pinv, N, n, part, o, tr, s);
    return 0;
}

template <typename T>
void kr_norm2(const T* a, const T* b, long long n, double* part, double* out, hipStream_t s,
              double* host)
{
    const int nb = krylov_blocks(n);
    k_norm2<T><<<nb, KB, 0, s>>>(a, b, n, part);
    k_reduce_cols<<<1, KB, 0, s>>>(part, nb, 1, out, 0, host);
}

template <typename T>
void kr_normalize_prec(int model, const T* w, const double* nrm2, T* v, T* z, const T* pinv,
                       long long N, double sign, hipStream_t s, int tr)
{
    if (model == 0)
        k_normalize_prec<T, 0><<<grid1(N), KB, 0, s>>>(w, nrm2, v, z, pinv, N, sign, tr);
    else if (model == 1)
        k_normalize_prec<T, 1><<<grid1(N), KB, 0, s>>>(w, nrm2, v, z, pinv, N, sign, tr);
    else
        k_normalize_prec<T, 2><<<grid1(N), KB, 0, s>>>(w, nrm2, v, z, pinv, N, sign, tr);
}

template <typename T>
void kr_update(int model, const T* V, long long ld, int k, const double* y, const T* pinv, T* x,
               long long N, hipStream_t s, int tr)
{
    if (model == 0)
        k_update<T, 0><<<grid1(N), KB, 0, s>>>(V, ld, k, y, pinv, x, N, tr);
    else if (model == 1)
        k_update<T, 1><<<grid1(N), KB, 0, s>>>(V, ld, k, y, pinv, x, N, tr);
    else
        k_update<T, 2><<<grid1(N), KB, 0, s>>>(V, ld, k, y, pinv, x, N, tr);
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
void kr_add_maxabs(T* x, const T* y, long long n, double* part, double* out, hipStream_t s,
                   double* host)
{
    const int nb = krylov_blocks(n);
    k_add_maxabs<T><<<nb, KB, 0, s>>>(x, y, n, part);
    k_max_pairs<<<1, KB, 0, s>>>(part, nb, out, host);
}

#define INST_KR(T)                                                                              \
    template int kr_cgs2<T>(int, const T*, long long, int, T*, T*, T*, const T*, long long, double*, \
                            const KrOut&, hipStream_t, int);                                     \
    template void kr_norm2<T>(const T*, const T*, long long, double*, double*, hipStream_t, double*); \
    template void kr_normalize_prec<T>(int, const T*, const double*, T*, T*, const T*, long long, \
                                       double, hipStream_t, int);                               \
    template void kr_update<T>(int, const T*, long long, int, const double*, const T*, T*,       \
                               long long, hipStream_t, int);                                    \
    template void kr_rsub<T>(const T*, T*, long long, hipStream_t);                              \
    template void kr_scale<T>(const T*, T*, double, long long, hipStream_t);                     \
    template void kr_add_maxabs<T>(T*, const T*, long long, double*, double*, hipStream_t, double*);
INST_KR(float)
INST_KR(double)

int cg_blocks(long long n) { return krylov_blocks(n); }

template <typename T>
void cg_start(const T* b, const T* pinv, T* r, T* z, T* p, T* x, long long n, double* part, double* st,
              double* host, double tol2, int maxit, hipStream_t s)
{
    k_cg_start<T><<<cg_blocks(n), KB, 0, s>>>(b, pinv, r, z, p, x, n, part, st, host, tol2, (double)maxit);
}
template <typename T>
void cg_dir(const T* z, T* p, long long n, const double* part, double* st, double* host, hipStream_t s)
{
    const int nb = cg_blocks(n);
    k_cg_dir<T><<<nb, KB, 0, s>>>(z, p, n, part, nb, st, host);
}
template <typename T>
void cg_pq(const T* p, const T* q, long long n, double* part2, const double* st, hipStream_t s)
{
    k_cg_pq<T><<<cg_blocks(n), KB, 0, s>>>(p, q, n, part2, st);
}
template <typename T>
void cg_alpha(T* x, T* r, T* z, const T* p, const T* q, const T* pinv, long long n, const double* part2,
              double* part, double* st, double* host, hipStream_t s, int nb2)
{
    const int nb = cg_blocks(n);
    k_cg_alpha<T><<<nb, KB, 0, s>>>(x, r, z, p, q, pinv, n, part2, nb2 > 0 ? nb2 : nb, part, st, host);
}
#define PF_CG_INST(T)                                                                                      \
    template void cg_start<T>(const T*, const T*, T*, T*, T*, T*, long long, double*, double*, double*,    \
                              double, int, hipStream_t);                                                   \
    template void cg_dir<T>(const T*, T*, long long, const double*, double*, double*, hipStream_t);        \
    template void cg_pq<T>(const T*, const T*, long long, double*, const double*, hipStream_t);            \
    template void cg_alpha<T>(T*, T*, T*, const T*, const T*, const T*, long long, const double*, double*, \
                              double*, double*, hipStream_t, int);
PF_CG_INST(float)
PF_CG_INST(double)
#undef PF_CG_INST

}  // namespace pfk
