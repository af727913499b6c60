// k_grain.hip -- multi-order-parameter Allen-Cahn (grain growth) on 2-D grids:
// p order parameters eta_1..eta_p, each following Eq. 1 with the same L and
// kappa, coupled through the multi-well energy of the grain-growth literature
//     f = sum_i (eta_i^4/4 - eta_i^2/2) + gamma sum_{i<j} eta_i^2 eta_j^2 + 1/4,
//     df/deta_i = eta_i (eta_i^2 (1 - 2 gamma) - 1 + 2 gamma S),  S = sum_j eta_j^2,
// so the coupling enters each Gauss point only through S (O(p) work per point,
// not O(p^2)); all order parameters are updated together, which is the paper's
// vectorisation across phase-field variables (Sec. 2.4).
//
// k_gg_tile2d: one 256-thread block per 16 x 16 tile of output nodes.
//   A. all p fields of the 18 x 18 node patch (halo 1) are staged in LDS;
//   B. each of the 17 x 17 patch elements forms S at its four Gauss points;
//   C. per field: each element evaluates df/deta_i at its Gauss points and
//      projects it onto its four nodes (LDS); each output node adds the shares
//      of its four elements, the closed 9-point stiffness of the staged patch,
//      and writes the step (or the residual).
// Every field is read once (with the 1.27x halo of 18^2/16^2) and written once.
// No-flux grids stage through the reflected indices; the update r/m needs no
// correction and the residual rows are divided by 2^b (see device.hpp).
#include <cmath>

#include "kernels.hpp"
#include "node_common.hpp"

namespace pfk {
namespace {

constexpr int GT = 16;       // output nodes per tile side
constexpr int GS = GT + 2;   // staged patch side
constexpr int GE = GT + 1;   // patch elements per side
constexpr int GB = GT * GT;  // threads per block

__device__ __forceinline__ int wrap_any(int i, int n)
{
    i %= n;
    return i < 0 ? i + n : i;
}

// the four Gauss-point values of an element from its nodes (bottom-left v00,
// bottom-right v10, top-left v01, top-right v11); point index qx + 2 qy
template <typename T>
__device__ __forceinline__ void qvals(T v00, T v10, T v01, T v11, T q[4])
{
    const T gp = (T)GP, gm = (T)GM;
    const T l0 = gp * v00 + gm * v01, l1 = gm * v00 + gp * v01;  // left column at qy = 0, 1
    const T r0 = gp * v10 + gm * v11, r1 = gm * v10 + gp * v11;  // right column
    q[0] = gp * l0 + gm * r0;
    q[1] = gm * l0 + gp * r0;
    q[2] = gp * l1 + gm * r1;
    q[3] = gm * l1 + gp * r1;
}

// MODE 0: out = eta - dtm * r (explicit step, dtm = dt / h^2); MODE 1: out = r
template <typename T, int MODE>
__global__ __launch_bounds__(GB) void k_gg_tile2d(Geom g, int P, T L, T kappa, T gam, T dtm,
                                                  const T* __restrict__ in, T* __restrict__ out,
                                                  int tiles_x)
{
    extern __shared__ unsigned char smem_raw[];
    T* sf = reinterpret_cast<T*>(smem_raw);  // P * GS * GS
    T* sS = sf + P * GS * GS;                 // GE * GE * 4
    T* sE = sS + GE * GE * 4;                 // GE * GE * 4
    const int tid = threadIdx.x;
    const int nx = g.n[0], ny = g.n[1];
    const long long N = g.N;
    const int tx0 = (int)(blockIdx.x % tiles_x) * GT, ty0 = (int)(blockIdx.x / tiles_x) * GT;

    // A. stage every field's patch
    for (int k = tid; k < P * GS * GS; k += GB) {
        const int f = k / (GS * GS), rem = k - f * (GS * GS);
        const int py = rem / GS, px = rem - py * GS;
        int gx = tx0 - 1 + px, gy = ty0 - 1 + py;
        gx = g.bc ? reflect(gx, nx) : wrap_any(gx, nx);
        gy = g.bc ? reflect(gy, ny) : wrap_any(gy, ny);
        sf[k] = in[(long long)f * N + (long long)gy * nx + gx];
    }
    __syncthreads();

    // B. S = sum_j eta_j^2 at the Gauss points of every patch element
    for (int e = tid; e < GE * GE; e += GB) {
        const int ex = e % GE, ey = e / GE;
        T s[4] = {T(0), T(0), T(0), T(0)};
        for (int f = 0; f < P; ++f) {
            const T* b = sf + f * GS * GS + ey * GS + ex;
            T q[4];
            qvals(b[0], b[1], b[GS], b[GS + 1], q);
#pragma unroll
            for (int i = 0; i < 4; ++i) s[i] = fmaT(q[i], q[i], s[i]);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) sS[4 * e + i] = s[i];
    }
    __syncthreads();

    const T h = (T)g.h;
    const T detJ = (T)0.25 * h * h;
    const T c3 = (T)1 - (T)2 * gam, c1 = (T)2 * gam;
    const int ox = tid % GT, oy = tid / GT;
    const int gxo = tx0 + ox, gyo = ty0 + oy;
    const bool valid = gxo < nx && gyo < ny;
    const T gp = (T)GP, gm = (T)GM;
    // C. one field at a time
    for (int f = 0; f < P; ++f) {
        const T* F = sf + f * GS * GS;
        for (int e = tid; e < GE * GE; e += GB) {
            const int ex = e % GE, ey = e / GE;
            const T* b = F + ey * GS + ex;
            T q[4];
            qvals(b[0], b[1], b[GS], b[GS + 1], q);
            T d[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) d[i] = q[i] * fmaT(q[i] * q[i], c3, fmaT(c1, sS[4 * e + i], (T)-1));
            // project onto the element's nodes: share_a = detJ sum_q phi_a(q) d_q (separable)
            const T a00 = gp * d[0] + gm * d[1], a10 = gm * d[0] + gp * d[1];  // x-projection, qy = 0
            const T a01 = gp * d[2] + gm * d[3], a11 = gm * d[2] + gp * d[3];  // qy = 1
            sE[4 * e + 0] = detJ * (gp * a00 + gm * a01);  // node (0, 0)
            sE[4 * e + 1] = detJ * (gp * a10 + gm * a11);  // node (1, 0)
            sE[4 * e + 2] = detJ * (gm * a00 + gp * a01);  // node (0, 1)
            sE[4 * e + 3] = detJ * (gm * a10 + gp * a11);  // node (1, 1)
        }
        __syncthreads();
        if (valid) {
            const int e00 = ox + GE * oy;  // the element below-left of the node
            const T Nn = sE[4 * e00 + 3] + sE[4 * (e00 + 1) + 2] + sE[4 * (e00 + GE) + 1] +
                         sE[4 * (e00 + GE + 1) + 0];
            T u[9];
#pragma unroll
            for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                for (int dx = 0; dx < 3; ++dx) u[dx + 3 * dy] = F[(oy + dy) * GS + ox + dx];
            const T r = L * (Nn + kappa * stiff<T, 2>(u, h));
            const long long o = (long long)f * N + (long long)gyo * nx + gxo;
            if (MODE == 0) {
                out[o] = u[4] - dtm * r;
            } else {
                out[o] = r / (T)bfactor<2>(g, gxo, gyo, 0);
            }
        }
        __syncthreads();
    }
}

// energy partials: node (i, j) owns the element with lower-left corner (i, j);
// out pairs (E_h share, sum_a m_a sum_i eta_i,a share)
template <typename T>
__global__ __launch_bounds__(256) void k_gg_energy2d(Geom g, int P, T kappa, T gam, const T* __restrict__ U,
                                                     double* __restrict__ part)
{
    const int nx = g.n[0], ny = g.n[1];
    const long long N = g.N;
    const double h = g.h, detJ = 0.25 * h * h;
    double en = 0.0, ms = 0.0;
    for (long long idx = (long long)blockIdx.x * 256 + threadIdx.x; idx < N; idx += (long long)gridDim.x * 256) {
        const int i = (int)(idx % nx), j = (int)(idx / nx);
        double sum_eta = 0.0;
        for (int f = 0; f < P; ++f) sum_eta += (double)U[(long long)f * N + idx];
        ms += h * h / bfactor<2>(g, i, j, 0) * sum_eta;
        if (g.bc && (i == nx - 1 || j == ny - 1)) continue;
        const int i1 = g.bc ? i + 1 : wrap_any(i + 1, nx), j1 = g.bc ? j + 1 : wrap_any(j + 1, ny);
        double S[4] = {0, 0, 0, 0}, Q4[4] = {0, 0, 0, 0}, A[4] = {0, 0, 0, 0}, G[4] = {0, 0, 0, 0};
        for (int f = 0; f < P; ++f) {
            const T* b = U + (long long)f * N;
            const double v00 = b[(long long)j * nx + i], v10 = b[(long long)j * nx + i1];
            const double v01 = b[(long long)j1 * nx + i], v11 = b[(long long)j1 * nx + i1];
            double q[4];
            qvals(v00, v10, v01, v11, q);
            // gradients at the Gauss points: d/dx along each Gauss row, d/dy along each column
            const double wy[2][2] = {{GP, GM}, {GM, GP}};  // [qy][bottom, top]
            for (int k = 0; k < 4; ++k) {
                const int qx = k & 1, qy = k >> 1;
                const double gx = (wy[qy][0] * (v10 - v00) + wy[qy][1] * (v11 - v01)) / h;
                const double gy = (wy[qx][0] * (v01 - v00) + wy[qx][1] * (v11 - v10)) / h;
                const double q2 = q[k] * q[k];
                S[k] += q2;
                Q4[k] += q2 * q2;
                A[k] += 0.25 * q2 * q2 - 0.5 * q2;
                G[k] += gx * gx + gy * gy;
            }
        }
        for (int k = 0; k < 4; ++k)
            en += detJ * (A[k] + 0.5 * (double)gam * (S[k] * S[k] - Q4[k]) + 0.25 + 0.5 * (double)kappa * G[k]);
    }
    __shared__ double se[256], sm[256];
    se[threadIdx.x] = en;
    sm[threadIdx.x] = ms;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            se[threadIdx.x] += se[threadIdx.x + s];
            sm[threadIdx.x] += sm[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = se[0];
        part[2 * blockIdx.x + 1] = sm[0];
    }
}

}  // namespace

size_t gg_tile_lds_bytes(int P, size_t esize) { return ((size_t)P * GS * GS + 2 * GE * GE * 4) * esize; }

template <typename T>
void launch_gg_tile2d(const Geom& g, int P, double L, double kappa, double gamma, double dt, const T* in,
                      T* out, int residual, hipStream_t s)
{
    const int tiles_x = (g.n[0] + GT - 1) / GT, tiles_y = (g.n[1] + GT - 1) / GT;
    const size_t lds = gg_tile_lds_bytes(P, sizeof(T));
    const T dtm = (T)(dt / (g.h * g.h));
    if (residual)
        k_gg_tile2d<T, 1><<<tiles_x * tiles_y, GB, lds, s>>>(g, P, (T)L, (T)kappa, (T)gamma, dtm, in, out,
                                                            tiles_x);
    else
        k_gg_tile2d<T, 0><<<tiles_x * tiles_y, GB, lds, s>>>(g, P, (T)L, (T)kappa, (T)gamma, dtm, in, out,
                                                            tiles_x);
}

template <typename T>
void launch_gg_energy2d(const Geom& g, int P, double kappa, double gamma, const T* U, double* part,
                        double* out, hipStream_t s)
{
    const int nb = energy_blocks(g);
    k_gg_energy2d<T><<<nb, 256, 0, s>>>(g, P, (T)kappa, (T)gamma, U, part);
    launch_reduce_pairs(part, nb, out, s);
}

#define GG_INST(T)                                                                                         \
    template void launch_gg_tile2d<T>(const Geom&, int, double, double, double, double, const T*, T*, int,  \
                                      hipStream_t);                                                         \
    template void launch_gg_energy2d<T>(const Geom&, int, double, double, const T*, double*, double*,       \
                                        hipStream_t);
GG_INST(float)
GG_INST(double)

}  // namespace pfk
