// k_grain.hip -- multi-order-parameter Allen-Cahn (grain growth) on 2-D grids:
// p order parameters eta_1..eta_p, each following Eq. 1 with the same L and
// kappa, coupled through the multi-well energy of the grain-growth literature
//     f = sum_i (eta_i^4/4 - eta_i^2/2) + gamma sum_{i<j} eta_i^2 eta_j^2 + 1/4,
//     df/deta_i = eta_i (eta_i^2 (1 - 2 gamma) - 1 + 2 gamma S),  S = sum_j eta_j^2,
// so the coupling enters each Gauss point only through S (O(p) work per point,
// not O(p^2)); all order parameters are updated together, which is the paper's
// vectorisation across phase-field variables (Sec. 2.4).
//
// k_gg_tile2d: one 256-thread block per 15 x 15 tile of output nodes; thread t
// owns element t of the 16 x 16 elements around the tile.
//   A. all p fields of the 17 x 17 node patch (halo 1) are staged in LDS;
//   B. each thread forms S at its element's four Gauss points (kept in registers);
//   C. per field: each element evaluates df/deta_i at its Gauss points and forms
//      its four nodal shares (the projection of df/deta_i plus the element
//      stiffness row kappa (4 u_a - u_x - u_y - 2 u_diag)/6 of the 2-D Q1 element);
//      each output node sums the shares of its four elements (LDS) and writes the
//      step (or the residual); four fields share one pair of barriers.
// Every field is read once (with the 1.28x halo of 17^2/15^2) and written once.
// No-flux grids stage through the reflected indices; the update r/m needs no
// correction and the residual rows are divided by 2^b (see device.hpp).
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "kernels.hpp"
#include "node_common.hpp"
#include "stream2d.hpp"

namespace pfk {
namespace {

constexpr int GT = 15;       // output nodes per tile side
constexpr int GS = GT + 2;   // staged patch side
constexpr int GE = GT + 1;   // patch elements per side (one per thread)
constexpr int GB = GE * GE;  // threads per block
constexpr int FG = 1;        // fields per barrier round

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

// MODE 0: out = eta - dtm * r (explicit step, dtm = dt / h^2);
// MODE 1: out = r, plus inv_dt m (eta - old) when old != nullptr (backward Euler);
// MODE 2: out = 1 / diag(dR/dU) (point Jacobi; inv_dt m on the diagonal)
template <typename T, int MODE>
__global__ __launch_bounds__(GB) void k_gg_tile2d(Geom g, int P, T L, T kappa, T gam, T dtm,
                                                  const T* __restrict__ in, T* __restrict__ out,
                                                  int tiles_x, const T* __restrict__ old, T inv_dt)
{
    extern __shared__ unsigned char smem_raw[];
    T* sf = reinterpret_cast<T*>(smem_raw);  // P * GS * GS
    T* sE = sf + P * GS * GS;                 // FG * 4 * GB nodal shares, [field][share][element]
    const int tid = threadIdx.x;
    const int nx = g.n[0], ny = g.n[1];
    const long long N = g.N;
    const int tx0 = (int)(blockIdx.x % tiles_x) * GT, ty0 = (int)(blockIdx.x / tiles_x) * GT;

    // A. stage every field's patch: each thread owns patch nodes tid and tid + GB
    //    (the second only for tid < GS*GS - GB), their grid offsets computed once
    long long off[2] = {0, 0};
    const int nslot = tid + GB < GS * GS ? 2 : 1;
    for (int k = 0; k < nslot; ++k) {
        const int slot = tid + k * GB, py = slot / GS, px = slot - py * GS;
        int gx = tx0 - 1 + px, gy = ty0 - 1 + py;
        gx = g.bc ? reflect(gx, nx) : wrap_any(gx, nx);
        gy = g.bc ? reflect(gy, ny) : wrap_any(gy, ny);
        off[k] = (long long)gy * nx + gx;
    }
    for (int f = 0; f < P; ++f) {
        const T* src = in + (long long)f * N;
        sf[f * GS * GS + tid] = src[off[0]];
        if (nslot == 2) sf[f * GS * GS + tid + GB] = src[off[1]];
    }
    __syncthreads();

    // B. S = sum_j eta_j^2 at the Gauss points of this thread's element
    const int ex = tid % GE, ey = tid / GE;
    const int eb = ey * GS + ex;  // the element's lower-left node in the patch
    T S[4] = {T(0), T(0), T(0), T(0)};
    for (int f = 0; f < P; ++f) {
        const T* b = sf + f * GS * GS + eb;
        T q[4];
        qvals(b[0], b[1], b[GS], b[GS + 1], q);
#pragma unroll
        for (int i = 0; i < 4; ++i) S[i] = fmaT(q[i], q[i], S[i]);
    }

    const T h = (T)g.h;
    const T detJ = (T)0.25 * h * h;
    const T c3 = (T)1 - (T)2 * gam, c1 = (T)2 * gam;
    const T ks = kappa * (T)(1.0 / 6.0);
    // the output node of this thread (the upper-right node of its element)
    const int gxo = tx0 + ex, gyo = ty0 + ey;
    const bool valid = ex < GT && ey < GT && gxo < nx && gyo < ny;
    const T gp = (T)GP, gm = (T)GM;
    // 2^-b of the output node's no-flux faces (1 on periodic grids), once per node
    const T ib = valid ? (T)1 / (T)bfactor<2>(g, gxo, gyo, 0) : (T)1;
    // C. FG fields per round: shares of FG fields to LDS, one barrier, node sums
    for (int f0 = 0; f0 < P; f0 += FG) {
        const int nf = min(FG, P - f0);
        for (int j = 0; j < nf; ++j) {
            const T* b = sf + (f0 + j) * GS * GS + eb;
            const T u00 = b[0], u10 = b[1], u01 = b[GS], u11 = b[GS + 1];
            T q[4];
            qvals(u00, u10, u01, u11, q);
            T d[4];
            // share c of this element at e[c * GB] (element-minor: the writes and the
            // node sums below touch consecutive words across lanes, no bank conflicts)
            T* e = sE + j * 4 * GB + tid;
            if (MODE == 2) {
                // diagonal: d2f/deta_i^2 = eta_i^2 (3 - 2 gamma) - 1 + 2 gamma S, projected
                // with phi_a^2, plus the element stiffness diagonal 4/6
#pragma unroll
                for (int i = 0; i < 4; ++i) d[i] = fmaT(q[i] * q[i], c3 + (T)2, fmaT(c1, S[i], (T)-1));
                const T p2 = gp * gp, m2 = gm * gm;
                const T a00 = p2 * d[0] + m2 * d[1], a10 = m2 * d[0] + p2 * d[1];
                const T a01 = p2 * d[2] + m2 * d[3], a11 = m2 * d[2] + p2 * d[3];
                const T kd = ks * (T)4;
                e[0] = fmaT(detJ, p2 * a00 + m2 * a01, kd);
                e[GB] = fmaT(detJ, p2 * a10 + m2 * a11, kd);
                e[2 * GB] = fmaT(detJ, m2 * a00 + p2 * a01, kd);
                e[3 * GB] = fmaT(detJ, m2 * a10 + p2 * a11, kd);
                continue;
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) d[i] = q[i] * fmaT(q[i] * q[i], c3, fmaT(c1, S[i], (T)-1));
            // nodal shares: detJ sum_q phi_a(q) d_q (separable) + element stiffness row
            const T a00 = gp * d[0] + gm * d[1], a10 = gm * d[0] + gp * d[1];  // x-projection, qy = 0
            const T a01 = gp * d[2] + gm * d[3], a11 = gm * d[2] + gp * d[3];  // qy = 1
            const T sum = (u00 + u10) + (u01 + u11);
            e[0] = fmaT(detJ, gp * a00 + gm * a01, ks * ((T)5 * u00 - u11 - sum));       // node (0, 0)
            e[GB] = fmaT(detJ, gp * a10 + gm * a11, ks * ((T)5 * u10 - u01 - sum));      // node (1, 0)
            e[2 * GB] = fmaT(detJ, gm * a00 + gp * a01, ks * ((T)5 * u01 - u10 - sum));  // node (0, 1)
            e[3 * GB] = fmaT(detJ, gm * a10 + gp * a11, ks * ((T)5 * u11 - u00 - sum));  // node (1, 1)
        }
        __syncthreads();
        if (valid) {
            for (int j = 0; j < nf; ++j) {
                // node (ex + 1, ey + 1) of the patch: share 3 of this element, 2 of the one
                // to the right, 1 of the one above, 0 of the one above-right
                const T* e = sE + j * 4 * GB;
                const T r = L * ((e[3 * GB + tid] + e[2 * GB + tid + 1]) +
                                 (e[GB + tid + GE] + e[tid + GE + 1]));
                const long long o = (long long)(f0 + j) * N + (long long)gyo * nx + gxo;
                const T uc = sf[(f0 + j) * GS * GS + eb + GS + 1];
                if (MODE == 0) {
                    out[o] = uc - dtm * r;
                } else if (MODE == 1) {
                    // the reflected row and h^2 are both 2^b times the no-flux ones
                    const T tt = old ? inv_dt * g.h * g.h * (uc - old[o]) : (T)0;
                    out[o] = (r + tt) * ib;
                } else {
                    out[o] = (T)bfactor<2>(g, gxo, gyo, 0) / (r + inv_dt * (T)(g.h * g.h));
                }
            }
        }
        __syncthreads();
    }
}

// The explicit step streamed row by row (the work layout of k_explicit2d): one
// 64-lane wave per strip of 62 output columns (lane = column, x-neighbours by DPP)
// and chunk of rows; every order parameter keeps its row window in registers:
// c of the previous row, its x-sums of the previous two rows, and the upward
// scatter of the element row below, with the next row's value in flight.  Per input
// row r, pass 1 forms S = sum_j eta_j^2 at the four Gauss points of element row
// (r-1, r) from all fields, pass 2 evaluates df/deta_i there, scatters it to the
// nodes (sum-factorised, as k_explicit2d's stage) and writes node row r-1:
//   out = eta - A N'(eta) - B (9 eta - box3x3 eta),  A = dt L |J| / m,  B = dt L kappa / (3 m)
// (the Q1 stiffness of a node is (9 u - box u) / 3 in 2-D).  Every field is read
// once (with a 64/62 column and (ty + 2)/ty row halo) and written once.
// No-flux grids read through the reflection of rows and columns, as the tile
// kernel does.  P is a template parameter: the field loops are unrolled without a
// branch, so the scheduler interleaves the fields' independent chains.
template <typename T>
struct GGCoef {
    T A, B;    // scales of the quadrature sum and of the stiffness
    T c3, c1;  // df/deta = q (q^2 c3 + c1 S - 1)
};

template <typename T, int P, bool MIRROR>
__global__ __launch_bounds__(256, 2) void k_gg_stream2d(const T* __restrict__ in, T* __restrict__ out, int nx,
                                                     int ny, int nstrips, int nwaves, int nchunks,
                                                     int fbytes, unsigned bytes, GGCoef<T> k)
{
    constexpr int OUTW = WAVE - 2;
    const int wave = uniform_wave();
    if (wave >= nwaves) return;  // uniform per wave
    const int chunk = wave / nstrips, strip = wave % nstrips;
    const int y0 = (int)((long long)chunk * ny / nchunks);
    const int y1 = (int)((long long)(chunk + 1) * ny / nchunks);
    const int lane = threadIdx.x & (WAVE - 1);
    const int xl = strip * OUTW - 1 + lane;
    const int x = MIRROR ? reflect(xl, nx) : wrap_any(xl, nx);
    const bool out_lane = lane >= 1 && lane < WAVE - 1 && xl < nx;
    const int vx = x * (int)sizeof(T);
    const int rowb = nx * (int)sizeof(T);
    const auto rin = make_rsrc(in, bytes);
    const auto rout = make_rsrc(out, bytes);
    const T gp = (T)GP, gm = (T)GM;
    T cur[P], c_m1[P], s3_m1[P], s3_m2[P], gu_l[P], gu_r[P];
#pragma unroll
    for (int f = 0; f < P; ++f) {
        cur[f] = c_m1[f] = s3_m1[f] = s3_m2[f] = gu_l[f] = gu_r[f] = (T)0;
    }
    auto phys = [&](int r) { return MIRROR ? reflect(r, ny) : wrap_any(r, ny); };
    {
        const int r0 = phys(y0 - 1);
#pragma unroll
        for (int f = 0; f < P; ++f) cur[f] = bload<T>(rin, vx, f * fbytes + r0 * rowb);
    }
    const int iters = (y1 - y0) + 2;  // input rows y0 - 1 .. y1
    for (int t = 0; t < iters; ++t) {
        // the next input row (past the last one the last row is read again)
        const int rn = phys(min(y0 + t, y1));
        // pass 1: S at the Gauss points of element row (r-1, r), r = y0 - 1 + t
        T S[4] = {(T)0, (T)0, (T)0, (T)0};
#pragma unroll
        for (int f = 0; f < P; ++f) {
            const T cc = cur[f], cm = c_m1[f];
            const T d0 = from_right(cc) - cc, d1 = from_right(cm) - cm;
            const T xl0 = fmaT(gm, d0, cc), xr0 = fmaT(gp, d0, cc);
            const T xl1 = fmaT(gm, d1, cm), xr1 = fmaT(gp, d1, cm);
            const T e0 = xl0 - xl1, e1 = xr0 - xr1;
            const T q0 = fmaT(gm, e0, xl1), q1 = fmaT(gp, e0, xl1);
            const T q2 = fmaT(gm, e1, xr1), q3 = fmaT(gp, e1, xr1);
            S[0] = fmaT(q0, q0, S[0]);
            S[1] = fmaT(q1, q1, S[1]);
            S[2] = fmaT(q2, q2, S[2]);
            S[3] = fmaT(q3, q3, S[3]);
        }
        T tq[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) tq[i] = fmaT(k.c1, S[i], (T)-1);
        // pass 2: df/deta_i at the Gauss points, scatter, node row r-1 (stored after
        // the loop, so that the fields' chains share one block for the scheduler)
        T vo[P];
#pragma unroll
        for (int f = 0; f < P; ++f) {
            {
                const T cc = cur[f], cm = c_m1[f];
                const T d0 = from_right(cc) - cc, d1 = from_right(cm) - cm;
                const T xl0 = fmaT(gm, d0, cc), xr0 = fmaT(gp, d0, cc);
                const T xl1 = fmaT(gm, d1, cm), xr1 = fmaT(gp, d1, cm);
                const T e0 = xl0 - xl1, e1 = xr0 - xr1;
                const T q0 = fmaT(gm, e0, xl1), q1 = fmaT(gp, e0, xl1);
                const T q2 = fmaT(gm, e1, xr1), q3 = fmaT(gp, e1, xr1);
                // left column: points 0 (nearer row r-1) and 1; right column: 2 and 3
                const T F0 = q0 * fmaT(q0 * q0, k.c3, tq[0]), F1 = q1 * fmaT(q1 * q1, k.c3, tq[1]);
                const T F2 = q2 * fmaT(q2 * q2, k.c3, tq[2]), F3 = q3 * fmaT(q3 * q3, k.c3, tq[3]);
                const T dL = F0 - F1, dR = F2 - F3;
                const T gdL = fmaT(gp, dL, F1), guL = fmaT(gm, dL, F1);
                const T gdR = fmaT(gp, dR, F3), guR = fmaT(gm, dR, F3);
                const T HL = gu_l[f] + gdL, HR = gu_r[f] + gdR;  // node row r-1 complete
                const T dH = HL - HR;
                const T pl = fmaT(gp, dH, HR), pr = fmaT(gm, dH, HR);
                const T Nn = pl + from_left(pr);
                const T s3 = from_left(cc) + cc + from_right(cc);
                const T box = s3_m2[f] + s3_m1[f] + s3;
                const T lap = fmaT((T)9, cm, -box);
                vo[f] = fmaT(-k.A, Nn, fmaT(-k.B, lap, cm));
                s3_m2[f] = s3_m1[f];
                s3_m1[f] = s3;
                gu_l[f] = guL;
                gu_r[f] = guR;
                c_m1[f] = cc;
                cur[f] = bload<T>(rin, vx, f * fbytes + rn * rowb);  // next row in flight
            }
        }
        if (t >= 2 && out_lane) {
            const int ro = (y0 - 2 + t) * rowb;
#pragma unroll
            for (int f = 0; f < P; ++f) bstore(vo[f], rout, vx, f * fbytes + ro);
        }
    }
}

// Jv = inv_dt m v + L [ sum_e sum_q detJ (H(eta_q) v_q)_i phi_a(q) + kappa K v_i ] with
// (H v)_i = v_i (eta_i^2 (3 - 6 gamma) - 1 + 2 gamma S) + 4 gamma eta_i T,
// S = sum_j eta_j^2, T = sum_j eta_j v_j (the Hessian of the multi-well energy is
// symmetric, so this is also the transpose product).  Same tiling as k_gg_tile2d
// with U and V staged.
template <typename T>
__global__ __launch_bounds__(GB) void k_gg_jvp2d(Geom g, int P, T L, T kappa, T gam, T inv_dt,
                                                 const T* __restrict__ U, const T* __restrict__ V,
                                                 T* __restrict__ out, int tiles_x)
{
    extern __shared__ unsigned char smem_raw[];
    T* su = reinterpret_cast<T*>(smem_raw);  // P * GS * GS
    T* sv = su + P * GS * GS;                 // P * GS * GS
    T* sE = sv + P * GS * GS;                 // 4 * GB nodal shares, [share][element]
    const int tid = threadIdx.x;
    const int nx = g.n[0], ny = g.n[1];
    const long long N = g.N;
    const int tx0 = (int)(blockIdx.x % tiles_x) * GT, ty0 = (int)(blockIdx.x / tiles_x) * GT;
    long long off[2] = {0, 0};
    const int nslot = tid + GB < GS * GS ? 2 : 1;
    for (int k = 0; k < nslot; ++k) {
        const int slot = tid + k * GB, py = slot / GS, px = slot - py * GS;
        int gx = tx0 - 1 + px, gy = ty0 - 1 + py;
        gx = g.bc ? reflect(gx, nx) : wrap_any(gx, nx);
        gy = g.bc ? reflect(gy, ny) : wrap_any(gy, ny);
        off[k] = (long long)gy * nx + gx;
    }
    for (int f = 0; f < P; ++f) {
        const long long fo = (long long)f * N;
        su[f * GS * GS + tid] = U[fo + off[0]];
        sv[f * GS * GS + tid] = V[fo + off[0]];
        if (nslot == 2) {
            su[f * GS * GS + tid + GB] = U[fo + off[1]];
            sv[f * GS * GS + tid + GB] = V[fo + off[1]];
        }
    }
    __syncthreads();
    const int ex = tid % GE, ey = tid / GE;
    const int eb = ey * GS + ex;
    T S[4] = {T(0), T(0), T(0), T(0)}, Tv[4] = {T(0), T(0), T(0), T(0)};
    for (int f = 0; f < P; ++f) {
        const T* b = su + f * GS * GS + eb;
        const T* c = sv + f * GS * GS + eb;
        T q[4], w[4];
        qvals(b[0], b[1], b[GS], b[GS + 1], q);
        qvals(c[0], c[1], c[GS], c[GS + 1], w);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            S[i] = fmaT(q[i], q[i], S[i]);
            Tv[i] = fmaT(q[i], w[i], Tv[i]);
        }
    }
    const T h = (T)g.h;
    const T detJ = (T)0.25 * h * h;
    const T c3 = (T)3 - (T)6 * gam, c1 = (T)2 * gam, c4 = (T)4 * gam;
    const T ks = kappa * (T)(1.0 / 6.0);
    const int gxo = tx0 + ex, gyo = ty0 + ey;
    const bool valid = ex < GT && ey < GT && gxo < nx && gyo < ny;
    const T gp = (T)GP, gm = (T)GM;
    const T ib = valid ? (T)1 / (T)bfactor<2>(g, gxo, gyo, 0) : (T)1;  // 2^-b, once per node
    for (int f = 0; f < P; ++f) {
        const T* b = su + f * GS * GS + eb;
        const T* c = sv + f * GS * GS + eb;
        const T v00 = c[0], v10 = c[1], v01 = c[GS], v11 = c[GS + 1];
        T q[4], w[4];
        qvals(b[0], b[1], b[GS], b[GS + 1], q);
        qvals(v00, v10, v01, v11, w);
        T d[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
            d[i] = fmaT(w[i], fmaT(q[i] * q[i], c3, fmaT(c1, S[i], (T)-1)), c4 * q[i] * Tv[i]);
        const T a00 = gp * d[0] + gm * d[1], a10 = gm * d[0] + gp * d[1];
        const T a01 = gp * d[2] + gm * d[3], a11 = gm * d[2] + gp * d[3];
        const T sum = (v00 + v10) + (v01 + v11);
        T* e = sE + tid;
        e[0] = fmaT(detJ, gp * a00 + gm * a01, ks * ((T)5 * v00 - v11 - sum));
        e[GB] = fmaT(detJ, gp * a10 + gm * a11, ks * ((T)5 * v10 - v01 - sum));
        e[2 * GB] = fmaT(detJ, gm * a00 + gp * a01, ks * ((T)5 * v01 - v10 - sum));
        e[3 * GB] = fmaT(detJ, gm * a10 + gp * a11, ks * ((T)5 * v11 - v00 - sum));
        __syncthreads();
        if (valid) {
            const T r = L * ((sE[3 * GB + tid] + sE[2 * GB + tid + 1]) +
                             (sE[GB + tid + GE] + sE[tid + GE + 1]));
            const long long o = (long long)f * N + (long long)gyo * nx + gxo;
            out[o] = fmaT(inv_dt * h * h, v11, r) * ib;
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
    const double ih2 = 1.0 / (h * h);  // the gradients are summed unscaled (no divide per point)
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
                const double gx = wy[qy][0] * (v10 - v00) + wy[qy][1] * (v11 - v01);  // h d/dx
                const double gy = wy[qx][0] * (v01 - v00) + wy[qx][1] * (v11 - v10);  // h d/dy
                const double q2 = q[k] * q[k];
                S[k] += q2;
                Q4[k] += q2 * q2;
                A[k] += 0.25 * q2 * q2 - 0.5 * q2;
                G[k] += gx * gx + gy * gy;
            }
        }
        for (int k = 0; k < 4; ++k)
            en += detJ * (A[k] + 0.5 * (double)gam * (S[k] * S[k] - Q4[k]) + 0.25 + 0.5 * (double)kappa * G[k] * ih2);
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

size_t gg_tile_lds_bytes(int P, size_t esize) { return ((size_t)P * GS * GS + FG * GB * 4) * esize; }

template <typename T>
void launch_gg_tile2d(const Geom& g, int P, double L, double kappa, double gamma, double dt, const T* in,
                      T* out, int mode, hipStream_t s, const T* old, double inv_dt)
{
    const int tiles_x = (g.n[0] + GT - 1) / GT, tiles_y = (g.n[1] + GT - 1) / GT;
    const size_t lds = gg_tile_lds_bytes(P, sizeof(T));
    const T dtm = (T)(dt / (g.h * g.h));
    const int nb = tiles_x * tiles_y;
    if (mode == 1)
        k_gg_tile2d<T, 1><<<nb, GB, lds, s>>>(g, P, (T)L, (T)kappa, (T)gamma, dtm, in, out, tiles_x, old,
                                              (T)inv_dt);
    else if (mode == 2)
        k_gg_tile2d<T, 2><<<nb, GB, lds, s>>>(g, P, (T)L, (T)kappa, (T)gamma, dtm, in, out, tiles_x, nullptr,
                                              (T)inv_dt);
    else
        k_gg_tile2d<T, 0><<<nb, GB, lds, s>>>(g, P, (T)L, (T)kappa, (T)gamma, dtm, in, out, tiles_x, nullptr,
                                              (T)0);
}

// one launch of k_gg_stream2d<T, P, MIRROR>: chunks sized so that strips x chunks
// just fills the waves the kernel's occupancy keeps resident (at least 8 rows each)
template <typename T, int P, bool MIRROR>
void gg_stream_launch(const Geom& g, const GGCoef<T>& k, const T* in, T* out, int cus, hipStream_t s)
{
    static const int per_cu = [] {
        int b = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_gg_stream2d<T, P, MIRROR>, 256, 0) != hipSuccess) {
            (void)hipGetLastError();
            b = 2;
        }
        return b < 1 ? 1 : b;
    }();
    const int nx = g.n[0], ny = g.n[1];
    const int nstrips = (nx + WAVE - 3) / (WAVE - 2);
    const long long resident = 4ll * per_cu * (cus > 0 ? cus : 256);  // waves: 4 per block
    long long nch = std::max<long long>(1, resident / nstrips);
    nch = std::min<long long>(nch, std::max(1, ny / 8));
    const int nchunks = (int)nch;
    const int nwaves = nstrips * nchunks;
    const int fbytes = (int)(g.N * sizeof(T));
    const unsigned bytes = (unsigned)((double)P * g.N * sizeof(T));
    k_gg_stream2d<T, P, MIRROR><<<(nwaves + 3) / 4, 256, 0, s>>>(in, out, nx, ny, nstrips, nwaves, nchunks,
                                                                  fbytes, bytes, k);
}

// The streamed explicit step when it applies (2-D, every field addressable with
// 32-bit offsets, P one of the instantiated field counts: 1-6 and 8 and, in FP32,
// 10, 12, 16, 20 -- larger counts would spill registers); returns false (nothing
// launched) otherwise.
template <typename T>
bool launch_gg_stream2d(const Geom& g, int P, double L, double kappa, double gamma, double dt, const T* in,
                        T* out, int cus, hipStream_t s)
{
    if (g.dim != 2 || P < 1 || tune_gg_stream() == 1) return false;
    if ((double)P * (double)g.N * sizeof(T) >= 2147483647.0) return false;
    const double m = g.h * g.h, detJ = 0.25 * g.h * g.h;
    const GGCoef<T> k{(T)(dt * L * detJ / m), (T)(dt * L * kappa / (3.0 * m)), (T)(1.0 - 2.0 * gamma),
                      (T)(2.0 * gamma)};
    auto go = [&](auto pc) {
        constexpr int PC = decltype(pc)::value;
        if (g.bc)
            gg_stream_launch<T, PC, true>(g, k, in, out, cus, s);
        else
            gg_stream_launch<T, PC, false>(g, k, in, out, cus, s);
        return true;
    };
    switch (P) {
        case 1: return go(std::integral_constant<int, 1>{});
        case 2: return go(std::integral_constant<int, 2>{});
        case 3: return go(std::integral_constant<int, 3>{});
        case 4: return go(std::integral_constant<int, 4>{});
        case 5: return go(std::integral_constant<int, 5>{});
        case 6: return go(std::integral_constant<int, 6>{});
        case 8: return go(std::integral_constant<int, 8>{});
        default: break;
    }
    if constexpr (sizeof(T) == 4) {
        switch (P) {
            case 10: return go(std::integral_constant<int, 10>{});
            case 12: return go(std::integral_constant<int, 12>{});
            case 16: return go(std::integral_constant<int, 16>{});
            case 20: return go(std::integral_constant<int, 20>{});
            default: break;
        }
    }
    return false;
}

size_t gg_jvp_lds_bytes(int P, size_t esize) { return ((size_t)2 * P * GS * GS + GB * 4) * esize; }

template <typename T>
void launch_gg_jvp2d(const Geom& g, int P, double L, double kappa, double gamma, double inv_dt, const T* U,
                     const T* V, T* Jv, hipStream_t s)
{
    const int tiles_x = (g.n[0] + GT - 1) / GT, tiles_y = (g.n[1] + GT - 1) / GT;
    k_gg_jvp2d<T><<<tiles_x * tiles_y, GB, gg_jvp_lds_bytes(P, sizeof(T)), s>>>(
        g, P, (T)L, (T)kappa, (T)gamma, (T)inv_dt, U, V, Jv, tiles_x);
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
                                      hipStream_t, const T*, double);                                       \
    template bool launch_gg_stream2d<T>(const Geom&, int, double, double, double, double, const T*, T*, int, \
                                        hipStream_t);                                                       \
    template void launch_gg_jvp2d<T>(const Geom&, int, double, double, double, double, const T*, const T*, \
                                     T*, hipStream_t);                                                      \
    template void launch_gg_energy2d<T>(const Geom&, int, double, double, const T*, double*, double*,       \
                                        hipStream_t);
GG_INST(float)
GG_INST(double)

}  // namespace pfk
