// k_jvp2d.hip -- Jacobian-vector product of the backward-Euler residual
// (Eq. 14, Sec. 2.3) on 2-D grids, row-streamed like the explicit step.
//
//   Allen-Cahn:     Jv    = inv_dt m v + L [ N'(u) v + kappa K v ]
//   Cahn-Hilliard:  Jv_c  = inv_dt m v_c + M K v_mu
//                   Jv_mu = m v_mu - [ N'(c) v_c + kappa K v_c ]
// with N'(u) v = sum_e sum_q |J| f''(u_q) v_q phi(q) (2 x 2 Gauss points per
// element) and the closed Q1 stencil K v = (9 v - box3x3 v) / 3.
//
// One 64-lane wave owns a strip of 62 output columns (lane = column, one halo
// lane per side) and marches up a chunk of rows.  x-neighbours come from the
// adjacent lanes by DPP; the rows r-2 .. r live in registers; each input row of
// u and of the direction is read once per wave, PF rows ahead.  The Gauss
// quadrature is sum-factorised as in the explicit step: per element row the
// x-interpolants of u and v at the two Gauss abscissae, the four quadrature
// values, f''(u_q) v_q, then the y- and x-scatters back to the nodes.
// No-flux grids read through the even extension about the end nodes; the row
// of a node on b boundary faces is then 2^b times the no-flux row, so the output
// is divided by 2^b (the node-centric kernel does the same).
// With nodal (Gauss-Lobatto) quadrature N'(u) v = m f''(u_a) v_a at the node and K
// is the 5-point stencil 4 v - (axis neighbours) (h-free in 2-D).
#include <algorithm>

#include "device.hpp"
#include "kernels.hpp"
#include "stream2d.hpp"

namespace pfk {
namespace {

template <typename T>
struct JCoef {
    T b0, b1, b2;  // f''(q) = b0 + q (b1 + b2 q)
    T mv;          // inv_dt m: the time term of the first row
    T nq;          // AC: L |J|; CH: |J|  (nodal quadrature: L m; m)
    T kv;          // AC: L kappa / 3; CH: kappa / 3  (nodal: L kappa; kappa)
    T kw;          // CH: M / 3  (nodal: M)
    T mw;          // CH: m
};

// One row of the pipeline: push the newest row r of u, v (and w = v_mu for
// Cahn-Hilliard) and get the output row r - 1.  v1 holds v of the output row
// until the push.
template <typename T, int MODEL, bool LOB = false>
struct JStage {
    T xlu = 0, xru = 0, xlv = 0, xrv = 0;  // x-interpolants of row r-1
    T guL = 0, guR = 0;                    // upward scatter of element row (r-2, r-1)
    T v1 = 0, s3v1 = 0, s3v2 = 0;          // v at row r-1; x-sums of v at rows r-1, r-2
    T w1 = 0, s3w1 = 0, s3w2 = 0;          // Cahn-Hilliard: the same for w

    __device__ __forceinline__ void push(T u, T v, T w, const JCoef<T>& k, T& o0, T& o1)
    {
        const T gp = (T)GP, gm = (T)GM;
        const T du = from_right(u) - u, dv = from_right(v) - v;
        const T xlu0 = fmaT(gm, du, u), xru0 = fmaT(gp, du, u);
        const T xlv0 = fmaT(gm, dv, v), xrv0 = fmaT(gp, dv, v);
        const T eu0 = xlu0 - xlu, eu1 = xru0 - xru;
        const T ev0 = xlv0 - xlv, ev1 = xrv0 - xrv;
        auto F = [&](T q, T p) { return fmaT(fmaT(k.b2, q, k.b1), q, k.b0) * p; };
        // element row (r-1, r): Gauss points (left/right abscissa, lower/upper ordinate)
        const T PL0 = F(fmaT(gm, eu0, xlu), fmaT(gm, ev0, xlv));
        const T PL1 = F(fmaT(gp, eu0, xlu), fmaT(gp, ev0, xlv));
        const T PR0 = F(fmaT(gm, eu1, xru), fmaT(gm, ev1, xrv));
        const T PR1 = F(fmaT(gp, eu1, xru), fmaT(gp, ev1, xrv));
        const T dL = PL0 - PL1, dR = PR0 - PR1;
        const T gdL = fmaT(gp, dL, PL1), guL0 = fmaT(gm, dL, PL1);
        const T gdR = fmaT(gp, dR, PR1), guR0 = fmaT(gm, dR, PR1);
        const T HL = guL + gdL, HR = guR + gdR;  // node row r-1 complete
        const T dH = HL - HR;
        const T pl = fmaT(gp, dH, HR), pr = fmaT(gm, dH, HR);
        const T Nn = pl + from_left(pr);  // sum_e sum_q f''(u_q) v_q phi(q) at row r-1
        const T s3v = from_left(v) + v + from_right(v);
        const T lapv = fmaT((T)9, v1, -(s3v2 + s3v1 + s3v));  // 9 v - box v at row r-1
        if constexpr (MODEL == 0) {
            o0 = fmaT(k.mv, v1, fmaT(k.nq, Nn, k.kv * lapv));
            o1 = (T)0;
        } else {
            const T s3w = from_left(w) + w + from_right(w);
            const T lapw = fmaT((T)9, w1, -(s3w2 + s3w1 + s3w));
            o0 = fmaT(k.mv, v1, k.kw * lapw);
            o1 = fmaT(k.mw, w1, -fmaT(k.nq, Nn, k.kv * lapv));
            w1 = w;
            s3w2 = s3w1;
            s3w1 = s3w;
        }
        xlu = xlu0;
        xru = xru0;
        xlv = xlv0;
        xrv = xrv0;
        guL = guL0;
        guR = guR0;
        v1 = v;
        s3v2 = s3v1;
        s3v1 = s3v;
    }
};

// Nodal quadrature: f''(u) v at the node and the 5-point stencil, no interpolation
// or scatter; the output row is r - 1 as above.
template <typename T, int MODEL>
struct JStage<T, MODEL, true> {
    T u1 = 0, v1 = 0, v2 = 0;  // u and v at row r-1, v at row r-2
    T w1 = 0, w2 = 0;          // Cahn-Hilliard: w at rows r-1, r-2

    __device__ __forceinline__ void push(T u, T v, T w, const JCoef<T>& k, T& o0, T& o1)
    {
        const T fv = fmaT(fmaT(k.b2, u1, k.b1), u1, k.b0) * v1;
        const T lapv = fmaT((T)4, v1, -((from_left(v1) + from_right(v1)) + (v2 + v)));
        if constexpr (MODEL == 0) {
            o0 = fmaT(k.mv, v1, fmaT(k.nq, fv, k.kv * lapv));
            o1 = (T)0;
        } else {
            const T lapw = fmaT((T)4, w1, -((from_left(w1) + from_right(w1)) + (w2 + w)));
            o0 = fmaT(k.mv, v1, k.kw * lapw);
            o1 = fmaT(k.mw, w1, -fmaT(k.nq, fv, k.kv * lapv));
            w2 = w1;
            w1 = w;
        }
        u1 = u;
        v2 = v1;
        v1 = v;
    }
};

constexpr int JPF = 4;  // rows in flight per field

// wave -> (strip, chunk), strips fastest (neighbouring waves share their rows);
// chunk c holds rows [c ty, min(ny, (c + 1) ty)).  bytes: one plane.
// PQ (Allen-Cahn, for conjugate gradients): also pq[block] = the block's share of
// v . Jv in FP64 (every node is stored by exactly one lane), fixed order.
template <typename T, int MODEL, bool MIRROR, bool PQ = false, bool LOB = false>
__global__ __launch_bounds__(256) void k_jvp2d(const T* __restrict__ U, const T* __restrict__ V,
                                               T* __restrict__ Jv, int nx, int ny, int nstrips, int nwaves,
                                               int ty, unsigned bytes, JCoef<T> k, double* __restrict__ pq)
{
    static_assert(!PQ || MODEL == 0, "v . Jv for the Allen-Cahn product");
    constexpr int OUTW = WAVE - 2;
    const int wid = uniform_wave();
    double pqs = 0.0;
    if (!PQ && wid >= nwaves) return;
    if (wid < nwaves) {
        const int strip = wid % nstrips, chunk = wid / nstrips;
        const int y0 = chunk * ty, y1 = min(ny, y0 + ty);
        const int lane = threadIdx.x & (WAVE - 1);
        const int xl = strip * OUTW - 1 + lane;
        int x;
        if constexpr (MIRROR) {
            x = reflect(xl, nx);
        } else {
            x = xl % nx;
            if (x < 0) x += nx;
        }
        const bool out_lane = lane >= 1 && lane < WAVE - 1 && xl < nx;
        T xs = (T)1;  // no-flux: 1 / 2 on the first and last columns
        if constexpr (MIRROR) xs = (x == 0 || x == nx - 1) ? (T)0.5 : (T)1;
        const int iters = (y1 - y0) + 2;  // rows y0-1 .. y1
        const int rowb = nx * (int)sizeof(T);
        const int vx = x * (int)sizeof(T);
        const auto ru = make_rsrc(U, bytes);
        const auto rv = make_rsrc(V, bytes);
        const auto rw = make_rsrc(MODEL == 1 ? V + (size_t)nx * ny : V, bytes);
        const auto r0 = make_rsrc(Jv, bytes);
        const auto r1 = make_rsrc(MODEL == 1 ? Jv + (size_t)nx * ny : Jv, bytes);
        // the rows read lie in [-1, ny]: one wrap (periodic) or one reflection about
        // the end row (no-flux; ny >= 2) maps them onto the grid
        auto row_off = [&](int t) {
            int r = min(y0 - 1 + t, y1);  // past the chunk the last row is read again (a cache hit)
            if constexpr (MIRROR) {
                r = r < 0 ? -r : (r >= ny ? 2 * (ny - 1) - r : r);
            } else {
                r = r < 0 ? r + ny : (r >= ny ? r - ny : r);
            }
            return r * rowb;
        };
        T ru_[JPF], rv_[JPF], rw_[JPF];
    #pragma unroll
        for (int u = 0; u < JPF; ++u) {
            const int off = row_off(u);
            ru_[u] = bload<T>(ru, vx, off);
            rv_[u] = bload<T>(rv, vx, off);
            rw_[u] = MODEL == 1 ? bload<T>(rw, vx, off) : (T)0;
        }
        JStage<T, MODEL, LOB> st;
        // the pipeline runs whole groups of JPF rows: the pushes past the chunk compute
        // rows nobody stores, so neither the loads nor the pushes need a branch
        for (int t0 = 0; t0 < iters; t0 += JPF) {
    #pragma unroll
            for (int u = 0; u < JPF; ++u) {
                const int t = t0 + u;
                const T cu = ru_[u], cv = rv_[u], cw = rw_[u];
                const int off = row_off(t + JPF);
                ru_[u] = bload<T>(ru, vx, off);
                rv_[u] = bload<T>(rv, vx, off);
                if constexpr (MODEL == 1) rw_[u] = bload<T>(rw, vx, off);
                const T vprev = st.v1;  // v at the output row
                T o0, o1;
                st.push(cu, cv, cw, k, o0, o1);
                if (t >= 2 && t < iters && out_lane) {
                    const int yo = y0 - 2 + t;  // output row
                    T sc = xs;
                    if constexpr (MIRROR) sc = (yo == 0 || yo == ny - 1) ? xs * (T)0.5 : xs;
                    const T q0 = MIRROR ? o0 * sc : o0;
                    bstore(q0, r0, vx, yo * rowb);
                    if constexpr (MODEL == 1) bstore(MIRROR ? o1 * sc : o1, r1, vx, yo * rowb);
                    if constexpr (PQ) pqs += (double)vprev * (double)q0;
                }
            }
        }
    }
    if constexpr (PQ) {
        for (int off = WAVE / 2; off > 0; off >>= 1) pqs += __shfl_down(pqs, off, WAVE);
        __shared__ double sh[4];
        if ((threadIdx.x & (WAVE - 1)) == 0) sh[threadIdx.x / WAVE] = pqs;
        __syncthreads();
        if (threadIdx.x == 0) pq[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    }
}

int device_cus()
{
    static const int n = [] {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
            return 256;
        return cus;
    }();
    return n;
}

}  // namespace

template <typename T>
bool launch_jvp2d_stream(const Geom& g, int model, const FreeEnergy& f, double kappa, double mob,
                         double inv_dt, const T* U, const T* v, T* Jv, hipStream_t s, double* pq, int* pq_blocks,
                         int pq_max)
{
    if (g.dim != 2 || g.cm || tune_jvp2d_stream() == 1) return false;
    if (pq && model != 0) return false;
    const int nx = g.n[0], ny = g.n[1];
    // buffer offsets are 32-bit: one plane must stay below 2^31 bytes
    if ((size_t)g.N * sizeof(T) >= (size_t(1) << 31)) return false;
    const double h = g.h, m = h * h, detJ = 0.25 * h * h;
    JCoef<T> k{};
    k.b0 = (T)f.b0;
    k.b1 = (T)f.b1;
    k.b2 = (T)f.b2;
    k.mv = (T)(inv_dt * m);
    // Gauss: |J| weights and the (9 v - box v) / 3 stencil; nodal: m and 4 v - nbrs
    const double wq = g.quad ? m : detJ, ks = g.quad ? 1.0 : 1.0 / 3.0;
    if (model == 0) {
        k.nq = (T)(mob * wq);
        k.kv = (T)(mob * kappa * ks);
    } else {
        k.nq = (T)wq;
        k.kv = (T)(kappa * ks);
        k.kw = (T)(mob * ks);
        k.mw = (T)m;
    }
    // chunks for about four waves per SIMD, never shorter than 8 rows
    // (PF_TUNE_STREAM2D_ROWS sets the rows per chunk instead)
    const int nstrips = (nx + WAVE - 3) / (WAVE - 2);
    long long nch = std::max<long long>(1, 16ll * device_cus() / nstrips);
    nch = std::min<long long>(nch, std::max(1, ny / 8));
    const int tov = tune_stream2d_rows();
    const int ty = tov > 0 ? std::min(tov, ny) : (int)((ny + nch - 1) / nch);
    const int nchunks = (ny + ty - 1) / ty;
    const long long nwaves = (long long)nstrips * nchunks;
    if (nwaves > (1ll << 30)) return false;
    const unsigned blocks = (unsigned)((nwaves + 3) / 4);
    if (pq && (int)blocks > pq_max) return false;
    const unsigned bytes = (unsigned)((size_t)g.N * sizeof(T));
#define JVP2D(MODEL, MIR, PQ)                                                                             \
    do {                                                                                                  \
        if (g.quad)                                                                                       \
            k_jvp2d<T, MODEL, MIR, PQ, true>                                                              \
                <<<blocks, 256, 0, s>>>(U, v, Jv, nx, ny, nstrips, (int)nwaves, ty, bytes, k, pq);        \
        else                                                                                              \
            k_jvp2d<T, MODEL, MIR, PQ, false>                                                             \
                <<<blocks, 256, 0, s>>>(U, v, Jv, nx, ny, nstrips, (int)nwaves, ty, bytes, k, pq);        \
    } while (0)
    if (pq) {
        if (g.bc) JVP2D(0, true, true); else JVP2D(0, false, true);
        *pq_blocks = (int)blocks;
    } else if (model == 0) {
        if (g.bc) JVP2D(0, true, false); else JVP2D(0, false, false);
    } else {
        if (g.bc) JVP2D(1, true, false); else JVP2D(1, false, false);
    }
#undef JVP2D
    return true;
}

template bool launch_jvp2d_stream<float>(const Geom&, int, const FreeEnergy&, double, double, double,
                                         const float*, const float*, float*, hipStream_t, double*, int*, int);
template bool launch_jvp2d_stream<double>(const Geom&, int, const FreeEnergy&, double, double, double,
                                          const double*, const double*, double*, hipStream_t, double*, int*, int);

}  // namespace pfk
