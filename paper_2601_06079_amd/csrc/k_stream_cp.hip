// k_stream_cp.hip -- fused explicit step of the coupled Allen-Cahn / Cahn-Hilliard
// model (Eq. 7, Supp. Note 3 free energies) on 2-D grids, periodic or no-flux.
//
// The row-streaming scheme of k_stream2d.hip with two streamed fields: one 64-lane
// wavefront owns a strip of columns, marches up a chunk of rows and keeps every
// intermediate in registers (x-neighbours by DPP, y-neighbours in a register
// window).  Per element row (r-1, r), c and eta are interpolated to the 4 Gauss
// points; there
//   A_q = f_a'(c_q)(1 - h(eta_q)) + f_b'(c_q) h(eta_q)     (mu source)
//   B_q = (f_b(c_q) - f_a(c_q)) h'(eta_q)                   (eta source)
// are formed once and scattered to the element's nodes (y then x, transposed
// interpolation).  Then, from the old state,
//   mu(r-1)    = |J|/m sum A
//   eta'(r-1)  = eta - dt M_eta/m [ |J| sum B + kappa K eta ]
//   c'(r-2)    = c - dt M_c/m K mu
// with K u = (9 u - box3x3(u)) / 3 (2-D Q1 stiffness, h-independent).  c' needs mu
// at x +- 1, so a strip outputs its 60 interior columns (halo 2 lanes per side)
// and chunks overlap by 2 rows.  Each field is read once and written once per step.
#include "device.hpp"
#include "kernels.hpp"
#include "stream2d.hpp"

namespace pfk {
namespace {

template <typename T>
struct CpCoef {
    T jm;  // |J| / m
    T kb;  // dt M_eta |J| / m
    T kk;  // dt M_eta kappa / (3 m)
    T kc;  // dt M_c / (3 m)
};

// the benchmark polynomials (Supp. Note 3)
template <typename T>
__device__ __forceinline__ void sources(T c, T e, T& A, T& B)
{
    const T fa = fmaT(fmaT(fmaT(fmaT((T)1.3687, c, (T)-2.7375), c, (T)5.1622), c, (T)-4.776), c, (T)-1.6704);
    const T dfa = fmaT(fmaT(fmaT((T)(4 * 1.3687), c, (T)(-3 * 2.7375)), c, (T)(2 * 5.1622)), c, (T)-4.776);
    const T fb = fmaT(fmaT((T)5.0, c, (T)-5.9746), c, (T)-1.5924);
    const T dfb = fmaT((T)10.0, c, (T)-5.9746);
    const T h = e * e * e * fmaT(fmaT((T)6, e, (T)-15), e, (T)10);
    const T t = e * ((T)1 - e);
    A = fmaT(dfb - dfa, h, dfa);
    B = (fb - fa) * ((T)30 * t * t);
}

// One step as a row pipeline: push(c, eta) of row r returns (c', eta') of row r - 2.
template <typename T>
struct CpStage {
    T c_m1 = 0, c_m2 = 0;                      // c at rows r-1, r-2
    T e_m1 = 0;                                // eta at row r-1
    T s3e_m1 = 0, s3e_m2 = 0;                  // 3-point x-sums of eta, rows r-1, r-2
    T cxl_m1 = 0, cxr_m1 = 0, exl_m1 = 0, exr_m1 = 0;  // x-interpolated row r-1
    T guAL = 0, guAR = 0, guBL = 0, guBR = 0;  // upward scatter of element row (r-2, r-1)
    T mu_m1 = 0;                               // mu at row r-2
    T s3mu_m1 = 0, s3mu_m2 = 0;                // x-sums of mu at rows r-2, r-3
    T en_m1 = 0;                               // eta' at row r-2

    __device__ __forceinline__ void push(T cc, T ee, const CpCoef<T>& k, T& c_out, T& e_out)
    {
        const T gp = (T)GP, gm = (T)GM;
        // x-interpolation of the new row to the two Gauss columns of element (x, x+1)
        const T cr = from_right(cc), er = from_right(ee);
        const T el = from_left(ee);
        const T dc = cr - cc, de = er - ee;
        const T cxl = fmaT(gm, dc, cc), cxr = fmaT(gp, dc, cc);
        const T exl = fmaT(gm, de, ee), exr = fmaT(gp, de, ee);
        const T s3e = el + ee + er;
        // y-interpolation to the 4 Gauss points of element row (r-1, r)
        const T dcl = cxl - cxl_m1, dcr = cxr - cxr_m1, del = exl - exl_m1, der = exr - exr_m1;
        T AL0, AL1, AR0, AR1, BL0, BL1, BR0, BR1;
        sources(fmaT(gm, dcl, cxl_m1), fmaT(gm, del, exl_m1), AL0, BL0);
        sources(fmaT(gp, dcl, cxl_m1), fmaT(gp, del, exl_m1), AL1, BL1);
        sources(fmaT(gm, dcr, cxr_m1), fmaT(gm, der, exr_m1), AR0, BR0);
        sources(fmaT(gp, dcr, cxr_m1), fmaT(gp, der, exr_m1), AR1, BR1);
        // y-scatter: to node row r-1 (down) and row r (up)
        const T dAL = AL0 - AL1, dAR = AR0 - AR1, dBL = BL0 - BL1, dBR = BR0 - BR1;
        const T HAL = guAL + fmaT(gp, dAL, AL1), HAR = guAR + fmaT(gp, dAR, AR1);
        const T HBL = guBL + fmaT(gp, dBL, BL1), HBR = guBR + fmaT(gp, dBR, BR1);
        guAL = fmaT(gm, dAL, AL1);
        guAR = fmaT(gm, dAR, AR1);
        guBL = fmaT(gm, dBL, BL1);
        guBR = fmaT(gm, dBR, BR1);
        // x-scatter: element (x, x+1) to node x (left) and x+1 (right)
        const T dHA = HAL - HAR, dHB = HBL - HBR;
        const T NA = fmaT(gp, dHA, HAR) + from_left(fmaT(gm, dHA, HAR));  // node (x, r-1)
        const T NB = fmaT(gp, dHB, HBR) + from_left(fmaT(gm, dHB, HBR));
        // mu and eta' at row r-1
        const T mu = k.jm * NA;
        const T boxe = s3e_m2 + s3e_m1 + s3e;
        const T en = e_m1 - fmaT(k.kb, NB, k.kk * fmaT((T)9, e_m1, -boxe));
        // c' at row r-2
        const T s3mu = from_left(mu) + mu + from_right(mu);
        const T boxmu = s3mu_m2 + s3mu_m1 + s3mu;
        c_out = c_m2 - k.kc * fmaT((T)9, mu_m1, -boxmu);
        e_out = en_m1;
        // shift the window
        en_m1 = en;
        s3mu_m2 = s3mu_m1;
        s3mu_m1 = s3mu;
        mu_m1 = mu;
        c_m2 = c_m1;
        c_m1 = cc;
        e_m1 = ee;
        s3e_m2 = s3e_m1;
        s3e_m1 = s3e;
        cxl_m1 = cxl;
        cxr_m1 = cxr;
        exl_m1 = exl;
        exr_m1 = exr;
    }
};

constexpr int CPH = 2;                 // halo (lanes and rows)
constexpr int CPOUT = WAVE - 2 * CPH;  // output columns per strip
constexpr int CPPF = 4;                // rows in flight per wave

template <typename T, bool MIRROR>
__global__ __launch_bounds__(256) void k_cp_explicit2d(const T* __restrict__ c_in, const T* __restrict__ e_in,
                                                       T* __restrict__ c_out, T* __restrict__ e_out,
                                                       int nx, int ny, int nstrips, int nwaves,
                                                       int nchunks, unsigned bytes, CpCoef<T> k)
{
    const int wave = uniform_wave();
    if (wave >= nwaves) return;  // uniform per wave
    const int chunk = wave / nstrips, strip = wave % nstrips;
    const int y0 = (int)((long long)chunk * ny / nchunks);
    const int y1 = (int)((long long)(chunk + 1) * ny / nchunks);
    const int lane = threadIdx.x & (WAVE - 1);
    const int xl = strip * CPOUT - CPH + lane;
    int x;
    if constexpr (MIRROR) {
        x = reflect(xl, nx);
    } else {
        x = xl % nx;
        if (x < 0) x += nx;
    }
    const bool out_lane = lane >= CPH && lane < WAVE - CPH && xl < nx;
    const int iters = (y1 - y0) + 2 * CPH;  // rows y0-2 .. y1+1
    const int rowb = nx * (int)sizeof(T);
    const int vx = x * (int)sizeof(T);
    const auto rc = make_rsrc(c_in, bytes), re = make_rsrc(e_in, bytes);
    const auto wc = make_rsrc(c_out, bytes), we = make_rsrc(e_out, bytes);

    // row cursor: periodic rl wraps; MIRROR reflects the logical row lr
    int lr = y0 - CPH, rl;
    if constexpr (MIRROR) {
        rl = reflect(lr, ny);
    } else {
        rl = lr;
        while (rl < 0) rl += ny;
    }
    auto advance = [&]() {
        if constexpr (MIRROR) {
            rl = reflect(++lr, ny);
        } else {
            if (++rl == ny) rl = 0;
        }
    };
    T rcv[CPPF], rev[CPPF];
#pragma unroll
    for (int u = 0; u < CPPF; ++u) {
        rcv[u] = u < iters ? bload<T>(rc, vx, rl * rowb) : (T)0;
        rev[u] = u < iters ? bload<T>(re, vx, rl * rowb) : (T)0;
        advance();
    }
    int rlast = y1 + CPH - 1;
    if constexpr (MIRROR) {
        rlast = reflect(rlast, ny);
    } else {
        while (rlast >= ny) rlast -= ny;
    }
    CpStage<T> st;
    for (int t0 = 0; t0 < iters; t0 += CPPF) {
#pragma unroll
        for (int u = 0; u < CPPF; ++u) {
            const int t = t0 + u;
            const T cv = rcv[u], ev = rev[u];
            // unconditional prefetch (the last row again once past the chunk)
            rcv[u] = bload<T>(rc, vx, rl * rowb);
            rev[u] = bload<T>(re, vx, rl * rowb);
            if (t + CPPF + 1 < iters) {
                advance();
            } else {
                rl = rlast;
            }
            T co, eo;
            st.push(cv, ev, k, co, eo);
            if (t >= 2 * CPH && t < iters && out_lane) {
                const int row = y0 - 2 * CPH + t;
                bstore(co, wc, vx, row * rowb);
                bstore(eo, we, vx, row * rowb);
            }
        }
    }
}

}  // namespace

template <typename T>
void launch_cp_explicit2d(const Geom& g, double kappa, double Mc, double Meta, double dt, const T* c_in,
                          const T* e_in, T* c_out, T* e_out, int rows, hipStream_t s)
{
    const int nx = g.n[0], ny = g.n[1];
    const double m = g.h * g.h, detJ = 0.25 * g.h * g.h;
    const int ty = rows > 0 ? rows : 32;
    const int nstrips = (nx + CPOUT - 1) / CPOUT;
    const int nchunks = (ny + ty - 1) / ty;
    const int nwaves = nstrips * nchunks;
    const int blocks = (nwaves + 3) / 4;
    const unsigned bytes = (unsigned)((size_t)g.N * sizeof(T));  // caller guarantees < 2^31
    CpCoef<T> k{(T)(detJ / m), (T)(dt * Meta * detJ / m), (T)(dt * Meta * kappa / (3.0 * m)),
                (T)(dt * Mc / (3.0 * m))};
    if (g.bc)
        k_cp_explicit2d<T, true><<<blocks, 256, 0, s>>>(c_in, e_in, c_out, e_out, nx, ny, nstrips, nwaves,
                                                        nchunks, bytes, k);
    else
        k_cp_explicit2d<T, false><<<blocks, 256, 0, s>>>(c_in, e_in, c_out, e_out, nx, ny, nstrips, nwaves,
                                                         nchunks, bytes, k);
}

template void launch_cp_explicit2d<float>(const Geom&, double, double, double, double, const float*,
                                          const float*, float*, float*, int, hipStream_t);
template void launch_cp_explicit2d<double>(const Geom&, double, double, double, double, const double*,
                                           const double*, double*, double*, int, hipStream_t);

}  // namespace pfk
