// elastic.hip -- the Eshelby-inclusion benchmark: small-strain linear elasticity
// with a dilatational eigenstrain (Eqs. 3-4; eigenstrain of Supp. Note 3,
// Eq. III.1), vector Q1 elements, solved matrix-free by conjugate gradients.
//
// Operator.  With one homogeneous isotropic stiffness (Lame constants lam, mu)
// the Q1 stiffness block that couples displacement component j of node b to
// equation i of node a is
//     K_ij = lam P_ij + mu P_ji + mu delta_ij (P_xx + P_yy + P_zz),
//     P_ij(a, b) = integral of d_i phi_a d_j phi_b,
// and on a structured grid every P_ij is a Kronecker product of three 1-D
// three-point operators (the 2-point Gauss rule is exact for them):
//     mass        M = (1/6, 2/3, 1/6) h
//     stiffness   A = (-1, 2, -1) / h
//     row-derivative    R = integral phi_a' phi_b = ( 1/2, 0, -1/2)
//     column-derivative C = integral phi_a phi_b' = (-1/2, 0,  1/2)
// (interior values; a node on the first or last plane of an axis keeps only the
// half that comes from its one element there).  P_ij takes A on axis i when
// i == j, R on axis i and C on axis j when i != j, and M on the other axes.
//
// Kernel k_el_apply.  One wave covers 64 consecutive nodes of an x-y plane
// (x fastest; 62 outputs, lanes 0 and 63 are halo) and marches along z over a
// chunk of planes.  Per plane it loads the three displacement components of
// its own column at rows y-1, y, y+1 (9 coalesced loads), reduces them with
// the four y-operators (12 row sums), keeps three planes of row sums in
// registers, combines them with the z-operators of the output plane into the
// per-column quantities each x-operator needs, and finishes the x-direction
// through DPP wave shifts.  Boundary nodes need no separate path: the 1-D
// operators of a node are built from two flags (element below / above exists),
// per lane for x and y and per wave for z.  About 150 FMA per node.
//
// Boundary conditions (the benchmark's quarter / octant model): symmetry on the
// planes through the origin (u_x = 0 on x = 0, u_y = 0 on y = 0, u_z = 0 on
// z = 0) as identity rows with those inputs masked out, so K stays symmetric
// positive definite; the other faces are traction-free (the natural boundary).
// In 2-D (plane strain) the kernel's y-axis is degenerate and the problem's y
// axis plays the marching axis.
//
// Solver.  Conjugate gradients in the one-reduction form of Chronopoulos and
// Gear: per iteration one apply w = K r fused with the per-block partial sums of
// gamma = r.r and delta = w.r (FP64), then one streaming update in which every
// block reduces those partials in the same fixed order, forms alpha and beta
// and applies p = r + beta p, s = w + beta s, x += alpha p, r -= alpha s.  No
// grid-wide fence or atomic is needed (an agent-scope release per block costs
// an L2 write-back on this multi-XCD part).  The host only polls the iteration
// count and residual through pinned memory; iterations enqueued after
// convergence return at once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>

#include "../../include/pf.h"
#include "api_internal.hpp"
#include "device.hpp"
#include "kernels.hpp"
#include "stream2d.hpp"

namespace pfel {

using pfk::WAVE;

constexpr int EL_BLOCK = 256;
constexpr int EL_WAVES = EL_BLOCK / WAVE;
constexpr int EL_OUT = WAVE - 2;  // outputs per wave
constexpr int EL_MAX_PARTS = 8192;

// device-side CG state (FP64), two slots in the workspace: iteration i reads
// slot i & 1 and writes slot (i + 1) & 1, so no kernel reads what it writes
enum { S_GAMMA_OLD = 0, S_ALPHA_OLD, S_TOL2, S_ITS, S_DONE, S_MAXIT, S_GAMMA, S_COUNT };
constexpr int S_SLOT = 8;  // doubles per slot
// host-visible mirror: its, done, gamma, gamma0
enum { H_ITS = 0, H_DONE, H_GAMMA, H_GAMMA0, H_COUNT };
enum { DONE_NO = 0, DONE_CONVERGED = 1, DONE_MAXIT = 2, DONE_BREAKDOWN = 3, DONE_NONFINITE = 4 };

struct Grid {
    int dim;
    int nx, ny, nz;  // kernel axes: x = lanes, y = row axis (1 in 2-D), z = marching axis
    long long N;     // nodes
    long long P;     // nodes per plane (nx * ny)
    int coff[3];     // component plane offsets in units of N (kernel comps x, y, z); -1 = absent
    double h;
};

Grid grid_of(const pf_elastic* p)
{
    Grid g{};
    g.dim = p->dim;
    g.h = p->h;
    g.nx = (int)p->n[0];
    if (p->dim == 3) {
        g.ny = (int)p->n[1];
        g.nz = (int)p->n[2];
        g.coff[0] = 0;
        g.coff[1] = 1;
        g.coff[2] = 2;
    } else {
        g.ny = 1;
        g.nz = (int)p->n[1];
        g.coff[0] = 0;
        g.coff[1] = -1;
        g.coff[2] = 1;
    }
    g.P = (long long)g.nx * g.ny;
    g.N = g.P * g.nz;
    return g;
}

// 1-D operators of one node along one axis; lo / hi: the element below / above exists
template <typename T>
struct Fac {
    T m[3], a[3], r[3], c[3];
};

template <typename T>
__device__ __forceinline__ Fac<T> fac(bool lo, bool hi)
{
    const T L = lo ? T(1) : T(0), H = hi ? T(1) : T(0);
    Fac<T> f;
    f.m[0] = L * T(1.0 / 6.0);
    f.m[1] = (L + H) * T(1.0 / 3.0);
    f.m[2] = H * T(1.0 / 6.0);
    f.a[0] = -L;
    f.a[1] = L + H;
    f.a[2] = -H;
    f.r[0] = L * T(0.5);
    f.r[1] = (L - H) * T(0.5);
    f.r[2] = -H * T(0.5);
    f.c[0] = -L * T(0.5);
    f.c[1] = (L - H) * T(0.5);
    f.c[2] = H * T(0.5);
    return f;
}

// lane i receives lane i-1 (left) / i+1 (right); lanes without a source get 0.
// bound_ctrl zeroing leaves no old value to initialise, so the move can fold into
// the VOP2 FMA that consumes it.
__device__ __forceinline__ float nb_left(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), pfk::DPP_WAVE_SHR1, 0xf, 0xf, true));
}
__device__ __forceinline__ float nb_right(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), pfk::DPP_WAVE_SHL1, 0xf, 0xf, true));
}
__device__ __forceinline__ double nb_left(double v) { return pfk::from_left(v); }
__device__ __forceinline__ double nb_right(double v) { return pfk::from_right(v); }

template <typename T>
__device__ __forceinline__ T tap3(const T w[3], T a, T b, T c)
{
    return pfk::fmaT(w[0], a, pfk::fmaT(w[1], b, w[2] * c));
}

// one plane of a column as the operator needs it: the y-operator row sums
// [M, A, R, C] of each component and the raw (unmasked) own values
template <typename T>
struct Plane {
    T s[3][4];
    T raw[3];
};

// wave-interleaved block -> logical block map: the hardware hands consecutive
// blocks to the eight XCDs in turn; give each XCD a contiguous range so that
// neighbouring segments (which share rows) meet in the same L2
__device__ __forceinline__ int xcd_block(int b, int nb)
{
    const int xcd = b & 7, idx = b >> 3;
    const int q = nb >> 3, r = nb & 7;
    return xcd * q + min(xcd, r) + idx;
}

template <typename T>
__device__ __forceinline__ void block_sum2(double& a, double& b, double* sh)
{
    for (int off = WAVE / 2; off > 0; off >>= 1) {
        a += __shfl_down(a, off, WAVE);
        b += __shfl_down(b, off, WAVE);
    }
    const int w = threadIdx.x / WAVE, l = threadIdx.x % WAVE;
    if (l == 0) {
        sh[2 * w] = a;
        sh[2 * w + 1] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        a = 0.0;
        b = 0.0;
        for (int i = 0; i < EL_WAVES; ++i) {
            a += sh[2 * i];
            b += sh[2 * i + 1];
        }
    }
}

struct CgArgs {
    double* part;        // 2 doubles per block of the apply
    const double* state; // the CG state slot this iteration reads (S_DONE); may be null
};

// Operator modes:
//   EL_PLAIN   y = K u (ident: identity rows on the fixed components, else zero rows)
//   EL_CG      y = K u, and per-block partial sums of u.u and y.u (CG; the update
//              kernel reduces them)
//   EL_RESID   y = b - K u
//   EL_JACOBI  y = u + omega D^-1 (b - K u), D the diagonal of K (one damped
//              Jacobi sweep; the multigrid smoother)
//   EL_JACOBI_DOT  the same sweep, and per-block partial sums of y.b and b.b
//              (the preconditioned CG's z.r and r.r from the last smoothing sweep)
// In every mode the launch returns at once if cg.state says the solve is done.
enum { EL_PLAIN = 0, EL_CG = 1, EL_RESID = 2, EL_JACOBI = 3, EL_JACOBI_DOT = 4 };
template <typename T, int D, int MODE>
__global__ void __launch_bounds__(EL_BLOCK) k_el_apply(Grid g, T lam, T mu, T scale, int ident,
                                                      const T* __restrict__ u, T* __restrict__ y,
                                                      int tz, int nseg, int nitems, CgArgs cg,
                                                      const T* __restrict__ bvec, T omega)
{
    constexpr bool CG = MODE == EL_CG;
    constexpr bool JAC = MODE == EL_JACOBI || MODE == EL_JACOBI_DOT;
    constexpr bool PART = CG || MODE == EL_JACOBI_DOT;
    __shared__ double sh[2 * EL_WAVES];
    if (cg.state && cg.state[S_DONE] != 0.0) return;
    const int lane = threadIdx.x % WAVE;
    // wave-uniform work item (kept in scalar registers: plane loop, z-operators and
    // plane base addresses are then scalar)
    const int wv = __builtin_amdgcn_readfirstlane(xcd_block(blockIdx.x, gridDim.x) * EL_WAVES +
                                                  (int)(threadIdx.x / WAVE));
    double pg = 0.0, pd = 0.0;
    // work items (segment, chunk of planes), grid-strided over at most the
    // resident waves
    for (int item = wv; item < nitems; item += (int)gridDim.x * EL_WAVES) {
        const int seg = item % nseg, chunk = item / nseg;
        const long long q0 = (long long)seg * EL_OUT - 1 + lane;
        const bool out_lane = lane >= 1 && lane <= EL_OUT && q0 >= 0 && q0 < g.P;
        const int q = (int)(q0 < 0 ? 0 : (q0 >= g.P ? g.P - 1 : q0));
        const int x = q % g.nx, yr = q / g.nx;
        const Fac<T> fx = fac<T>(x > 0, x < g.nx - 1);
        const Fac<T> fy = fac<T>(yr > 0, yr < g.ny - 1);
        // byte offsets inside a plane (planes hold < 2^29 nodes)
        const unsigned ob = (unsigned)q * sizeof(T);
        const unsigned obm = (unsigned)((D == 3 && yr > 0) ? q - g.nx : q) * sizeof(T);
        const unsigned obp = (unsigned)((D == 3 && yr < g.ny - 1) ? q + g.nx : q) * sizeof(T);
        const long long N = g.N, P = g.P;
        const char* ux = reinterpret_cast<const char*>(u + (long long)g.coff[0] * N);
        const char* uy = reinterpret_cast<const char*>(D == 3 ? u + (long long)g.coff[1] * N : u);
        const char* uz = reinterpret_cast<const char*>(u + (long long)g.coff[2] * N);
        const T zx = x == 0 ? T(0) : T(1);         // u_x fixed on x = 0
        const T zym = (yr - 1 == 0) ? T(0) : T(1);  // u_y fixed on y = 0 (row y-1)
        const T zy0 = (yr == 0) ? T(0) : T(1);      // (row y)
        const T lm2 = lam + T(2) * mu;
        constexpr int NL = D == 3 ? 9 : 2;
        // loads of one plane through a buffer descriptor of that plane (scalar
        // set-up; the lane offsets are the only per-lane address state).  A plane
        // index beyond the grid is clamped to the edge plane: its values only meet
        // z-operator weights that are zero there (kz is wave-uniform).
        const unsigned plane_bytes = (unsigned)(P * (long long)sizeof(T));
        auto issue = [&](int kz, T* L) {
            kz = kz < 0 ? 0 : (kz >= g.nz ? g.nz - 1 : kz);
            const long long pb = (long long)kz * P * (long long)sizeof(T);
            const auto rx = pfk::make_rsrc(ux + pb, plane_bytes);
            const auto rz = pfk::make_rsrc(uz + pb, plane_bytes);
            if (D == 3) {
                const auto ry = pfk::make_rsrc(uy + pb, plane_bytes);
                L[0] = pfk::bload<T>(rx, (int)obm, 0);
                L[1] = pfk::bload<T>(rx, (int)ob, 0);
                L[2] = pfk::bload<T>(rx, (int)obp, 0);
                L[3] = pfk::bload<T>(ry, (int)obm, 0);
                L[4] = pfk::bload<T>(ry, (int)ob, 0);
                L[5] = pfk::bload<T>(ry, (int)obp, 0);
                L[6] = pfk::bload<T>(rz, (int)obm, 0);
                L[7] = pfk::bload<T>(rz, (int)ob, 0);
                L[8] = pfk::bload<T>(rz, (int)obp, 0);
            } else {
                L[0] = pfk::bload<T>(rx, (int)ob, 0);
                L[1] = pfk::bload<T>(rz, (int)ob, 0);
            }
        };
        // row sums of a loaded plane; ZMASK: the plane may be z = 0 (u_z fixed there)
        auto rows = [&](const T* L, int kz, Plane<T>& o, bool zmask) {
            if (D == 3) {
                o.raw[0] = L[1];
                o.raw[1] = L[4];
                o.raw[2] = L[7];
                const T zz = (zmask && kz == 0) ? T(0) : T(1);
                const T a0 = L[0] * zx, a1 = L[1] * zx, a2 = L[2] * zx;
                const T b0 = L[3] * zym, b1 = L[4] * zy0, b2 = L[5];
                T c0 = L[6], c1 = L[7], c2 = L[8];
                if (zmask) {
                    c0 *= zz;
                    c1 *= zz;
                    c2 *= zz;
                }
                o.s[0][0] = tap3(fy.m, a0, a1, a2);
                o.s[0][1] = tap3(fy.a, a0, a1, a2);
                o.s[0][2] = tap3(fy.r, a0, a1, a2);
                o.s[0][3] = tap3(fy.c, a0, a1, a2);
                o.s[1][0] = tap3(fy.m, b0, b1, b2);
                o.s[1][1] = tap3(fy.a, b0, b1, b2);
                o.s[1][2] = tap3(fy.r, b0, b1, b2);
                o.s[1][3] = tap3(fy.c, b0, b1, b2);
                o.s[2][0] = tap3(fy.m, c0, c1, c2);
                o.s[2][1] = tap3(fy.a, c0, c1, c2);
                o.s[2][2] = tap3(fy.r, c0, c1, c2);
                o.s[2][3] = tap3(fy.c, c0, c1, c2);
            } else {
                o.raw[0] = L[0];
                o.raw[1] = T(0);
                o.raw[2] = L[1];
                o.s[0][0] = L[0] * zx;
                o.s[2][0] = (zmask && kz == 0) ? T(0) : L[1];
            }
        };
        // outputs of plane k from the row sums of planes k-1, k, k+1
        auto emit = [&](int k, const Plane<T>& A_, const Plane<T>& B_, const Plane<T>& C_) {
            const Fac<T> fz = fac<T>(k > 0, k < g.nz - 1);
            enum { M = 0, A = 1, R = 2, C = 3 };
            auto Q = [&](int c, int F, const T* G) { return tap3(G, A_.s[c][F], B_.s[c][F], C_.s[c][F]); };
            T SA0, SM0, SR0, SC0, SA2, SM2, SR2, SC2, SA1 = T(0), SM1 = T(0), SR1 = T(0), SC1 = T(0);
            {
                const T q0MM = Q(0, M, fz.m), q0MA = Q(0, M, fz.a), q0MR = Q(0, M, fz.r), q0MC = Q(0, M, fz.c);
                const T q2MM = Q(2, M, fz.m), q2MA = Q(2, M, fz.a), q2MR = Q(2, M, fz.r), q2MC = Q(2, M, fz.c);
                SA0 = lm2 * q0MM;
                SM0 = mu * q0MA;
                SR0 = lam * q2MC;
                SC0 = mu * q2MR;
                SM2 = lm2 * q2MA;
                SA2 = mu * q2MM;
                SC2 = lam * q0MR;
                SR2 = mu * q0MC;
                if (D == 3) {
                    const T q0AM = Q(0, A, fz.m), q0RM = Q(0, R, fz.m), q0CM = Q(0, C, fz.m);
                    const T q1MM = Q(1, M, fz.m), q1AM = Q(1, A, fz.m), q1MA = Q(1, M, fz.a),
                            q1CM = Q(1, C, fz.m), q1RM = Q(1, R, fz.m), q1CR = Q(1, C, fz.r),
                            q1RC = Q(1, R, fz.c);
                    const T q2AM = Q(2, A, fz.m), q2RC = Q(2, R, fz.c), q2CR = Q(2, C, fz.r);
                    SM0 = mu * (q0AM + q0MA);
                    SR0 = lam * (q1CM + q2MC);
                    SC0 = mu * (q1RM + q2MR);
                    SM1 = pfk::fmaT(lm2, q1AM, pfk::fmaT(mu, q1MA, pfk::fmaT(lam, q2RC, mu * q2CR)));
                    SA1 = mu * q1MM;
                    SC1 = lam * q0RM;
                    SR1 = mu * q0CM;
                    SM2 = pfk::fmaT(lm2, q2MA, pfk::fmaT(mu, q2AM, pfk::fmaT(lam, q1CR, mu * q1RC)));
                }
            }
            auto xsum = [&](T sa, T sm, T sr, T sc) {
                T acc = pfk::fmaT(fx.a[1], sa, pfk::fmaT(fx.m[1], sm, pfk::fmaT(fx.r[1], sr, fx.c[1] * sc)));
                acc = pfk::fmaT(nb_left(sa), fx.a[0], acc);
                acc = pfk::fmaT(nb_left(sm), fx.m[0], acc);
                acc = pfk::fmaT(nb_left(sr), fx.r[0], acc);
                acc = pfk::fmaT(nb_left(sc), fx.c[0], acc);
                acc = pfk::fmaT(nb_right(sa), fx.a[2], acc);
                acc = pfk::fmaT(nb_right(sm), fx.m[2], acc);
                acc = pfk::fmaT(nb_right(sr), fx.r[2], acc);
                acc = pfk::fmaT(nb_right(sc), fx.c[2], acc);
                return acc * scale;
            };
            const T w0 = xsum(SA0, SM0, SR0, SC0);
            const T w2 = xsum(SA2, SM2, SR2, SC2);
            T w1 = T(0);
            if (D == 3) w1 = xsum(SA1, SM1, SR1, SC1);
            if (out_lane && (MODE == EL_RESID || JAC)) {
                const long long o = (long long)k * P + q;
                const T r0 = B_.raw[0], r1 = B_.raw[1], r2 = B_.raw[2];
                const bool f0 = x == 0, f1 = yr == 0, f2 = k == 0;  // fixed components
                const T k0v = f0 ? r0 : w0, k2v = f2 ? r2 : w2, k1v = f1 ? r1 : w1;
                const long long o0 = (long long)g.coff[0] * N + o, o2 = (long long)g.coff[2] * N + o;
                if (MODE == EL_RESID) {
                    y[o0] = bvec[o0] - k0v;
                    y[o2] = bvec[o2] - k2v;
                    if (D == 3) y[(long long)g.coff[1] * N + o] = bvec[(long long)g.coff[1] * N + o] - k1v;
                } else {
                    // the diagonal from the same 1-D operators (centre entries)
                    T d0, d1 = T(1), d2;
                    if (D == 3) {
                        const T pxx = fx.a[1] * fy.m[1] * fz.m[1], pyy = fx.m[1] * fy.a[1] * fz.m[1],
                                pzz = fx.m[1] * fy.m[1] * fz.a[1];
                        d0 = scale * (lm2 * pxx + mu * (pyy + pzz));
                        d1 = scale * (lm2 * pyy + mu * (pxx + pzz));
                        d2 = scale * (lm2 * pzz + mu * (pxx + pyy));
                    } else {
                        const T pxx = fx.a[1] * fz.m[1], pzz = fx.m[1] * fz.a[1];
                        d0 = lm2 * pxx + mu * pzz;
                        d2 = lm2 * pzz + mu * pxx;
                    }
                    d0 = f0 ? T(1) : d0;
                    d1 = f1 ? T(1) : d1;
                    d2 = f2 ? T(1) : d2;
                    const T b0 = bvec[o0], b2 = bvec[o2];
                    const T y0 = r0 + omega * (b0 - k0v) / d0;
                    const T y2 = r2 + omega * (b2 - k2v) / d2;
                    y[o0] = y0;
                    y[o2] = y2;
                    T y1 = T(0), b1 = T(0);
                    if (D == 3) {
                        const long long o1 = (long long)g.coff[1] * N + o;
                        b1 = bvec[o1];
                        y1 = r1 + omega * (b1 - k1v) / d1;
                        y[o1] = y1;
                    }
                    if (PART) {
                        pg += (double)y0 * b0 + (double)y2 * b2 + (D == 3 ? (double)y1 * b1 : 0.0);
                        pd += (double)b0 * b0 + (double)b2 * b2 + (D == 3 ? (double)b1 * b1 : 0.0);
                    }
                }
            } else if (out_lane) {
                const long long o = (long long)k * P + q;
                const T r0 = B_.raw[0], r1 = B_.raw[1], r2 = B_.raw[2];
                const T y0 = x == 0 ? (ident ? r0 : T(0)) : w0;
                const T y2 = k == 0 ? (ident ? r2 : T(0)) : w2;
                y[(long long)g.coff[0] * N + o] = y0;
                y[(long long)g.coff[2] * N + o] = y2;
                T y1 = T(0);
                if (D == 3) {
                    y1 = yr == 0 ? (ident ? r1 : T(0)) : w1;
                    y[(long long)g.coff[1] * N + o] = y1;
                }
                if (CG) {
                    pg += (double)r0 * r0 + (double)r2 * r2 + (D == 3 ? (double)r1 * r1 : 0.0);
                    pd += (double)y0 * r0 + (double)y2 * r2 + (D == 3 ? (double)y1 * r1 : 0.0);
                }
            }
        };
        const int k0 = chunk * tz, k1 = min(g.nz, k0 + tz);
        Plane<T> pA, pB, pC;
        T L[NL];
        issue(k0 - 1, L);
        rows(L, k0 - 1, pA, true);
        issue(k0, L);
        rows(L, k0, pB, true);
        issue(k0 + 1, L);
        // three-way unrolled plane loop: the ring roles rotate statically (no moves);
        // the loads of the plane after next are in flight while a plane is emitted
        for (int k = k0; k < k1; k += 3) {
            rows(L, k + 1, pC, false);
            issue(k + 2, L);
            emit(k, pA, pB, pC);
            if (k + 1 >= k1) break;
            rows(L, k + 2, pA, false);
            issue(k + 3, L);
            emit(k + 1, pB, pC, pA);
            if (k + 2 >= k1) break;
            rows(L, k + 3, pB, false);
            issue(k + 4, L);
            emit(k + 2, pC, pA, pB);
        }
    }
    if (!PART) return;
    block_sum2<T>(pg, pd, sh);
    if (threadIdx.x == 0) {
        cg.part[2 * blockIdx.x] = pg;
        cg.part[2 * blockIdx.x + 1] = pd;
    }
}

// One CG iteration's scalar step and vector update.  Every block reduces the
// apply's partial sums in the same fixed order (so all blocks agree bit for
// bit), forms gamma = r.r, delta = w.r and
//     beta = gamma / gamma_old,  alpha = gamma / (delta - beta gamma / alpha_old)
// (beta = 0 on the first iteration), stops on ||r||^2 <= rtol^2 ||b||^2, the
// iteration limit, a non-positive denominator or a non-finite value, and else
// updates p = r + beta p;  s = w + beta s;  x += alpha p;  r -= alpha s.
// Block 0 writes the next state slot and the host mirror.
template <typename T>
__global__ void __launch_bounds__(EL_BLOCK) k_el_cg_update(long long n, const double* __restrict__ part, int nparts,
                                                          const double* __restrict__ sin, double* __restrict__ sout,
                                                          double* host, T* __restrict__ x, T* __restrict__ r,
                                                          T* __restrict__ p, T* __restrict__ s,
                                                          const T* __restrict__ w)
{
    __shared__ double sh[2 * EL_WAVES];
    __shared__ double sc[2];
    if (sin[S_DONE] != 0.0) {
        if (blockIdx.x == 0 && threadIdx.x < S_SLOT) sout[threadIdx.x] = sin[threadIdx.x];
        return;
    }
    double ga = 0.0, de = 0.0;
    for (int i = threadIdx.x; i < nparts; i += EL_BLOCK) {
        ga += part[2 * i];
        de += part[2 * i + 1];
    }
    block_sum2<T>(ga, de, sh);
    if (threadIdx.x == 0) {
        const double its = sin[S_ITS];
        const double tol2 = its == 0.0 ? sin[S_TOL2] * ga : sin[S_TOL2];
        double done = DONE_NO, alpha = 0.0, beta = 0.0;
        if (!(std::isfinite(ga) && std::isfinite(de))) {
            done = DONE_NONFINITE;
        } else if (ga <= tol2) {
            done = DONE_CONVERGED;
        } else if (its >= sin[S_MAXIT]) {
            done = DONE_MAXIT;
        } else {
            beta = its == 0.0 ? 0.0 : ga / sin[S_GAMMA_OLD];
            const double den = its == 0.0 ? de : de - beta * ga / sin[S_ALPHA_OLD];
            if (!(den > 0.0)) done = DONE_BREAKDOWN;
            else alpha = ga / den;
        }
        sc[0] = done == DONE_NO ? alpha : 0.0;
        sc[1] = done == DONE_NO ? beta : 0.0;
        if (blockIdx.x == 0) {
            sout[S_GAMMA_OLD] = done == DONE_NO ? ga : sin[S_GAMMA_OLD];
            sout[S_ALPHA_OLD] = done == DONE_NO ? alpha : sin[S_ALPHA_OLD];
            sout[S_TOL2] = tol2;
            sout[S_ITS] = done == DONE_NO ? its + 1.0 : its;
            sout[S_DONE] = done;
            sout[S_MAXIT] = sin[S_MAXIT];
            sout[S_GAMMA] = ga;
            if (its == 0.0)
                __hip_atomic_store(&host[H_GAMMA0], ga, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            __hip_atomic_store(&host[H_GAMMA], ga, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            __hip_atomic_store(&host[H_ITS], done == DONE_NO ? its + 1.0 : its, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_SYSTEM);
            __hip_atomic_store(&host[H_DONE], done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
    __syncthreads();
    const T alpha = (T)sc[0], beta = (T)sc[1];
    if (sc[0] == 0.0) return;  // stopped (alpha > 0 on every real iteration)
    constexpr int VW = 16 / sizeof(T);
    using V = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
    const long long nv = n / VW;
    const long long stride = (long long)gridDim.x * EL_BLOCK;
    for (long long i = blockIdx.x * (long long)EL_BLOCK + threadIdx.x; i < nv; i += stride) {
        V rv = reinterpret_cast<const V*>(r)[i], pv = reinterpret_cast<const V*>(p)[i];
        V sv = reinterpret_cast<const V*>(s)[i], wv = reinterpret_cast<const V*>(w)[i];
        V xv = reinterpret_cast<const V*>(x)[i];
        T* R = reinterpret_cast<T*>(&rv);
        T* Pp = reinterpret_cast<T*>(&pv);
        T* S = reinterpret_cast<T*>(&sv);
        T* W = reinterpret_cast<T*>(&wv);
        T* X = reinterpret_cast<T*>(&xv);
#pragma unroll
        for (int j = 0; j < VW; ++j) {
            Pp[j] = pfk::fmaT(beta, Pp[j], R[j]);
            S[j] = pfk::fmaT(beta, S[j], W[j]);
            X[j] = pfk::fmaT(alpha, Pp[j], X[j]);
            R[j] = pfk::fmaT(-alpha, S[j], R[j]);
        }
        reinterpret_cast<V*>(p)[i] = pv;
        reinterpret_cast<V*>(s)[i] = sv;
        reinterpret_cast<V*>(x)[i] = xv;
        reinterpret_cast<V*>(r)[i] = rv;
    }
    for (long long i = nv * VW + blockIdx.x * (long long)EL_BLOCK + threadIdx.x; i < n; i += stride) {
        const T pn = pfk::fmaT(beta, p[i], r[i]);
        const T sn = pfk::fmaT(beta, s[i], w[i]);
        p[i] = pn;
        s[i] = sn;
        x[i] = pfk::fmaT(alpha, pn, x[i]);
        r[i] = pfk::fmaT(-alpha, sn, r[i]);
    }
}

// Eigenstrain load f_i(a) = sum over the node's elements and their Gauss points
// of |J| coef e0(|x_q|) d_i phi_a(x_q), e0 of Eq. III.1; zero on fixed components.
// A block owns a tile of nodes (8 x 8 x 4 in 3-D, 16 x 16 in 2-D): it first
// evaluates |J| coef e0 once at every Gauss point of the elements touching the
// tile (into LDS; the profile's tanh is the costly part, and each point serves
// up to 2^D nodes), then every node sums its 2^D elements' points.
template <int D>
struct RhsTile {
    static constexpr int TX = D == 3 ? 8 : 16, TY = D == 3 ? 8 : 16, TZ = D == 3 ? 4 : 1;
    // Gauss points per axis over the tile's elements (tile + 1 elements, 2 each)
    static constexpr int QX = 2 * (TX + 1), QY = 2 * (TY + 1), QZ = D == 3 ? 2 * (TZ + 1) : 1;
    static constexpr int NQ = QX * QY * QZ;
};

template <typename T, int D>
__global__ void __launch_bounds__(EL_BLOCK) k_el_rhs(Grid g, double coef, double m, double a, double l,
                                                    T* __restrict__ f, int tiles_x, int tiles_y)
{
    using RT = RhsTile<D>;
    static_assert(RT::TX * RT::TY * RT::TZ == EL_BLOCK, "one node per thread");
    __shared__ double wq[RT::NQ];
    int n[3];
    // problem axes (not kernel axes): 2-D uses (x, y), 3-D (x, y, z)
    n[0] = g.nx;
    n[1] = D == 3 ? g.ny : g.nz;
    n[2] = D == 3 ? g.nz : 1;
    const int bx = blockIdx.x % tiles_x, by = (blockIdx.x / tiles_x) % tiles_y, bz = blockIdx.x / (tiles_x * tiles_y);
    const int t0[3] = {bx * RT::TX, by * RT::TY, bz * RT::TZ};
    const double h = g.h;
    const double gq = 0.57735026918962576451;  // 1/sqrt(3)
    const double detJ = D == 3 ? 0.125 * h * h * h : 0.25 * h * h;
    // phase 1: the tile's Gauss-point weights; local point q on an axis belongs to
    // element t0 - 1 + q / 2, at its lower (even q) or upper Gauss coordinate
    for (int qi = threadIdx.x; qi < RT::NQ; qi += EL_BLOCK) {
        const int q[3] = {qi % RT::QX, (qi / RT::QX) % RT::QY, qi / (RT::QX * RT::QY)};
        double r2 = 0.0;
        bool ok = true;
        for (int k = 0; k < D; ++k) {
            const int el = t0[k] - 1 + (q[k] >> 1);
            ok = ok && el >= 0 && el < n[k] - 1;
            const double xi = (q[k] & 1) ? gq : -gq;  // reference coordinate in [-1, 1]
            const double xk = h * (el + 0.5 * (1.0 + xi));
            r2 += xk * xk;
        }
        wq[qi] = ok ? detJ * coef * (m * (0.5 - 0.5 * tanh(l * (sqrt(r2) - a)))) : 0.0;
    }
    __syncthreads();
    // phase 2: one node per thread
    const int lt[3] = {(int)(threadIdx.x % RT::TX), (int)((threadIdx.x / RT::TX) % RT::TY),
                       (int)(threadIdx.x / (RT::TX * RT::TY))};
    int idx[3];
    bool inside = true;
    for (int k = 0; k < 3; ++k) {
        idx[k] = t0[k] + lt[k];
        inside = inside && idx[k] < n[k];
    }
    if (!inside) return;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int e = 0; e < (1 << D); ++e) {
        // element whose local node bit b_k (0 = lower, 1 = upper) on axis k is e's
        // bit: local element lt_k + 1 - b_k of the tile's range
        for (int qp = 0; qp < (1 << D); ++qp) {
            int qloc[3] = {0, 0, 0};
            double val[3], der[3];
            for (int k = 0; k < D; ++k) {
                const int qb = (qp >> k) & 1, b = (e >> k) & 1;
                qloc[k] = 2 * (lt[k] + 1 - b) + qb;
                const double xi = qb ? gq : -gq;
                const double sgn = b ? 1.0 : -1.0;
                val[k] = 0.5 * (1.0 + sgn * xi);
                der[k] = sgn / h;
            }
            const double w = wq[qloc[0] + RT::QX * (qloc[1] + RT::QY * qloc[2])];
            for (int c = 0; c < D; ++c) {
                double gc = der[c];
                for (int k = 0; k < D; ++k)
                    if (k != c) gc *= val[k];
                acc[c] += w * gc;
            }
        }
    }
    const long long i = idx[0] + (long long)n[0] * (idx[1] + (long long)n[1] * idx[2]);
    for (int c = 0; c < D; ++c) f[c * g.N + i] = idx[c] == 0 ? T(0) : (T)acc[c];
}

// Coordinates on the problem axes (n[0] fastest) of node i; 32-bit division when
// the grid has fewer than 2^32 nodes (64-bit division is a long instruction
// sequence on the GPU).
template <int D>
__device__ __forceinline__ void node_coords(long long i, const int* n, long long N, int* idx)
{
    if (N <= 0xffffffffll) {
        const unsigned u = (unsigned)i, q = u / (unsigned)n[0];
        idx[0] = (int)(u - q * (unsigned)n[0]);
        if (D == 3) {
            const unsigned q2 = q / (unsigned)n[1];
            idx[1] = (int)(q - q2 * (unsigned)n[1]);
            idx[2] = (int)q2;
        } else {
            idx[1] = (int)q;
            idx[2] = 0;
        }
    } else {
        idx[0] = (int)(i % n[0]);
        idx[1] = (int)((i / n[0]) % n[1]);
        idx[2] = D == 3 ? (int)(i / ((long long)n[0] * n[1])) : 0;
    }
}

// volume-change weights: integral of d_i phi_a over the body, i.e. the outward
// face normal times the face share of the node (nonzero on the far faces only)
template <int D>
__device__ __forceinline__ double vol_weight(const int* idx, const int* n, int c, double h)
{
    if (idx[c] == 0 || idx[c] != n[c] - 1) return 0.0;
    double w = 1.0;
    for (int k = 0; k < D; ++k)
        if (k != c) w *= (idx[k] == 0 || idx[k] == n[k] - 1) ? 0.5 * h : h;
    return w;
}

// partial sums of g . u (g == nullptr: the volume-change weights), one per block
template <typename T, int D>
__global__ void __launch_bounds__(EL_BLOCK) k_el_dot(Grid g, const T* __restrict__ gw, const T* __restrict__ u,
                                                    double* __restrict__ part)
{
    __shared__ double sh[2 * EL_WAVES];
    int n[3];
    n[0] = g.nx;
    n[1] = D == 3 ? g.ny : g.nz;
    n[2] = D == 3 ? g.nz : 1;
    double acc = 0.0, dummy = 0.0;
    const long long stride = (long long)gridDim.x * EL_BLOCK;
    for (long long i = blockIdx.x * (long long)EL_BLOCK + threadIdx.x; i < g.N; i += stride) {
        int idx[3];
        node_coords<D>(i, n, g.N, idx);
        for (int c = 0; c < D; ++c) {
            const double wc = gw ? (double)gw[c * g.N + i] : vol_weight<D>(idx, n, c, g.h);
            acc += wc * (double)u[c * g.N + i];
        }
    }
    block_sum2<T>(acc, dummy, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// one block: out[0] = sum of part[0..nb) in a fixed order
__global__ void __launch_bounds__(EL_BLOCK) k_el_sum(const double* __restrict__ part, int nb,
                                                    double* __restrict__ out)
{
    __shared__ double sh[2 * EL_WAVES];
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < nb; i += EL_BLOCK) a += part[i];
    block_sum2<float>(a, b, sh);
    if (threadIdx.x == 0) out[0] = a;
}

// CG state initialisation: slot 0 (slot 1 cleared) and the host mirror
__global__ void k_el_cg_init(double* state, double* host, double rtol2, double maxit)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        for (int i = 0; i < 2 * S_SLOT; ++i) state[i] = 0.0;
        state[S_ALPHA_OLD] = 1.0;
        state[S_TOL2] = rtol2;
        state[S_MAXIT] = maxit;
        for (int i = 0; i < H_COUNT; ++i)
            __hip_atomic_store(&host[i], 0.0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

template <typename T>
__global__ void __launch_bounds__(EL_BLOCK) k_el_fill(long long n, T* __restrict__ a, const T* __restrict__ src)
{
    const long long stride = (long long)gridDim.x * EL_BLOCK;
    for (long long i = blockIdx.x * (long long)EL_BLOCK + threadIdx.x; i < n; i += stride)
        a[i] = src ? src[i] : T(0);
}

// dst = src with the fixed components zeroed (src == nullptr: the volume-change weights)
template <typename T, int D>
__global__ void __launch_bounds__(EL_BLOCK) k_el_weights(Grid g, const T* __restrict__ src, T* __restrict__ dst)
{
    const long long i = blockIdx.x * (long long)EL_BLOCK + threadIdx.x;
    if (i >= g.N) return;
    int n[3], idx[3];
    n[0] = g.nx;
    n[1] = D == 3 ? g.ny : g.nz;
    n[2] = D == 3 ? g.nz : 1;
    node_coords<D>(i, n, g.N, idx);
    for (int c = 0; c < D; ++c) {
        const long long o = c * g.N + i;
        dst[o] = idx[c] == 0 ? T(0) : (src ? src[o] : (T)vol_weight<D>(idx, n, c, g.h));
    }
}

// ---------------------------------------------------------------------------
// Geometric multigrid (V-cycle) preconditioner and the preconditioned CG.
// The Q1 spaces of the grids n, (n - 1)/2 + 1, ... are nested, and with one
// homogeneous stiffness the Galerkin coarse operator P^T K P equals the Q1
// stiffness rediscretised at 2h, so every level runs k_el_apply with its own
// spacing.  Restriction is the transpose of the trilinear prolongation; the
// symmetry-plane components stay fixed (zero) on every level.

constexpr int MG_MAXL = 12;
constexpr int MG_PRE = 2, MG_POST = 2;  // damped-Jacobi sweeps (even, >= 2: results land back in x)
// sweeps on the coarsest grid: twice its longest axis (even), within [4, 32]
constexpr int MG_COARSE_MIN = 4, MG_COARSE_MAX = 32;
// Jacobi damping omega = MG_SMOOTH / lambda_max(D^-1 K).  lambda_max depends on
// the dimension and nu only (2.0 to 3.5 in 2-D, 2.2 to 6.2 in 3-D for nu in
// [0, 0.49]; its modes sit at the free surfaces), and a 9^d grid already has the
// large-grid value; MG_POWER power steps from a pseudo-random start come within
// about 1.5 %, which keeps omega lambda_max well below 2.
constexpr double MG_SMOOTH = 1.6;
constexpr int MG_EIG_N = 9, MG_POWER = 64;

// PCG state (FP64, one slot; the done flag sits where k_el_apply looks for it)
enum { P_RHO = 0, P_RHO_OLD = 1, P_TOL2 = 2, P_ITS = 3, P_DONE = 4, P_MAXIT = 5, P_RR = 6, P_RTOL2 = 7 };
static_assert(P_DONE == S_DONE, "the operator's early exit reads the same done flag");

template <int D>
__device__ __forceinline__ void prob_axes(const Grid& g, int* n)
{
    n[0] = g.nx;
    n[1] = D == 3 ? g.ny : g.nz;
    n[2] = D == 3 ? g.nz : 1;
}

// The first smoothing sweep from x = 0: y = omega D^-1 b (no operator
// needed), D the diagonal of K from the centre entries of the 1-D operators
// (1 on the fixed components)
template <typename T, int D>
__global__ void __launch_bounds__(EL_BLOCK) k_el_jacobi0(Grid g, T lam, T mu, T scale, const T* __restrict__ b,
                                                        T* __restrict__ y, T omega, const double* __restrict__ st)
{
    if (st && st[P_DONE] != 0.0) return;
    const long long i = blockIdx.x * (long long)EL_BLOCK + threadIdx.x;
    if (i >= g.N) return;
    int n[3], idx[3];
    prob_axes<D>(g, n);
    node_coords<D>(i, n, g.N, idx);
    T mc[3], ac[3];
    for (int k = 0; k < D; ++k) {
        const Fac<T> f = fac<T>(idx[k] > 0, idx[k] < n[k] - 1);
        mc[k] = f.m[1];
        ac[k] = f.a[1];
    }
    const T lm2 = lam + T(2) * mu;
    for (int c = 0; c < D; ++c) {
        // P_kk centre entry: a on axis k, m on the others
        T diag = T(0);
        for (int k = 0; k < D; ++k) {
            T pkk = ac[k];
            for (int j = 0; j < D; ++j)
                if (j != k) pkk *= mc[j];
            diag += (k == c ? lm2 : mu) * pkk;
        }
        diag *= scale;
        const long long o = c * g.N + i;
        y[o] = idx[c] == 0 ? omega * b[o] : omega * b[o] / diag;
    }
}

// rc = P^T rf: coarse node I gathers the fine nodes 2I + o (|o_k| <= 1, inside the
// grid) with weights prod_k (o_k == 0 ? 1 : 1/2); fixed coarse components are zero
template <typename T, int D>
__global__ void __launch_bounds__(EL_BLOCK) k_el_restrict(Grid gf, Grid gc, const T* __restrict__ rf,
                                                         T* __restrict__ rc, const double* __restrict__ st)
{
    if (st && st[P_DONE] != 0.0) return;
    const long long I = blockIdx.x * (long long)EL_BLOCK + threadIdx.x;
    if (I >= gc.N) return;
    int nc[3], nf[3], ic[3];
    prob_axes<D>(gc, nc);
    prob_axes<D>(gf, nf);
    node_coords<D>(I, nc, gc.N, ic);
    T acc[3] = {T(0), T(0), T(0)};
    for (int oz = (D == 3 ? -1 : 0); oz <= (D == 3 ? 1 : 0); ++oz)
        for (int oy = -1; oy <= 1; ++oy)
            for (int ox = -1; ox <= 1; ++ox) {
                const int fx = 2 * ic[0] + ox, fy = 2 * ic[1] + oy, fz = 2 * ic[2] + oz;
                if (fx < 0 || fx >= nf[0] || fy < 0 || fy >= nf[1] || fz < 0 || fz >= nf[2]) continue;
                const T w = (ox ? T(0.5) : T(1)) * (oy ? T(0.5) : T(1)) * (oz ? T(0.5) : T(1));
                const long long fi = fx + (long long)nf[0] * (fy + (long long)nf[1] * fz);
                for (int c = 0; c < D; ++c) acc[c] = pfk::fmaT(w, rf[c * gf.N + fi], acc[c]);
            }
    for (int c = 0; c < D; ++c) rc[c * gc.N + I] = ic[c] == 0 ? T(0) : acc[c];
}

// xf += P ec (trilinear interpolation of the coarse correction)
template <typename T, int D>
__global__ void __launch_bounds__(EL_BLOCK) k_el_prolong(Grid gc, Grid gf, const T* __restrict__ ec,
                                                        T* __restrict__ xf, const double* __restrict__ st)
{
    if (st && st[P_DONE] != 0.0) return;
    const long long F = blockIdx.x * (long long)EL_BLOCK + threadIdx.x;
    if (F >= gf.N) return;
    int nc[3], nf[3], f[3];
    prob_axes<D>(gc, nc);
    prob_axes<D>(gf, nf);
    node_coords<D>(F, nf, gf.N, f);
    int lo[3], hi[3];
    for (int k = 0; k < 3; ++k) {
        lo[k] = f[k] >> 1;
        hi[k] = (f[k] & 1) ? lo[k] + 1 : lo[k];
    }
    T acc[3] = {T(0), T(0), T(0)};
    for (int bz = 0; bz < (D == 3 ? 2 : 1); ++bz)
        for (int by = 0; by < 2; ++by)
            for (int bx = 0; bx < 2; ++bx) {
                const int cx = bx ? hi[0] : lo[0], cy = by ? hi[1] : lo[1], cz = bz ? hi[2] : lo[2];
                // a node on a coarse line takes its one coarse value once (weight 1)
                const T w = ((f[0] & 1) ? T(0.5) : (bx ? T(0) : T(1))) * ((f[1] & 1) ? T(0.5) : (by ? T(0) : T(1))) *
                            (D == 3 ? ((f[2] & 1) ? T(0.5) : (bz ? T(0) : T(1))) : T(1));
                if (w == T(0)) continue;
                const long long ci = cx + (long long)nc[0] * (cy + (long long)nc[1] * cz);
                for (int c = 0; c < D; ++c) acc[c] = pfk::fmaT(w, ec[c * gc.N + ci], acc[c]);
            }
    for (int c = 0; c < D; ++c) xf[c * gf.N + F] += acc[c];
}

// The done flag as one block-wide decision: block 0 of k_pcg_rho / k_pcg_alpha
// may set it while other blocks start, and a block whose waves disagreed would
// split at its barriers.
__device__ __forceinline__ bool pcg_block_done(const double* st)
{
    __shared__ int flag;
    if (threadIdx.x == 0) flag = st[P_DONE] != 0.0;
    __syncthreads();
    return flag != 0;
}

// reduce nparts (z.r, r.r) pairs in a fixed order (every block gets the same sums)
__device__ __forceinline__ void reduce_pairs_block(const double* __restrict__ part, int nparts, double* sh,
                                                   double& a, double& b)
{
    a = 0.0;
    b = 0.0;
    for (int i = threadIdx.x; i < nparts; i += EL_BLOCK) {
        a += part[2 * i];
        b += part[2 * i + 1];
    }
    block_sum2<float>(a, b, sh);
}

// rho = z.r; stop on ||r||^2 <= rtol^2 ||b||^2, the iteration limit or a
// non-positive rho; else beta = rho / rho_old (0 on the first iteration) and
// p = z + beta p.  Block 0 records the state and the host mirror.
template <typename T>
__global__ void __launch_bounds__(EL_BLOCK) k_pcg_rho(long long n, const double* __restrict__ part, int nparts,
                                                     double* st, double* host, const T* __restrict__ z,
                                                     T* __restrict__ p)
{
    __shared__ double sh[2 * EL_WAVES];
    __shared__ double sc[2];
    if (pcg_block_done(st)) return;
    double zr, rr;
    reduce_pairs_block(part, nparts, sh, zr, rr);
    if (threadIdx.x == 0) {
        const double its = st[P_ITS];
        const double tol2 = its == 0.0 ? st[P_RTOL2] * rr : st[P_TOL2];
        double done = DONE_NO;
        if (!(std::isfinite(zr) && std::isfinite(rr))) done = DONE_NONFINITE;
        else if (rr <= tol2) done = DONE_CONVERGED;
        else if (its >= st[P_MAXIT]) done = DONE_MAXIT;
        else if (!(zr > 0.0)) done = DONE_BREAKDOWN;
        sc[0] = done;
        sc[1] = (done == DONE_NO && its > 0.0) ? zr / st[P_RHO_OLD] : 0.0;
        if (blockIdx.x == 0) {
            st[P_RHO] = zr;
            st[P_RR] = rr;
            if (its == 0.0) {
                st[P_TOL2] = tol2;
                __hip_atomic_store(&host[H_GAMMA0], rr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            }
            __hip_atomic_store(&host[H_GAMMA], rr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            __hip_atomic_store(&host[H_ITS], its, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            __hip_atomic_store(&host[H_DONE], done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            if (done != DONE_NO) st[P_DONE] = done;
        }
    }
    __syncthreads();
    if (sc[0] != DONE_NO) return;
    const T beta = (T)sc[1];
    const long long stride = (long long)gridDim.x * EL_BLOCK;
    for (long long i = blockIdx.x * (long long)EL_BLOCK + threadIdx.x; i < n; i += stride)
        p[i] = pfk::fmaT(beta, p[i], z[i]);
}

// alpha = rho / (p . K p) from the operator's partials (second of each pair);
// x += alpha p, r -= alpha q, and per-block partial sums of the new r.r (rpart)
template <typename T>
__global__ void __launch_bounds__(EL_BLOCK) k_pcg_alpha(long long n, const double* __restrict__ part, int nparts,
                                                       double* st, double* host, T* __restrict__ x,
                                                       T* __restrict__ r, const T* __restrict__ p,
                                                       const T* __restrict__ q, double* __restrict__ rpart)
{
    __shared__ double sh[2 * EL_WAVES];
    __shared__ double sc[1];
    if (pcg_block_done(st)) return;
    double pp, pq;
    reduce_pairs_block(part, nparts, sh, pp, pq);
    if (threadIdx.x == 0) {
        const bool ok = pq > 0.0 && std::isfinite(pq);
        sc[0] = ok ? st[P_RHO] / pq : 0.0;
        if (blockIdx.x == 0) {
            if (ok) {
                st[P_RHO_OLD] = st[P_RHO];
                st[P_ITS] = st[P_ITS] + 1.0;
                __hip_atomic_store(&host[H_ITS], st[P_ITS], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            } else {
                st[P_DONE] = std::isfinite(pq) ? (double)DONE_BREAKDOWN : (double)DONE_NONFINITE;
                __hip_atomic_store(&host[H_DONE], st[P_DONE], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            }
        }
    }
    __syncthreads();
    if (sc[0] == 0.0) return;
    const T alpha = (T)sc[0];
    const long long stride = (long long)gridDim.x * EL_BLOCK;
    double rr = 0.0, dummy = 0.0;
    for (long long i = blockIdx.x * (long long)EL_BLOCK + threadIdx.x; i < n; i += stride) {
        x[i] = pfk::fmaT(alpha, p[i], x[i]);
        const T rv = pfk::fmaT(-alpha, q[i], r[i]);
        r[i] = rv;
        rr += (double)rv * rv;
    }
    __syncthreads();  // sh is reused
    block_sum2<T>(rr, dummy, sh);
    if (threadIdx.x == 0) rpart[blockIdx.x] = rr;
}

// The stop test on the updated residual, before the next V-cycle: one block
// reduces k_pcg_alpha's partials; ||r||^2 <= rtol^2 ||b||^2, a non-finite value or
// the iteration limit end the solve (every later launch then returns at once).
__global__ void __launch_bounds__(EL_BLOCK) k_pcg_check(const double* __restrict__ rpart, int nparts, double* st,
                                                       double* host)
{
    __shared__ double sh[2 * EL_WAVES];
    if (st[P_DONE] != 0.0) return;
    double rr = 0.0, dummy = 0.0;
    for (int i = threadIdx.x; i < nparts; i += EL_BLOCK) rr += rpart[i];
    block_sum2<float>(rr, dummy, sh);
    if (threadIdx.x == 0) {
        double done = DONE_NO;
        if (!std::isfinite(rr)) done = DONE_NONFINITE;
        else if (rr <= st[P_TOL2]) done = DONE_CONVERGED;
        else if (st[P_ITS] >= st[P_MAXIT]) done = DONE_MAXIT;
        st[P_RR] = rr;
        __hip_atomic_store(&host[H_GAMMA], rr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        if (done != DONE_NO) {
            st[P_DONE] = done;
            __hip_atomic_store(&host[H_DONE], done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
}

__global__ void k_pcg_init(double* st, double* host, double rtol2, double maxit)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        for (int i = 0; i < S_SLOT; ++i) st[i] = 0.0;
        st[P_RTOL2] = rtol2;
        st[P_MAXIT] = maxit;
        for (int i = 0; i < H_COUNT; ++i)
            __hip_atomic_store(&host[i], 0.0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// Power iteration for the largest eigenvalue of D^-1 K (the smoother's damping).
// Seed: a fixed pseudo-random vector in [-1, 1) (an integer hash of the index),
// which has a component along the oscillatory top mode.
__global__ void __launch_bounds__(EL_BLOCK) k_el_seed(long long n, double* __restrict__ v)
{
    const long long stride = (long long)gridDim.x * EL_BLOCK;
    for (long long i = blockIdx.x * (long long)EL_BLOCK + threadIdx.x; i < n; i += stride) {
        unsigned long long z = (unsigned long long)i + 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        v[i] = (double)(z >> 11) * 0x1.0p-52 - 1.0;
    }
}

// One block: out[0] = ||v||, then v /= ||v||
__global__ void __launch_bounds__(EL_BLOCK) k_el_normalize(long long n, double* __restrict__ v,
                                                          double* __restrict__ out)
{
    __shared__ double sh[2 * EL_WAVES];
    __shared__ double nrm;
    double a = 0.0, b = 0.0;
    for (long long i = threadIdx.x; i < n; i += EL_BLOCK) a += v[i] * v[i];
    block_sum2<double>(a, b, sh);
    if (threadIdx.x == 0) {
        nrm = std::sqrt(a);
        out[0] = nrm;
    }
    __syncthreads();
    const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
    for (long long i = threadIdx.x; i < n; i += EL_BLOCK) v[i] *= inv;
}

// ---------------------------------------------------------------------------
// The coarse end of the V-cycle in one workgroup.  On the smallest grids every
// launch costs its fixed dispatch latency (3-5 us) for almost no work, so the
// levels from a few hundred nodes down run inside one 1024-thread block with
// all their vectors (x, b, t per level) in LDS: the same smoothing, residual,
// transfer and coarsest-grid steps as the multi-launch cycle, with the operator
// assembled per node from the same 1-D operators.

constexpr int MG_BOTTOM_MAXL = 8;
constexpr int MG_BOTTOM_THREADS = 1024;
// nodes per level at most.  Measured: in 2-D the block with grids up to 33^2
// makes a 1025^2 solve 1.3x faster (2.33 vs 3.04 ms) and a 257^2 one 1.5x; in
// 3-D one block is slower than the launches it replaces (a 9^3 pass has 27
// neighbours x 3 x 3 couplings per node on one CU), so 3-D keeps every launch.
constexpr long long MG_BOTTOM_NODES_3D = 0, MG_BOTTOM_NODES_2D = 1200;
constexpr size_t MG_BOTTOM_LDS = 48 * 1024;       // bytes of LDS for all its vectors

template <typename T>
struct BottomArgs {
    int nl;             // levels run in the block (the first is the entry level)
    int coarse_sweeps;  // smoothing sweeps on the coarsest level
    int n[MG_BOTTOM_MAXL][3];
    int N[MG_BOTTOM_MAXL];
    int off[MG_BOTTOM_MAXL];  // LDS offset (elements) of the level's x; b and t follow
    T scale[MG_BOTTOM_MAXL];  // the operator's row scale (h in 3-D, 1 in 2-D)
    T lam, mu, omega;
};

// (K u) at node idx on one level, all D components, and the diagonal of K there;
// K_cd(o) = lam P_cd + mu P_dc + mu delta_cd sum_k P_kk, each P a product of 1-D
// operators (A on the differentiated axis, R / C on the two axes of a mixed
// term, M elsewhere).  Fixed components: identity rows, masked columns.
template <typename T, int D>
__device__ void bottom_ku(const T* __restrict__ u, int N, const int* n, const int* idx, T lam, T mu, T scale,
                          T* ku, T* dg)
{
    Fac<T> F[3];
    for (int k = 0; k < D; ++k) F[k] = fac<T>(idx[k] > 0, idx[k] < n[k] - 1);
    const T lm2 = lam + T(2) * mu;
    T acc[3] = {T(0), T(0), T(0)};
    const int i = idx[0] + n[0] * (idx[1] + n[1] * idx[2]);
    constexpr int NO = D == 3 ? 27 : 9;
    for (int oi = 0; oi < NO; ++oi) {
        const int o[3] = {oi % 3, (oi / 3) % 3, D == 3 ? oi / 9 : 1};
        int nb[3] = {0, 0, 0};
        bool inside = true;
        for (int k = 0; k < D; ++k) {
            nb[k] = idx[k] + o[k] - 1;
            inside = inside && nb[k] >= 0 && nb[k] < n[k];
        }
        if (!inside) continue;  // the 1-D weights towards a missing neighbour are zero
        // (selects rather than indexing by o: keeps the factors in registers)
        auto pick = [](const T* w, int j) { return j == 0 ? w[0] : (j == 1 ? w[1] : w[2]); };
        T m[3], a[3], r[3], c[3];
        for (int k = 0; k < D; ++k) {
            m[k] = pick(F[k].m, o[k]);
            a[k] = pick(F[k].a, o[k]);
            r[k] = pick(F[k].r, o[k]);
            c[k] = pick(F[k].c, o[k]);
        }
        T pkk[3], sp = T(0);
        for (int k = 0; k < D; ++k) {
            T v = a[k];
            for (int j = 0; j < D; ++j)
                if (j != k) v *= m[j];
            pkk[k] = v;
            sp += v;
        }
        const int nbi = nb[0] + n[0] * (nb[1] + n[1] * nb[2]);
        for (int cc = 0; cc < D; ++cc) {
            for (int d = 0; d < D; ++d) {
                if (nb[d] == 0) continue;  // the neighbour's component d is fixed (masked)
                T coef;
                if (cc == d) {
                    coef = lm2 * pkk[cc] + mu * (sp - pkk[cc]);
                } else {
                    T rest = T(1);
                    for (int j = 0; j < D; ++j)
                        if (j != cc && j != d) rest *= m[j];
                    coef = (lam * (r[cc] * c[d]) + mu * (r[d] * c[cc])) * rest;
                }
                acc[cc] += coef * u[d * N + nbi];
            }
            if (oi == NO / 2) dg[cc] = (lm2 * pkk[cc] + mu * (sp - pkk[cc])) * scale;
        }
    }
    for (int cc = 0; cc < D; ++cc) {
        const bool fixed = idx[cc] == 0;
        ku[cc] = fixed ? u[cc * N + i] : acc[cc] * scale;
        if (fixed) dg[cc] = T(1);
    }
}

// the diagonal of K at node idx (1 on fixed components)
template <typename T, int D>
__device__ void bottom_dg(const int* n, const int* idx, T lam, T mu, T scale, T* dg)
{
    T mc[3], ac[3];
    for (int k = 0; k < D; ++k) {
        const Fac<T> f = fac<T>(idx[k] > 0, idx[k] < n[k] - 1);
        mc[k] = f.m[1];
        ac[k] = f.a[1];
    }
    const T lm2 = lam + T(2) * mu;
    T pkk[3], sp = T(0);
    for (int k = 0; k < D; ++k) {
        T v = ac[k];
        for (int j = 0; j < D; ++j)
            if (j != k) v *= mc[j];
        pkk[k] = v;
        sp += v;
    }
    for (int c = 0; c < D; ++c) dg[c] = idx[c] == 0 ? T(1) : (lm2 * pkk[c] + mu * (sp - pkk[c])) * scale;
}

template <int D>
__device__ __forceinline__ void bottom_coords(int i, const int* n, int* idx)
{
    idx[0] = i % n[0];
    idx[1] = (i / n[0]) % n[1];
    idx[2] = D == 3 ? i / (n[0] * n[1]) : 0;
}

template <typename T, int D>
__global__ void __launch_bounds__(MG_BOTTOM_THREADS) k_el_bottom(BottomArgs<T> a, const T* __restrict__ bin,
                                                                T* __restrict__ xout, const double* __restrict__ st)
{
    if (st && st[P_DONE] != 0.0) return;
    extern __shared__ double bottom_smem[];
    T* lds = reinterpret_cast<T*>(bottom_smem);
    const int tid = threadIdx.x;
    auto X = [&](int l) { return lds + a.off[l]; };
    auto B = [&](int l) { return lds + a.off[l] + D * a.N[l]; };
    auto Tt = [&](int l) { return lds + a.off[l] + 2 * D * a.N[l]; };
    for (int i = tid; i < D * a.N[0]; i += MG_BOTTOM_THREADS) B(0)[i] = bin[i];
    __syncthreads();
    // y = u + omega D^-1 (b - K u) on level l (from_zero: y = omega D^-1 b);
    // resid: y = b - K u
    auto pass = [&](int l, const T* u, T* y, bool from_zero, bool resid) {
        const T* b = B(l);
        const int N = a.N[l];
        for (int i = tid; i < N; i += MG_BOTTOM_THREADS) {
            int idx[3];
            bottom_coords<D>(i, a.n[l], idx);
            T ku[3] = {T(0), T(0), T(0)}, dg[3] = {T(1), T(1), T(1)};
            if (from_zero)
                bottom_dg<T, D>(a.n[l], idx, a.lam, a.mu, a.scale[l], dg);
            else
                bottom_ku<T, D>(u, N, a.n[l], idx, a.lam, a.mu, a.scale[l], ku, dg);
            for (int c = 0; c < D; ++c) {
                const int o = c * N + i;
                if (resid) y[o] = b[o] - ku[c];
                else if (from_zero) y[o] = a.omega * b[o] / dg[c];
                else y[o] = u[o] + a.omega * (b[o] - ku[c]) / dg[c];
            }
        }
        __syncthreads();
    };
    // bit l of cur: which of (x, t) holds level l's iterate (1 = t)
    unsigned cur = 0;
    for (int l = 0; l < a.nl; ++l) {
        const bool coarsest = l == a.nl - 1;
        const int pre = coarsest ? a.coarse_sweeps : MG_PRE;
        T* v[2] = {X(l), Tt(l)};
        int c = 0;
        pass(l, nullptr, v[c], true, false);
        for (int s = 1; s < pre; ++s) {
            pass(l, v[c], v[c ^ 1], false, false);
            c ^= 1;
        }
        cur |= (unsigned)c << l;
        if (coarsest) break;
        // residual into the other vector, restricted into the next level's b
        pass(l, v[c], v[c ^ 1], false, true);
        const T* rf = v[c ^ 1];
        T* rc = B(l + 1);
        const int Nc = a.N[l + 1], Nf = a.N[l];
        for (int I = tid; I < Nc; I += MG_BOTTOM_THREADS) {
            int ic[3];
            bottom_coords<D>(I, a.n[l + 1], ic);
            T acc[3] = {T(0), T(0), T(0)};
            for (int oz = (D == 3 ? -1 : 0); oz <= (D == 3 ? 1 : 0); ++oz)
                for (int oy = -1; oy <= 1; ++oy)
                    for (int ox = -1; ox <= 1; ++ox) {
                        const int fx = 2 * ic[0] + ox, fy = 2 * ic[1] + oy, fz = 2 * ic[2] + oz;
                        if (fx < 0 || fx >= a.n[l][0] || fy < 0 || fy >= a.n[l][1] || fz < 0 ||
                            fz >= (D == 3 ? a.n[l][2] : 1))
                            continue;
                        const T w = (ox ? T(0.5) : T(1)) * (oy ? T(0.5) : T(1)) * (oz ? T(0.5) : T(1));
                        const int fi = fx + a.n[l][0] * (fy + a.n[l][1] * fz);
                        for (int cc = 0; cc < D; ++cc) acc[cc] += w * rf[cc * Nf + fi];
                    }
            for (int cc = 0; cc < D; ++cc) rc[cc * Nc + I] = ic[cc] == 0 ? T(0) : acc[cc];
        }
        __syncthreads();
    }
    for (int l = a.nl - 2; l >= 0; --l) {
        T* v[2] = {X(l), Tt(l)};
        int c = (cur >> l) & 1;
        // prolongation of the coarser level's iterate into this level's
        const T* ec = ((cur >> (l + 1)) & 1) ? Tt(l + 1) : X(l + 1);
        const int Nc = a.N[l + 1], Nf = a.N[l];
        for (int F = tid; F < Nf; F += MG_BOTTOM_THREADS) {
            int f[3];
            bottom_coords<D>(F, a.n[l], f);
            int lo[3], hi[3];
            for (int k = 0; k < 3; ++k) {
                lo[k] = f[k] >> 1;
                hi[k] = (f[k] & 1) ? lo[k] + 1 : lo[k];
            }
            T acc[3] = {T(0), T(0), T(0)};
            for (int bz = 0; bz < (D == 3 ? 2 : 1); ++bz)
                for (int by = 0; by < 2; ++by)
                    for (int bx = 0; bx < 2; ++bx) {
                        const T w = ((f[0] & 1) ? T(0.5) : (bx ? T(0) : T(1))) *
                                    ((f[1] & 1) ? T(0.5) : (by ? T(0) : T(1))) *
                                    (D == 3 ? ((f[2] & 1) ? T(0.5) : (bz ? T(0) : T(1))) : T(1));
                        if (w == T(0)) continue;
                        const int cx = bx ? hi[0] : lo[0], cy = by ? hi[1] : lo[1], cz = bz ? hi[2] : lo[2];
                        const int ci = cx + a.n[l + 1][0] * (cy + a.n[l + 1][1] * cz);
                        for (int cc = 0; cc < D; ++cc) acc[cc] += w * ec[cc * Nc + ci];
                    }
            for (int cc = 0; cc < D; ++cc) v[c][cc * Nf + F] += acc[cc];
        }
        __syncthreads();
        for (int s = 0; s < MG_POST; ++s) {
            pass(l, v[c], v[c ^ 1], false, false);
            c ^= 1;
        }
        cur = (cur & ~(1u << l)) | ((unsigned)c << l);
    }
    const T* res = (cur & 1) ? Tt(0) : X(0);
    for (int i = tid; i < D * a.N[0]; i += MG_BOTTOM_THREADS) xout[i] = res[i];
}

// ---------------------------------------------------------------------------
// host side

struct ApplyShape {
    int tz, nseg, nwaves, blocks;  // nwaves: work items (segment, chunk)
};

// Resident waves of a kernel (its occupancy times the CU count), queried once.
template <typename K>
int resident_waves(K kernel)
{
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, EL_BLOCK, 0) != hipSuccess ||
        hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        return 4096;
    }
    return std::max(1, per_cu) * std::max(1, cus) * EL_WAVES;
}

// Planes per work item: each item pays two warm-up planes and the grid holds at
// most the resident waves, which loop over the items; pick the chunk length that
// minimises (items per wave) x (planes + 2) (measured on MI355X: a grid just over
// one round of resident waves runs ~1.3x slower than one just under it).
ApplyShape apply_shape(const Grid& g, int slots)
{
    ApplyShape s{};
    s.nseg = (int)((g.P + EL_OUT - 1) / EL_OUT);
    int tz = 1;
    long long best = -1;
    for (int t = 2; t <= 64; ++t) {
        const long long items = (long long)s.nseg * ((g.nz + t - 1) / t);
        const long long cost = ((items + slots - 1) / slots) * (std::min(t, g.nz) + 2);
        if (best < 0 || cost < best) {
            best = cost;
            tz = t;
        }
    }
    if (pfk::tune_el_planes() > 0) tz = pfk::tune_el_planes();
    tz = std::min(tz, g.nz);
    while ((long long)s.nseg * ((g.nz + tz - 1) / tz) > (1ll << 30)) ++tz;  // item index fits an int
    s.tz = tz;
    const long long items = (long long)s.nseg * ((g.nz + tz - 1) / tz);
    s.nwaves = (int)items;
    const long long waves = std::min<long long>(items, slots);
    s.blocks = (int)((waves + EL_WAVES - 1) / EL_WAVES);
    return s;
}

template <typename T, int D, int MODE>
ApplyShape apply_shape_for(const Grid& g)
{
    static const int slots = resident_waves(k_el_apply<T, D, MODE>);
    return apply_shape(g, slots);
}

// y = K u in the given mode (see k_el_apply); b and omega for EL_RESID / EL_JACOBI
template <typename T>
void launch_apply_mode(int mode, const Grid& g, double lam, double mu, int ident, const T* u, T* y,
                       const CgArgs* cg, hipStream_t st, const T* b = nullptr, double omega = 0.0)
{
    const T scale = (T)(g.dim == 3 ? g.h : 1.0);
    CgArgs a = cg ? *cg : CgArgs{nullptr, nullptr};
    auto go = [&](auto kernel, const ApplyShape& s) {
        kernel<<<s.blocks, EL_BLOCK, 0, st>>>(g, (T)lam, (T)mu, scale, ident, u, y, s.tz, s.nseg, s.nwaves, a, b,
                                              (T)omega);
    };
#define EL_GO(DD, MM) go(k_el_apply<T, DD, MM>, apply_shape_for<T, DD, MM>(g))
    if (g.dim == 3) {
        if (mode == EL_CG) EL_GO(3, EL_CG);
        else if (mode == EL_RESID) EL_GO(3, EL_RESID);
        else if (mode == EL_JACOBI) EL_GO(3, EL_JACOBI);
        else if (mode == EL_JACOBI_DOT) EL_GO(3, EL_JACOBI_DOT);
        else EL_GO(3, EL_PLAIN);
    } else {
        if (mode == EL_CG) EL_GO(2, EL_CG);
        else if (mode == EL_RESID) EL_GO(2, EL_RESID);
        else if (mode == EL_JACOBI) EL_GO(2, EL_JACOBI);
        else if (mode == EL_JACOBI_DOT) EL_GO(2, EL_JACOBI_DOT);
        else EL_GO(2, EL_PLAIN);
    }
#undef EL_GO
}

template <typename T>
void launch_apply(const Grid& g, double lam, double mu, int ident, const T* u, T* y, const CgArgs* cg,
                  hipStream_t st)
{
    launch_apply_mode<T>(cg ? EL_CG : EL_PLAIN, g, lam, mu, ident, u, y, cg, st);
}

template <typename T>
ApplyShape cg_apply_shape(const Grid& g)
{
    return g.dim == 3 ? apply_shape_for<T, 3, EL_CG>(g) : apply_shape_for<T, 2, EL_CG>(g);
}

int stream_blocks(long long n)
{
    return (int)std::min<long long>(2048, std::max<long long>(1, (n + 4 * EL_BLOCK - 1) / (4 * EL_BLOCK)));
}

template <typename T>
void launch_rhs(const Grid& g, double coef, const pf_elastic* p, T* f, hipStream_t st)
{
    int n[3];
    n[0] = g.nx;
    n[1] = g.dim == 3 ? g.ny : g.nz;
    n[2] = g.dim == 3 ? g.nz : 1;
    if (g.dim == 3) {
        using RT = RhsTile<3>;
        const int tx = (n[0] + RT::TX - 1) / RT::TX, ty = (n[1] + RT::TY - 1) / RT::TY,
                  tz = (n[2] + RT::TZ - 1) / RT::TZ;
        k_el_rhs<T, 3><<<tx * ty * tz, EL_BLOCK, 0, st>>>(g, coef, p->m, p->a, p->l, f, tx, ty);
    } else {
        using RT = RhsTile<2>;
        const int tx = (n[0] + RT::TX - 1) / RT::TX, ty = (n[1] + RT::TY - 1) / RT::TY;
        k_el_rhs<T, 2><<<tx * ty, EL_BLOCK, 0, st>>>(g, coef, p->m, p->a, p->l, f, tx, ty);
    }
}

constexpr int DOT_BLOCKS = 1024;

template <typename T>
void launch_dot(const Grid& g, const T* gw, const T* u, double* part, double* out, hipStream_t st)
{
    const int blocks = (int)std::min<long long>(DOT_BLOCKS, (g.N + EL_BLOCK - 1) / EL_BLOCK);
    if (g.dim == 3)
        k_el_dot<T, 3><<<blocks, EL_BLOCK, 0, st>>>(g, gw, u, part);
    else
        k_el_dot<T, 2><<<blocks, EL_BLOCK, 0, st>>>(g, gw, u, part);
    k_el_sum<<<1, EL_BLOCK, 0, st>>>(part, blocks, out);
}

void lame(const pf_elastic* p, double* lam, double* mu)
{
    *lam = p->E * p->nu / ((1.0 + p->nu) * (1.0 - 2.0 * p->nu));
    *mu = p->E / (2.0 * (1.0 + p->nu));
}

int validate(const pf_elastic* p)
{
    using pfapi::fail;
    if (!p) return fail(PF_EINVAL, "elastic problem is NULL");
    if (p->dim != 2 && p->dim != 3) return fail(PF_EINVAL, "dim must be 2 or 3 (got %d)", p->dim);
    if (p->dtype != PF_F32 && p->dtype != PF_F64) return fail(PF_EINVAL, "unknown dtype %d", p->dtype);
    long long N = 1, P = 1;
    for (int k = 0; k < p->dim; ++k) {
        if (p->n[k] < 2) return fail(PF_EINVAL, "n[%d] = %lld must be >= 2", k, (long long)p->n[k]);
        if (p->n[k] > (1ll << 30)) return fail(PF_EINVAL, "n[%d] too large", k);
        N *= p->n[k];
        if (k < p->dim - 1) P *= p->n[k];
    }
    if (N * p->dim > (1ll << 38)) return fail(PF_EINVAL, "grid too large");
    if (P >= (1ll << 28)) return fail(PF_EINVAL, "an x-y plane (2-D: a row) holds too many nodes");
    if (!(p->h > 0.0) || !std::isfinite(p->h)) return fail(PF_EINVAL, "h must be finite and > 0");
    if (!(p->E > 0.0) || !std::isfinite(p->E)) return fail(PF_EINVAL, "E must be finite and > 0");
    if (!(p->nu > -1.0 && p->nu < 0.5)) return fail(PF_EINVAL, "nu must lie in (-1, 0.5)");
    if (!std::isfinite(p->m) || !std::isfinite(p->a) || !std::isfinite(p->l))
        return fail(PF_EINVAL, "m, a and l must be finite");
    return PF_OK;
}

long long ndof(const pf_elastic* p)
{
    long long N = 1;
    for (int k = 0; k < p->dim; ++k) N *= p->n[k];
    return N * p->dim;
}

size_t esz(const pf_elastic* p) { return p->dtype == PF_F64 ? 8 : 4; }

int check_vec(const void* v, const pf_elastic* p, const char* name)
{
    if (!v) return pfapi::fail(PF_EINVAL, "%s is NULL", name);
    if (reinterpret_cast<uintptr_t>(v) % 16)
        return pfapi::fail(PF_EINVAL, "%s must be 16-byte aligned", name);
    (void)p;
    return PF_OK;
}

struct Levels {
    int nl = 1;
    int coarse_sweeps = MG_COARSE_MIN;
    int bottom = 1;  // first level run by k_el_bottom (nl: none)
    Grid g[MG_MAXL];
    long long ndof[MG_MAXL];
};

// the grid hierarchy: halve every axis while all keep an odd node count >= 3
// (pf_tune_set(PF_TUNE_EL_MG, 1) keeps one level: plain CG)
Levels mg_levels(const pf_elastic* p)
{
    Levels L;
    L.g[0] = grid_of(p);
    L.ndof[0] = ndof(p);
    if (pfk::tune_el_mg() == 1) return L;
    pf_elastic q = *p;
    while (L.nl < MG_MAXL) {
        bool ok = true;
        for (int k = 0; k < p->dim; ++k) ok = ok && (q.n[k] - 1) % 2 == 0 && q.n[k] >= 5;
        if (!ok) break;
        for (int k = 0; k < p->dim; ++k) q.n[k] = (q.n[k] - 1) / 2 + 1;
        q.h *= 2.0;
        L.g[L.nl] = grid_of(&q);
        L.ndof[L.nl] = ndof(&q);
        ++L.nl;
    }
    long long longest = 0;
    for (int k = 0; k < p->dim; ++k) longest = std::max<long long>(longest, q.n[k]);
    L.coarse_sweeps = (int)std::min<long long>(MG_COARSE_MAX, std::max<long long>(MG_COARSE_MIN, 2 * longest));
    // the coarse end that fits one block's LDS (never the finest level: the PCG
    // takes its dot products from the finest level's last sweep)
    L.bottom = L.nl;
    const int tm = pfk::tune_el_mg();
    if (tm != 2) {
        const long long cap = tm >= 3 ? tm : (p->dim == 3 ? MG_BOTTOM_NODES_3D : MG_BOTTOM_NODES_2D);
        size_t bytes = 0;
        for (int l = L.nl - 1; l >= 1 && L.nl - l <= MG_BOTTOM_MAXL; --l) {
            bytes += 3 * (size_t)L.ndof[l] * esz(p);
            if (L.g[l].N > cap || bytes > MG_BOTTOM_LDS) break;
            L.bottom = l;
        }
    }
    return L;
}

// workspace: CG vectors r, p, s, w, then (sensitivity) lambda, g, t; partials; CG
// state; multigrid: a fine temporary and (x, b, t) on every coarser level
struct Ws {
    void* r;
    void* p;
    void* s;
    void* w;
    void* lam;
    void* g;
    void* t;
    double* part;
    double* scal;
    double* rpart;  // k_pcg_alpha's r.r partials
    void* mg[MG_MAXL][3];
    double* eig;  // power iteration: two vectors and the zero load on a 9^d grid, then a norm
};

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

size_t ws_bytes(const pf_elastic* p, Ws* out, void* base)
{
    const size_t vb = align256((size_t)ndof(p) * esz(p));
    char* b = (char*)base;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        void* q = b ? b + off : nullptr;
        off += align256(bytes);
        return q;
    };
    Ws w{};
    w.r = take(vb);
    w.p = take(vb);
    w.s = take(vb);
    w.w = take(vb);
    w.lam = take(vb);
    w.g = take(vb);
    w.t = take(vb);
    w.part = (double*)take(sizeof(double) * 2 * EL_MAX_PARTS);
    w.scal = (double*)take(sizeof(double) * (2 * S_SLOT + 8));
    const Levels Lv = mg_levels(p);
    if (Lv.nl > 1) {
        w.eig = (double*)take(sizeof(double) * (3 * 3 * MG_EIG_N * MG_EIG_N * MG_EIG_N + 8));
        w.rpart = (double*)take(sizeof(double) * EL_MAX_PARTS);
        w.mg[0][2] = take(vb);
        for (int l = 1; l < Lv.nl; ++l)
            for (int k = 0; k < 3; ++k) w.mg[l][k] = take(align256((size_t)Lv.ndof[l] * esz(p)));
    }
    if (out) *out = w;
    return off;
}

// The pinned mirror the CG kernels store their scalars into (owned by the
// context, made by pf_create) with its two events; this is a view of it.
struct HostMirror {
    double* host = nullptr;
    double* dev = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
};

HostMirror host_mirror(const pf_ctx* ctx)
{
    HostMirror m;
    m.host = ctx->cg.host;
    m.dev = ctx->cg.dev;
    m.ev[0] = ctx->cg.ev[0];
    m.ev[1] = ctx->cg.ev[1];
    return m;
}

// CG on K x = b (b already in W.r); x is overwritten.  Host-synchronous.
template <typename T>
int cg_solve(const pf_ctx* ctx, const pf_elastic* p, const Grid& g, T* x, const Ws& W, double rtol, int maxit,
             pf_el_report* rep, hipStream_t st)
{
    double lam, mu;
    lame(p, &lam, &mu);
    const HostMirror hmv = host_mirror(ctx);
    const HostMirror* hm = &hmv;
    const long long n = ndof(p);
    const int sb = stream_blocks(n);
    k_el_fill<T><<<sb, EL_BLOCK, 0, st>>>(n, x, nullptr);
    k_el_fill<T><<<sb, EL_BLOCK, 0, st>>>(n, (T*)W.p, nullptr);
    k_el_fill<T><<<sb, EL_BLOCK, 0, st>>>(n, (T*)W.s, nullptr);
    k_el_cg_init<<<1, 64, 0, st>>>(W.scal, hm->dev, rtol * rtol, (double)maxit);
    if (int rc = pfapi::check_launch("CG setup")) return rc;
    const ApplyShape shp = cg_apply_shape<T>(g);
    if (shp.blocks > EL_MAX_PARTS) return pfapi::fail(PF_EINVAL, "grid too large for the CG reduction");
    const int ub = std::min(sb, 1024);
    // enqueue batches of iterations; poll the previous batch while the next runs
    int batch = 8, enq = 0, slot = 0;
    bool pending = false;
    double done = 0.0, its = 0.0, gam = 0.0, gam0 = 0.0;
    for (;;) {
        const int nb = std::min(batch, maxit + 1 - enq);
        for (int i = 0; i < nb; ++i) {
            const int it = enq + i;
            double* sin = W.scal + S_SLOT * (it & 1);
            double* sout = W.scal + S_SLOT * ((it + 1) & 1);
            const CgArgs cg{W.part, sin};
            launch_apply<T>(g, lam, mu, 1, (const T*)W.r, (T*)W.w, &cg, st);
            k_el_cg_update<T><<<ub, EL_BLOCK, 0, st>>>(n, W.part, shp.blocks, sin, sout, hm->dev, x, (T*)W.r,
                                                       (T*)W.p, (T*)W.s, (const T*)W.w);
        }
        enq += nb;
        if (int rc = pfapi::check_launch("CG iteration")) return rc;
        if (hipEventRecord(hm->ev[slot], st) != hipSuccess) return pfapi::check_launch("CG event");
        if (pending) {
            if (hipEventSynchronize(hm->ev[slot ^ 1]) != hipSuccess) return pfapi::check_launch("CG wait");
            done = *(volatile double*)&hm->host[H_DONE];
            if (done != 0.0) break;
        }
        pending = true;
        slot ^= 1;
        if (enq > maxit) {
            if (hipEventSynchronize(hm->ev[slot ^ 1]) != hipSuccess) return pfapi::check_launch("CG wait");
            break;
        }
        batch = std::min(batch * 2, 64);
    }
    if (hipStreamSynchronize(st) != hipSuccess) return pfapi::check_launch("CG sync");
    done = *(volatile double*)&hm->host[H_DONE];
    its = *(volatile double*)&hm->host[H_ITS];
    gam = *(volatile double*)&hm->host[H_GAMMA];
    gam0 = *(volatile double*)&hm->host[H_GAMMA0];
    if (rep) {
        rep->iterations = (int32_t)its;
        rep->converged = done == DONE_CONVERGED;
        rep->status = (int32_t)done;
        rep->levels = 1;
        rep->res_norm = std::sqrt(std::max(gam, 0.0));
        rep->rhs_norm = std::sqrt(std::max(gam0, 0.0));
    }
    if (done == DONE_NONFINITE) return pfapi::fail(PF_ENONFINITE, "CG met a non-finite value");
    if (done != DONE_CONVERGED)
        return pfapi::fail(PF_ENOCONV, "CG stopped after %d iterations without reaching rtol (status %d)",
                           (int)its, (int)done);
    return PF_OK;
}

template <typename T>
void launch_restrict(const Grid& gf, const Grid& gc, const T* rf, T* rc, const double* st, hipStream_t s)
{
    const int nb = (int)((gc.N + EL_BLOCK - 1) / EL_BLOCK);
    if (gf.dim == 3)
        k_el_restrict<T, 3><<<nb, EL_BLOCK, 0, s>>>(gf, gc, rf, rc, st);
    else
        k_el_restrict<T, 2><<<nb, EL_BLOCK, 0, s>>>(gf, gc, rf, rc, st);
}

template <typename T>
void launch_prolong(const Grid& gc, const Grid& gf, const T* ec, T* xf, const double* st, hipStream_t s)
{
    const int nb = (int)((gf.N + EL_BLOCK - 1) / EL_BLOCK);
    if (gf.dim == 3)
        k_el_prolong<T, 3><<<nb, EL_BLOCK, 0, s>>>(gc, gf, ec, xf, st);
    else
        k_el_prolong<T, 2><<<nb, EL_BLOCK, 0, s>>>(gc, gf, ec, xf, st);
}

// x = V(b) on level l (x, t: this level's vectors): pre-smoothing from x = 0
// (its first sweep pointwise), residual, restriction, the coarser cycle,
// prolongation, post-smoothing; the coarsest level only smooths.  The cycle is
// a fixed symmetric operator.  part != nullptr: the last sweep also leaves the
// partial sums of x.b and b.b there.
template <typename T>
void launch_jacobi0(const Grid& g, double lam, double mu, const T* b, T* y, double omega, const double* st,
                    hipStream_t s)
{
    const int nb = (int)((g.N + EL_BLOCK - 1) / EL_BLOCK);
    const T scale = (T)(g.dim == 3 ? g.h : 1.0);
    if (g.dim == 3)
        k_el_jacobi0<T, 3><<<nb, EL_BLOCK, 0, s>>>(g, (T)lam, (T)mu, scale, b, y, (T)omega, st);
    else
        k_el_jacobi0<T, 2><<<nb, EL_BLOCK, 0, s>>>(g, (T)lam, (T)mu, scale, b, y, (T)omega, st);
}

// levels l .. nl-1 of the cycle in one block (k_el_bottom): b and x in global memory
template <typename T>
void launch_bottom(const Levels& Lv, int l0, const T* b, T* x, double lam, double mu, double omega,
                   const double* st, hipStream_t s)
{
    BottomArgs<T> a{};
    a.nl = Lv.nl - l0;
    a.coarse_sweeps = Lv.coarse_sweeps;
    a.lam = (T)lam;
    a.mu = (T)mu;
    a.omega = (T)omega;
    const int D = Lv.g[l0].dim;
    int off = 0;
    for (int k = 0; k < a.nl; ++k) {
        const Grid& g = Lv.g[l0 + k];
        a.n[k][0] = g.nx;
        a.n[k][1] = D == 3 ? g.ny : g.nz;
        a.n[k][2] = D == 3 ? g.nz : 1;
        a.N[k] = (int)g.N;
        a.off[k] = off;
        a.scale[k] = (T)(D == 3 ? g.h : 1.0);
        off += 3 * D * (int)g.N;
    }
    const size_t bytes = (size_t)off * sizeof(T);
    if (D == 3)
        k_el_bottom<T, 3><<<1, MG_BOTTOM_THREADS, bytes, s>>>(a, b, x, st);
    else
        k_el_bottom<T, 2><<<1, MG_BOTTOM_THREADS, bytes, s>>>(a, b, x, st);
}

template <typename T>
void vcycle(const Levels& Lv, int l, const T* b, T* x, T* t, const Ws& W, double lam, double mu, double omega,
            const double* st, double* part, hipStream_t s)
{
    const Grid& g = Lv.g[l];
    if (l == Lv.bottom && part == nullptr) {
        launch_bottom<T>(Lv, l, b, x, lam, mu, omega, st, s);
        return;
    }
    const CgArgs ca{nullptr, st}, cd{part, st};
    const bool coarsest = l == Lv.nl - 1;
    // sweeps alternate between the two vectors; an odd count moves the result
    auto sweeps = [&](T* cur, T* oth, int m, bool dot_last) {
        for (int i = 0; i < m; ++i) {
            const bool dot = dot_last && i == m - 1;
            launch_apply_mode<T>(dot ? EL_JACOBI_DOT : EL_JACOBI, g, lam, mu, 1, cur, oth, dot ? &cd : &ca, s, b,
                                 omega);
            std::swap(cur, oth);
        }
    };
    const int pre = coarsest ? Lv.coarse_sweeps : MG_PRE;  // even: x0 -> t, then an odd count back to x
    launch_jacobi0<T>(g, lam, mu, b, t, omega, st, s);
    sweeps(t, x, pre - 1, coarsest && part);
    if (coarsest) return;
    launch_apply_mode<T>(EL_RESID, g, lam, mu, 1, x, t, &ca, s, b);
    T* xc = (T*)W.mg[l + 1][0];
    T* bc = (T*)W.mg[l + 1][1];
    T* tc = (T*)W.mg[l + 1][2];
    launch_restrict<T>(g, Lv.g[l + 1], t, bc, st, s);
    vcycle<T>(Lv, l + 1, bc, xc, tc, W, lam, mu, omega, st, nullptr, s);
    launch_prolong<T>(Lv.g[l + 1], g, xc, x, st, s);
    sweeps(x, t, MG_POST, part != nullptr);
}

// lambda_max(D^-1 K) for this dimension and nu: power iteration on I + D^-1 K
// (the Jacobi-mode operator with omega = -1 and a zero load) on a 9^d grid in
// FP64, through the same operator kernel; cached per (dim, nu) in the context.
int jacobi_lmax(pf_ctx* ctx, const pf_elastic* p, const Ws& W, hipStream_t st, double* out)
{
    const std::pair<int, double> key(p->dim, p->nu);
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        auto it = ctx->el_lmax.find(key);
        if (it != ctx->el_lmax.end()) {
            *out = it->second;
            return PF_OK;
        }
    }
    pf_elastic q = *p;
    for (int k = 0; k < 3; ++k) q.n[k] = k < p->dim ? MG_EIG_N : 1;
    q.h = 1.0;
    q.dtype = PF_F64;
    const Grid g = grid_of(&q);
    double lam, mu;
    lame(&q, &lam, &mu);
    const long long n = ndof(&q);
    double* v = W.eig;
    double* w = v + n;
    double* zero = w + n;
    double* nrm = zero + n;
    k_el_seed<<<1, EL_BLOCK, 0, st>>>(n, v);
    k_el_fill<double><<<1, EL_BLOCK, 0, st>>>(n, zero, nullptr);
    k_el_normalize<<<1, EL_BLOCK, 0, st>>>(n, v, nrm);
    for (int i = 0; i < MG_POWER; ++i) {
        launch_apply_mode<double>(EL_JACOBI, g, lam, mu, 1, v, w, nullptr, st, zero, -1.0);
        k_el_normalize<<<1, EL_BLOCK, 0, st>>>(n, w, nrm);
        std::swap(v, w);
    }
    double h = 0.0;
    if (hipMemcpyAsync(&h, nrm, sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return pfapi::check_launch("smoother eigenvalue estimate");
    const double lmax = h - 1.0;
    if (!(std::isfinite(lmax) && lmax > 0.5))
        return pfapi::fail(PF_ENONFINITE, "smoother eigenvalue estimate failed (%g)", lmax);
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->el_lmax[key] = lmax;
    *out = lmax;
    return PF_OK;
}

// Preconditioned CG (multigrid V-cycle) on K x = b (b already in W.r); x is
// overwritten.  Per iteration: z = V(r) (its last sweep also sums z.r and
// ||r||^2 for the stop test); p = z + beta p; q = K p with p.q; x += alpha p,
// r -= alpha q.  Scalars
// stay on the device; the host polls a pinned mirror.  Host-synchronous.
template <typename T>
int pcg_solve(pf_ctx* ctx, const pf_elastic* p, const Levels& Lv, T* x, const Ws& W, double rtol, int maxit,
              pf_el_report* rep, hipStream_t st)
{
    double lam, mu;
    lame(p, &lam, &mu);
    const HostMirror hmv = host_mirror(ctx);
    const HostMirror* hm = &hmv;
    const Grid& g = Lv.g[0];
    const long long n = Lv.ndof[0];
    const int sb = stream_blocks(n);
    double* S = W.scal;
    double lmax = 0.0;
    if (int rc = jacobi_lmax(ctx, p, W, st, &lmax)) return rc;
    const double omega = MG_SMOOTH / lmax;
    k_el_fill<T><<<sb, EL_BLOCK, 0, st>>>(n, x, nullptr);
    k_el_fill<T><<<sb, EL_BLOCK, 0, st>>>(n, (T*)W.p, nullptr);
    k_pcg_init<<<1, 64, 0, st>>>(S, hm->dev, rtol * rtol, (double)maxit);
    if (int rc = pfapi::check_launch("PCG setup")) return rc;
    const ApplyShape shp = cg_apply_shape<T>(g);
    const int jparts = g.dim == 3 ? apply_shape_for<T, 3, EL_JACOBI_DOT>(g).blocks
                                  : apply_shape_for<T, 2, EL_JACOBI_DOT>(g).blocks;
    if (shp.blocks > EL_MAX_PARTS || jparts > EL_MAX_PARTS)
        return pfapi::fail(PF_EINVAL, "grid too large for the CG reduction");
    const int db = std::min(sb, 1024);
    // one iteration per poll: the host enqueues iteration k + 1 while k runs and
    // reads k - 1's state, so at most one iteration is enqueued past convergence
    const int batch = 1;
    int enq = 0, slot = 0;
    bool pending = false;
    double done = 0.0;
    for (;;) {
        const int nb = std::min(batch, maxit + 1 - enq);
        for (int i = 0; i < nb; ++i) {
            vcycle<T>(Lv, 0, (const T*)W.r, (T*)W.s, (T*)W.mg[0][2], W, lam, mu, omega, S, W.part, st);
            k_pcg_rho<T><<<db, EL_BLOCK, 0, st>>>(n, W.part, jparts, S, hm->dev, (const T*)W.s, (T*)W.p);
            const CgArgs cg{W.part, S};
            launch_apply<T>(g, lam, mu, 1, (const T*)W.p, (T*)W.w, &cg, st);
            k_pcg_alpha<T><<<db, EL_BLOCK, 0, st>>>(n, W.part, shp.blocks, S, hm->dev, x, (T*)W.r,
                                                   (const T*)W.p, (const T*)W.w, W.rpart);
            k_pcg_check<<<1, EL_BLOCK, 0, st>>>(W.rpart, db, S, hm->dev);
        }
        enq += nb;
        if (int rc = pfapi::check_launch("PCG iteration")) return rc;
        if (hipEventRecord(hm->ev[slot], st) != hipSuccess) return pfapi::check_launch("PCG event");
        if (pending) {
            if (hipEventSynchronize(hm->ev[slot ^ 1]) != hipSuccess) return pfapi::check_launch("PCG wait");
            done = *(volatile double*)&hm->host[H_DONE];
            if (done != 0.0) break;
        }
        pending = true;
        slot ^= 1;
        if (enq > maxit) {
            if (hipEventSynchronize(hm->ev[slot ^ 1]) != hipSuccess) return pfapi::check_launch("PCG wait");
            break;
        }
    }
    if (hipStreamSynchronize(st) != hipSuccess) return pfapi::check_launch("PCG sync");
    done = *(volatile double*)&hm->host[H_DONE];
    const double its = *(volatile double*)&hm->host[H_ITS];
    const double gam = *(volatile double*)&hm->host[H_GAMMA];
    const double gam0 = *(volatile double*)&hm->host[H_GAMMA0];
    if (rep) {
        rep->iterations = (int32_t)its;
        rep->converged = done == DONE_CONVERGED;
        rep->status = (int32_t)done;
        rep->levels = Lv.nl;
        rep->res_norm = std::sqrt(std::max(gam, 0.0));
        rep->rhs_norm = std::sqrt(std::max(gam0, 0.0));
    }
    if (done == DONE_NONFINITE) return pfapi::fail(PF_ENONFINITE, "PCG met a non-finite value");
    if (done != DONE_CONVERGED)
        return pfapi::fail(PF_ENOCONV, "PCG stopped after %d iterations without reaching rtol (status %d)",
                           (int)its, (int)done);
    return PF_OK;
}

// the solver for K x = b (b in W.r): multigrid-preconditioned CG when the grid
// coarsens, else plain CG
template <typename T>
int el_solve_any(pf_ctx* ctx, const pf_elastic* p, const Grid& g, T* x, const Ws& W, double rtol, int maxit,
                 pf_el_report* rep, hipStream_t st)
{
    const Levels Lv = mg_levels(p);
    if (Lv.nl > 1) return pcg_solve<T>(ctx, p, Lv, x, W, rtol, maxit, rep, st);
    return cg_solve<T>(ctx, p, g, x, W, rtol, maxit, rep, st);
}

template <typename T>
int solve_t(pf_ctx* ctx, const pf_elastic* p, const void* b, void* u, double rtol, int maxit, pf_el_report* rep,
            const Ws& W, hipStream_t st)
{
    const Grid g = grid_of(p);
    double lam, mu;
    lame(p, &lam, &mu);
    const long long n = ndof(p);
    if (b)
        k_el_fill<T><<<stream_blocks(n), EL_BLOCK, 0, st>>>(n, (T*)W.r, (const T*)b);
    else
        launch_rhs<T>(g, p->dim * lam + 2.0 * mu, p, (T*)W.r, st);
    return el_solve_any<T>(ctx, p, g, (T*)u, W, rtol, maxit, rep, st);
}

// Sensitivities of O = g . u with respect to (E, nu) at the equilibrium u:
// adjoint K lam_a = g (K is symmetric), then with K = lam K_l + mu K_m and
// f = (d lam + 2 mu) f1 (f1: the load for unit coefficient)
//   dO/dlam = lam_a . (d f1 - K_l u),   dO/dmu = lam_a . (2 f1 - K_m u),
// mapped to (E, nu) by the chain rule.
template <typename T>
int sensitivity_t(pf_ctx* ctx, const pf_elastic* p, const void* gw, const void* u, double* out, double rtol,
                  int maxit, pf_el_report* rep, const Ws& W, hipStream_t st)
{
    const Grid g = grid_of(p);
    const long long n = ndof(p);
    const int bl = (int)((g.N + EL_BLOCK - 1) / EL_BLOCK);
    if (g.dim == 3)
        k_el_weights<T, 3><<<bl, EL_BLOCK, 0, st>>>(g, (const T*)gw, (T*)W.g);
    else
        k_el_weights<T, 2><<<bl, EL_BLOCK, 0, st>>>(g, (const T*)gw, (T*)W.g);
    k_el_fill<T><<<stream_blocks(n), EL_BLOCK, 0, st>>>(n, (T*)W.r, (const T*)W.g);
    if (int rc = pfapi::check_launch("adjoint set-up")) return rc;
    if (int rc = el_solve_any<T>(ctx, p, g, (T*)W.lam, W, rtol, maxit, rep, st)) return rc;
    double* dots = W.scal + 2 * S_SLOT;  // 4 device doubles after the CG state
    double* part = W.part;
    launch_dot<T>(g, (const T*)W.g, (const T*)u, part, dots + 0, st);
    launch_rhs<T>(g, 1.0, p, (T*)W.t, st);
    launch_dot<T>(g, (const T*)W.lam, (const T*)W.t, part, dots + 1, st);
    launch_apply<T>(g, 1.0, 0.0, 0, (const T*)u, (T*)W.t, nullptr, st);
    launch_dot<T>(g, (const T*)W.lam, (const T*)W.t, part, dots + 2, st);
    launch_apply<T>(g, 0.0, 1.0, 0, (const T*)u, (T*)W.t, nullptr, st);
    launch_dot<T>(g, (const T*)W.lam, (const T*)W.t, part, dots + 3, st);
    if (int rc = pfapi::check_launch("sensitivity")) return rc;
    double h[4];
    if (hipMemcpyAsync(h, dots, sizeof h, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return pfapi::check_launch("sensitivity readback");
    const double d = p->dim, E = p->E, nu = p->nu;
    const double dl = d * h[1] - h[2], dm = 2.0 * h[1] - h[3];
    const double D = (1.0 + nu) * (1.0 - 2.0 * nu);
    out[0] = h[0];
    out[1] = dl * (nu / D) + dm * (1.0 / (2.0 * (1.0 + nu)));
    out[2] = dl * (E * (1.0 + 2.0 * nu * nu) / (D * D)) + dm * (-E / (2.0 * (1.0 + nu) * (1.0 + nu)));
    return PF_OK;
}

}  // namespace pfel

using namespace pfel;
using pfapi::fail;

namespace pfapi {
size_t elastic_pinned_doubles() { return 64; }
}  // namespace pfapi

extern "C" {

int pf_el_workspace_size(const pf_ctx* ctx, const pf_elastic* p, size_t* bytes)
{
    return pfapi::guarded("pf_el_workspace_size", [&]() -> int {
        if (int rc = pfapi::check_ctx(ctx)) return rc;
        if (int rc = pfel::validate(p)) return rc;
        if (!bytes) return fail(PF_EINVAL, "bytes is NULL");
        *bytes = ws_bytes(p, nullptr, nullptr);
        return PF_OK;
    });
}

int pf_el_apply(pf_ctx* ctx, const pf_elastic* p, const void* u, void* y, void* stream)
{
    return pfapi::guarded("pf_el_apply", [&]() -> int {
        if (int rc = pfapi::check_ctx(ctx)) return rc;
        if (int rc = pfel::validate(p)) return rc;
        if (int rc = check_vec(u, p, "u")) return rc;
        if (int rc = check_vec(y, p, "y")) return rc;
        if (u == y) return fail(PF_EINVAL, "u and y must not alias");
        if (int rc = pfapi::require_device(ctx)) return rc;
        const Grid g = grid_of(p);
        double lam, mu;
        lame(p, &lam, &mu);
        hipStream_t st = (hipStream_t)stream;
        if (p->dtype == PF_F32)
            launch_apply<float>(g, lam, mu, 1, (const float*)u, (float*)y, nullptr, st);
        else
            launch_apply<double>(g, lam, mu, 1, (const double*)u, (double*)y, nullptr, st);
        return pfapi::check_launch("pf_el_apply");
    });
}

int pf_el_rhs(pf_ctx* ctx, const pf_elastic* p, void* f, void* stream)
{
    return pfapi::guarded("pf_el_rhs", [&]() -> int {
        if (int rc = pfapi::check_ctx(ctx)) return rc;
        if (int rc = pfel::validate(p)) return rc;
        if (int rc = check_vec(f, p, "f")) return rc;
        if (int rc = pfapi::require_device(ctx)) return rc;
        const Grid g = grid_of(p);
        double lam, mu;
        lame(p, &lam, &mu);
        hipStream_t st = (hipStream_t)stream;
        if (p->dtype == PF_F32)
            launch_rhs<float>(g, p->dim * lam + 2.0 * mu, p, (float*)f, st);
        else
            launch_rhs<double>(g, p->dim * lam + 2.0 * mu, p, (double*)f, st);
        return pfapi::check_launch("pf_el_rhs");
    });
}

int pf_el_solve(pf_ctx* ctx, const pf_elastic* p, const void* b, void* u, double rtol, int32_t maxit,
                pf_el_report* rep, void* ws, void* stream)
{
    return pfapi::guarded("pf_el_solve", [&]() -> int {
        if (int rc = pfapi::check_ctx(ctx)) return rc;
        if (int rc = pfel::validate(p)) return rc;
        if (b)
            if (int rc = check_vec(b, p, "b")) return rc;
        if (int rc = check_vec(u, p, "u")) return rc;
        if (!ws || reinterpret_cast<uintptr_t>(ws) % 256) return fail(PF_EINVAL, "ws is NULL or not 256-byte aligned");
        if (!(rtol > 0.0) || !std::isfinite(rtol)) return fail(PF_EINVAL, "rtol must be finite and > 0");
        if (maxit < 1) return fail(PF_EINVAL, "maxit must be >= 1");
        if (b == u) return fail(PF_EINVAL, "b and u must not alias");
        if (int rc = pfapi::require_device(ctx)) return rc;
        Ws W;
        ws_bytes(p, &W, ws);
        hipStream_t st = (hipStream_t)stream;
        if (p->dtype == PF_F32) return solve_t<float>(ctx, p, b, u, rtol, maxit, rep, W, st);
        return solve_t<double>(ctx, p, b, u, rtol, maxit, rep, W, st);
    });
}

int pf_el_objective(pf_ctx* ctx, const pf_elastic* p, const void* gw, const void* u, double* out, void* ws,
                    void* stream)
{
    return pfapi::guarded("pf_el_objective", [&]() -> int {
        if (int rc = pfapi::check_ctx(ctx)) return rc;
        if (int rc = pfel::validate(p)) return rc;
        if (gw)
            if (int rc = check_vec(gw, p, "g")) return rc;
        if (int rc = check_vec(u, p, "u")) return rc;
        if (!out || reinterpret_cast<uintptr_t>(out) % 8) return fail(PF_EINVAL, "out is NULL or misaligned");
        if (!ws || reinterpret_cast<uintptr_t>(ws) % 256) return fail(PF_EINVAL, "ws is NULL or not 256-byte aligned");
        if (int rc = pfapi::require_device(ctx)) return rc;
        Ws W;
        ws_bytes(p, &W, ws);
        const Grid g = grid_of(p);
        hipStream_t st = (hipStream_t)stream;
        if (p->dtype == PF_F32)
            launch_dot<float>(g, (const float*)gw, (const float*)u, W.part, out, st);
        else
            launch_dot<double>(g, (const double*)gw, (const double*)u, W.part, out, st);
        return pfapi::check_launch("pf_el_objective");
    });
}

int pf_el_sensitivity(pf_ctx* ctx, const pf_elastic* p, const void* gw, const void* u, double* out, double rtol,
                      int32_t maxit, pf_el_report* rep, void* ws, void* stream)
{
    return pfapi::guarded("pf_el_sensitivity", [&]() -> int {
        if (int rc = pfapi::check_ctx(ctx)) return rc;
        if (int rc = pfel::validate(p)) return rc;
        if (gw)
            if (int rc = check_vec(gw, p, "g")) return rc;
        if (int rc = check_vec(u, p, "u")) return rc;
        if (!out) return fail(PF_EINVAL, "out is NULL");
        if (!ws || reinterpret_cast<uintptr_t>(ws) % 256) return fail(PF_EINVAL, "ws is NULL or not 256-byte aligned");
        if (!(rtol > 0.0) || !std::isfinite(rtol)) return fail(PF_EINVAL, "rtol must be finite and > 0");
        if (maxit < 1) return fail(PF_EINVAL, "maxit must be >= 1");
        if (int rc = pfapi::require_device(ctx)) return rc;
        Ws W;
        ws_bytes(p, &W, ws);
        hipStream_t st = (hipStream_t)stream;
        if (p->dtype == PF_F32) return sensitivity_t<float>(ctx, p, gw, u, out, rtol, maxit, rep, W, st);
        return sensitivity_t<double>(ctx, p, gw, u, out, rtol, maxit, rep, W, st);
    });
}

}  // extern "C"
