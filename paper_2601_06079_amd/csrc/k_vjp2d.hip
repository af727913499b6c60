// k_vjp2d.hip -- adjoint of the Allen-Cahn explicit step (Eq. 12) for ragged
// batches of 2-D periodic grids, streamed row by row like the forward kernel
// (one 64-lane wavefront per strip of columns, DPP for x-neighbours, a register
// window for y-neighbours, both fields prefetched PF rows ahead).  The work
// items are those of the forward plan: a strip of a plan built for ks fused
// steps outputs its 64 - 2 ks columns (the adjoint itself needs one halo lane).
//
// One step is eta' = eta - (dt L / m) r(eta), r = N(eta) + kappa K eta, with
// N(eta)_i = sum over the node's elements and quadrature points of
// |J| f'(eta_q) phi_i(q).  The Jacobian of r is symmetric, so the adjoint maps
// the sensitivity lam' of eta' to
//   lam_i = lam'_i - (dt L / m) [ |J| sum_q f''(eta_q) lam'_q phi_i(q) + kappa (K lam')_i ]
// (Supp. Note 2, Eqs. II.5-II.6 for one step).  The step's parameter
// sensitivities lam'^T d(eta')/d(L, kappa, W) need only two sums per sample:
// sum_i lam'_i N(eta)_i equals the quadrature of f'(eta_q) lam'_q (lam'_q the
// interpolated adjoint), and sum_i lam'_i (K eta)_i is a dot product, which K's
// symmetry on the periodic grid turns into sum_i eta_i (K lam')_i -- and K lam' the
// step needs anyway -- so with
//   A = sum_q f'_1(eta_q) lam'_q          (f'_1: f' at W = 1)
//   B = sum_i eta_i (9 lam'_i - box3x3(lam')_i)      (= 3 eta^T K lam' = 3 lam'^T K eta)
// the gradient contributions are
//   dL     = -(dt/m) (W |J| A + kappa B / 3)
//   dkappa = -(dt/m) L B / 3
//   dW     = -(dt/m) L |J| A.
// A lane sums its terms down the chunk in the field's precision; the wave sums
// them in FP64 and each work item (sample, strip, chunk) adds its A and B to its
// own FP64 slot, so successive launches accumulate a whole trajectory in a fixed
// order without atomics; one reduction per sample turns the slots into gradients.
#include "device.hpp"
#include "kernels.hpp"
#include "stream2d.hpp"

namespace pfk {
namespace {

template <typename T>
struct VjpCoef {
    T b0, b1, b2;  // f''(q) = b0 + b1 q + b2 q^2 with dt L |J| / m folded in
    T a1, a2, a3;  // f'_1(q) = q (a1 + a2 q + a3 q^2), W = 1
    T beta;        // dt L kappa / (3 m)
};

// push(eta_r, lam'_r) takes row r and returns lam of row r - 1.  a: the 4
// quadrature points of this lane's element (x, x+1) x (r-1, r), summed
// f'_1(eta_q) lam'_q; b: eta(x, r-1) (9 lam' - box lam')(x, r-1).  SYM: the
// symmetric double well (f'' = b0 + b2 q^2, f'_1 = q (a1 + a3 q^2)), whose two
// polynomials share q^2.
template <typename T, bool SYM>
struct VjpStage {
    T l_m1 = 0, e_m1 = 0;          // lam', eta at row r-1
    T s3l_m1 = 0, s3l_m2 = 0;      // 3-point x-sums of lam' at rows r-1, r-2
    T exl_m1 = 0, exr_m1 = 0;      // x-interpolated eta of row r-1
    T lxl_m1 = 0, lxr_m1 = 0;      // x-interpolated lam' of row r-1
    T guL_m1 = 0, guR_m1 = 0;      // upward scatter of element row (r-2, r-1)

    __device__ __forceinline__ T push(T ec, T lc, const VjpCoef<T>& k, T& a, T& b)
    {
        const T gp = (T)GP, gm = (T)GM;
        const T er = from_right(ec);
        const T ll = from_left(lc), lr = from_right(lc);
        const T s3l = ll + lc + lr;
        const T de = er - ec, dl = lr - lc;
        const T exl = fmaT(gm, de, ec), exr = fmaT(gp, de, ec);
        const T lxl = fmaT(gm, dl, lc), lxr = fmaT(gp, dl, lc);
        const T e0 = exl - exl_m1, e1 = exr - exr_m1;
        const T f0 = lxl - lxl_m1, f1 = lxr - lxr_m1;
        // quadrature points: left/right column point, lower (0) / upper (1) row point
        const T qL0 = fmaT(gm, e0, exl_m1), qL1 = fmaT(gp, e0, exl_m1);
        const T qR0 = fmaT(gm, e1, exr_m1), qR1 = fmaT(gp, e1, exr_m1);
        const T pL0 = fmaT(gm, f0, lxl_m1), pL1 = fmaT(gp, f0, lxl_m1);
        const T pR0 = fmaT(gm, f1, lxr_m1), pR1 = fmaT(gp, f1, lxr_m1);
        T PL0, PL1, PR0, PR1;
        if constexpr (SYM) {
            const T sL0 = qL0 * qL0, sL1 = qL1 * qL1, sR0 = qR0 * qR0, sR1 = qR1 * qR1;
            PL0 = fmaT(k.b2, sL0, k.b0) * pL0;
            PL1 = fmaT(k.b2, sL1, k.b0) * pL1;
            PR0 = fmaT(k.b2, sR0, k.b0) * pR0;
            PR1 = fmaT(k.b2, sR1, k.b0) * pR1;
            T s = fmaT(k.a3, sL0, k.a1) * (qL0 * pL0);
            s = fmaT(fmaT(k.a3, sL1, k.a1), qL1 * pL1, s);
            s = fmaT(fmaT(k.a3, sR0, k.a1), qR0 * pR0, s);
            a = fmaT(fmaT(k.a3, sR1, k.a1), qR1 * pR1, s);
        } else {
            PL0 = fmaT(fmaT(k.b2, qL0, k.b1), qL0, k.b0) * pL0;
            PL1 = fmaT(fmaT(k.b2, qL1, k.b1), qL1, k.b0) * pL1;
            PR0 = fmaT(fmaT(k.b2, qR0, k.b1), qR0, k.b0) * pR0;
            PR1 = fmaT(fmaT(k.b2, qR1, k.b1), qR1, k.b0) * pR1;
            T s = cubic(qL0, k.a1, k.a2, k.a3) * pL0;
            s = fmaT(cubic(qL1, k.a1, k.a2, k.a3), pL1, s);
            s = fmaT(cubic(qR0, k.a1, k.a2, k.a3), pR0, s);
            a = fmaT(cubic(qR1, k.a1, k.a2, k.a3), pR1, s);
        }
        // scatter of f'' lam' to the nodes, as the forward scatters f'
        const T dL = PL0 - PL1, dR = PR0 - PR1;
        const T gdL = fmaT(gp, dL, PL1), guL = fmaT(gm, dL, PL1);
        const T gdR = fmaT(gp, dR, PR1), guR = fmaT(gm, dR, PR1);
        const T HL = guL_m1 + gdL, HR = guR_m1 + gdR;  // node row r-1 complete
        const T dH = HL - HR;
        const T pl = fmaT(gp, dH, HR), pr = fmaT(gm, dH, HR);
        const T N2 = pl + from_left(pr);
        const T lapl = fmaT((T)9, l_m1, -(s3l_m2 + s3l_m1 + s3l));
        const T out = l_m1 - N2 - k.beta * lapl;
        b = e_m1 * lapl;
        l_m1 = lc;
        e_m1 = ec;
        s3l_m2 = s3l_m1;
        s3l_m1 = s3l;
        exl_m1 = exl;
        exr_m1 = exr;
        lxl_m1 = lxl;
        lxr_m1 = lxr;
        guL_m1 = guL;
        guR_m1 = guR;
        return out;
    }
};

// 1 or 0 from a wave-uniform condition, selected in a scalar register
template <typename T>
__device__ __forceinline__ T unit_if(bool c);
template <>
__device__ __forceinline__ float unit_if<float>(bool c)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(c ? 0x3f800000 : 0));
}
template <>
__device__ __forceinline__ double unit_if<double>(bool c)
{
    return __hiloint2double(__builtin_amdgcn_readfirstlane(c ? 0x3ff00000 : 0), 0);
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
    return v;
}

// One work item of KS (1 or 2) adjoint steps: lam over the chunk's rows of the
// strip, and this wave's (A, B) summed over the KS steps.  With KS = 2 the
// first stage maps (eta_hi, lam_in) = (eta_k, lam_{k+1}) to lam_k row by row
// and the second maps (eta_lo, lam_k) = (eta_{k-1}, lam_k) to lam_{k-1}, one
// row behind, so lam_k never leaves registers (temporal blocking in reverse).
// hk: the plan's strip halo (its strips output 64 - 2 hk columns; hk >= KS).
// Must be called by a whole wave with wave-uniform arguments.
template <typename T, int PF, int KS, bool SYM>
__device__ __forceinline__ void vjp_item(const T* __restrict__ eta_hi, const T* __restrict__ eta_lo,
                                         const T* __restrict__ lam_in, T* __restrict__ lam_out,
                                         int nx, int ny, int strip, int chunk, int ty, int hk,
                                         unsigned bytes, const VjpCoef<T>& k, double& A, double& B)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int xl = strip * (WAVE - 2 * hk) - hk + lane;
    int x = xl % nx;
    if (x < 0) x += nx;
    const bool out_lane = lane >= hk && lane < WAVE - hk && xl < nx;
    const int y0 = chunk * ty;
    const int y1 = min(y0 + ty, ny);
    const int iters = (y1 - y0) + 2 * KS;  // rows y0-KS .. y1+KS-1
    const int rowb = nx * (int)sizeof(T);
    const int vx = x * (int)sizeof(T);
    const auto rh = make_rsrc(eta_hi, bytes);
    const auto rlo = make_rsrc(KS == 2 ? eta_lo : eta_hi, bytes);
    const auto rl = make_rsrc(lam_in, bytes);
    const auto ro = make_rsrc(lam_out, bytes);
    VjpStage<T, SYM> st[KS];
    T ringh[PF], ringl[PF], ringo[PF];
    int row = y0 - KS;
    while (row < 0) row += ny;
#pragma unroll
    for (int u = 0; u < PF; ++u) {
        ringh[u] = u < iters ? bload<T>(rh, vx, row * rowb) : (T)0;
        ringl[u] = u < iters ? bload<T>(rl, vx, row * rowb) : (T)0;
        if constexpr (KS == 2) ringo[u] = u < iters ? bload<T>(rlo, vx, row * rowb) : (T)0;
        if (++row == ny) row = 0;
    }
    int rlast = y1 + KS - 1;
    while (rlast >= ny) rlast -= ny;
    T elo_prev = 0;  // eta_lo of the row before the current one (KS = 2)
    // the lane's sums down the chunk in the field's precision (FP64 from the
    // wave sum on); rows outside the chunk enter with a wave-uniform weight 0
    T accA = 0, accB = 0;
    for (int t0 = 0; t0 < iters; t0 += PF) {
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const int t = t0 + u;
            const T vh = ringh[u], vl = ringl[u];
            T vo = 0;
            // unconditional prefetch (past the chunk the last row is re-read)
            ringh[u] = bload<T>(rh, vx, row * rowb);
            ringl[u] = bload<T>(rl, vx, row * rowb);
            if constexpr (KS == 2) {
                vo = ringo[u];
                ringo[u] = bload<T>(rlo, vx, row * rowb);
            }
            if (t + PF + 1 < iters) {
                if (++row == ny) row = 0;
            } else {
                row = rlast;
            }
            // stage 0 finishes row y0 - KS - 1 + t (and the element row above it)
            T a, b;
            T v = st[0].push(vh, vl, k, a, b);
            const T w0 = unit_if<T>(t >= KS + 1 && t < (y1 - y0) + KS + 1);
            accA = fmaT(w0, a, accA);
            accB = fmaT(w0, b, accB);
            if constexpr (KS == 2) {
                // stage 1 finishes row y0 - 4 + t from lam_k of row y0 - 3 + t
                v = st[1].push(elo_prev, v, k, a, b);
                elo_prev = vo;
                const T w1 = unit_if<T>(t >= 4 && t < iters);
                accA = fmaT(w1, a, accA);
                accB = fmaT(w1, b, accB);
            }
            if (t >= 2 * KS && t < iters && out_lane) bstore(v, ro, vx, (y0 - 2 * KS + t) * rowb);
        }
    }
    A = out_lane ? (double)accA : 0.0;
    B = out_lane ? (double)accB : 0.0;
}

// The two-step FP32 kernel holds about 100 VGPRs when the compiler is free to
// choose; capped at 96 it runs five waves per SIMD instead of four and the
// adjoint step takes 8% less time.  The symmetric-well variant then spills three
// values, one of which is stored and reloaded once per two rows.
template <typename T, int PF, int KS, bool SYM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(KS == 2 && sizeof(T) == 4 ? 5 : 1)))
void k_vjp2d_batched(const T* __restrict__ eta_hi, const T* __restrict__ eta_lo, const T* __restrict__ lam_in,
                     T* __restrict__ lam_out, const BatchSample* __restrict__ smp,
                     const BatchItem* __restrict__ items, int n_items, int ty, int hk, double* __restrict__ part)
{
    const int wave = uniform_wave();
    if (wave >= n_items) return;
    const BatchItem it = items[wave];
    const BatchSample& sm = smp[it.sample];
    const double m = sm.h * sm.h, detJ = 0.25 * sm.h * sm.h, sc = sm.dt * sm.mob * detJ / m;
    const FreeEnergy fw = make_free_energy(sm.fe, sm.W), f1 = make_free_energy(sm.fe, 1.0);
    const VjpCoef<T> k{(T)(sc * fw.b0), (T)(sc * fw.b1), (T)(sc * fw.b2), (T)f1.a1, (T)f1.a2,
                       (T)f1.a3, (T)(sm.dt * sm.mob * sm.kappa / (3.0 * m))};
    const unsigned bytes = (unsigned)((long long)sm.nx * sm.ny * (long long)sizeof(T));
    double A, B;
    vjp_item<T, PF, KS, SYM>(eta_hi + sm.offset, eta_lo + sm.offset, lam_in + sm.offset,
                        lam_out + sm.offset, sm.nx, sm.ny, it.strip, it.chunk, ty, hk, bytes, k, A, B);
    A = wave_sum(A);
    B = wave_sum(B);
    if ((threadIdx.x & (WAVE - 1)) == 0) {
        part[2 * (long long)wave] += A;
        part[2 * (long long)wave + 1] += B;
    }
}

// theta_bar[s] += gradient of the sample's accumulated (A, B), slots summed in
// item order by a fixed-shape tree (bitwise reproducible)
constexpr int RB = 256;
__global__ __launch_bounds__(RB) void k_vjp2d_reduce(const double* __restrict__ part,
                                                     const BatchSample* __restrict__ smp, int ty,
                                                     double* __restrict__ theta_bar)
{
    const BatchSample& sm = smp[blockIdx.x];
    const int nitems = sm.nstrips * ((sm.ny + ty - 1) / ty);
    __shared__ double sh[2][RB];
    double a = 0.0, b = 0.0;
    for (int j = threadIdx.x; j < nitems; j += RB) {
        a += part[2 * (long long)(sm.first_item + j)];
        b += part[2 * (long long)(sm.first_item + j) + 1];
    }
    sh[0][threadIdx.x] = a;
    sh[1][threadIdx.x] = b;
    __syncthreads();
    for (int w = RB / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + w];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double m = sm.h * sm.h, detJ = 0.25 * sm.h * sm.h, c = -sm.dt / m;
        const double A = sh[0][0], B = sh[1][0];
        theta_bar[3 * blockIdx.x + 0] += c * (sm.W * detJ * A + sm.kappa * B / 3.0);
        theta_bar[3 * blockIdx.x + 1] += c * sm.mob * B / 3.0;
        theta_bar[3 * blockIdx.x + 2] += c * sm.mob * detJ * A;
    }
}

}  // namespace

template <typename T>
void launch_vjp2d_batched(const T* eta_hi, const T* eta_lo, const T* lam_in, T* lam_out,
                          const BatchSample* smp, const BatchItem* items, int n_items, int ty, int hk,
                          int depth, int ksteps, bool sym, double* part, hipStream_t s)
{
    const int blocks = (n_items + 3) / 4;
#define VJP_LAUNCH(PF, KS)                                                                                  \
    do {                                                                                                    \
        if (sym)                                                                                            \
            k_vjp2d_batched<T, PF, KS, true><<<blocks, 256, 0, s>>>(eta_hi, eta_lo, lam_in, lam_out, smp,   \
                                                                    items, n_items, ty, hk, part);          \
        else                                                                                                \
            k_vjp2d_batched<T, PF, KS, false><<<blocks, 256, 0, s>>>(eta_hi, eta_lo, lam_in, lam_out, smp,  \
                                                                     items, n_items, ty, hk, part);         \
    } while (0)
    if (ksteps == 2) {
        // three streamed fields: a 2-row ring keeps enough loads in flight and
        // the register count low enough for five waves per SIMD
        VJP_LAUNCH(2, 2);
        (void)depth;
    } else {
        if (depth <= 4)
            VJP_LAUNCH(4, 1);
        else
            VJP_LAUNCH(8, 1);
    }
#undef VJP_LAUNCH
}

void launch_vjp2d_reduce(const double* part, const BatchSample* smp, int count, int ty,
                         double* theta_bar, hipStream_t s)
{
    k_vjp2d_reduce<<<count, RB, 0, s>>>(part, smp, ty, theta_bar);
}

template void launch_vjp2d_batched<float>(const float*, const float*, const float*, float*,
                                          const BatchSample*, const BatchItem*, int, int, int, int,
                                          int, bool, double*, hipStream_t);
template void launch_vjp2d_batched<double>(const double*, const double*, const double*, double*,
                                           const BatchSample*, const BatchItem*, int, int, int, int,
                                           int, bool, double*, hipStream_t);

}  // namespace pfk
