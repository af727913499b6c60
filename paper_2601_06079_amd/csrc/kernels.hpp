// kernels.hpp -- host-side launchers of the HIP kernels (internal to libpfhip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pfk {

// Geometry of a structured grid (x fastest).  bc 0: periodic; bc 1: no-flux
// (natural boundary, n - 1 elements per axis).
struct Geom {
    int dim;
    int n[3];
    long long N;  // nodes
    double h;
    int bc;
    int cm;  // 1: consistent mass in the implicit-path kernels (residual, JVP, adjoint)
    int quad;  // 1: Gauss-Lobatto (nodal) quadrature; 0: 2-point Gauss-Legendre
};

// Free-energy polynomials with W folded in.
//   f'(q)  = q (a1 + q (a2 + a3 q))
//   f''(q) = b0 + q (b1 + b2 q)
//   fe     = which f for the energy (0: W (q^2-1)^2 / 4, 1: W q^2 (1-q)^2)
struct FreeEnergy {
    double a1, a2, a3;
    double b0, b1, b2;
    double W;
    int fe;
};

// the two double wells: f' = a1 q + a2 q^2 + a3 q^3, f'' = b0 + b1 q + b2 q^2 (W folded in)
__host__ __device__ inline FreeEnergy make_free_energy(int fe, double W)
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

// ---- ragged batches: device plan entries (written by the host, batch.cpp) -----
struct BatchSample {
    long long offset;          // element offset of the sample in the packed arrays
    int nx, ny;                // nodes per axis
    int nstrips, first_item;   // work items of this sample (strips x chunks)
    int fe, reserved;          // free energy (0: W (c^2-1)^2/4, 1: W c^2 (1-c)^2)
    double a1, a2, a3, beta, gamma;  // fused-kernel coefficients (dt folded in)
    double W, kappa, mob, h, dt;     // raw parameters (sensitivities)
};
struct BatchItem {
    int sample, strip, chunk, pad;
};

// ---- per-node kernels (k_node.hip); T = float or double ---------------------
// r(U) of Eq. 11; with Uold != nullptr the backward-Euler residual of Eq. 14
template <typename T>
void launch_residual(const Geom& g, int model, const FreeEnergy& f, double kappa, double mob,
                     const T* U, T* r, hipStream_t s, const T* Uold = nullptr, double inv_dt = 0.0);
// Jv = (dR/dU) v (trans: transpose product; acc: Jv += ...)
template <typename T>
void launch_jvp(const Geom& g, int model, const FreeEnergy& f, double kappa, double mob,
                double inv_dt, const T* U, const T* v, T* Jv, hipStream_t s, int trans = 0,
                int acc = 0);
// z-planes per block of launch_jvp3d set by pf_tune_set (0: automatic)
int tune_jvp3d_planes();
int tune_el_planes();  // z-planes per wave of the elasticity operator (0 = automatic)
int tune_el_mg();      // 1: plain CG for the elasticity solves
int tune_stream2d_seam();  // 1: fused 2-D launches recompute chunk seams (no LDS sharing)
int tune_nn_group();       // samples per forward group of the surrogate (0: automatic)
int tune_gs_reorth();      // Gram-Schmidt re-orthogonalisation threshold (0: default)
int tune_gg_stream();      // 1: grain steps on the tile kernel
int tune_jvp2d_stream();   // 1: 2-D Jacobian products on the node-centric kernel
int tune_stream2d_rows();  // rows per wave of the 2-D streaming kernels (0: automatic)
// Row-streaming 2-D Jacobian product (k_jvp2d.hip): Gauss quadrature, lumped
// mass, periodic or no-flux; the non-transposed product, which for Allen-Cahn is
// also its transpose.  Returns false (nothing launched) where it does not apply.
// pq (Allen-Cahn only): also the per-block FP64 partial sums of v . Jv, at most
// pq_max of them, their count in *pq_blocks.
template <typename T>
bool launch_jvp2d_stream(const Geom& g, int model, const FreeEnergy& f, double kappa, double mob,
                         double inv_dt, const T* U, const T* v, T* Jv, hipStream_t s, double* pq = nullptr,
                         int* pq_blocks = nullptr, int pq_max = 0);

// grain growth (PF_GRAIN, 2-D): one explicit step (residual = 0) or the residual
// (residual = 1) of all P order parameters; LDS bytes per block of the tile kernel
size_t gg_tile_lds_bytes(int P, size_t esize);
// mode 0: one explicit step (dt); 1: the residual, with the backward-Euler time term
// inv_dt m (U - old) when old != nullptr; 2: the point-Jacobi inverse diagonal of
// dR/dU (inv_dt m + ...) into out
template <typename T>
void launch_gg_tile2d(const Geom& g, int P, double L, double kappa, double gamma, double dt, const T* in,
                      T* out, int mode, hipStream_t s, const T* old = nullptr, double inv_dt = 0.0);
// one explicit step streamed row by row (k_gg_stream2d) when it applies: 2-D, P in
// 1-6, 8 (and 10, 12, 16, 20 in FP32), P N elements addressable with 32-bit offsets, not
// switched off by PF_TUNE_GG_STREAM; false (nothing launched) otherwise
template <typename T>
bool launch_gg_stream2d(const Geom& g, int P, double L, double kappa, double gamma, double dt, const T* in,
                        T* out, int cus, hipStream_t s);
// Jv = dR/dU v of the backward-Euler residual (symmetric); LDS bytes per block
size_t gg_jvp_lds_bytes(int P, size_t esize);
template <typename T>
void launch_gg_jvp2d(const Geom& g, int P, double L, double kappa, double gamma, double inv_dt, const T* U,
                     const T* V, T* Jv, hipStream_t s);
// out[0] = E_h, out[1] = sum m sum_i eta_i; partials: 2 * energy_blocks(g) doubles
template <typename T>
void launch_gg_energy2d(const Geom& g, int P, double kappa, double gamma, const T* U, double* part,
                        double* out, hipStream_t s);  // z-planes per wave of the elasticity operator (0 = automatic)
// 3-D Jv (acc = 0) by element-wise sum factorisation through z-marching LDS tiles
template <typename T>
void launch_jvp3d(const Geom& g, int model, const FreeEnergy& f, double kappa, double mob,
                  double inv_dt, const T* U, const T* v, T* Jv, hipStream_t s, int trans);
// (block-)Jacobi inverse of dR/dU at U: N (Allen-Cahn) or 4N (Cahn-Hilliard) values
template <typename T>
void launch_prec(const Geom& g, int model, const FreeEnergy& f, double kappa, double mob,
                 double inv_dt, const T* U, T* pinv, hipStream_t s);
// mu = [N(c) + kappa K c] / m
template <typename T>
void launch_chem(const Geom& g, const FreeEnergy& f, double kappa, const T* c, T* mu,
                 hipStream_t s);
// c_out = c - dt M K mu / m
template <typename T>
void launch_ch_update(const Geom& g, double dtM, const T* c, const T* mu, T* c_out,
                      hipStream_t s);
// eta_out = eta - dt r(eta) / m   (Allen-Cahn, any dim)
template <typename T>
void launch_ac_step(const Geom& g, const FreeEnergy& f, double kappa, double dtL, const T* eta,
                    T* eta_out, hipStream_t s);
// out[0] = E_h, out[1] = sum m c ; partials: 2 * energy_blocks(g) doubles
template <typename T>
void launch_energy(const Geom& g, const FreeEnergy& f, double kappa, const T* c, double* partials,
                   double* out, hipStream_t s);
int energy_blocks(const Geom& g);

// out[0] = sum_b part[2b], out[1] = sum_b part[2b+1] (one block, fixed order)
void launch_reduce_pairs(const double* part, int nb, double* out, hipStream_t s);

// ---- coupled Allen-Cahn / Cahn-Hilliard (k_coupled.hip); states [c ; mu ; eta] --
// mu = g(c, eta)/m; with eta_out != nullptr also eta_out = eta - dt M_eta r_eta/M_eta/m
template <typename T>
void launch_cp_mu_eta(const Geom& g, double kappa, double dt_Meta, const T* c, const T* eta, T* mu,
                      T* eta_out, hipStream_t s);
// r = [M_c K mu ; m mu - g(c, eta) ; M_eta (s(c, eta) + kappa K eta)] (+ inv_dt M (U - Uold))
template <typename T>
void launch_cp_residual(const Geom& g, double kappa, double Mc, double Meta, const T* U, T* r,
                        hipStream_t s, const T* Uold = nullptr, double inv_dt = 0.0);
// Jv of the backward-Euler residual (inv_dt = 0: of r)
template <typename T>
void launch_cp_jvp(const Geom& g, double kappa, double Mc, double Meta, double inv_dt, const T* U,
                   const T* v, T* Jv, hipStream_t s);
// 3x3 block-Jacobi inverse (9 values per node, row-major)
template <typename T>
void launch_cp_prec(const Geom& g, double kappa, double Mc, double Meta, double inv_dt, const T* U,
                    T* pinv, hipStream_t s);
// one fused explicit step of the coupled model on a 2-D grid (k_stream_cp.hip):
// (c_in, e_in) -> (c_out, e_out); rows: rows per wavefront (0: 32)
template <typename T>
void launch_cp_explicit2d(const Geom& g, double kappa, double Mc, double Meta, double dt, const T* c_in,
                          const T* e_in, T* c_out, T* e_out, int rows, hipStream_t s);
// out[0] = E_h(c, eta), out[1] = sum m c; partials: 2 * energy_blocks(g) doubles
template <typename T>
void launch_cp_energy(const Geom& g, double kappa, const T* U, double* partials, double* out,
                      hipStream_t s);

// ---- sensitivities (k_adjoint.hip) -----------------------------------------
// theta_bar[0..3) += scale * w^T dr/dtheta at U (part: 3 * ceil(N/256) doubles)
template <typename T>
void launch_dtheta(const Geom& g, int model, const FreeEnergy& f, double kappa, double mob,
                   const T* U, const T* w, double scale, double* part, double* theta_bar,
                   hipStream_t s);
// ubar[0..N) += inv_dt m lam[0..N)
template <typename T>
void launch_mass_axpy(const Geom& g, double inv_dt, const T* lam, T* ub, hipStream_t s);
// one explicit step S at U: ubar += (dS/dU)^T vbar, theta_bar += (dS/dtheta)^T vbar
// (Cahn-Hilliard: c planes only).  scratch: 2N values.
template <typename T>
void launch_vjp_explicit(const Geom& g, int model, const FreeEnergy& f, double kappa, double mob,
                         double dt, const T* U, const T* vbar, T* ubar, T* scratch, double* part,
                         double* theta_bar, hipStream_t s);

// ---- fused 2-D explicit streaming kernels (k_stream2d.hip) ------------------
struct Stream2DConfig {
    int ty;     // rows per wave
    int depth;  // rows in flight per wave (4, 8 or 16)
    int ks;     // explicit steps fused per launch (1..4)
};
// cfg.ks explicit steps in -> out (out != in).  model 0: Allen-Cahn, 1: Cahn-Hilliard c-plane.
template <typename T>
void launch_explicit2d(const Geom& g, int model, const FreeEnergy& f, double kappa, double mob,
                       double dt, const T* in, T* out, const Stream2DConfig& cfg, hipStream_t s);

// ---- ragged batch kernels ------------------------------------------------------
// cfg.ks explicit steps of every sample: one launch for the whole batch.  With
// mid != nullptr two steps are fused and the state after the first is also
// written to mid (trajectory mode; cfg.ks is ignored).
template <typename T>
void launch_explicit2d_batched(int model, const T* in, T* out, const BatchSample* smp,
                               const BatchItem* items, int n_items, const Stream2DConfig& cfg,
                               hipStream_t s, T* mid = nullptr);
// Allen-Cahn step adjoint over a ragged batch (streamed like the forward kernel),
// ksteps (1 or 2 <= hk) steps per launch: lam_out = S_lo^T S_hi^T lam_in with
// S^T lam = lam - (dt L/m) J_r(eta)^T lam at eta_hi (= eta_k) and, for two
// steps, eta_lo (= eta_{k-1}); part[2 w .. 2 w + 2) += (A, B) of work item w
// (see k_vjp2d.hip); hk: the plan's strip halo (H ks); sym: every sample has the
// symmetric double well W (c^2 - 1)^2 / 4
template <typename T>
void launch_vjp2d_batched(const T* eta_hi, const T* eta_lo, const T* lam_in, T* lam_out,
                          const BatchSample* smp, const BatchItem* items, int n_items, int ty, int hk,
                          int depth, int ksteps, bool sym, double* part, hipStream_t s);
// theta_bar[s][0..3) += the gradient of sample s's accumulated (A, B) (fixed order)
void launch_vjp2d_reduce(const double* part, const BatchSample* smp, int count, int ty,
                         double* theta_bar, hipStream_t s);

}  // namespace pfk
