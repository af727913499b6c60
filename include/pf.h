/*
 * pf.h -- C ABI of the MI355X (gfx950) phase-field step library libpfhip.so.
 *
 * The library evaluates and advances the finite-element phase-field models of
 * arXiv 2601.06079 on structured 2-D / 3-D grids:
 *   Allen-Cahn       d eta/dt = -L (f'(eta) - kappa lap eta)              (Sec. 2.1, Eq. 1, Eq. 5)
 *   Cahn-Hilliard    dc/dt = div(M grad mu), mu = f'(c) - kappa lap c     (Sec. 2.2, Eqs. 9-10)
 * semi-discretised as M dU/dt + r(U, theta) = 0 (Eq. 11) with Q1 (bi/tri-linear)
 * Lagrange elements, 2-point Gauss-Legendre quadrature per axis and the
 * row-sum lumped mass matrix (nodal mass m = h^d on periodic grids).
 *
 * Conventions shared by every entry point
 *   - Fields are contiguous device arrays, node index i + n0*(j + n1*k)
 *     (x fastest).  Cahn-Hilliard states U hold the c plane at offset 0 and
 *     the mu plane at offset N (N = number of nodes).  Element type is
 *     float (PF_F32) or double (PF_F64) as pf_problem.dtype says.
 *   - Every call that enqueues device work takes a context (pf_ctx, made by
 *     pf_create for one device) and must be made with that device current.
 *     The context holds what persists between calls: the device properties
 *     the launchers size their grids with, the pinned host slots the Newton,
 *     GMRES and CG kernels store their scalars into (allocated by pf_create,
 *     never inside a compute call), the elasticity smoother's eigenvalue cache
 *     and the batch autotuner's results.  Calls that share a context must not
 *     run concurrently on different host threads (one context per thread, or
 *     external locking).
 *   - The caller owns every buffer.  The library allocates no device memory
 *     on any compute path and never frees caller memory.  Scratch needs are
 *     reported by pf_workspace_size and passed in as `ws` (device memory,
 *     256-byte aligned).
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  All
 *     work is enqueued on it; calls return before the work finishes unless
 *     stated otherwise.
 *   - Return value is a pf_status.  PF_EINVAL is returned before anything is
 *     enqueued for a malformed problem or argument; pf_last_error() then
 *     gives a thread-local message.  No C++ exception crosses this ABI: a
 *     host allocation that fails inside a call returns PF_EDEVICE.
 *   - Thread safety: calls on different streams from different host threads
 *     are independent; concurrent calls that share buffers race.
 */
#ifndef PF_H
#define PF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum pf_status {
    PF_OK = 0,
    PF_EINVAL = 1,      /* malformed problem or argument; nothing enqueued */
    PF_EDEVICE = 2,     /* a HIP runtime call failed (message in pf_last_error) */
    PF_ENOCONV = 3,     /* Newton did not converge; U holds the last iterate */
    PF_ENONFINITE = 4,  /* a non-finite residual norm was met */
    PF_EUNSUPPORTED = 5 /* valid request the library does not implement */
} pf_status;

/* Per-device context (opaque).  See pf_create. */
typedef struct pf_ctx pf_ctx;
enum { PF_HOST_ONLY = -1 }; /* pf_create device: a context for sizing and validation only */

enum { PF_PERIODIC = 0, PF_NOFLUX = 1 };       /* boundary condition (Supp. Note 3) */
enum { PF_ALLEN_CAHN = 0, PF_CAHN_HILLIARD = 1,
       PF_COUPLED = 2 }; /* coupled Allen-Cahn / Cahn-Hilliard of Eq. 7 with the benchmark
                          * free energies of Supp. Note 3 (fe and W are ignored):
                          *   f_a(c) = -1.6704 - 4.776c + 5.1622c^2 - 2.7375c^3 + 1.3687c^4,
                          *   f_b(c) = 5.0c^2 - 5.9746c - 1.5924,
                          *   h(eta) = 10 eta^3 - 15 eta^4 + 6 eta^5;
                          * states [c ; mu ; eta], mobility = M_c, mobility_eta = M_eta,
                          * kappa = kappa_eta (no composition gradient energy).  Supported by
                          * pf_residual, pf_step_explicit, pf_energy, pf_jvp and
                          * pf_newton_step (3x3 block-Jacobi); pf_vjp and the batch calls
                          * return PF_EUNSUPPORTED. */
enum { PF_GRAIN = 3 };   /* grain growth: nfields order parameters eta_1..eta_p, each an
                          * Allen-Cahn field (Eq. 1; mobility = L, kappa) coupled through the
                          * multi-well energy of the grain-growth literature (the paper does
                          * not print it):
                          *   f = sum_i (eta_i^4/4 - eta_i^2/2) + gamma sum_{i<j} eta_i^2 eta_j^2 + 1/4;
                          * all order parameters are updated in one launch (Sec. 2.4).
                          * States [eta_1 (N) ; ... ; eta_p (N)].  2-D only; fe and W are
                          * ignored; nfields <= 32 (PF_F32) or <= 12 (PF_F64).  Supported by
                          * pf_residual, pf_step_explicit, pf_energy (out[1] = sum m
                          * sum_i eta_i), and with nfields <= 24 (PF_F32) by pf_jvp and
                          * pf_newton_step (point Jacobi over all p N unknowns); pf_vjp and
                          * the batch calls return PF_EUNSUPPORTED. */
enum { PF_F_SYM = 0,  /* f(c) = W (c^2 - 1)^2 / 4 */
       PF_F_01 = 1 }; /* f(c) = W c^2 (1 - c)^2  (Supp. Note 3: f' = 4c(c-1)(c-1/2) at W = 1) */
enum { PF_F32 = 0, PF_F64 = 1 };
/* Mass matrix of the implicit path.  PF_MASS_LUMPED: the row-sum lumped mass
 * everywhere (the default; required by the explicit step, its adjoint and the
 * batches).  PF_MASS_CONSISTENT: every term of the weak form Gauss-integrated,
 * so the backward-Euler time term M (U - U_old)/dt and the Cahn-Hilliard
 * mu-row M mu carry M_ab = int phi_a phi_b (Eqs. 11, 13-14); supported by
 * pf_residual, pf_jvp, pf_newton_step and pf_vjp (PF_VJP_RESIDUAL,
 * PF_VJP_NEWTON_STEP) for Allen-Cahn and Cahn-Hilliard; the explicit step,
 * PF_VJP_EXPLICIT_STEP, the batches and the coupled model return
 * PF_EUNSUPPORTED.  Energies and sum m c are the same for both (the row sums of
 * the consistent mass are the lumped mass). */
enum { PF_MASS_LUMPED = 0, PF_MASS_CONSISTENT = 1 };
/* Quadrature of every element integral (Sec. 2.2 leaves it open).
 * PF_QUAD_GAUSS: 2-point Gauss-Legendre per axis (the default).
 * PF_QUAD_LOBATTO: 2-point Gauss-Lobatto per axis, whose points are the element's
 * nodes (nodal quadrature): the nonlinear term becomes m_a f'(c_a), the Q1
 * stiffness the 5-point stencil 4 c_i - (axis neighbours) in 2-D and
 * h (6 c_i - axis neighbours) in 3-D, the energy sum_a m_a f(c_a) + kappa/2 c.Kc,
 * and the mass diagonal (PF_MASS_CONSISTENT then equals PF_MASS_LUMPED).
 * Allen-Cahn and Cahn-Hilliard, 2-D and 3-D, periodic and no-flux: pf_residual,
 * pf_step_explicit, pf_energy, pf_jvp and pf_newton_step; pf_vjp, the batches and
 * the coupled and grain models return PF_EUNSUPPORTED. */
enum { PF_QUAD_GAUSS = 0, PF_QUAD_LOBATTO = 1 };

/* Problem statement: grid, boundary condition, model, free energy and the
 * material parameters theta = (mobility, kappa, W) of Eqs. 1, 5-6, 9-10.
 * Periodic grids have n elements per axis (domain length n h); no-flux grids
 * (the natural boundary condition of the weak form, Supp. Note 3) have n - 1,
 * and the lumped mass of a node on b boundary faces is h^dim / 2^b. */
typedef struct pf_problem {
    int32_t dim;      /* 2 or 3 */
    int32_t bc;       /* PF_PERIODIC or PF_NOFLUX (natural boundary; batches: periodic only) */
    int32_t model;    /* PF_ALLEN_CAHN or PF_CAHN_HILLIARD */
    int32_t fe;       /* PF_F_SYM or PF_F_01 */
    int32_t dtype;    /* PF_F32 or PF_F64 */
    int32_t mass;     /* PF_MASS_LUMPED (0) or PF_MASS_CONSISTENT (implicit path) */
    int64_t n[3];     /* nodes per axis, each >= 2 (n[2] ignored when dim == 2) */
    double h;         /* grid spacing > 0 */
    double W;         /* barrier height of f */
    double kappa;     /* gradient-energy coefficient */
    double mobility;  /* L (Allen-Cahn) or M (Cahn-Hilliard); M_c (coupled) */
    double mobility_eta; /* coupled model: M_eta (ignored by the other models) */
    int32_t nfields;  /* PF_GRAIN: number of order parameters (ignored by the other models) */
    int32_t quad;     /* PF_QUAD_GAUSS (0) or PF_QUAD_LOBATTO (see below) */
    double gamma;     /* PF_GRAIN: pair coupling of the multi-well energy */
} pf_problem;

/* Operation codes for pf_workspace_size. */
enum {
    PF_OP_RESIDUAL = 0,
    PF_OP_STEP_EXPLICIT = 1,
    PF_OP_ENERGY = 2,
    PF_OP_NEWTON = 3,
    PF_OP_VJP = 4,
    PF_OP_JVP = 5
};

/* Thread-local description of the last non-OK status returned on this thread. */
const char* pf_last_error(void);

/* Library ABI version (major * 100 + minor). */
int pf_version(void);

/* Make a context for device `device` (a HIP device ordinal): queries its
 * properties and allocates the pinned host slots that the Newton/GMRES, CG and
 * elasticity solvers read their scalars from.  The current device is left as it
 * was.  device = PF_HOST_ONLY makes a context without a device, accepted by the
 * host-only queries (pf_workspace_size, pf_launch_shape, pf_el_workspace_size)
 * and by argument validation; calls that enqueue device work return PF_EINVAL
 * with it.  *out receives the context (NULL on failure).  PF_EDEVICE if the
 * device does not exist or an allocation fails. */
int pf_create(int device, pf_ctx** out);
/* Free a context and everything it owns (NULL is accepted).  No call may be
 * using it; work already enqueued with it need not have finished. */
int pf_destroy(pf_ctx* ctx);
/* The device ordinal of a context (PF_HOST_ONLY for a host-only one). */
int pf_ctx_device(const pf_ctx* ctx, int* device);

/* Copy `bytes` (a multiple of 16; src, dst 16-byte aligned, not overlapping)
 * with 16-byte loads and stores: the practical HBM (or Infinity Cache)
 * bandwidth against which the stencil kernels are measured.  Asynchronous. */
int pf_stream_copy(pf_ctx* ctx, const void* src, void* dst, size_t bytes, void* stream);
/* `blocks` blocks of 256 threads, each running 8 independent non-packed FP32 FMA
 * chains for `iters` rounds (16 iters flops per thread) and writing one float to
 * out[block * 256 + thread] (device, 256 blocks floats): the practical FP32 VALU
 * ceiling of the explicit step.  Asynchronous. */
int pf_fma_probe(pf_ctx* ctx, int blocks, int iters, float* out, void* stream);

/* Launch-shape overrides, process-global (value 0 restores the automatic
 * choice).  Used by the autotuner; results never depend on them, except that on
 * no-flux grids the steps fused per launch change boundary-adjacent values in
 * the last bits (a fused stage evaluates the reflected ghost rows).
 *   PF_TUNE_STREAM2D_ROWS:  rows per wavefront of the fused 2-D explicit kernel and of
 *                           the row-streaming 2-D Jacobian product;
 *   PF_TUNE_STREAM2D_DEPTH: rows it keeps in flight per wavefront (<=4, <=8, else 16);
 *   PF_TUNE_STREAM2D_FUSE:  explicit steps fused per launch by temporal blocking (1..4);
 *   PF_TUNE_JVP3D_PLANES:   z-planes per block of the 3-D Jacobian product;
 *   PF_TUNE_EL_PLANES:      z-planes (2-D: rows) per wave of the elasticity operator;
 *   PF_TUNE_STREAM2D_SEAM:  1 = fused 2-D launches recompute the rows where chunks meet
 *                           (each wave alone); 0 = the waves of a workgroup share them
 *                           through LDS where the chunk plan allows (periodic grids);
 *   PF_TUNE_NN_GROUP:       samples per group of the surrogate's forward pass (0: as
 *                           many as keep one 32-channel activation within 128 MiB);
 *   PF_TUNE_GS_REORTH:      v >= 1: GMRES re-orthogonalises (a second Gram-Schmidt
 *                           pass) when one projection keeps less than (v - 1) / 1000
 *                           of ||w||^2 (1: never, 2001: always); 0: 1/10 (default);
 *   PF_TUNE_GG_STREAM:      1 = explicit grain-growth steps on the LDS tile kernel; 0 =
 *                           the row-streaming kernel where it applies (default);
 *   PF_TUNE_JVP2D_STREAM:   1 = 2-D Jacobian products (pf_jvp, the Newton Krylov
 *                           solves) on the node-centric kernel; 0 = the row-streaming
 *                           kernel where it applies (default: Gauss quadrature,
 *                           lumped mass, Allen-Cahn and Cahn-Hilliard);
 *   PF_TUNE_EL_MG:          1 = plain CG for the elasticity solves (no multigrid);
 *                           2 = multigrid with every level launched separately;
 *                           v >= 3 = the multigrid's coarse grids of at most v
 *                           nodes run in one workgroup (default: 1200 in 2-D,
 *                           none in 3-D). */
enum { PF_TUNE_STREAM2D_ROWS = 0, PF_TUNE_STREAM2D_DEPTH = 1, PF_TUNE_STREAM2D_FUSE = 2,
       PF_TUNE_JVP3D_PLANES = 3, PF_TUNE_EL_PLANES = 4, PF_TUNE_EL_MG = 5, PF_TUNE_STREAM2D_SEAM = 6,
       PF_TUNE_NN_GROUP = 7, PF_TUNE_GS_REORTH = 8, PF_TUNE_GG_STREAM = 9,
       PF_TUNE_JVP2D_STREAM = 10 };
int pf_tune_set(int key, int value);
int pf_tune_get(int key, int* value);
/* The launch shape pf_step_explicit uses for p (2-D) on the context's device:
 * steps fused per launch, rows per wavefront, prefetch depth.  Host-only. */
int pf_launch_shape(const pf_ctx* ctx, const pf_problem* p, int* ks, int* ty, int* depth);

/* Bytes of device scratch `ws` that operation `op` needs for problem p
 * (0 when none).  Host-only; enqueues nothing. */
int pf_workspace_size(const pf_ctx* ctx, const pf_problem* p, int op, size_t* bytes);

/* r = r(U, theta) of Eq. 11 (no mass/time term).
 *   Allen-Cahn:     r = L [ N(eta) + kappa K eta ]
 *   Cahn-Hilliard:  r_c  = M K mu
 *                   r_mu = m mu - [ N(c) + kappa K c ]
 * where N(u)_a = sum_e sum_q |J| f'(u_q) phi_a(q) (Gauss points q) and K is
 * the Q1 stiffness matrix.  With this r the implicit residual of Eq. 14 is
 * R = M (U - U_old)/dt + r(U) with mass matrix diag(m) (Allen-Cahn) or
 * diag(m, 0) (Cahn-Hilliard).
 *   Coupled (Eq. 7):  r_c   = M_c K mu
 *                     r_mu  = m mu - sum_e sum_q |J| [f_a'(c_q)(1 - h(eta_q)) + f_b'(c_q) h(eta_q)] phi_a
 *                     r_eta = M_eta [ sum_e sum_q |J| (f_b - f_a)(c_q) h'(eta_q) phi_a + kappa K eta ]
 * U and r: device, ndof elements (N, 2N or 3N), must not alias.  ws: the
 * pf_workspace_size(PF_OP_RESIDUAL) scratch, which is 0 bytes (NULL is
 * accepted).  Asynchronous. */
int pf_residual(pf_ctx* ctx, const pf_problem* p, const void* U, void* r, void* ws, void* stream);

/* nsteps forward-Euler steps of Eq. 12 with the lumped mass, in place on U:
 *   Allen-Cahn:     eta <- eta - dt r(eta) / m
 *   Cahn-Hilliard:  mu <- [N(c) + kappa K c] / m, then c <- c - dt M K mu / m
 *                   (the algebraic mu-row of the split form solved each step);
 *                   on return the mu plane holds [N(c) + kappa K c]/m of the
 *                   final c.
 *   Coupled:        mu <- g(c, eta)/m and eta <- eta - dt r_eta(c, eta)/m from the
 *                   old state, then c <- c - dt M_c K mu / m; on return the mu
 *                   plane holds g/m of the final state.
 * ws: device scratch of pf_workspace_size(PF_OP_STEP_EXPLICIT) bytes (one
 * ping-pong field; two for the coupled model).  nsteps >= 0, dt > 0.
 * Asynchronous. */
int pf_step_explicit(pf_ctx* ctx, const pf_problem* p, double dt, int64_t nsteps, void* U, void* ws,
                     void* stream);

/* out[0] = E_h(U) = sum_e sum_q |J| [ f(c_q) + kappa/2 |grad c_q|^2 ]  (Eqs. 5-6)
 *          (coupled model: [f_a(c_q)(1 - h(eta_q)) + f_b(c_q) h(eta_q) + kappa/2 |grad eta_q|^2],
 *          Eq. 7, with U the whole [c ; mu ; eta] state)
 * out[1] = sum_a m_a c_a  (total conserved quantity)
 * out: device pointer to 2 doubles; accumulation in FP64 with a fixed
 * reduction order (bitwise reproducible).  ws: pf_workspace_size(PF_OP_ENERGY).
 * Asynchronous. */
int pf_energy(pf_ctx* ctx, const pf_problem* p, const void* U, double* out, void* ws, void* stream);

/* pf_energy without a workspace, for callers that cannot allocate device memory
 * (code under HIP graph capture, loops that forbid allocation): the same result,
 * bitwise, with the reduction's partial sums kept in a static array of the library
 * (1 MiB per device, held until the process ends).  Grids of at most 2^24 nodes;
 * larger ones return PF_EINVAL before anything is enqueued.  Calls that overlap on
 * one device share that array and race; serialise them (one stream, or events).
 * Allocates nothing.  Asynchronous. */
int pf_energy_noalloc(pf_ctx* ctx, const pf_problem* p, const void* U, double* out, void* stream);

/* Jv = (dR/dU) v for R = inv_dt M (U - U_old) + r(U) (Eq. 14; inv_dt = 0
 * gives dr/dU):
 *   Allen-Cahn:     Jv = inv_dt m v + L [ N'(eta) v + kappa K v ]
 *   Cahn-Hilliard:  Jv_c  = inv_dt m v_c + M K v_mu
 *                   Jv_mu = m v_mu - [ N'(c) v_c + kappa K v_c ]
 * N'(u) v = sum_e sum_q |J| f''(u_q) v_q phi_a(q).  Matrix-free (the Jacobian
 * of Sec. 2.3 is never formed).  U, v, Jv: device, ndof elements; Jv must not
 * alias U or v.  Asynchronous. */
int pf_jvp(pf_ctx* ctx, const pf_problem* p, double inv_dt, const void* U, const void* v, void* Jv,
           void* stream);

/* ---------------------------------------------------------------------- */
/* Backward-Euler Newton step (Eqs. 13-14, Sec. 2.3)                        */
/* ---------------------------------------------------------------------- */
enum { PF_PRECOND_NONE = 0, PF_PRECOND_JACOBI = 1 /* point (AC) / 2x2 block (CH) */ };
/* Linear solver of each Newton correction.  PF_KRYLOV_CG (preconditioned
 * conjugate gradients, device-resident scalars) needs a symmetric positive
 * definite Jacobian: Allen-Cahn only, and dt * mobility * W < 1 (then
 * (m/dt) M + L (N'(eta) + kappa K) is positive definite for every eta, since
 * f'' >= -W for both double wells); otherwise pf_newton_step returns PF_EINVAL. */
enum { PF_KRYLOV_GMRES = 0, PF_KRYLOV_CG = 1 };

typedef struct pf_newton_opts {
    double rtol;            /* stop when ||R||_2 <= rtol ||R(U_initial)||_2 (default 1e-8) */
    double atol;            /* or ||R||_2 <= atol (default 0) */
    int32_t max_newton;     /* Newton corrections (default 20) */
    int32_t gmres_restart;  /* Krylov dimension m of GMRES(m), 1..64 (default 30) */
    int32_t gmres_max_its;  /* Arnoldi steps per Newton correction (default 600) */
    int32_t precond;        /* PF_PRECOND_* (default PF_PRECOND_JACOBI) */
    double lin_rtol_max;    /* inexact-Newton forcing: linear rtol = clamp(0.1 ||R_k||/||R_0||, */
    double lin_rtol_min;    /*   lin_rtol_min, lin_rtol_max) (defaults 1e-2, 1e-6) */
    int32_t stagnation;     /* 1: also stop at the field precision's rounding floor: after
                             * >= 2 corrections ||R_k|| > ||R_{k-1}||/2 while the last
                             * correction is <= 8 eps max|U|, or ||R_k|| > 0.9 ||R_{k-1}||
                             * after a correction <= sqrt(eps) max|U| */
    int32_t krylov;         /* PF_KRYLOV_GMRES (default) or PF_KRYLOV_CG; gmres_restart is
                             * ignored by CG, gmres_max_its bounds its iterations */
} pf_newton_opts;

typedef struct pf_newton_report {
    int32_t newton_its;      /* corrections applied */
    int32_t gmres_its;       /* Krylov iterations over all corrections (Arnoldi steps or CG) */
    int32_t converged;       /* 1 if a stop test passed */
    int32_t reason;          /* 0 rtol, 1 atol, 2 rounding floor, -1 max_newton, -2 non-finite */
    double res_norm[33];     /* ||R||_2 per iterate (FP64), entries 0..newton_its (<= 32 kept) */
} pf_newton_report;

/* Fill opts with the defaults listed above. */
void pf_newton_default_opts(pf_newton_opts* o);

/* One backward-Euler step: solve R(U) = M (U - U_old)/dt + r(U) = 0 for U by
 * Newton-Raphson with matrix-free Jacobian-vector products inside restarted,
 * right-preconditioned GMRES (classical Gram-Schmidt with one
 * re-orthogonalisation; FP64 dot products and Hessenberg even for PF_F32
 * fields), or, with opts->krylov = PF_KRYLOV_CG (Allen-Cahn, dt L W < 1),
 * Jacobi-preconditioned conjugate gradients with FP64 scalars.  U holds the initial guess on entry and the last iterate on exit.
 * U_old is not modified.  ws: pf_workspace_size(PF_OP_NEWTON) bytes.
 * Host-synchronous: returns when the step is done (PF_OK or PF_ENOCONV /
 * PF_ENONFINITE with rep filled).  rep may be NULL. */
int pf_newton_step(pf_ctx* ctx, const pf_problem* p, double dt, const void* U_old, void* U,
                   const pf_newton_opts* opts, pf_newton_report* rep, void* ws, void* stream);

/* ---------------------------------------------------------------------- */
/* Sensitivities (Eq. 18, Supp. Note 2, Eqs. II.1-II.6)                     */
/* ---------------------------------------------------------------------- */
enum { PF_VJP_RESIDUAL = 0, PF_VJP_EXPLICIT_STEP = 1, PF_VJP_NEWTON_STEP = 2 };

enum { PF_VJP_THETA_HOST = 1 }; /* pf_vjp flags: theta_bar is a host pointer */
/* Vector-Jacobian products of one building block, accumulated into Ubar and
 * theta_bar (3 doubles: mobility, kappa, W; a device pointer, or a host pointer
 * with flags = PF_VJP_THETA_HOST, which makes the call host-synchronous):
 *   PF_VJP_RESIDUAL:       U_old == NULL: the residual r of Eq. 11:
 *                            Ubar += (dr/dU)^T vbar, theta_bar += (dr/dtheta)^T vbar at U;
 *                          U_old != NULL: the backward-Euler residual of Eq. 14,
 *                            R = M (U - U_old)/dt + r(U): Ubar += (dR/dU)^T vbar
 *                            = (M/dt) vbar + (dr/dU)^T vbar (M symmetric), theta_bar as
 *                            above (U_old enters R linearly and its values are not
 *                            needed; dt must be > 0)
 *   PF_VJP_EXPLICIT_STEP:  for S(U) = one pf_step_explicit step from U:
 *                          Ubar += (dS/dU)^T vbar,  theta_bar += (dS/dtheta)^T vbar
 *                          (Cahn-Hilliard: c planes only; mu is a derived output)
 *   PF_VJP_NEWTON_STEP:    U is the converged root of one backward-Euler step:
 *                          solve (dR/dU)^T lambda = vbar (GMRES, same opts as
 *                          the forward step), then Ubar(U_old) += (M/dt) lambda,
 *                          theta_bar -= (dr/dtheta)^T lambda   (II.5-II.6).
 * U_old is read only by PF_VJP_RESIDUAL (see there) and may be NULL otherwise.
 * theta_bar accumulates in FP64 with a fixed reduction order.  dt is ignored
 * for PF_VJP_RESIDUAL without U_old.  ws: pf_workspace_size(PF_OP_VJP).
 * Asynchronous, except PF_VJP_NEWTON_STEP (host-synchronous like
 * pf_newton_step) and PF_VJP_THETA_HOST. */
int pf_vjp(pf_ctx* ctx, const pf_problem* p, int kind, double dt, const void* U, const void* U_old,
           const void* vbar, void* Ubar, double* theta_bar, int flags, void* ws, void* stream);

/* ---------------------------------------------------------------------- */
/* Ragged batches of independent 2-D problems (many samples in one launch) */
/* ---------------------------------------------------------------------- */
/* One sample of a batch: its own grid and material parameters.  All samples
 * share the base problem's model, free energy, dtype and (periodic) boundary.
 * A batch holds 1 .. PF_BATCH_MAX_COUNT samples. */
enum { PF_BATCH_MAX_COUNT = 1 << 20 };
typedef struct pf_batch_sample {
    int64_t offset; /* element offset of this sample's field in the packed arrays */
    int64_t n[3];   /* nodes per axis (n[2] ignored); each sample < 2 GiB */
    double h, W, kappa, mobility;
} pf_batch_sample;

/* Host-side description of a device plan (filled by pf_batch_plan). */
typedef struct pf_batch_info {
    int32_t count, n_items, fe;        /* samples, work items (sample, strip, chunk), free energy */
    int32_t ks, ty, depth;             /* fused steps, rows per wave, prefetch depth */
    int32_t model, dtype;
    int64_t total;                     /* elements of each packed array (max offset + nodes) */
    int64_t plan_bytes;
    double dt;
    int64_t off_samples, off_items, reserved1; /* byte offsets of the plan's tables; 0 */
} pf_batch_info;

/* Bytes of the device plan for these samples with ks fused steps and ty rows
 * per wave (0 = the largest automatic choice may need).  Host-only. */
int pf_batch_plan_size(const pf_problem* base, const pf_batch_sample* samples, int count, int ks,
                       int ty, size_t* bytes);

/* Build the launch plan of a batch (work items of the explicit kernel, per-sample
 * coefficients for step dt) on the host and copy it to plan_dev (caller-owned
 * device memory, 256-byte aligned, plan_bytes long).  ks/ty/depth = 0 take the
 * autotuned choice for this batch shape if pf_batch_autotune ran, else the
 * defaults.  Sample ranges must not overlap.  Host-synchronous (waits for the
 * copy).  base supplies dim (2), bc (periodic), model, fe and dtype only. */
int pf_batch_plan(pf_ctx* ctx, const pf_problem* base, const pf_batch_sample* samples, int count, double dt,
                  int ks, int ty, int depth, void* plan_dev, size_t plan_bytes,
                  pf_batch_info* info, void* stream);

/* Workspace of a batched call: PF_OP_STEP_EXPLICIT (one packed field) or
 * PF_OP_VJP (one packed field + two FP64 slots per work item of info). */
int pf_batch_workspace_size(const pf_batch_info* info, int op, size_t* bytes);

/* nsteps explicit steps (Eq. 12) of every sample, one launch per info->ks steps
 * for the whole batch.  traj == NULL: in place on U (nsteps a multiple of ks;
 * ws one packed field); elements of U outside every sample are unspecified on
 * return.  traj != NULL: U is only read, and the state after step k
 * (k = 1..nsteps) is written to traj + (k-1) * info->total; with a plan built for
 * ks >= 2 each launch advances two steps and writes both states (bitwise those
 * of single steps).
 * Allen-Cahn and the Cahn-Hilliard c plane (mu is not produced).  Asynchronous. */
int pf_step_explicit_batched(pf_ctx* ctx, const pf_batch_info* info, const void* plan, int64_t nsteps,
                             void* U, void* ws, void* traj, void* stream);

/* Adjoint of nsteps batched Allen-Cahn explicit steps (Supp. Note 2 applied
 * step by step).  states + k * info->total holds the input of step k+1
 * (k = 0..nsteps-1).  On entry lam holds dO/dU of the final state; on return
 * dO/dU of the first input.  The steps stream over the plan's work items, two
 * steps per launch when the plan was built for ks >= 2 (paired from the last
 * step; lam is bitwise that of single steps), else one.  Sensitivities of
 * theta = (mobility, kappa, W)
 * accumulate per work item in FP64 slots kept in ws (each lane's terms summed
 * down its chunk in the field precision first); with PF_VJP_BEGIN the
 * slots are zeroed first, with PF_VJP_END they are summed (fixed order) into
 * theta_bar (device, count x 3 doubles).  A trajectory processed in segments
 * (checkpointing) with BEGIN on the first call and END on the last gives
 * bitwise the gradient of one call over all steps (with a ks >= 2 plan: when
 * every segment has an even number of steps).  Cahn-Hilliard plans:
 * PF_EUNSUPPORTED.  ws: pf_batch_workspace_size(PF_OP_VJP) of the same info,
 * kept between the calls of one trajectory.  Asynchronous. */
enum { PF_VJP_BEGIN = 1, PF_VJP_END = 2 };
int pf_vjp_explicit_batched(pf_ctx* ctx, const pf_batch_info* info, const void* plan, int64_t nsteps,
                            const void* states, void* lam, double* theta_bar, void* ws, int flags,
                            void* stream);

/* Launch-shape autotuner: times the batched explicit kernel for every
 * (ks, ty, depth) candidate with HIP events on U_scratch (overwritten) and ws,
 * keeps the fastest per step, records it in the context for later
 * pf_batch_plan calls with zero shape arguments, and leaves its plan in
 * plan_dev / *best.  Candidates: ks 1..4, ty 16..48, depth 4 or 8; a candidate whose
 * plan does not fit plan_bytes is skipped, so plan_bytes should be
 * pf_batch_plan_size(..., 4, 16, ...) (the narrowest strips, shortest chunks).
 * Host-synchronous. */
int pf_batch_autotune(pf_ctx* ctx, const pf_problem* base, const pf_batch_sample* samples, int count, double dt,
                      void* U_scratch, void* ws, void* plan_dev, size_t plan_bytes,
                      pf_batch_info* best, double* best_us_per_step, void* stream);

/* ---------------------------------------------------------------------- */
/* Eshelby inclusion: linear elasticity with an eigenstrain (Eqs. 3-4,      */
/* Supp. Note 3 Eq. III.1) and its (E, nu) sensitivities (Eq. 18, Eq. 21)   */
/* ---------------------------------------------------------------------- */
/* Small-strain equilibrium div sigma = 0 with sigma = C : (eps(u) - eps0), C
 * isotropic with Young's modulus E and Poisson's ratio nu (Lame constants
 * lam = E nu / ((1 + nu)(1 - 2 nu)), mu = E / (2 (1 + nu))), and the
 * dilatational eigenstrain eps0 = e0(r) I with
 *     e0(r) = m (1/2 - 1/2 tanh(l (r - a))),  r = distance from the origin,
 * which is m inside the inclusion of radius a and 0 far outside (the printed
 * formula has "+" before the tanh, which would put the misfit outside the
 * inclusion; the library follows the text: m is the misfit inside).
 * Grid [0, (n-1) h]^dim with n - 1 vector Q1 elements per axis, 2-point Gauss
 * quadrature (eps0 evaluated at the Gauss points); dim 2 is plane strain with
 * an in-plane eigenstrain.  The inclusion sits at the origin corner: symmetry
 * planes through the origin (u_x = 0 on x = 0, u_y = 0 on y = 0, u_z = 0 on
 * z = 0) and traction-free outer faces.  Fields hold dim components, component
 * c of node i at c N + i (N nodes, node index i + n0 (j + n1 k)); vectors must
 * be 16-byte aligned.  The fixed components are identity rows of K whose
 * inputs do not act on the free rows, so K is symmetric positive definite. */
typedef struct pf_elastic {
    int32_t dim;    /* 2 (plane strain) or 3 */
    int32_t dtype;  /* PF_F32 or PF_F64 (fields); CG scalars and dot products are FP64 */
    int64_t n[3];   /* nodes per axis, each >= 2 (n[2] ignored when dim == 2) */
    double h;       /* grid spacing > 0 */
    double E, nu;   /* E > 0, -1 < nu < 0.5 */
    double m, a, l; /* misfit magnitude, inclusion radius, interface sharpness */
} pf_elastic;

typedef struct pf_el_report {
    int32_t iterations; /* CG iterations */
    int32_t converged;  /* 1 if ||r|| <= rtol ||b|| (recursively updated residual) */
    int32_t status;     /* 1 converged, 2 iteration limit, 3 breakdown, 4 non-finite */
    int32_t levels;     /* multigrid levels of the preconditioner (1: plain CG) */
    double res_norm;    /* final ||r||_2 */
    double rhs_norm;    /* ||b||_2 */
} pf_el_report;

/* Workspace bytes for pf_el_solve, pf_el_objective and pf_el_sensitivity
 * (seven fields plus FP64 partial sums; with multigrid also one more field,
 * three fields per coarser grid (under 1/7 of a field in 2-D, 1/2 in 3-D, in
 * total) and the 9^d eigenvalue-estimate vectors). */
int pf_el_workspace_size(const pf_ctx* ctx, const pf_elastic* p, size_t* bytes);

/* y = K u (the stiffness of Eqs. 3-4 with the identity rows above).  u, y
 * device, distinct.  Asynchronous. */
int pf_el_apply(pf_ctx* ctx, const pf_elastic* p, const void* u, void* y, void* stream);

/* f = the eigenstrain load: f_i(a) = sum over elements and Gauss points of
 * |J| (dim lam + 2 mu) e0(|x_q|) d_i phi_a(x_q); 0 on the fixed components.
 * Evaluated in FP64.  Asynchronous. */
int pf_el_rhs(pf_ctx* ctx, const pf_elastic* p, void* f, void* stream);

/* Solve K u = b by conjugate gradients from u = 0 until ||r|| <= rtol ||b||
 * or maxit iterations; b = NULL solves for the eigenstrain load.  When every
 * axis has an odd node count of at least 5, the CG is preconditioned by a
 * geometric multigrid V-cycle: the grid halves while that holds (rep->levels
 * grids), Q1 rediscretised at 2h, trilinear transfers, two damped-Jacobi sweeps
 * before and after and 2 x (longest axis) on the coarsest grid (4 to 32),
 * damping 1.6 / lambda_max of D^-1 K.  lambda_max depends on dim and nu
 * only; the first solve of a (dim, nu) pair on a context estimates it by
 * power iteration on a 9^d grid (about a millisecond).  Other grids, or
 * pf_tune_set(PF_TUNE_EL_MG, 1), use plain CG.  The fixed components are identity rows of K (u there matches b to
 * the tolerance).  Host-synchronous; returns PF_OK, PF_ENOCONV (u holds the
 * last iterate) or PF_ENONFINITE; rep may be NULL. */
int pf_el_solve(pf_ctx* ctx, const pf_elastic* p, const void* b, void* u, double rtol, int32_t maxit,
                pf_el_report* rep, void* ws, void* stream);

/* out[0] (device double) = g . u, accumulated in FP64 in a fixed order;
 * g = NULL selects the volume change int div u dV of Eq. 21 (the outward
 * face-normal component of u weighted by each node's face share).
 * Asynchronous. */
int pf_el_objective(pf_ctx* ctx, const pf_elastic* p, const void* g, const void* u, double* out, void* ws,
                    void* stream);

/* Sensitivities of O = g . u (g = NULL: the volume change) at the equilibrium u
 * (as returned by pf_el_solve) with respect to theta = (E, nu), by the adjoint
 * method of Eq. 18: solve K lambda = g (fixed components of g ignored), then
 * dO/dtheta = lambda . (df/dtheta - dK/dtheta u).  out (host, 3 doubles) =
 * {O, dO/dE, dO/dnu}.  Host-synchronous; the adjoint solve uses rtol / maxit. */
int pf_el_sensitivity(pf_ctx* ctx, const pf_elastic* p, const void* g, const void* u, double* out,
                      double rtol, int32_t maxit, pf_el_report* rep, void* ws, void* stream);

/* ---------------------------------------------------------------------- */
/* Learned K-step surrogate for 2-D Cahn-Hilliard (added by this library;  */
/* the paper has no learned component).  BF16 matrix-core kernels with     */
/* FP32 accumulation; FP32 master parameters.                              */
/* ---------------------------------------------------------------------- */
/* Network: a0 = (c, M, kappa) per pixel; three 3x3 periodic convolutions of
 * width 32 with bias and relu; a 3x3 convolution to one channel d;
 * c_hat = c + d - mean(d) per sample (mass conserved exactly).
 * Parameters (FP32, this order): W1 [3][3][3][32], b1 [32], W2 [3][3][32][32],
 * b2 [32], W3 [3][3][32][32], b3 [32], W4 [3][3][32], b4 [1]; W[ky][kx][cin][cout]
 * multiplies the input at (y + ky - 1, x + kx - 1).  Inputs, weights and hidden
 * activations (and their gradients) are rounded to bfloat16, ties to even. */
int pf_nn_param_count(void);

/* Workspace bytes for B samples of H x W pixels (W a multiple of 32). */
int pf_nn_workspace_size(int B, int H, int W, size_t* bytes);

/* c_hat [B, H, W] from c [B, H, W], M [B], kappa [B] (all FP32 device). */
int pf_nn_forward(const float* params, int B, int H, int W, const float* c, const float* M,
                  const float* kappa, float* c_hat, void* ws, void* stream);

/* Forward and backward: grad (FP32 device, pf_nn_param_count values) = dL/dparams of
 * L = sum_b mean_p (c_hat - target)^2; loss (device, B doubles, may be NULL) gets
 * each sample's mean squared error.  Asynchronous. */
int pf_nn_backward(const float* params, int B, int H, int W, const float* c, const float* M,
                   const float* kappa, const float* target, double* loss, float* grad, void* ws,
                   void* stream);

/* One bias-corrected Adam step (step count t >= 1) on params with moments m, v. */
int pf_nn_adam(float* params, float* m, float* v, const float* grad, int t, double lr,
               double beta1, double beta2, double eps, void* stream);

/* Residual check of a surrogate jump c_prev -> c_hat over K steps of size dt, given
 * c_step = one explicit step of c_hat (so (c_hat - c_step)/dt = M K mu(c_hat)/m).
 * Per sample, out[3 b + 0] = ||R_BE|| / ||m (c_hat - c_prev)/(K dt)|| with the
 * backward-Euler residual R_BE of Eq. 14 for the jump; out[3 b + 1] =
 * sum (c_hat - c_prev); out[3 b + 2] = ||c_hat - c_prev|| / (K dt).  FP64 sums. */
int pf_nn_check(int B, int H, int W, const float* c_hat, const float* c_prev, const float* c_step,
                double K_dt, double dt, double* out, void* ws, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* PF_H */
