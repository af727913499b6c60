// krylov.hpp -- launchers of the GMRES vector kernels (k_krylov.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace pfk {

// number of partial-sum blocks used for vectors of length n (fixed per n)
int krylov_blocks(long long n);

// largest basis handled by one Gram-Schmidt step
constexpr int KR_MAXK = 32;
// Outputs of one Gram-Schmidt step: device buffers (h1, h2: KR_MAXK + 1
// doubles, nrm2: 1), and optional host-mapped copies of the same values
// (written with system-scope stores; null to skip).
struct KrOut {
    double *h1, *h2, *nrm2;
    double *host_h1, *host_h2, *host_nrm2;
};
// One Arnoldi orthogonalisation of w against the k basis vectors V (N nodes, 1
// plane for model 0, 2 for model 1, 3 for model 2; leading dimension ld),
// classical Gram-Schmidt with selective re-orthogonalisation:
//   h1[0..k) = V^T w, h1[k] = ||w||^2;
//   if ||w||^2 - ||h1||^2 >= ||w||^2 / 10 (one projection is enough): h2 = 0,
//     nrm2[0] = ||w - V h1||^2, vnext = (w - V h1) / sqrt(nrm2[0]), w untouched;
//   else: w <- w - V h1, h2[0..k) = V^T w, h2[k] = ||w||^2,
//     nrm2[0] = ||w - V h2||^2, vnext = (w - V h2) / sqrt(nrm2[0]);
//   (vnext = 0 if nrm2[0] is 0), z = P^-1 vnext.  The Hessenberg column is h1 + h2.
//   part: (k + 1) * krylov_blocks(n) doubles.  Returns -1 (nothing launched) for k
//   outside 1..KR_MAXK.
template <typename T>
int kr_cgs2(int model, const T* V, long long ld, int k, T* w, T* vnext, T* z, const T* pinv,
            long long N, double* part, const KrOut& o, hipStream_t s, int tr = 0);
// out[0] = ||a - b||^2 (b may be null); host: optional host-mapped copy
template <typename T>
void kr_norm2(const T* a, const T* b, long long n, double* part, double* out, hipStream_t s,
              double* host = nullptr);
// v = sign * w / sqrt(nrm2[0]) ; z = P^-1 v (pinv null: identity; z null: skipped;
// tr = 1: transposed blocks).  N = nodes (the vectors hold 1, 2 or 3 planes; blocks
// 1x1, 2x2 or 3x3 per node).
template <typename T>
void kr_normalize_prec(int model, const T* w, const double* nrm2, T* v, T* z, const T* pinv,
                       long long N, double sign, hipStream_t s, int tr = 0);
// x += P^-1 (V y)
template <typename T>
void kr_update(int model, const T* V, long long ld, int k, const double* y, const T* pinv, T* x,
               long long N, hipStream_t s, int tr = 0);
// w = b - w
template <typename T>
void kr_rsub(const T* b, T* w, long long n, hipStream_t s);
// y = alpha x
template <typename T>
void kr_scale(const T* x, T* y, double alpha, long long n, hipStream_t s);
// x += y ; out[0] = max|y|, out[1] = max|x| (part: 2 krylov_blocks(n) doubles;
// host: optional host-mapped copy of out)
template <typename T>
void kr_add_maxabs(T* x, const T* y, long long n, double* part, double* out, hipStream_t s,
                   double* host = nullptr);

// ---- preconditioned conjugate gradients (symmetric positive definite J) ----
// Scalars live on the device (state: CG_NSTATE doubles); every block of a step
// kernel reduces the previous kernel's partial sums in the same fixed order, so
// all blocks agree on alpha and beta without a separate reduction launch.  The
// host reads a pinned mirror (its, done, r.r) once per iteration.
enum { CG_RZ = 0, CG_RZOLD = 1, CG_TOL2 = 2, CG_ITS = 3, CG_DONE = 4, CG_MAXIT = 5, CG_RR = 6, CG_NSTATE = 8 };
enum { CG_H_ITS = 0, CG_H_DONE = 1, CG_H_RR = 2 };
enum { CG_CONVERGED = 1, CG_MAXITS = 2, CG_BREAKDOWN = 3, CG_NONFINITE = 4 };
// partial-sum blocks of the CG kernels for n unknowns (2 doubles each in part)
int cg_blocks(long long n);
// x = 0, r = b, z = P^-1 b, p = 0; partials (r.z, r.r); state reset (stop when
// r.r <= tol2 or after maxit iterations); host mirror cleared
template <typename T>
void cg_start(const T* b, const T* pinv, T* r, T* z, T* p, T* x, long long n, double* part, double* st,
              double* host, double tol2, int maxit, hipStream_t s);
// the stop tests on (r.z, r.r); beta; p = z + beta p
template <typename T>
void cg_dir(const T* z, T* p, long long n, const double* part, double* st, double* host, hipStream_t s);
// partials of p.q (q = J p)
template <typename T>
void cg_pq(const T* p, const T* q, long long n, double* part2, const double* st, hipStream_t s);
// alpha = r.z / p.q; x += alpha p, r -= alpha q, z = P^-1 r; partials (r.z, r.r).
// nb2: the number of p.q partials in part2 (0: cg_blocks(n), as cg_pq writes them)
template <typename T>
void cg_alpha(T* x, T* r, T* z, const T* p, const T* q, const T* pinv, long long n, const double* part2,
              double* part, double* st, double* host, hipStream_t s, int nb2 = 0);

}  // namespace pfk
