// krylov.hpp -- launchers of the GMRES vector kernels (k_krylov.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace pfk {

// number of partial-sum blocks used for vectors of length n (fixed per n)
int krylov_blocks(long long n);

// out[0..k) (+)= V^T w ; part: k * krylov_blocks(n) doubles
template <typename T>
void kr_mdot(const T* V, long long ld, int k, const T* w, long long n, double* part, double* out,
             int accumulate, hipStream_t s);
// w -= V h ; out[0..k) = V^T w
template <typename T>
void kr_axpy_mdot(const T* V, long long ld, int k, const double* h, T* w, long long n, double* part,
                  double* out, hipStream_t s);
// w -= V h ; out[0] = ||w||^2
template <typename T>
void kr_axpy_norm(const T* V, long long ld, int k, const double* h, T* w, long long n, double* part,
                  double* out, hipStream_t s);
// out[0] = ||a - b||^2 (b may be null)
template <typename T>
void kr_norm2(const T* a, const T* b, long long n, double* part, double* out, hipStream_t s);
// v = sign * w / sqrt(nrm2[0]) ; z = P^-1 v (pinv null: identity; z null: skipped;
// tr = 1: transposed 2x2 blocks).  N = nodes (the vectors hold 1 or 2 planes).
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
// x += y ; part[2b] = max|y|, part[2b+1] = max|x| per block (krylov_blocks(n) blocks)
template <typename T>
void kr_add_maxabs(T* x, const T* y, long long n, double* part, hipStream_t s);

}  // namespace pfk
