// device.hpp -- gfx950 device helpers shared by the phase-field kernels.
//
// Q1 element, 2-point Gauss-Legendre rule.  Along one axis an element has two
// nodes (local a = 0, 1) and two quadrature points xi = -1/sqrt(3), +1/sqrt(3);
// the 1-D shape-function values there are
//     B[q][a] = [[GP, GM], [GM, GP]],  GP = (1 + 1/sqrt(3))/2, GM = (1 - 1/sqrt(3))/2,
// and the d-dimensional values are tensor products.  B is symmetric, so the
// same two numbers interpolate nodal values to the quadrature points and
// scatter quadrature contributions back to the nodes.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pfk {

constexpr double GP = 0.78867513459481288225457439025098;  // (1 + 1/sqrt 3) / 2
constexpr double GM = 0.21132486540518711774542560974902;  // (1 - 1/sqrt 3) / 2

constexpr int WAVE = 64;

// ---- cross-lane moves inside one 64-lane wavefront (DPP, no LDS) ----------
// wave_shr:1 -> lane i receives lane i-1; wave_shl:1 -> lane i receives lane i+1.
// Lanes without a source (0 resp. 63) receive 0; callers treat those lanes as
// halo and never use what they compute.
constexpr int DPP_WAVE_SHL1 = 0x130;
constexpr int DPP_WAVE_SHR1 = 0x138;

__device__ __forceinline__ int dpp_i32_from_left(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, DPP_WAVE_SHR1, 0xf, 0xf, false);
}
__device__ __forceinline__ int dpp_i32_from_right(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, DPP_WAVE_SHL1, 0xf, 0xf, false);
}

__device__ __forceinline__ float from_left(float v)
{
    return __int_as_float(dpp_i32_from_left(__float_as_int(v)));
}
__device__ __forceinline__ float from_right(float v)
{
    return __int_as_float(dpp_i32_from_right(__float_as_int(v)));
}
__device__ __forceinline__ double from_left(double v)
{
    long long b = __double_as_longlong(v);
    int lo = dpp_i32_from_left((int)(b & 0xffffffffll));
    int hi = dpp_i32_from_left((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double from_right(double v)
{
    long long b = __double_as_longlong(v);
    int lo = dpp_i32_from_right((int)(b & 0xffffffffll));
    int hi = dpp_i32_from_right((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// fused multiply-add with the operand type fixed (no promotion to double)
__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Cubic local-energy derivative in Horner form:  q * (a1 + q * (a2 + a3 q)).
// Both free energies of this library have f'(0) = 0, so f' has no constant
// term; the caller folds every constant factor into (a1, a2, a3).
template <typename T>
__device__ __forceinline__ T cubic(T q, T a1, T a2, T a3)
{
    return q * fmaT(fmaT(a3, q, a2), q, a1);
}

// Nodal values (u[-1], u[0], u[+1]) along one axis -> the 4 quadrature points
// of the two elements that share node 0 (lower element first).
template <typename T>
__device__ __forceinline__ void interp3to4(T a, T b, T c, T q[4])
{
    const T d0 = b - a, d1 = c - b;
    q[0] = fmaT((T)GM, d0, a);
    q[1] = fmaT((T)GP, d0, a);
    q[2] = fmaT((T)GM, d1, b);
    q[3] = fmaT((T)GP, d1, b);
}

// Weight of those 4 quadrature points in the centre node's shape function:
// phi_1 at the lower element's points, phi_0 at the upper element's points.
template <typename T>
__device__ __forceinline__ T wsum4(const T v[4])
{
    return (T)GM * (v[0] + v[3]) + (T)GP * (v[1] + v[2]);
}

__host__ __device__ __forceinline__ int wrap(int i, int n)
{
    return i < 0 ? i + n : (i >= n ? i - n : i);
}

// Node index i (any integer) reflected about the end nodes 0 and n - 1 (n >= 2):
// the even extension of a no-flux grid, period 2 (n - 1).
__host__ __device__ __forceinline__ int reflect(int i, int n)
{
    const int p = 2 * (n - 1);
    i %= p;
    if (i < 0) i += p;
    return i < n ? i : p - i;
}

// No-flux grids by reflection.  On the even extension of a field about the end
// nodes, every ghost element is the mirror image of a real element and adds the
// same contribution to the boundary node.  So at a node on b boundary faces the
// periodic-style node formula applied to reflected neighbours gives 2^b times
// the no-flux row (and the periodic lumped mass is 2^b times the no-flux one);
// dividing by 2^b restores the row, and ratios such as r/m need no correction.
__host__ __device__ __forceinline__ int edge_count(int i, int n) { return (i == 0) + (i == n - 1); }

}  // namespace pfk
