// node_common.hpp -- device helpers of the node-centric kernels.
//
// One thread owns one node.  It reads the 3^d neighbourhood of the node and
// evaluates the node's row of the weak form directly, summing over the 2^d
// elements that share the node (no atomics, fixed summation order):
//   nonlinear term  N(u)_a = sum_e sum_q |J| f'(u_q) phi_a(q)        (Eqs. 5-6, 10)
//   gradient term   (K u)_a = sum_e sum_q |J| grad u_q . grad phi_a   (exact: a closed
//                   tensor stencil, K = sum_k Khat_k (x) Mhat_others, Khat = [-1 2 -1]/h,
//                   Mhat = h [1 4 1] / 6)
// The 4^d quadrature values of the 2^d elements are produced by sum
// factorisation: interp3to4 along x, then y (then z).
#pragma once
#include "device.hpp"
#include "kernels.hpp"

namespace pfk {
namespace {

template <int D>
struct NB {
    static constexpr int K = D == 2 ? 9 : 27;
};

// neighbour i + d (d = -1, +1) of node i on an axis of n nodes: periodic wrap,
// or reflection about the end node on a no-flux grid
__device__ __forceinline__ int nbr(int i, int d, int n, int bc)
{
    const int t = i + d;
    if (bc) return t < 0 ? 1 : (t >= n ? n - 2 : t);
    return t < 0 ? t + n : (t >= n ? t - n : t);
}

// 2^b for a node on b boundary faces of a no-flux grid (1 on periodic grids)
template <int D>
__device__ __forceinline__ int bfactor(const Geom& g, int i, int j, int k)
{
    if (!g.bc) return 1;
    int b = (i == 0 || i == g.n[0] - 1) + (j == 0 || j == g.n[1] - 1);
    if (D == 3) b += (k == 0 || k == g.n[2] - 1);
    return 1 << b;
}

// Neighbourhood index: (dx+1) + 3 (dy+1) + 9 (dz+1).  SCALED multiplies every
// gathered value by its node's 2^b (used where an operator acts on D u).
template <typename T, int D, bool SCALED = false>
__device__ __forceinline__ void gather(const T* __restrict__ u, const Geom& g, int i, int j, int k,
                                       T out[NB<D>::K])
{
    const int xs[3] = {nbr(i, -1, g.n[0], g.bc), i, nbr(i, 1, g.n[0], g.bc)};
    const int ys[3] = {nbr(j, -1, g.n[1], g.bc), j, nbr(j, 1, g.n[1], g.bc)};
    T fx[3] = {(T)1, (T)1, (T)1}, fy[3] = {(T)1, (T)1, (T)1}, fz[3] = {(T)1, (T)1, (T)1};
    if (SCALED && g.bc) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            fx[a] = (T)(1 << edge_count(xs[a], g.n[0]));
            fy[a] = (T)(1 << edge_count(ys[a], g.n[1]));
        }
    }
    if constexpr (D == 2) {
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                out[a + 3 * b] = u[(long long)ys[b] * g.n[0] + xs[a]];
                if (SCALED) out[a + 3 * b] *= fx[a] * fy[b];
            }
    } else {
        const int zs[3] = {nbr(k, -1, g.n[2], g.bc), k, nbr(k, 1, g.n[2], g.bc)};
        if (SCALED && g.bc)
#pragma unroll
            for (int c = 0; c < 3; ++c) fz[c] = (T)(1 << edge_count(zs[c], g.n[2]));
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int b = 0; b < 3; ++b)
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    out[a + 3 * b + 9 * c] =
                        u[((long long)zs[c] * g.n[1] + ys[b]) * g.n[0] + xs[a]];
                    if (SCALED) out[a + 3 * b + 9 * c] *= fx[a] * fy[b] * fz[c];
                }
    }
}

// Unit-coefficient Q1 stiffness row at the centre node (2-D: h-free; 3-D: times h).
template <typename T, int D>
__device__ __forceinline__ T stiff(const T* u, T h)
{
    if constexpr (D == 2) {
        T kx[3], mx[3];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            kx[b] = (T)2 * u[1 + 3 * b] - u[3 * b] - u[2 + 3 * b];
            mx[b] = (T)4 * u[1 + 3 * b] + u[3 * b] + u[2 + 3 * b];
        }
        const T km = kx[0] + (T)4 * kx[1] + kx[2];  // Khat_x (x) Mhat_y
        const T mk = (T)2 * mx[1] - mx[0] - mx[2];  // Mhat_x (x) Khat_y
        return (km + mk) * (T)(1.0 / 6.0);
    } else {
        T km[3], mk[3], mm[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            T kx[3], mx[3];
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const T* r = u + 3 * b + 9 * c;
                kx[b] = (T)2 * r[1] - r[0] - r[2];
                mx[b] = (T)4 * r[1] + r[0] + r[2];
            }
            km[c] = kx[0] + (T)4 * kx[1] + kx[2];
            mk[c] = (T)2 * mx[1] - mx[0] - mx[2];
            mm[c] = mx[0] + (T)4 * mx[1] + mx[2];
        }
        const T a = (km[0] + mk[0]) + (T)4 * (km[1] + mk[1]) + (km[2] + mk[2]);  // (..) (x) Mhat_z
        const T b = (T)2 * mm[1] - mm[0] - mm[2];                              // Mhat Mhat Khat_z
        return (a + b) * h * (T)(1.0 / 36.0);
    }
}

// sum_q w_q F(u_q[, v_q]) over the 4^D quadrature points around the centre node;
// w = tensor product of (GM, GP, GP, GM).  |J| is applied by the caller.
template <typename T, int D, bool WITHV, typename Fn>
__device__ __forceinline__ T quad_sum(const T* u, const T* v, Fn F)
{
    if constexpr (D == 2) {
        T Xu[3][4], Xv[3][4];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            interp3to4(u[3 * b], u[3 * b + 1], u[3 * b + 2], Xu[b]);
            if constexpr (WITHV) interp3to4(v[3 * b], v[3 * b + 1], v[3 * b + 2], Xv[b]);
        }
        T col[4];
#pragma unroll
        for (int qx = 0; qx < 4; ++qx) {
            T qu[4], qv[4], fv[4];
            interp3to4(Xu[0][qx], Xu[1][qx], Xu[2][qx], qu);
            if constexpr (WITHV) interp3to4(Xv[0][qx], Xv[1][qx], Xv[2][qx], qv);
#pragma unroll
            for (int qy = 0; qy < 4; ++qy) fv[qy] = F(qu[qy], WITHV ? qv[qy] : (T)0);
            col[qx] = wsum4(fv);
        }
        return wsum4(col);
    } else {
        T Xu[9][4], Xv[9][4];
#pragma unroll
        for (int r = 0; r < 9; ++r) {
            interp3to4(u[3 * r], u[3 * r + 1], u[3 * r + 2], Xu[r]);
            if constexpr (WITHV) interp3to4(v[3 * r], v[3 * r + 1], v[3 * r + 2], Xv[r]);
        }
        T plane[4];
#pragma unroll
        for (int qx = 0; qx < 4; ++qx) {
            T Yu[3][4], Yv[3][4];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                interp3to4(Xu[3 * c][qx], Xu[3 * c + 1][qx], Xu[3 * c + 2][qx], Yu[c]);
                if constexpr (WITHV)
                    interp3to4(Xv[3 * c][qx], Xv[3 * c + 1][qx], Xv[3 * c + 2][qx], Yv[c]);
            }
            T row[4];
#pragma unroll
            for (int qy = 0; qy < 4; ++qy) {
                T qu[4], qv[4], fv[4];
                interp3to4(Yu[0][qy], Yu[1][qy], Yu[2][qy], qu);
                if constexpr (WITHV) interp3to4(Yv[0][qy], Yv[1][qy], Yv[2][qy], qv);
#pragma unroll
                for (int qz = 0; qz < 4; ++qz) fv[qz] = F(qu[qz], WITHV ? qv[qz] : (T)0);
                row[qy] = wsum4(fv);
            }
            plane[qx] = wsum4(row);
        }
        return wsum4(plane);
    }
}

// sum_q w_q^2 F(u_q): the diagonal entry sum_e sum_q f''(u_q) phi_a(q)^2 (no |J|)
template <typename T, int D, typename Fn>
__device__ __forceinline__ T quad_sum_sq(const T* u, Fn F)
{
    const T w2[4] = {(T)(GM * GM), (T)(GP * GP), (T)(GP * GP), (T)(GM * GM)};
    auto ws = [&](const T v[4]) { return w2[0] * v[0] + w2[1] * v[1] + w2[2] * v[2] + w2[3] * v[3]; };
    if constexpr (D == 2) {
        T Xu[3][4];
#pragma unroll
        for (int b = 0; b < 3; ++b) interp3to4(u[3 * b], u[3 * b + 1], u[3 * b + 2], Xu[b]);
        T col[4];
#pragma unroll
        for (int qx = 0; qx < 4; ++qx) {
            T qu[4], fv[4];
            interp3to4(Xu[0][qx], Xu[1][qx], Xu[2][qx], qu);
#pragma unroll
            for (int qy = 0; qy < 4; ++qy) fv[qy] = F(qu[qy], (T)1);
            col[qx] = ws(fv);
        }
        return ws(col);
    } else {
        T Xu[9][4];
#pragma unroll
        for (int r = 0; r < 9; ++r) interp3to4(u[3 * r], u[3 * r + 1], u[3 * r + 2], Xu[r]);
        T plane[4];
#pragma unroll
        for (int qx = 0; qx < 4; ++qx) {
            T Yu[3][4];
#pragma unroll
            for (int c = 0; c < 3; ++c) interp3to4(Xu[3 * c][qx], Xu[3 * c + 1][qx], Xu[3 * c + 2][qx], Yu[c]);
            T row[4];
#pragma unroll
            for (int qy = 0; qy < 4; ++qy) {
                T qu[4], fv[4];
                interp3to4(Yu[0][qy], Yu[1][qy], Yu[2][qy], qu);
#pragma unroll
                for (int qz = 0; qz < 4; ++qz) fv[qz] = F(qu[qz], (T)1);
                row[qy] = ws(fv);
            }
            plane[qx] = ws(row);
        }
        return ws(plane);
    }
}

// sum_q w_q^2 F(u_q, v_q) over the 4^D points (w = phi of the centre node): the
// diagonal entry of a two-field second-derivative operator (no |J|)
template <typename T, int D, typename Fn>
__device__ __forceinline__ T quad_sum_sq2(const T* u, const T* v, Fn F)
{
    const T w2[4] = {(T)(GM * GM), (T)(GP * GP), (T)(GP * GP), (T)(GM * GM)};
    auto ws = [&](const T x[4]) { return w2[0] * x[0] + w2[1] * x[1] + w2[2] * x[2] + w2[3] * x[3]; };
    if constexpr (D == 2) {
        T Xu[3][4], Xv[3][4];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            interp3to4(u[3 * b], u[3 * b + 1], u[3 * b + 2], Xu[b]);
            interp3to4(v[3 * b], v[3 * b + 1], v[3 * b + 2], Xv[b]);
        }
        T col[4];
#pragma unroll
        for (int qx = 0; qx < 4; ++qx) {
            T qu[4], qv[4], fv[4];
            interp3to4(Xu[0][qx], Xu[1][qx], Xu[2][qx], qu);
            interp3to4(Xv[0][qx], Xv[1][qx], Xv[2][qx], qv);
#pragma unroll
            for (int qy = 0; qy < 4; ++qy) fv[qy] = F(qu[qy], qv[qy]);
            col[qx] = ws(fv);
        }
        return ws(col);
    } else {
        T Xu[9][4], Xv[9][4];
#pragma unroll
        for (int r = 0; r < 9; ++r) {
            interp3to4(u[3 * r], u[3 * r + 1], u[3 * r + 2], Xu[r]);
            interp3to4(v[3 * r], v[3 * r + 1], v[3 * r + 2], Xv[r]);
        }
        T plane[4];
#pragma unroll
        for (int qx = 0; qx < 4; ++qx) {
            T Yu[3][4], Yv[3][4];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                interp3to4(Xu[3 * c][qx], Xu[3 * c + 1][qx], Xu[3 * c + 2][qx], Yu[c]);
                interp3to4(Xv[3 * c][qx], Xv[3 * c + 1][qx], Xv[3 * c + 2][qx], Yv[c]);
            }
            T row[4];
#pragma unroll
            for (int qy = 0; qy < 4; ++qy) {
                T qu[4], qv[4], fv[4];
                interp3to4(Yu[0][qy], Yu[1][qy], Yu[2][qy], qu);
                interp3to4(Yv[0][qy], Yv[1][qy], Yv[2][qy], qv);
#pragma unroll
                for (int qz = 0; qz < 4; ++qz) fv[qz] = F(qu[qz], qv[qz]);
                row[qy] = ws(fv);
            }
            plane[qx] = ws(row);
        }
        return ws(plane);
    }
}

// diagonal entry of the unit Q1 stiffness at any periodic node
// Consistent Q1 mass on a gathered 3^d neighbourhood: the tensor product of the
// 1-D (h/6)(1, 4, 1) (2-point Gauss integrates phi_a phi_b exactly).
template <typename T, int D>
__device__ __forceinline__ T cmass(const T* u, T h)
{
    if constexpr (D == 2) {
        T mx[3];
#pragma unroll
        for (int b = 0; b < 3; ++b) mx[b] = (T)4 * u[1 + 3 * b] + u[3 * b] + u[2 + 3 * b];
        return (mx[0] + (T)4 * mx[1] + mx[2]) * h * h * (T)(1.0 / 36.0);
    } else {
        T mm[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            T mx[3];
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const T* r = u + 3 * b + 9 * c;
                mx[b] = (T)4 * r[1] + r[0] + r[2];
            }
            mm[c] = mx[0] + (T)4 * mx[1] + mx[2];
        }
        return (mm[0] + (T)4 * mm[1] + mm[2]) * h * h * h * (T)(1.0 / 216.0);
    }
}

template <typename T, int D>
__device__ __forceinline__ T stiff_diag(T h)
{
    return D == 2 ? (T)(8.0 / 3.0) : (T)(8.0 / 3.0) * h;
}

// Gauss-Lobatto (nodal) quadrature: the quadrature points are the nodes, so the
// nonlinear term is m f'(u_a) at the node and the Q1 stiffness integrated at the
// nodes is the unit 5-point stencil (2-D, h-free) or h times the 7-point one (3-D).
template <typename T, int D>
__device__ __forceinline__ T stiff_lob(const T* u, T h)
{
    if constexpr (D == 2) {
        return (T)4 * u[4] - ((u[3] + u[5]) + (u[1] + u[7]));
    } else {
        return ((T)6 * u[13] - ((u[12] + u[14]) + (u[10] + u[16]) + (u[4] + u[22]))) * h;
    }
}

template <typename T, int D>
__device__ __forceinline__ T stiff_lob_diag(T h)
{
    return D == 2 ? (T)4 : (T)6 * h;
}

// the stiffness row of the grid's quadrature
template <typename T, int D>
__device__ __forceinline__ T stiff_q(const Geom& g, const T* u, T h)
{
    return g.quad ? stiff_lob<T, D>(u, h) : stiff<T, D>(u, h);
}

template <int D>
__device__ __forceinline__ bool node_of(const Geom& g, long long idx, int& i, int& j, int& k)
{
    if (idx >= g.N) return false;
    if (g.N <= 0xffffffffll) {
        // 32-bit division (a 64-bit one is a long instruction sequence on the GPU)
        const unsigned u = (unsigned)idx, n0 = (unsigned)g.n[0], n1 = (unsigned)g.n[1];
        const unsigned r = u / n0;
        i = (int)(u - r * n0);
        if (D == 3) {
            const unsigned r2 = r / n1;
            j = (int)(r - r2 * n1);
            k = (int)r2;
        } else {
            j = (int)r;
            k = 0;
        }
        return true;
    }
    i = (int)(idx % g.n[0]);
    long long r = idx / g.n[0];
    j = (int)(r % g.n[1]);
    k = D == 3 ? (int)(r / g.n[1]) : 0;
    return true;
}

template <typename T>
struct Cub {
    T a1, a2, a3;
    __device__ T operator()(T q, T) const { return cubic(q, a1, a2, a3); }
};
template <typename T>
struct Lin {  // f''(q) v
    T b0, b1, b2;
    __device__ T operator()(T q, T v) const { return fmaT(fmaT(b2, q, b1), q, b0) * v; }
};

}  // namespace
}  // namespace pfk
