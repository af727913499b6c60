// k_jvp3d.hip -- Jacobian product of the 3-D backward-Euler residual (Eqs. 13-14)
// by element-wise sum factorisation, marching along z through an LDS tile.
//
// The node-centric kernel evaluates, for every node, the 64 quadrature points of
// its 8 elements; every point is thus evaluated 8 times.  Here every element is
// evaluated once per tile:
//   - a block owns 15 x 15 output columns (x, y) and a run of tz planes in z;
//   - the 17 x 17 node patch (one halo node on each side, wrapped on periodic
//     grids, reflected about the end nodes on no-flux grids) of every z-plane is
//     staged in LDS; the 16 x 16 elements of each slab between two planes are
//     computed one per thread: nodal c and v interpolated to the 8 Gauss points
//     (three 1-D passes), f''(c_q) v_q |J| formed there and scattered back to the
//     8 element nodes (the transposed passes);
//   - each node sums the loads of its 8 elements: 4 from the slab below its
//     plane, 4 from the slab above (fixed order, no atomics);
//   - the stiffness term uses the closed 27-point Q1 stencil, factored per plane:
//     when a plane arrives each node forms (Khat Mhat + Mhat Khat) and Mhat Mhat of
//     its 3 x 3 in-plane patch, and keeps the last three planes in registers.
// Work per node: one element (x 1.14 for the tile halo) plus the stencil, against
// 8 elements' worth of quadrature in the node-centric kernel.
#include <cmath>

#include "device.hpp"
#include "kernels.hpp"

namespace pfk {
namespace {

constexpr int OT = 15;           // output nodes per tile edge (x and y)
constexpr int ET = OT + 1;       // elements per tile edge
constexpr int PT = OT + 2;       // staged nodes per tile edge
constexpr int PA = PT * PT;      // staged nodes per plane
constexpr int NT = ET * ET;      // threads per block (one element each)
static_assert(NT == 256, "one element per thread");

template <typename T>
__device__ __forceinline__ void lerp2(T a, T b, T& q0, T& q1)
{
    const T d = b - a;
    q0 = fmaT((T)GM, d, a);
    q1 = fmaT((T)GP, d, a);
}

// transpose of lerp2: the two point values back to the two nodes
template <typename T>
__device__ __forceinline__ void spread2(T p0, T p1, T& r0, T& r1)
{
    r0 = fmaT((T)GP, p0, (T)GM * p1);
    r1 = fmaT((T)GM, p0, (T)GP * p1);
}

// Nodal loads r[az][ay][ax] = sum_q phi_a(q) |J| f''(c_q) v_q of one element
// from its nodal values c, v (same indexing); b0..b2 carry |J|.
template <typename T>
__device__ __forceinline__ void element_loads(const T (&c)[2][2][2], const T (&v)[2][2][2], T b0,
                                              T b1, T b2, T (&r)[2][2][2])
{
    T cx[2][2][2], vx[2][2][2];  // [az][ay][qx]
#pragma unroll
    for (int az = 0; az < 2; ++az)
#pragma unroll
        for (int ay = 0; ay < 2; ++ay) {
            lerp2(c[az][ay][0], c[az][ay][1], cx[az][ay][0], cx[az][ay][1]);
            lerp2(v[az][ay][0], v[az][ay][1], vx[az][ay][0], vx[az][ay][1]);
        }
    T cy[2][2][2], vy[2][2][2];  // [az][qy][qx]
#pragma unroll
    for (int az = 0; az < 2; ++az)
#pragma unroll
        for (int qx = 0; qx < 2; ++qx) {
            lerp2(cx[az][0][qx], cx[az][1][qx], cy[az][0][qx], cy[az][1][qx]);
            lerp2(vx[az][0][qx], vx[az][1][qx], vy[az][0][qx], vy[az][1][qx]);
        }
    T p[2][2][2];  // [qz][qy][qx]
#pragma unroll
    for (int qy = 0; qy < 2; ++qy)
#pragma unroll
        for (int qx = 0; qx < 2; ++qx) {
            T cq[2], vq[2];
            lerp2(cy[0][qy][qx], cy[1][qy][qx], cq[0], cq[1]);
            lerp2(vy[0][qy][qx], vy[1][qy][qx], vq[0], vq[1]);
#pragma unroll
            for (int qz = 0; qz < 2; ++qz) p[qz][qy][qx] = fmaT(fmaT(b2, cq[qz], b1), cq[qz], b0) * vq[qz];
        }
    T sz[2][2][2];  // [az][qy][qx]
#pragma unroll
    for (int qy = 0; qy < 2; ++qy)
#pragma unroll
        for (int qx = 0; qx < 2; ++qx) spread2(p[0][qy][qx], p[1][qy][qx], sz[0][qy][qx], sz[1][qy][qx]);
    T sy[2][2][2];  // [az][ay][qx]
#pragma unroll
    for (int az = 0; az < 2; ++az)
#pragma unroll
        for (int qx = 0; qx < 2; ++qx) spread2(sz[az][0][qx], sz[az][1][qx], sy[az][0][qx], sy[az][1][qx]);
#pragma unroll
    for (int az = 0; az < 2; ++az)
#pragma unroll
        for (int ay = 0; ay < 2; ++ay) spread2(sy[az][ay][0], sy[az][ay][1], r[az][ay][0], r[az][ay][1]);
}

// In-plane factors of the unit 3-D Q1 stiffness at the centre of a 3 x 3 patch:
// s = (Khat_x Mhat_y + Mhat_x Khat_y) u, mm = (Mhat_x Mhat_y) u (Khat = [-1 2 -1],
// Mhat = [1 4 1]; the scale h / 36 is applied by the caller).
template <typename T>
__device__ __forceinline__ void plane_factors(const T* L, int ly, int lx, T& s, T& mm)
{
    T kx[3], mx[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const T* r = L + (ly - 1 + b) * PT + lx - 1;
        kx[b] = (T)2 * r[1] - r[0] - r[2];
        mx[b] = (T)4 * r[1] + r[0] + r[2];
    }
    s = (kx[0] + (T)4 * kx[1] + kx[2]) + ((T)2 * mx[1] - mx[0] - mx[2]);
    mm = mx[0] + (T)4 * mx[1] + mx[2];
}

// ring of the last three planes' stiffness factors and centre values of one field
template <typename T>
struct PlaneRing {
    T s[3], mm[3], c[3];
    __device__ __forceinline__ void push(T s2, T m2, T c2)
    {
        s[0] = s[1]; s[1] = s[2]; s[2] = s2;
        mm[0] = mm[1]; mm[1] = mm[2]; mm[2] = m2;
        c[0] = c[1]; c[1] = c[2]; c[2] = c2;
    }
    // unit stiffness row at the middle plane, times h / 36
    __device__ __forceinline__ T stiff(T h36) const
    {
        return ((s[0] + (T)4 * s[1] + s[2]) + ((T)2 * mm[1] - mm[0] - mm[2])) * h36;
    }
};

// MODEL 0 (Allen-Cahn): fields {c, v};  Jv = inv_dt m v + L (N'(c) v + kappa K v)
// MODEL 1 (Cahn-Hilliard): fields {c, v_c, v_mu};
//   TRANS 0: [inv_dt m v_c + M K v_mu ;  m v_mu - (N'(c) v_c + kappa K v_c)]
//   TRANS 1: [inv_dt m v_c - (N'(c) v_mu + kappa K v_mu) ;  M K v_c + m v_mu]
template <typename T, int MODEL, int TRANS>
__global__ __launch_bounds__(NT) void k_jvp3d(const T* __restrict__ U, const T* __restrict__ V,
                                              T* __restrict__ Jv, Geom g, T b0, T b1, T b2,
                                              T kappa, T mob, T m, T inv_dt, T h36, int tz)
{
    constexpr int NF = MODEL == 0 ? 2 : 3;  // staged fields: c, then the direction plane(s)
    constexpr int VN = MODEL == 0 ? 1 : 1 + TRANS;  // staged field the f'' term acts on
    constexpr int NLD = (NF * PA + NT - 1) / NT;    // staged values per thread per plane
    __shared__ T pl[2][NF * PA + 1];    // two planes of the staged fields (+1 spare word)
    __shared__ T eb[4][NT], et[2][4][NT];  // element loads: bottom corners, top corners (2 slabs)

    const int n0 = g.n[0], n1 = g.n[1], n2 = g.n[2];
    const long long plane = (long long)n0 * n1;
    const int t = threadIdx.x;
    const int x0 = blockIdx.x * OT, y0 = blockIdx.y * OT, z0 = blockIdx.z * tz;
    const int nz = min(tz, n2 - z0);
    const int ox = min(OT, n0 - x0), oy = min(OT, n1 - y0);

    // this thread's staged values: source (field + in-plane offset, periodic wrap)
    // and LDS slot; slots past the patch read the plane's first U value (in
    // bounds) into a spare LDS word
    const T* ld_src[NLD];
    int ld_l[NLD];
#pragma unroll
    for (int k = 0; k < NLD; ++k) {
        const int q = t + k * NT;
        const int f = q < NF * PA ? q / PA : -1;
        const int r = q % PA;
        const int gx = g.bc ? reflect(x0 - 1 + r % PT, n0) : ((x0 - 1 + r % PT) % n0 + n0) % n0;
        const int gy = g.bc ? reflect(y0 - 1 + r / PT, n1) : ((y0 - 1 + r / PT) % n1 + n1) % n1;
        ld_src[k] = f < 0 ? U : (f == 0 ? U : (f == 1 ? V : V + g.N)) + (long long)gy * n0 + gx;
        ld_l[k] = f < 0 ? NF * PA : q;
    }
    auto fetch = [&](int p, T (&buf)[NLD]) {
        const long long zo = (long long)(g.bc ? reflect(p, n2) : ((p % n2) + n2) % n2) * plane;
#pragma unroll
        for (int k = 0; k < NLD; ++k) buf[k] = ld_src[k][zo];
    };

    const int ix = t % OT, iy = t / OT;  // output node of this thread (t < OT * OT)
    const bool node_thread = t < OT * OT;
    const int ex = t % ET, ey = t / ET;  // element of this thread (lower corner at patch (ex, ey))

    PlaneRing<T> ring[NF - 1];
#pragma unroll
    for (int f = 0; f < NF - 1; ++f)
#pragma unroll
        for (int i = 0; i < 3; ++i) ring[f].s[i] = ring[f].mm[i] = ring[f].c[i] = (T)0;

    T buf[NLD];
    fetch(z0 - 1, buf);
    for (int it = 0; it < nz + 2; ++it) {
        const int slot = it & 1;
#pragma unroll
        for (int k = 0; k < NLD; ++k) pl[slot][ld_l[k]] = buf[k];
        if (it + 1 < nz + 2) fetch(z0 + it, buf);  // next plane, in flight during the compute
        __syncthreads();
        if (node_thread) {
#pragma unroll
            for (int f = 0; f < NF - 1; ++f) {
                T s, mm;
                plane_factors(pl[slot] + (f + 1) * PA, iy + 1, ix + 1, s, mm);
                ring[f].push(s, mm, pl[slot][(f + 1) * PA + (iy + 1) * PT + ix + 1]);
            }
        }
        if (it >= 1) {
            T c[2][2][2], v[2][2][2], r[2][2][2];
#pragma unroll
            for (int az = 0; az < 2; ++az) {
                const int sl = az ? slot : slot ^ 1;
#pragma unroll
                for (int ay = 0; ay < 2; ++ay)
#pragma unroll
                    for (int ax = 0; ax < 2; ++ax) {
                        const int l = (ey + ay) * PT + ex + ax;
                        c[az][ay][ax] = pl[sl][l];
                        v[az][ay][ax] = pl[sl][VN * PA + l];
                    }
            }
            element_loads(c, v, b0, b1, b2, r);
#pragma unroll
            for (int ay = 0; ay < 2; ++ay)
#pragma unroll
                for (int ax = 0; ax < 2; ++ax) {
                    eb[ay * 2 + ax][t] = r[0][ay][ax];
                    et[slot][ay * 2 + ax][t] = r[1][ay][ax];
                }
        }
        __syncthreads();
        if (it >= 2 && node_thread && ix < ox && iy < oy) {
            // loads of the 8 elements around the node of plane z0 + it - 2
            T nv = (T)0;
#pragma unroll
            for (int ay = 0; ay < 2; ++ay)
#pragma unroll
                for (int ax = 0; ax < 2; ++ax) {
                    const int e = (iy + 1 - ay) * ET + (ix + 1 - ax);
                    nv += et[slot ^ 1][ay * 2 + ax][e] + eb[ay * 2 + ax][e];
                }
            const int zc = z0 + it - 2;
            const long long o = (long long)zc * plane + (long long)(y0 + iy) * n0 + x0 + ix;
            // no-flux: the reflected rows are 2^b times the node's row
            T ib = (T)1;
            if (g.bc)
                ib = (T)1 / (T)(1 << (edge_count(x0 + ix, n0) + edge_count(y0 + iy, n1) + edge_count(zc, n2)));
            if constexpr (MODEL == 0) {
                const T kv = ring[0].stiff(h36);
                Jv[o] = (inv_dt * m * ring[0].c[1] + mob * (nv + kappa * kv)) * ib;
            } else {
                const T kc = ring[0].stiff(h36), km = ring[1].stiff(h36);
                const T vc = ring[0].c[1], vm = ring[1].c[1];
                if constexpr (TRANS == 0) {
                    Jv[o] = (inv_dt * m * vc + mob * km) * ib;
                    Jv[g.N + o] = (m * vm - (nv + kappa * kc)) * ib;
                } else {
                    Jv[o] = (inv_dt * m * vc - (nv + kappa * km)) * ib;
                    Jv[g.N + o] = (mob * kc + m * vm) * ib;
                }
            }
        }
    }
}

}  // namespace

template <typename T>
void launch_jvp3d(const Geom& g, int model, const FreeEnergy& f, double kappa, double mob,
                  double inv_dt, const T* U, const T* v, T* Jv, hipStream_t s, int trans)
{
    const double detJ = std::pow(0.5 * g.h, 3), m = std::pow(g.h, 3);
    const int gx = (g.n[0] + OT - 1) / OT, gy = (g.n[1] + OT - 1) / OT;
    // about 1024 blocks (4 per CU); fewer planes per block cost more z halo
    const int want = std::max(1, 1024 / (gx * gy));
    int tz = std::max(1, (g.n[2] + want - 1) / want);
    if (tz < 4) tz = std::min(4, g.n[2]);
    if (const int ov = tune_jvp3d_planes()) tz = std::min(ov, g.n[2]);
    const int gz = (g.n[2] + tz - 1) / tz;
    const dim3 grid((unsigned)gx, (unsigned)gy, (unsigned)gz);
    const T b0 = (T)(detJ * f.b0), b1 = (T)(detJ * f.b1), b2 = (T)(detJ * f.b2);
    const T h36 = (T)(g.h / 36.0);
#define JVP3(MODEL, TR)                                                                          \
    k_jvp3d<T, MODEL, TR><<<grid, NT, 0, s>>>(U, v, Jv, g, b0, b1, b2, (T)kappa, (T)mob, (T)m,  \
                                              (T)inv_dt, h36, tz)
    if (model == 0)
        JVP3(0, 0);
    else if (!trans)
        JVP3(1, 0);
    else
        JVP3(1, 1);
#undef JVP3
}

template void launch_jvp3d<float>(const Geom&, int, const FreeEnergy&, double, double, double,
                                  const float*, const float*, float*, hipStream_t, int);
template void launch_jvp3d<double>(const Geom&, int, const FreeEnergy&, double, double, double,
                                   const double*, const double*, double*, hipStream_t, int);

}  // namespace pfk
