// k_stream2d.hip -- fused explicit step (Eq. 12) for 2-D periodic grids.
//
// Layout of the work.  One 64-lane wavefront owns a strip of 64 consecutive
// columns (lane = column) and marches upward through a chunk of rows,
// keeping every intermediate in registers:
//   - x-neighbours come from the adjacent lane through DPP wave shifts (no LDS,
//     no shared-memory traffic);
//   - y-neighbours are the previous rows, held in a short register window;
//   - each input row is read from HBM once per wave, PF rows ahead of use.
// A strip outputs its 64 - 2H interior columns (H = 1 for Allen-Cahn, 2 for
// the Cahn-Hilliard split step, whose mu must be known at x +- 1); the H halo
// lanes on each side recompute what they need.  Chunks overlap by H rows in
// the same way.  No LDS, no atomics, no inter-wave synchronisation.
//
// Per element row (r-1, r) the Q1 quadrature is sum-factorised:
//   X_r[qx]   = sum_ax B[qx][ax] c(x+ax, r)              (2 values / node)
//   c_q       = sum_ay B[qy][ay] X_{r-1+ay}[qx]           (4 quad values / element)
//   G[qx][ay] = sum_qy B[qy][ay] f'(c_q)                  (y-scatter)
//   N(x, r-1) = sum_qx B[qx][1] Hsum(x-1)[qx] + B[qx][0] Hsum(x)[qx]   (x-scatter)
// with B = [[GP, GM], [GM, GP]].  The gradient term is the closed Q1 stencil
// K c = (9 c - sum_{3x3} c) / 3 (2-D, h-independent).
#include <type_traits>

#include "device.hpp"
#include "kernels.hpp"
#include "stream2d.hpp"

namespace pfk {
namespace {

template <typename T>
struct Coef {
    T a1, a2, a3;  // cubic f' with every constant factor folded in
    T beta;        // multiplies (9 c - box3x3(c))
    T gamma;       // Cahn-Hilliard: multiplies (9 mu - box3x3(mu))
};

// One explicit step as a row pipeline.  push(cc) takes c of the newest row
// r (per lane = column) and returns the stepped value of row r - H
// (H = 1 Allen-Cahn, 2 Cahn-Hilliard); the register window holds the rows
// in between.  Lane validity shrinks by H lanes per side per stage.
//   MODEL 0: Allen-Cahn    out = c - [dt L |J|/m] N'(c) - [dt L kappa/(3m)] (9c - box c)
//   MODEL 1: Cahn-Hilliard mu  = [|J|/m] N'(c) + [kappa/(3m)] (9c - box c)
//                          out = c - [dt M/(3m)] (9 mu - box mu)
// N' is the quadrature sum with the scaled cubic (a1, a2, a3); box = 3x3 sum.
template <typename T, int MODEL, bool LOB = false>
struct Stage {
    T c_m1 = 0, c_m2 = 0;        // c at rows r-1, r-2
    T s3_m1 = 0, s3_m2 = 0;      // 3-point x-sums of c at rows r-1, r-2
    T xl_m1 = 0, xr_m1 = 0;      // x-interpolated values of row r-1
    T guL_m1 = 0, guR_m1 = 0;    // upward scatter of element row (r-2, r-1)
    T mu_m1 = 0;                 // CH: mu at row r-2
    T s3mu_m1 = 0, s3mu_m2 = 0;  // CH: x-sums of mu at rows r-2, r-3

    __device__ __forceinline__ T push(T cc, const Coef<T>& k)
    {
        const T gp = (T)GP, gm = (T)GM;
        const T cl = from_left(cc), cr = from_right(cc);
        const T s3 = cl + cc + cr;
        const T d = cr - cc;
        const T xl_0 = fmaT(gm, d, cc), xr_0 = fmaT(gp, d, cc);
        const T e0 = xl_0 - xl_m1, e1 = xr_0 - xr_m1;
        const T FL0 = cubic(fmaT(gm, e0, xl_m1), k.a1, k.a2, k.a3);
        const T FL1 = cubic(fmaT(gp, e0, xl_m1), k.a1, k.a2, k.a3);
        const T FR0 = cubic(fmaT(gm, e1, xr_m1), k.a1, k.a2, k.a3);
        const T FR1 = cubic(fmaT(gp, e1, xr_m1), k.a1, k.a2, k.a3);
        const T dL = FL0 - FL1, dR = FR0 - FR1;
        const T gdL = fmaT(gp, dL, FL1), guL = fmaT(gm, dL, FL1);
        const T gdR = fmaT(gp, dR, FR1), guR = fmaT(gm, dR, FR1);
        const T HL = guL_m1 + gdL, HR = guR_m1 + gdR;  // node row r-1 complete
        const T dH = HL - HR;
        const T pl = fmaT(gp, dH, HR), pr = fmaT(gm, dH, HR);
        const T Nn = pl + from_left(pr);
        const T box = s3_m2 + s3_m1 + s3;
        const T lap = fmaT((T)9, c_m1, -box);
        T v;
        if constexpr (MODEL == 0) {
            v = c_m1 - Nn - k.beta * lap;
        } else {
            const T mu = fmaT(k.beta, lap, Nn);  // mu at row r-1
            const T s3mu = from_left(mu) + mu + from_right(mu);
            const T boxmu = s3mu_m2 + s3mu_m1 + s3mu;  // around row r-2
            v = c_m2 - k.gamma * fmaT((T)9, mu_m1, -boxmu);
            s3mu_m2 = s3mu_m1;
            s3mu_m1 = s3mu;
            mu_m1 = mu;
        }
        c_m2 = c_m1;
        c_m1 = cc;
        s3_m2 = s3_m1;
        s3_m1 = s3;
        xl_m1 = xl_0;
        xr_m1 = xr_0;
        guL_m1 = guL;
        guR_m1 = guR;
        return v;
    }
};

// The same pipeline with Gauss-Lobatto (nodal) quadrature: the nonlinear term is
// m f'(c) at the node and the stiffness the 5-point stencil (4 c - axis neighbours,
// h-free in 2-D), so no interpolation or scatter remains:
//   MODEL 0: out = c - [dt L] f'(c) - [dt L kappa/m] (4c - nbrs c)
//   MODEL 1: mu  = f'(c) + [kappa/m] (4c - nbrs c);  out = c - [dt M/m] (4 mu - nbrs mu)
template <typename T, int MODEL>
struct Stage<T, MODEL, true> {
    T c_m1 = 0, c_m2 = 0;    // c at rows r-1, r-2
    T mu_m1 = 0, mu_m2 = 0;  // CH: mu at rows r-2, r-3

    __device__ __forceinline__ T push(T cc, const Coef<T>& k)
    {
        const T lap = fmaT((T)4, c_m1, -((from_left(c_m1) + from_right(c_m1)) + (c_m2 + cc)));  // row r-1
        T v;
        if constexpr (MODEL == 0) {
            v = c_m1 - cubic(c_m1, k.a1, k.a2, k.a3) - k.beta * lap;
        } else {
            const T mu = fmaT(k.beta, lap, cubic(c_m1, k.a1, k.a2, k.a3));  // mu at row r-1
            const T lapmu = fmaT((T)4, mu_m1, -((from_left(mu_m1) + from_right(mu_m1)) + (mu_m2 + mu)));
            v = c_m2 - k.gamma * lapmu;  // row r-2
            mu_m2 = mu_m1;
            mu_m1 = mu;
        }
        c_m2 = c_m1;
        c_m1 = cc;
        return v;
    }
};

// KS explicit steps of one (strip, chunk) work item (temporal blocking):
// stage s consumes the rows stage s-1 produces, so a row is read from memory
// once and written once per KS steps.  Each stage performs exactly the
// arithmetic of a single-step launch, so the result is bitwise that of KS
// single steps.  PF: rows in flight per wave (register prefetch ring depth).
// Must be called by a whole wave with wave-uniform arguments.
// MIRROR: no-flux grid, read through the even extension about the end rows and
// columns (reflect); the lumped update r/m of a boundary node is then exactly the
// interior formula (see reflect in device.hpp), for every fused stage.
template <typename T, int MODEL, int PF, int KS, bool MID = false, bool MIRROR = false, bool LOB = false>
__device__ __forceinline__ void stream_item(const T* __restrict__ in, T* __restrict__ out, int nx,
                                            int ny, int strip, int y0, int y1, unsigned bytes,
                                            const Coef<T>& k, T* __restrict__ mid = nullptr)
{
    constexpr int H = MODEL == 0 ? 1 : 2;
    constexpr int HK = H * KS;            // halo of the whole pass
    constexpr int OUTW = WAVE - 2 * HK;   // output columns per strip
    const int lane = threadIdx.x & (WAVE - 1);
    const int x0 = strip * OUTW;
    const int xl = x0 - HK + lane;
    int x;
    if constexpr (MIRROR) {
        x = reflect(xl, nx);
    } else {
        x = xl % nx;
        if (x < 0) x += nx;
    }
    const bool out_lane = lane >= HK && lane < WAVE - HK && xl < nx;
    const int iters = (y1 - y0) + 2 * HK;  // rows y0-HK .. y1+HK-1
    const int rowb = nx * (int)sizeof(T);  // bytes per row
    const int vx = x * (int)sizeof(T);
    const auto rin = make_rsrc(in, bytes);
    const auto rout = make_rsrc(out, bytes);
    const auto rmid = make_rsrc(MID ? mid : out, bytes);

    Stage<T, MODEL, LOB> st[KS];

    // prefetch ring: slot (t mod PF) holds row y0 - HK + t.  Every row runs the
    // pipeline unconditionally (rows past the chunk compute values nobody
    // stores), so the register window never needs merging; only the prefetch
    // and the store are predicated.
    T ring[PF];
    // periodic: rl is the physical row and wraps; MIRROR: lr is the logical row
    // and rl its reflection
    int lr = y0 - HK;
    int rl = lr;
    if constexpr (MIRROR) {
        rl = reflect(lr, ny);
    } else {
        while (rl < 0) rl += ny;
    }
    auto advance = [&]() {
        if constexpr (MIRROR) {
            rl = reflect(++lr, ny);
        } else {
            if (++rl == ny) rl = 0;
        }
    };
#pragma unroll
    for (int u = 0; u < PF; ++u) {
        ring[u] = u < iters ? bload<T>(rin, vx, rl * rowb) : (T)0;
        advance();
    }
    // The prefetch load itself is unconditional: once the chunk's last row has
    // been requested the row index stops advancing and the same row is read
    // again (a cache hit).  A conditional load would make the compiler wait for
    // it immediately.
    int rlast = y1 + HK - 1;
    if constexpr (MIRROR) {
        rlast = reflect(rlast, ny);
    } else {
        while (rlast >= ny) rlast -= ny;
    }
    // stage s >= 1 receives only pipeline fill (garbage) before t = 2 H s: it skips
    // those pushes (its window then starts from zeros, which the 2H pushes before
    // its first valid output overwrite), which the first FIRST iterations handle
    // with compile-time loop indices; the steady loop pushes every stage
    constexpr int FIRST = (2 * H * (KS - 1) + PF - 1) / PF * PF;  // <= 2 HK <= iters
    auto row = [&](int t, int u, bool head) {
        T v = ring[u];
        ring[u] = bload<T>(rin, vx, rl * rowb);
        if (t + PF + 1 < iters) {
            advance();
        } else {
            rl = rlast;
        }
        v = st[0].push(v, k);
        if constexpr (MID) {
            // trajectory mode: the first stage's row y0 - HK - H + t is the state
            // after one step (bitwise a single-step launch's)
            if (t >= HK + H && t < HK + H + (y1 - y0) && out_lane)
                bstore(v, rmid, vx, (y0 - HK - H + t) * rowb);
        }
#pragma unroll
        for (int sidx = 1; sidx < KS; ++sidx)
            if (!head || t >= 2 * H * sidx) v = st[sidx].push(v, k);
        // the last stage just finished row y0 - 2 HK + t
        if (t >= 2 * HK && t < iters && out_lane) bstore(v, rout, vx, (y0 - 2 * HK + t) * rowb);
    };
#pragma unroll
    for (int t = 0; t < FIRST; ++t) row(t, t % PF, true);
    for (int t0 = FIRST; t0 < iters; t0 += PF) {
#pragma unroll
        for (int u = 0; u < PF; ++u) row(t0 + u, u, false);
    }
}

template <typename T, int MODEL, int PF, int KS, bool MIRROR = false, bool LOB = false>
__global__ __launch_bounds__(256) void k_explicit2d(const T* __restrict__ in, T* __restrict__ out,
                                                    int nx, int ny, int nstrips, int nwaves, int nchunks,
                                                    unsigned bytes, Coef<T> k)
{
    const int wave = uniform_wave();
    if (wave >= nwaves) return;  // uniform per wave
    // balanced chunks: chunk c of a strip owns rows [c ny / nchunks, (c + 1) ny / nchunks)
    const int chunk = wave / nstrips;
    const int y0 = (int)((long long)chunk * ny / nchunks);
    const int y1 = (int)((long long)(chunk + 1) * ny / nchunks);
    stream_item<T, MODEL, PF, KS, false, MIRROR, LOB>(in, out, nx, ny, wave % nstrips, y0, y1, bytes, k);
}

// Fused steps with the chunk seams shared through LDS (periodic grids).
//
// A workgroup holds SEAM_NW consecutive chunks of one strip, one per wave.  Stage s
// of the chunk with rows [y0, y1) produces rows [y0 + s H, y1 + s H): the stages
// form a parallelogram in (row, step).  Stage s >= 1 then consumes stage s-1's rows
// [y0 + (s-1) H, y1 + (s+1) H); the top 2H of them are the first 2H rows the chunk
// above produces at stage s-1.  Every wave leaves those first rows of each stage
// but the last in LDS; after one barrier, the wave below pushes them through its
// next stage at the end of its sweep instead of computing them again.  The top wave
// of a workgroup has no neighbour above in LDS and computes its rows itself.
//
// Per chunk and KS steps a wave pushes KS (ty + 2H) rows (the top wave of the
// workgroup H KS (KS - 1) more), against KS (ty + 2 H KS) for k_explicit2d.  Every
// stage runs exactly the arithmetic of a single step on the same inputs, so the
// result is bitwise that of KS single-step launches.
//
// Loop index t = 0 .. ty + 2 KS H - 1: input row y0 - H + t enters stage 0; stage
// s emits row y0 - (s + 2) H + t, valid once t >= 2 H (s + 1).  Must be launched
// with whole workgroups (nchunks a multiple of SEAM_NW): every wave reaches the one
// barrier.
constexpr int SEAM_NW = 4;  // waves (chunks) per workgroup

template <typename T, int MODEL, int KS, bool LOB>
__global__ __launch_bounds__(256) void k_explicit2d_seam(const T* __restrict__ in, T* __restrict__ out, int nx,
                                                         int ny, int nchunks, int nblocks, unsigned bytes,
                                                         Coef<T> k)
{
    constexpr int PF = 4;
    constexpr int H = MODEL == 0 ? 1 : 2;
    constexpr int HK = H * KS;
    constexpr int OUTW = WAVE - 2 * HK;
    constexpr int FILL = 2 * H * KS;                     // first loop index of a valid output
    constexpr int FIRST = (FILL + PF - 1) / PF * PF;     // seam rows are all in LDS after these
    static_assert(KS >= 2, "seam kernel: fused steps only");
    __shared__ T seam[SEAM_NW][KS - 1][2 * H][WAVE];

    // blocks are dealt round-robin to the 8 XCDs: give each XCD a contiguous range of
    // workgroups, so that the rows neighbouring chunks share stay in one L2
    const int b = (int)blockIdx.x, xcd = b % 8, per = nblocks / 8, rem = nblocks % 8;
    const int blk = xcd * per + min(xcd, rem) + b / 8;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
    const int wave = blk * SEAM_NW + wv;
    const int strip = wave / nchunks, chunk = wave % nchunks;
    const bool top = wv == SEAM_NW - 1;  // no neighbour above in this workgroup
    // the workgroups of a strip take balanced row ranges; inside one, the top chunk is
    // H (KS - 1) rows shorter, as its wave pushes H KS (KS - 1) more rows, so that
    // every wave of the workgroup does the same work
    const int nwg = nchunks / SEAM_NW, grp = chunk / SEAM_NW;
    const int Y0 = (int)((long long)grp * ny / nwg), Y1 = (int)((long long)(grp + 1) * ny / nwg);
    const int span = Y1 - Y0 + H * (KS - 1);
    const int y0 = Y0 + wv * span / SEAM_NW;
    const int y1 = top ? Y1 : Y0 + (wv + 1) * span / SEAM_NW;
    const int ty = y1 - y0;
    const int iters = ty + FILL;
    const int lane = threadIdx.x & (WAVE - 1);
    const int xl = strip * OUTW - HK + lane;
    int x = xl % nx;
    if (x < 0) x += nx;
    const bool out_lane = lane >= HK && lane < WAVE - HK && xl < nx;
    const int rowb = nx * (int)sizeof(T);
    const int vx = x * (int)sizeof(T);
    const auto rin = make_rsrc(in, bytes);
    const auto rout = make_rsrc(out, bytes);

    Stage<T, MODEL, LOB> st[KS];
    T ring[PF];
    // input rows y0 - H .. (the top wave reads 2 H (KS - 1) rows further)
    int rl = y0 - H;
    while (rl < 0) rl += ny;
    int rlast = y0 - H + (top ? iters : ty + 2 * H) - 1;
    while (rlast >= ny) rlast -= ny;
    int ro = y0 + (KS - 1) * H;  // first output row (the last stage's), wraps
    while (ro >= ny) ro -= ny;
#pragma unroll
    for (int u = 0; u < PF; ++u) {
        ring[u] = bload<T>(rin, vx, rl * rowb);
        if (++rl == ny) rl = 0;
    }
    const int need = (top ? iters : ty + 2 * H);  // input rows this wave reads
    auto fetch = [&](int t, int u) {
        T v = ring[u];
        ring[u] = bload<T>(rin, vx, rl * rowb);
        if (t + PF + 1 < need) {
            if (++rl == ny) rl = 0;
        } else {
            rl = rlast;
        }
        return v;
    };
    auto store = [&](T o) {
        if (out_lane) bstore(o, rout, vx, ro * rowb);
        if (++ro == ny) ro = 0;
    };
    // Three phases, each with its stage set known at compile time:
    //  warm-up (t < FIRST): stage s pushes from t = 2 H s; every stage but the last
    //    leaves its first 2H valid rows (t in [2H (s+1), 2H (s+2))) in LDS;
    //  steady (FIRST <= t < tend): every stage pushes its own rows, one output row;
    //    tend = ty + 2H below the top of the workgroup, iters for the top wave;
    //  seam tail (below the top only): segment j takes the 2H rows stage j of the
    //    wave above left in LDS and pushes them through stages j+1 .. KS-1.
    // The launcher guarantees ty + 2H >= FIRST + PF, so no stage of the warm-up
    // reaches its own end and no seam row is read before the barrier.
    auto warm = [&](int t) {  // t is a constant once the warm-up loop is unrolled
        T o = fetch(t, t % PF);
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            if (t >= 2 * H * s) o = st[s].push(o, k);
            if (s < KS - 1 && t >= 2 * H * (s + 1) && t < 2 * H * (s + 2))
                seam[wv][s][t - 2 * H * (s + 1)][lane] = o;
        }
        if (t >= FILL) store(o);
    };
    auto steady = [&](int t, int u) {
        T o = fetch(t, u);
#pragma unroll
        for (int s = 0; s < KS; ++s) o = st[s].push(o, k);
        store(o);
    };
#pragma unroll
    for (int t = 0; t < FIRST; ++t) warm(t);
    __syncthreads();
    const int tend = top ? iters : ty + 2 * H;
    const int t2 = FIRST + (tend - FIRST) / PF * PF;
    for (int t0 = FIRST; t0 < t2; t0 += PF) {
#pragma unroll
        for (int u = 0; u < PF; ++u) steady(t0 + u, u);
    }
#pragma unroll
    for (int u = 0; u < PF - 1; ++u)
        if (t2 + u < tend) steady(t2 + u, u);
    if (top) return;
#pragma unroll
    for (int j = 0; j < KS - 1; ++j) {
#pragma unroll
        for (int r = 0; r < 2 * H; ++r) {
            T o = seam[wv + 1][j][r][lane];
#pragma unroll
            for (int s = j + 1; s < KS; ++s) o = st[s].push(o, k);
            store(o);
        }
    }
}

// Ragged batch: wave w processes work item items[w] = (sample, strip, chunk)
// of a batch of independent problems packed in one array (see BatchSample).
template <typename T, int MODEL, int PF, int KS, bool MID = false>
__global__ __launch_bounds__(256) void k_explicit2d_batched(const T* __restrict__ in,
                                                            T* __restrict__ out,
                                                            const BatchSample* __restrict__ smp,
                                                            const BatchItem* __restrict__ items,
                                                            int n_items, int ty, T* __restrict__ mid)
{
    const int wave = uniform_wave();
    if (wave >= n_items) return;
    const BatchItem it = items[wave];
    const BatchSample& sm = smp[it.sample];
    const Coef<T> k{(T)sm.a1, (T)sm.a2, (T)sm.a3, (T)sm.beta, (T)sm.gamma};
    const unsigned bytes = (unsigned)((long long)sm.nx * sm.ny * (long long)sizeof(T));
    const int y0 = it.chunk * ty;
    stream_item<T, MODEL, PF, KS, MID>(in + sm.offset, out + sm.offset, sm.nx, sm.ny, it.strip, y0,
                                       min(y0 + ty, sm.ny), bytes, k, MID ? mid + sm.offset : nullptr);
}

template <typename T, int MODEL, int KS>
void launch_depth(int depth, int blocks, hipStream_t s, const T* in, T* out, int nx, int ny,
                  int nstrips, int nwaves, int nchunks, unsigned bytes, const Coef<T>& k, int bc, int quad)
{
    if (quad) {  // Gauss-Lobatto: one prefetch depth
        if (bc)
            k_explicit2d<T, MODEL, 4, KS, true, true><<<blocks, 256, 0, s>>>(in, out, nx, ny, nstrips, nwaves, nchunks, bytes, k);
        else
            k_explicit2d<T, MODEL, 4, KS, false, true><<<blocks, 256, 0, s>>>(in, out, nx, ny, nstrips, nwaves, nchunks, bytes, k);
        return;
    }
    if (bc)  // no-flux grids: one prefetch depth
        k_explicit2d<T, MODEL, 4, KS, true><<<blocks, 256, 0, s>>>(in, out, nx, ny, nstrips, nwaves, nchunks, bytes, k);
    else if (depth <= 4)
        k_explicit2d<T, MODEL, 4, KS><<<blocks, 256, 0, s>>>(in, out, nx, ny, nstrips, nwaves, nchunks, bytes, k);
    else if (depth <= 8)
        k_explicit2d<T, MODEL, 8, KS><<<blocks, 256, 0, s>>>(in, out, nx, ny, nstrips, nwaves, nchunks, bytes, k);
    else
        k_explicit2d<T, MODEL, 16, KS><<<blocks, 256, 0, s>>>(in, out, nx, ny, nstrips, nwaves, nchunks, bytes, k);
}

// The seam kernel for a periodic grid when its chunk plan fits (nchunks a multiple
// of SEAM_NW, chunks long enough that no seam row is read before the barrier).
// Returns false (nothing launched) otherwise.
template <typename T, int MODEL, bool LOB>
bool launch_seam(int ks, int ty, hipStream_t s, const T* in, T* out, int nx, int ny, int nstrips,
                 unsigned bytes, const Coef<T>& k)
{
    constexpr int H = MODEL == 0 ? 1 : 2;
    if (ks < 2 || ks > 4 || tune_stream2d_seam() == 1) return false;
    int nch = (ny + ty - 1) / ty;
    nch = (nch + SEAM_NW - 1) / SEAM_NW * SEAM_NW;
    const int fill = 2 * H * ks, first = (fill + 3) / 4 * 4;
    // shortest chunk: the top one of the smallest workgroup range (rows
    // [Y0 + 3 span / 4, Y1) with span = Y1 - Y0 + H (ks - 1); no longer for a longer range)
    const int rmin = ny / (nch / SEAM_NW), sh = H * (ks - 1);
    const int shortest = rmin - (SEAM_NW - 1) * (rmin + sh) / SEAM_NW;
    if (shortest < first + 4 - 2 * H || shortest < 8) return false;
    const long long waves = (long long)nstrips * nch;
    if (waves / SEAM_NW > (1ll << 30)) return false;
    const int nblocks = (int)(waves / SEAM_NW);
    switch (ks) {
        case 2: k_explicit2d_seam<T, MODEL, 2, LOB><<<nblocks, 256, 0, s>>>(in, out, nx, ny, nch, nblocks, bytes, k); break;
        case 3: k_explicit2d_seam<T, MODEL, 3, LOB><<<nblocks, 256, 0, s>>>(in, out, nx, ny, nch, nblocks, bytes, k); break;
        default: k_explicit2d_seam<T, MODEL, 4, LOB><<<nblocks, 256, 0, s>>>(in, out, nx, ny, nch, nblocks, bytes, k); break;
    }
    return true;
}

template <typename T, int MODEL>
void launch_ks(int ks, int depth, int blocks, hipStream_t s, const T* in, T* out, int nx, int ny,
               int nstrips, int nwaves, int nchunks, unsigned bytes, const Coef<T>& k, int bc, int quad)
{
    switch (ks) {
        case 1: launch_depth<T, MODEL, 1>(depth, blocks, s, in, out, nx, ny, nstrips, nwaves, nchunks, bytes, k, bc, quad); break;
        case 2: launch_depth<T, MODEL, 2>(depth, blocks, s, in, out, nx, ny, nstrips, nwaves, nchunks, bytes, k, bc, quad); break;
        case 3: launch_depth<T, MODEL, 3>(depth, blocks, s, in, out, nx, ny, nstrips, nwaves, nchunks, bytes, k, bc, quad); break;
        default: launch_depth<T, MODEL, 4>(depth, blocks, s, in, out, nx, ny, nstrips, nwaves, nchunks, bytes, k, bc, quad); break;
    }
}

}  // namespace

template <typename T, int MODEL, int KS, bool MID>
void launch_batched_depth(int depth, int blocks, hipStream_t s, const T* in, T* out,
                          const BatchSample* smp, const BatchItem* items, int n_items, int ty, T* mid)
{
    if (depth <= 4)
        k_explicit2d_batched<T, MODEL, 4, KS, MID><<<blocks, 256, 0, s>>>(in, out, smp, items, n_items, ty, mid);
    else if (depth <= 8)
        k_explicit2d_batched<T, MODEL, 8, KS, MID><<<blocks, 256, 0, s>>>(in, out, smp, items, n_items, ty, mid);
    else
        k_explicit2d_batched<T, MODEL, 16, KS, MID><<<blocks, 256, 0, s>>>(in, out, smp, items, n_items, ty, mid);
}

template <typename T>
void launch_explicit2d_batched(int model, const T* in, T* out, const BatchSample* smp,
                               const BatchItem* items, int n_items, const Stream2DConfig& cfg,
                               hipStream_t s, T* mid)
{
    const int blocks = (n_items + 3) / 4;
    const int d = cfg.depth, ty = cfg.ty;
#define BATCHED_KS(MODEL)                                                                                  \
    if (mid) {                                                                                             \
        launch_batched_depth<T, MODEL, 2, true>(d, blocks, s, in, out, smp, items, n_items, ty, mid);      \
    } else {                                                                                               \
        switch (cfg.ks) {                                                                                  \
            case 1: launch_batched_depth<T, MODEL, 1, false>(d, blocks, s, in, out, smp, items, n_items, ty, nullptr); break; \
            case 2: launch_batched_depth<T, MODEL, 2, false>(d, blocks, s, in, out, smp, items, n_items, ty, nullptr); break; \
            case 3: launch_batched_depth<T, MODEL, 3, false>(d, blocks, s, in, out, smp, items, n_items, ty, nullptr); break; \
            default: launch_batched_depth<T, MODEL, 4, false>(d, blocks, s, in, out, smp, items, n_items, ty, nullptr); break; \
        }                                                                                                  \
    }
    if (model == 0) {
        BATCHED_KS(0)
    } else {
        BATCHED_KS(1)
    }
#undef BATCHED_KS
}

template void launch_explicit2d_batched<float>(int, const float*, float*, const BatchSample*,
                                               const BatchItem*, int, const Stream2DConfig&,
                                               hipStream_t, float*);
template void launch_explicit2d_batched<double>(int, const double*, double*, const BatchSample*,
                                                const BatchItem*, int, const Stream2DConfig&,
                                                hipStream_t, double*);

template <typename T>
void launch_explicit2d(const Geom& g, int model, const FreeEnergy& f, double kappa, double mob,
                       double dt, const T* in, T* out, const Stream2DConfig& cfg, hipStream_t s)
{
    const int nx = g.n[0], ny = g.n[1];
    const double h = g.h, m = h * h, detJ = 0.25 * h * h;
    const int H = model == 0 ? 1 : 2;
    const int ks = cfg.ks >= 1 && cfg.ks <= 4 ? cfg.ks : 1;
    const int outw = WAVE - 2 * H * ks;
    const int ty = cfg.ty > 0 ? cfg.ty : 32;
    const int nstrips = (nx + outw - 1) / outw;
    const int nchunks = (ny + ty - 1) / ty;
    const int nwaves = nstrips * nchunks;
    const int blocks = (nwaves + 3) / 4;
    const unsigned bytes = (unsigned)((size_t)g.N * sizeof(T));  // caller guarantees < 2^31
    Coef<T> k{};
    // Gauss: the quadrature sum N carries detJ and the box stencil (9c - box)/3;
    // Gauss-Lobatto: N = m f'(c) and the 5-point stencil 4c - nbrs (both h-free in 2-D).
    // (The products keep the association the batched plans use, so a sample there is
    // bitwise the same problem stepped alone.)
    const double nsc = g.quad ? m : detJ, kd = g.quad ? m : 3.0 * m;
    auto seam_or_halo = [&](auto model_tag) {
        constexpr int MODEL = decltype(model_tag)::value;
        const bool seam = !g.bc && (cfg.depth <= 4 || g.quad) &&
                          (g.quad ? launch_seam<T, MODEL, true>(ks, ty, s, in, out, nx, ny, nstrips, bytes, k)
                                  : launch_seam<T, MODEL, false>(ks, ty, s, in, out, nx, ny, nstrips, bytes, k));
        if (!seam)
            launch_ks<T, MODEL>(ks, cfg.depth, blocks, s, in, out, nx, ny, nstrips, nwaves, nchunks, bytes, k, g.bc,
                                g.quad);
    };
    if (model == 0) {
        const double sc = dt * mob * nsc / m;
        k.a1 = (T)(sc * f.a1); k.a2 = (T)(sc * f.a2); k.a3 = (T)(sc * f.a3);
        k.beta = (T)(dt * mob * kappa / kd);
        seam_or_halo(std::integral_constant<int, 0>{});
    } else {
        const double sc = nsc / m;
        k.a1 = (T)(sc * f.a1); k.a2 = (T)(sc * f.a2); k.a3 = (T)(sc * f.a3);
        k.beta = (T)(kappa / kd);
        k.gamma = (T)(dt * mob / kd);
        seam_or_halo(std::integral_constant<int, 1>{});
    }
}

template void launch_explicit2d<float>(const Geom&, int, const FreeEnergy&, double, double, double,
                                       const float*, float*, const Stream2DConfig&, hipStream_t);
template void launch_explicit2d<double>(const Geom&, int, const FreeEnergy&, double, double, double,
                                        const double*, double*, const Stream2DConfig&, hipStream_t);

}  // namespace pfk
