// k_nn.hip -- convolutional surrogate on BF16 matrix cores (a learned component
// this library adds; the paper has none).
//
// Network (width 32, 3x3 periodic convolutions, NHWC activations):
//   a0 = (c, M, kappa, 0 ... 0)                      16 channels, bf16
//   a_l = bf16(relu(conv(a_{l-1}; W_l) + b_l)), l = 1..3   32 channels, bf16
//   d = conv(a_3; W_4) + b_4                          1 channel, fp32
//   c_hat = c + d - mean(d)                           per sample (exact mass)
// Loss: sum over samples of mean_p (c_hat - target)^2.
//
// Hidden layers and their input-gradient (dgrad) and weight-gradient (wgrad)
// products run on v_mfma_f32_32x32x16_bf16 with FP32 accumulation:
//   forward/dgrad: persistent blocks (as many as are resident) walk tiles of CR
//     rows x 32 pixels; each stages the tile's (CR+2) x (32+2) halo in LDS (the
//     next tile's loads in flight during this tile's MFMAs), and each of its 4
//     waves computes CR/4 rows of 32 pixels x 32 channels, its A operand (pixels
//     x input channels of one tap) read from the tile, its B operand (the
//     weights of that tap) from a copy of the fragments the block made in LDS
//     once.  K = 9 taps x Cin.
//   wgrad: dW[tap] (Cin x Cout) = sum over pixels of a_in(p + tap) g_out(p)^T,
//     K = pixels; every block accumulates a fixed stride of pixel tiles in
//     registers (split-K) and writes one FP32 partial; a second kernel sums the
//     partials in block order (bitwise reproducible).
// The 32 -> 1 output layer (2.9% of the flops) runs on the VALU in training.
// Inference fuses: the first layer into the second's tiles (MODE 4: a1 never
// reaches memory), and the output layer's channel sums into the third's epilogue
// (MODE 3: 9 FP32 tap planes, then a gather, k_out_taps).
//
// MFMA operand layout (32x32x16): lane l supplies A[l % 32][8 (l / 32) + j] and
// B[8 (l / 32) + j][l % 32] for j = 0..7, and receives
// C[8 (i / 4) + 4 (l / 32) + (i % 4)][l % 32] in accumulator i = 0..15.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "device.hpp"
#include "nn.hpp"

namespace pfk {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned short u16;

constexpr int TW = 32;        // pixels per wave row
constexpr int TR = 4;         // rows per wgrad tile (one per wave)
constexpr int CR = 4;         // rows per forward/dgrad tile (CR / 4 per wave)
constexpr int NBLK = 256;

// fp32 -> bf16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ u16 bf16_bits(float f)
{
    unsigned u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (u16)(u >> 16);
}
__device__ __forceinline__ float bf16_val(u16 b) { return __uint_as_float((unsigned)b << 16); }
// two fp32 -> packed bf16 bits (lo, hi), round to nearest even (v_cvt_pk_bf16_f32)
__device__ __forceinline__ unsigned bf16_pair(float lo, float hi)
{
    const bf16x2 v = {(__bf16)lo, (__bf16)hi};
    return __builtin_bit_cast(unsigned, v);
}

__device__ __forceinline__ int wrapi(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }
// Row of a tile's halo, i in [-2, n + 9]: periodic for i <= n + 1; rows further out
// (only when n is below the tile's reach) feed only outputs past the grid, which are
// never stored, so they are clamped to the last row (every read stays in the sample).
__device__ __forceinline__ int halo_row(int i, int n)
{
    int r = i < 0 ? i + n : i;
    r = r < 0 ? r + n : r;  // n = 1
    r = r >= n ? r - n : r;
    return r < n ? r : n - 1;
}

// LDS tile: (ROWS + 2) rows x (TW + 2) pixels, CIN channels, pixel stride padded by
// 16 bytes: a stride of 4k banks with k odd (k = 5 for 32 channels, 3 for 16) puts
// the 16-byte reads of 8 consecutive pixels on 8 disjoint bank quads
template <int CIN, int ROWS = TR>
struct Tile {
    static constexpr int PSTRIDE = CIN * 2 + 16;  // bytes per pixel in LDS
    static constexpr int BYTES = (ROWS + 2) * (TW + 2) * PSTRIDE;
};

// stage the halo tile of rows y0-1 .. y0+ROWS, pixels x0-1 .. x0+TW (periodic)
template <int CIN, int ROWS = TR>
__device__ __forceinline__ void stage_tile(const u16* __restrict__ act, int b, int H, int W, int y0,
                                           int x0, unsigned char* lds)
{
    constexpr int CHUNKS = CIN * 2 / 16;  // 16-byte chunks per pixel
    constexpr int TOTAL = (ROWS + 2) * (TW + 2) * CHUNKS;
    for (int t = threadIdx.x; t < TOTAL; t += NBLK) {
        const int ch = t % CHUNKS, pix = t / CHUNKS;
        const int px = pix % (TW + 2), ry = pix / (TW + 2);
        const int gy = halo_row(y0 - 1 + ry, H), gx = wrapi(x0 - 1 + px, W);
        const uint4 v = *reinterpret_cast<const uint4*>(
            act + (((size_t)b * H + gy) * W + gx) * CIN + ch * 8);
        *reinterpret_cast<uint4*>(lds + (ry * (TW + 2) + px) * Tile<CIN, ROWS>::PSTRIDE + ch * 16) = v;
    }
}

// MODE 0: out = bf16(relu(acc + bias))          (forward, hidden layers)
// MODE 1: out = bf16(acc * (mask[p][co] > 0))    (dgrad: relu mask of the layer input)
// MODE 4: the second layer with the first computed while staging (forward only):
//         the tile reads the c plane only, and forms its 6 x 34 halo of
//         a1 = bf16(relu(sum_tap W1[tap][0] bf16(c(p + tap)) + beff)) on the matrix
//         cores, one MFMA per 32 pixels (A = the 9 taps of c, zero-padded to 16).
//         M and kappa are constant over a sample, so their channels reduce to the
//         bias beff = b1 + bf16(M) sum_tap W1[tap][1] + bf16(kappa) sum_tap W1[tap][2];
//         a1 never reaches memory
// MODE 3: as MODE 0 for the last hidden layer, followed by the output layer's
//         channel contraction: instead of a3 it stores the 9 planes
//         P[tap][p] = sum_ci W4[tap][ci] a3[p][ci] (FP32), which a gather sums over
//         the taps' neighbours (forward only; training keeps a3 for the gradients)
// wfrag: B fragments [9][CIN/16][64 lanes][8] bf16 for this layer/use
// Persistent: the grid holds the resident blocks, each loads its weight fragments
// into registers once (LDS then carries only the A operands) and walks the tiles
// blockIdx.x, blockIdx.x + gridDim.x, ...; the next tile's global loads are
// issued into registers before the current tile's MFMAs, so staging overlaps
// compute.  Every output is the same MFMA chain as with one tile per block.
struct InPlanes {  // MODE 4 only
    const float* c;      // [B][H][W]
    const float* M;      // [B]
    const float* kappa;  // [B]
    const float* w1;     // FP32 W1 [9][3][32]
    const float* b1;     // FP32 b1 [32]
};
struct TapPlanes {
    const u16* w4;    // bf16 W4 [9][32]
    float* P;         // [9][B][H][W]
    long long plane;  // B H W
};

template <int CIN, int MODE>
__global__ __launch_bounds__(NBLK, 3) void k_conv_mfma(const u16* __restrict__ in,
                                                    const u16* __restrict__ wfrag,
                                                    const float* __restrict__ bias,
                                                    const u16* __restrict__ mask,
                                                    u16* __restrict__ out, int B, int H, int W, int ntiles,
                                                    InPlanes ip, TapPlanes tp)
{
    static_assert(MODE != 4 || CIN == 32, "the fused first layer feeds the second");
    constexpr int KS = CIN / 16;
    constexpr int PS = Tile<CIN, CR>::PSTRIDE;
    constexpr int CHUNKS = CIN * 2 / 16;  // 16-byte chunks per pixel
    constexpr int TOTAL = (CR + 2) * (TW + 2) * CHUNKS;
    constexpr int PER = (TOTAL + NBLK - 1) / NBLK;  // staged chunks per thread
    constexpr int OST = 80;  // bytes per pixel row of the epilogue transpose (64 + 16: no bank overlap)
    constexpr int LB = Tile<CIN, CR>::BYTES > 4 * TW * OST ? Tile<CIN, CR>::BYTES : 4 * TW * OST;
    __shared__ __align__(16) unsigned char lds[LB];  // the halo tile, then the transpose
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int tiles_x = W / TW, tiles_y = (H + CR - 1) / CR;
    // this lane's weight fragments for every (tap, k-slice), kept for all tiles
    bf16x8 bw[9 * KS];
#pragma unroll
    for (int q = 0; q < 9 * KS; ++q)
        bw[q] = *reinterpret_cast<const bf16x8*>(wfrag + ((size_t)q * 64 + lane) * 8);
    const int m = lane & 31, kh = lane >> 5;
    const int co = m;
    __shared__ __align__(16) float sbias[32];
    if (MODE != 1 && threadIdx.x < 32) sbias[threadIdx.x] = bias[threadIdx.x];  // read after the loop's barrier
    // MODE 3: W4 as the A operand of the contraction, A[tap][k = ci] = W4[tap][16 ks + k]
    // (rows 9..31 zero), kept in LDS (rows of 40 bf16: conflict-free 16-byte reads);
    // lane l reads tap l % 32, channels 16 ks + 8 (l / 32) + j
    constexpr int W4S = 40;
    __shared__ __align__(16) u16 sw4[MODE == 3 ? 32 * W4S : 1];
    if constexpr (MODE == 3) {
        for (int i = threadIdx.x; i < 32 * 32; i += NBLK) {
            const int tap = i / 32, ci = i % 32;
            sw4[tap * W4S + ci] = tap < 9 ? tp.w4[tap * 32 + ci] : (u16)0;
        }
    }
    // MODE 4: the first layer's B fragment (B[k = tap][co] = W1[tap][0][co], k < 9),
    // the per-sample bias terms and the c patch (rows y0-2 .. y0+CR+1, pixels
    // x0-2 .. x0+TW+1) in LDS as bf16
    constexpr int CPW = TW + 4, CPN = (CR + 4) * CPW;  // 36 x 8 = 288 values
    bf16x8 l1f = {};
    float l1s1 = 0.0f, l1s2 = 0.0f, l1b = 0.0f;
    float cs0 = 0.0f, cs1 = 0.0f;  // the next tile's c values (2 per thread)
    __shared__ u16 cpt[MODE == 4 ? CPN : 1];
    __shared__ __align__(16) float sbeff[MODE == 4 ? 32 : 1];  // the tile's sample's beff per channel
    if constexpr (MODE == 4) {
        static_assert(CPN <= 2 * NBLK, "two c values per thread");
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = 8 * kh + j;
            l1f[j] = __builtin_bit_cast(__bf16, k < 9 ? bf16_bits(ip.w1[(k * 3) * 32 + co]) : (u16)0);
        }
        for (int tap = 0; tap < 9; ++tap) {
            l1s1 += bf16_val(bf16_bits(ip.w1[(tap * 3 + 1) * 32 + co]));
            l1s2 += bf16_val(bf16_bits(ip.w1[(tap * 3 + 2) * 32 + co]));
        }
        l1b = ip.b1[co];
    }
    // the halo tile of rows y0-1 .. y0+CR, pixels x0-1 .. x0+TW (periodic) of a tile,
    // PER 16-byte chunks per thread (chunks past TOTAL load a valid dummy)
    uint4 s0, s1, s2, s3;
    static_assert(PER <= 4, "staging registers");
#define PF_CONV_FETCH(T_)                                                                                   \
    do {                                                                                                    \
        const int tt_ = (T_);                                                                               \
        const int tx_ = tt_ % tiles_x, ty_ = (tt_ / tiles_x) % tiles_y, b_ = tt_ / (tiles_x * tiles_y);     \
        const int x0_ = tx_ * TW, y0_ = ty_ * CR;                                                           \
        if (MODE == 4) {                                                                                    \
            float* cdst_[2] = {&cs0, &cs1};                                                                 \
            _Pragma("unroll") for (int q = 0; q < 2; ++q)                                                   \
            {                                                                                               \
                int i_ = threadIdx.x + q * NBLK;                                                            \
                i_ = i_ < CPN ? i_ : CPN - 1;                                                               \
                const int gy = halo_row(y0_ - 2 + i_ / CPW, H), gx = wrapi(x0_ - 2 + i_ % CPW, W);         \
                *cdst_[q] = ip.c[((size_t)b_ * H + gy) * W + gx];                                           \
            }                                                                                               \
            break;                                                                                          \
        }                                                                                                   \
        uint4* dst_[4] = {&s0, &s1, &s2, &s3};                                                              \
        _Pragma("unroll") for (int q = 0; q < PER; ++q)                                                     \
        {                                                                                                   \
            int c = threadIdx.x + q * NBLK;                                                                 \
            c = c < TOTAL ? c : TOTAL - 1;                                                                  \
            const int ch = c % CHUNKS, pix = c / CHUNKS;                                                    \
            const int px = pix % (TW + 2), ry = pix / (TW + 2);                                             \
            const int gy = halo_row(y0_ - 1 + ry, H), gx = wrapi(x0_ - 1 + px, W);                          \
            const size_t gp_ = ((size_t)b_ * H + gy) * W + gx;                                              \
            *dst_[q] = *reinterpret_cast<const uint4*>(in + gp_ * CIN + ch * 8);                            \
        }                                                                                                   \
    } while (0)
    int t = blockIdx.x;
    if (t < ntiles) PF_CONV_FETCH(t);
    for (; t < ntiles; t += gridDim.x) {
        __syncthreads();  // the previous tile's reads of the LDS tile are done
        if constexpr (MODE == 4) {
            cpt[threadIdx.x] = bf16_bits(cs0);
            if (threadIdx.x + NBLK < CPN) cpt[threadIdx.x + NBLK] = bf16_bits(cs1);
            if (threadIdx.x < 32) {
                const int bt = t / (tiles_x * tiles_y);
                sbeff[co] = l1b + bf16_val(bf16_bits(ip.M[bt])) * l1s1 + bf16_val(bf16_bits(ip.kappa[bt])) * l1s2;
            }
        } else {
            const uint4 src[4] = {s0, s1, s2, s3};
#pragma unroll
            for (int q = 0; q < PER; ++q) {
                const int c = threadIdx.x + q * NBLK;
                if (c < TOTAL) *reinterpret_cast<uint4*>(lds + (c / CHUNKS) * PS + (c % CHUNKS) * 16) = src[q];
            }
        }
        __syncthreads();
        if (t + (int)gridDim.x < ntiles) PF_CONV_FETCH(t + (int)gridDim.x);
        const int tx = t % tiles_x, ty = (t / tiles_x) % tiles_y, b = t / (tiles_x * tiles_y);
        const int x0 = tx * TW, y0 = ty * CR;
        if constexpr (MODE == 4) {
            // the first layer on the (CR+2) x (TW+2) = 204 halo pixels, 32 per MFMA:
            // wave wv takes groups wv and wv + 4; tile pixel s = 34 ry + px sits at
            // c patch rows ry .. ry+2, pixels px .. px+2.  W1 is the A operand, so the
            // product is transposed: lane l holds pixel 32 grp + l % 32, channels
            // 8 g + 4 (l / 32) + r in accumulator 4 g + r, stored 4 channels at a time
            constexpr int NPX = (CR + 2) * (TW + 2);
#pragma unroll
            for (int gq = 0; gq < 2; ++gq) {
                const int grp = wv + 4 * gq;
                if (32 * grp < NPX) {
                    const int sp = min(32 * grp + m, NPX - 1);
                    const int ry = sp / (TW + 2), px = sp % (TW + 2);
                    bf16x8 a;
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        const int k = 8 * kh + j;
                        const u16 bits = k < 9 ? cpt[(ry + k / 3) * CPW + px + k % 3] : (u16)0;
                        a[j] = __builtin_bit_cast(__bf16, bits);
                    }
                    f32x16 a1 = {};
                    a1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(l1f, a, a1, 0, 0, 0);
                    const int s = 32 * grp + m;
                    if (s < NPX) {
#pragma unroll
                        for (int g4 = 0; g4 < 4; ++g4) {
                            const float4 be = *reinterpret_cast<const float4*>(sbeff + 8 * g4 + 4 * kh);
                            const uint2 o = make_uint2(
                                bf16_pair(fmaxf(a1[4 * g4] + be.x, 0.0f), fmaxf(a1[4 * g4 + 1] + be.y, 0.0f)),
                                bf16_pair(fmaxf(a1[4 * g4 + 2] + be.z, 0.0f), fmaxf(a1[4 * g4 + 3] + be.w, 0.0f)));
                            *reinterpret_cast<uint2*>(lds + s * PS + (8 * g4 + 4 * kh) * 2) = o;
                        }
                    }
                }
            }
            __syncthreads();
        }
        static_assert(CR == 4, "one output row per wave");
        const int rt = wv;  // tile row of this wave's output row
        const int y = y0 + rt;
        f32x16 acc = {};
        if (y < H) {
#pragma unroll
            for (int tap = 0; tap < 9; ++tap) {
                const int dy = tap / 3, dx = tap % 3;  // tile coordinates: row rt + dy, pixel m + dx
                const unsigned char* rowp = lds + ((rt + dy) * (TW + 2) + (m + dx)) * PS;
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) {
                    const bf16x8 a = *reinterpret_cast<const bf16x8*>(rowp + (ks * 16 + kh * 8) * 2);
                    // the weights as the A operand: the product is transposed, so the
                    // epilogue packs whole channel groups of a pixel
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(bw[tap * KS + ks], a, acc, 0, 0, 0);
                }
            }
        }
        // epilogue: the wave's 32 pixels x 32 channels go through LDS (the tile is
        // free once every wave has its products) so that each lane stores whole
        // 16-byte channel groups: lane l writes pixel l / 2, channels 16 (l % 2) ...
        __syncthreads();
        // lane l holds pixel l % 32, channels 8 g + 4 (l / 32) + r in accumulator 4 g + r:
        // four channels (8 bytes) per write into the wave's [pixel][channel] transpose
        unsigned char* ot = lds + wv * TW * OST;
#pragma unroll
        for (int g4 = 0; g4 < 4; ++g4) {
            float v[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) v[r] = acc[4 * g4 + r];
            if constexpr (MODE != 1) {
                const float4 bg = *reinterpret_cast<const float4*>(sbias + 8 * g4 + 4 * kh);
                v[0] = fmaxf(v[0] + bg.x, 0.0f);
                v[1] = fmaxf(v[1] + bg.y, 0.0f);
                v[2] = fmaxf(v[2] + bg.z, 0.0f);
                v[3] = fmaxf(v[3] + bg.w, 0.0f);
            }
            *reinterpret_cast<uint2*>(ot + m * OST + (8 * g4 + 4 * kh) * 2) =
                make_uint2(bf16_pair(v[0], v[1]), bf16_pair(v[2], v[3]));
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if constexpr (MODE == 3) {
            // P^T = W4 a3^T on the matrix cores: B[k = ci][n = pixel] is the wave's bf16
            // a3 row read back from the transpose (pixel m, channels 16 ks + 8 kh ...);
            // lane l then holds pixel l % 32, taps 4 (l / 32) + i (i < 4) and, for
            // l < 32, tap 8 in accumulator 4
            const bf16x8 a0 = *reinterpret_cast<const bf16x8*>(ot + m * OST + kh * 16);
            const bf16x8 a1 = *reinterpret_cast<const bf16x8*>(ot + m * OST + 32 + kh * 16);
            const bf16x8 w0 = *reinterpret_cast<const bf16x8*>(sw4 + m * W4S + kh * 8);
            const bf16x8 w1 = *reinterpret_cast<const bf16x8*>(sw4 + m * W4S + 16 + kh * 8);
            f32x16 pacc = {};
            pacc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w0, a0, pacc, 0, 0, 0);
            pacc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w1, a1, pacc, 0, 0, 0);
            if (y < H) {
                float* dst = tp.P + ((size_t)b * H + y) * W + x0 + m;
#pragma unroll
                for (int r = 0; r < 4; ++r) dst[(size_t)(4 * kh + r) * tp.plane] = pacc[r];
                if (kh == 0) dst[(size_t)8 * tp.plane] = pacc[4];
            }
        } else if (y < H) {
            const int p = lane >> 1, half = lane & 1;
            uint4 v0 = *reinterpret_cast<const uint4*>(ot + p * OST + half * 32);
            uint4 v1 = *reinterpret_cast<const uint4*>(ot + p * OST + half * 32 + 16);
            const size_t pidx = ((size_t)b * H + y) * W + x0 + p;
            if (MODE == 1) {
                // dgrad: keep the entries whose layer input was positive
                const uint4* mk = reinterpret_cast<const uint4*>(mask + pidx * 32 + half * 16);
                const uint4 m0 = mk[0], m1 = mk[1];
                // a bf16 is > 0 iff its sign bit is clear and it lies in (0, +inf]
                auto pos = [](unsigned h) { return h != 0u && h <= 0x7f80u; };
                auto gate = [&](unsigned g, unsigned mword) {
                    const unsigned lo = pos(mword & 0xffffu) ? 0xffffu : 0u;
                    const unsigned hi = pos(mword >> 16) ? 0xffff0000u : 0u;
                    return g & (lo | hi);
                };
                v0 = make_uint4(gate(v0.x, m0.x), gate(v0.y, m0.y), gate(v0.z, m0.z), gate(v0.w, m0.w));
                v1 = make_uint4(gate(v1.x, m1.x), gate(v1.y, m1.y), gate(v1.z, m1.z), gate(v1.w, m1.w));
            }
            uint4* dst = reinterpret_cast<uint4*>(out + pidx * 32 + half * 16);
            dst[0] = v0;
            dst[1] = v1;
        }
    }
#undef PF_CONV_FETCH
}

// wgrad of a hidden layer: part[block][tap][ci][co] = sum over this block's pixel
// tiles of a_in(p + tap)[ci] g(p)[co]; partb[block][co] = sum g(p)[co].
// CIN = 16 (first layer, channels 16..31 of the M tile are zero) or 32.
template <int CIN>
__global__ __launch_bounds__(NBLK) void k_wgrad_mfma(const u16* __restrict__ ain,
                                                     const u16* __restrict__ g, float* __restrict__ part,
                                                     float* __restrict__ partb, int B, int H, int W)
{
    __shared__ __align__(16) unsigned char la[Tile<CIN>::BYTES];
    __shared__ __align__(16) u16 lg[TR * TW * 32 + 8];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int m = lane & 31, kh = lane >> 5;
    const int tiles_x = W / TW, tiles_y = (H + TR - 1) / TR;
    const int ntiles = tiles_x * tiles_y * B;
    // wave wv owns taps wv, wv + 4, wv + 8
    f32x16 acc[3] = {{}, {}, {}};
    float db = 0.0f;
    for (int t0 = blockIdx.x; t0 < ntiles; t0 += gridDim.x) {
        int t = t0;
        const int tx = t % tiles_x;
        t /= tiles_x;
        const int ty = t % tiles_y;
        const int b = t / tiles_y;
        const int x0 = tx * TW, y0 = ty * TR;
        __syncthreads();
        stage_tile<CIN>(ain, b, H, W, y0, x0, la);
        for (int q = threadIdx.x; q < TR * TW * 4; q += NBLK) {  // 16-byte chunks of g
            const int ch = q & 3, pix = q >> 2;
            const int r = pix / TW, px = pix % TW;
            uint4 v = {0, 0, 0, 0};
            if (y0 + r < H)
                v = *reinterpret_cast<const uint4*>(g + ((((size_t)b * H + y0 + r) * W + x0 + px) * 32 + ch * 8));
            *reinterpret_cast<uint4*>(lg + pix * 32 + ch * 8) = v;
        }
        __syncthreads();
        // K loop over the tile's 128 pixels, 16 at a time (rows past H hold g = 0)
#pragma unroll 1
        for (int k0 = 0; k0 < TR * TW; k0 += 16) {
            // B operand: g[pixel k0 + 8 kh + j][co = m]
            bf16x8 bg;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const u16 bits = lg[(k0 + 8 * kh + j) * 32 + m];
                bg[j] = __builtin_bit_cast(__bf16, bits);
                if (wv == 0) db += bf16_val(bits);  // the bias gradient: lane (co, kh) sums its half
            }
#pragma unroll
            for (int s = 0; s < 3; ++s) {
                const int tap = wv + 4 * s;
                if (tap < 9) {
                    const int dy = tap / 3, dx = tap % 3;
                    bf16x8 aa;
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        const int p = k0 + 8 * kh + j;  // pixel of the tile: row p / TW, column p % TW
                        const int r = p / TW, px = p % TW;
                        u16 bits = 0;
                        if (m < CIN)
                            bits = *reinterpret_cast<const u16*>(
                                la + ((r + dy) * (TW + 2) + px + dx) * Tile<CIN>::PSTRIDE + m * 2);
                        aa[j] = __builtin_bit_cast(__bf16, bits);
                    }
                    acc[s] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aa, bg, acc[s], 0, 0, 0);
                }
            }
        }
    }
    // lanes co and co + 32 of wave 0 hold the two halves of the pixels
    db += __shfl_down(db, 32);
    // write this block's partial: C[ci][co] tile per tap
    float* pb = part + (size_t)blockIdx.x * 9 * 32 * 32;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        const int tap = wv + 4 * s;
        if (tap < 9)
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int ci = 8 * (i >> 2) + 4 * kh + (i & 3);
                pb[((size_t)tap * 32 + ci) * 32 + m] = acc[s][i];
            }
    }
    if (wv == 0 && lane < 32) partb[(size_t)blockIdx.x * 32 + lane] = db;
}

// out[i] = sum over blocks of part[block][i]  (i < n), fixed order: a block
// owns 32 columns; its 8 thread groups sum every 8th partial row (coalesced
// 128-byte row segments), then one fixed 8-way combine.
__global__ __launch_bounds__(NBLK) void k_sum_partials(const float* __restrict__ part, int nb,
                                                       int n, float* __restrict__ out)
{
    const int c = threadIdx.x & 31, grp = threadIdx.x >> 5;
    const int i = blockIdx.x * 32 + c;
    double s = 0.0;
    if (i < n)
        for (int b = grp; b < nb; b += NBLK / 32) s += (double)part[(size_t)b * n + i];
    __shared__ double sh[NBLK / 32][32];
    sh[grp][c] = s;
    __syncthreads();
    if (grp == 0 && i < n) {
        double t = 0.0;
        for (int q = 0; q < NBLK / 32; ++q) t += sh[q][c];
        out[i] = (float)t;
    }
}

// a0 = bf16 (c, M, kappa, 0 x 13) per pixel
__global__ __launch_bounds__(NBLK) void k_pack_input(const float* __restrict__ c,
                                                     const float* __restrict__ Mv,
                                                     const float* __restrict__ kv, u16* __restrict__ a0,
                                                     int B, int HW)
{
    const size_t p = (size_t)blockIdx.x * NBLK + threadIdx.x;
    if (p >= (size_t)B * HW) return;
    const int b = (int)(p / HW);
    u16 v[16] = {};
    v[0] = bf16_bits(c[p]);
    v[1] = bf16_bits(Mv[b]);
    v[2] = bf16_bits(kv[b]);
    uint4* dst = reinterpret_cast<uint4*>(a0 + p * 16);
    dst[0] = *reinterpret_cast<uint4*>(&v[0]);
    dst[1] = *reinterpret_cast<uint4*>(&v[8]);
}

// FP32 master parameters -> bf16 B fragments.  Hidden layer l, use u (0 forward, 1 dgrad):
//   forward: B[k = 16 ks + j'][n = co] = W[tap][ci = 16 ks + j'][co]
//   dgrad:   B[k = 16 ks + j'][n = ci] = W[8 - tap][ci' = ... ] with the roles of ci, co swapped
// frag layout [tap][ks][lane][8]: lane supplies k = 16 ks + 8 (lane / 32) + j, n = lane % 32.
__global__ __launch_bounds__(NBLK) void k_prep_weights(const float* __restrict__ params,
                                                       NNOffsets off, u16* __restrict__ frag,
                                                       NNFragOffsets fo, u16* __restrict__ w4)
{
    const int t = blockIdx.x * NBLK + threadIdx.x;
    // hidden layers: 3 forward fragments (cin 16/32/32) + 2 dgrad fragments (layers 2, 3)
    const int n1 = 9 * 1 * 64 * 8, n2 = 9 * 2 * 64 * 8;
    if (t < n1) {  // layer 1 forward, CIN padded 3 -> 16
        const int j = t & 7, lane = (t >> 3) & 63, tap = t / (64 * 8);
        const int k = 8 * (lane >> 5) + j, co = lane & 31;
        const float w = k < 3 ? params[off.w1 + (tap * 3 + k) * 32 + co] : 0.0f;
        frag[fo.f1 + t] = bf16_bits(w);
        return;
    }
    int u = t - n1;
    for (int l = 0; l < 2; ++l) {       // layers 2, 3 forward
        if (u < n2) {
            const int j = u & 7, lane = (u >> 3) & 63, q = u / (64 * 8);
            const int tap = q / 2, ks = q % 2;
            const int ci = 16 * ks + 8 * (lane >> 5) + j, co = lane & 31;
            const size_t wo = (l == 0 ? off.w2 : off.w3) + ((size_t)tap * 32 + ci) * 32 + co;
            frag[(l == 0 ? fo.f2 : fo.f3) + u] = bf16_bits(params[wo]);
            return;
        }
        u -= n2;
    }
    for (int l = 0; l < 2; ++l) {       // layers 2, 3 dgrad: out channel = ci, k = co, tap flipped
        if (u < n2) {
            const int j = u & 7, lane = (u >> 3) & 63, q = u / (64 * 8);
            const int tap = q / 2, ks = q % 2;
            const int co = 16 * ks + 8 * (lane >> 5) + j, ci = lane & 31;
            const size_t wo = (l == 0 ? off.w2 : off.w3) + ((size_t)(8 - tap) * 32 + ci) * 32 + co;
            frag[(l == 0 ? fo.d2 : fo.d3) + u] = bf16_bits(params[wo]);
            return;
        }
        u -= n2;
    }
    if (u < 9 * 32) w4[u] = bf16_bits(params[off.w4 + u]);
}

// output layer forward: d[p] = b4 + sum_tap sum_ci W4[tap][ci] a3[p + tap][ci]  (fp32)
// Output layer (32 -> 1): a block stages the a3 halo tile of OR rows x 32 pixels
// in LDS (the conflict-free stride of the hidden layers) and each thread forms one
// pixel's 288-term sum with the packed bf16 dot instruction (two products per
// step, FP32 accumulation), the weights broadcast from LDS.
constexpr int OR = NBLK / TW;  // 8 rows: one pixel per thread
__global__ __launch_bounds__(NBLK) void k_out_fwd(const u16* __restrict__ a3, const u16* __restrict__ w4,
                                                  const float* __restrict__ params, NNOffsets off,
                                                  float* __restrict__ d, int B, int H, int W)
{
    constexpr int PS = Tile<32, OR>::PSTRIDE;
    __shared__ __align__(16) unsigned char la[Tile<32, OR>::BYTES];
    __shared__ uint4 sw[9 * 4];  // weights as bf16 pairs [tap][16 pairs]
    const int tiles_x = W / TW, tiles_y = (H + OR - 1) / OR;
    const int tx = blockIdx.x % tiles_x, ty = (blockIdx.x / tiles_x) % tiles_y, b = blockIdx.x / (tiles_x * tiles_y);
    const int x0 = tx * TW, y0 = ty * OR;
    if (threadIdx.x < 9 * 4) sw[threadIdx.x] = reinterpret_cast<const uint4*>(w4)[threadIdx.x];
    stage_tile<32, OR>(a3, b, H, W, y0, x0, la);
    __syncthreads();
    const int r = threadIdx.x / TW, m = threadIdx.x % TW;
    const int y = y0 + r;
    if (y >= H) return;
    auto dot8 = [](const uint4& a, const uint4& w, float acc) {
        acc = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2, a.x), __builtin_bit_cast(bf16x2, w.x), acc,
                                              false);
        acc = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2, a.y), __builtin_bit_cast(bf16x2, w.y), acc,
                                              false);
        acc = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2, a.z), __builtin_bit_cast(bf16x2, w.z), acc,
                                              false);
        return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2, a.w), __builtin_bit_cast(bf16x2, w.w),
                                               acc, false);
    };
    float sum = params[off.b4];
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
        const int dy = tap / 3, dx = tap % 3;
        const uint4* ap = reinterpret_cast<const uint4*>(la + ((r + dy) * (TW + 2) + (m + dx)) * PS);
#pragma unroll
        for (int q = 0; q < 4; ++q) sum = dot8(ap[q], sw[tap * 4 + q], sum);
    }
    d[((size_t)b * H + y) * W + x0 + m] = sum;
}

// Output layer from the tap planes of MODE 3: d[p] = b4 + sum_tap P[tap][p + tap]
// (periodic neighbours, taps in order), and the per-sample partial sums of d that
// k_sample_sum would form (same blocks, same reduction tree): part[b * nbs + blk].
__global__ __launch_bounds__(NBLK) void k_out_taps(const float* __restrict__ P, long long plane,
                                                   const float* __restrict__ params, NNOffsets off,
                                                   float* __restrict__ d, double* __restrict__ part, int H,
                                                   int W)
{
    const int HW = H * W, nbs = (HW + NBLK - 1) / NBLK;
    const int b = blockIdx.x / nbs, blk = blockIdx.x % nbs;
    const int i = blk * NBLK + threadIdx.x;
    double v = 0.0;
    if (i < HW) {
        const int y = i / W, x = i % W;
        const int ym = y == 0 ? H - 1 : y - 1, yp = y == H - 1 ? 0 : y + 1;
        const int xm = x == 0 ? W - 1 : x - 1, xp = x == W - 1 ? 0 : x + 1;
        const int rows[3] = {ym, y, yp}, cols[3] = {xm, x, xp};
        const float* Pb = P + (size_t)b * HW;
        float s = params[off.b4];
#pragma unroll
        for (int tap = 0; tap < 9; ++tap)
            s += Pb[(size_t)tap * plane + (size_t)rows[tap / 3] * W + cols[tap % 3]];
        d[(size_t)b * HW + i] = s;
        v = (double)s;
    }
    __shared__ double sh[NBLK];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int st = NBLK / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// per-sample partial sums of x over blocks of NBLK pixels: part[b * nbs + blk]
__global__ __launch_bounds__(NBLK) void k_sample_sum(const float* __restrict__ x, int HW,
                                                     double* __restrict__ part)
{
    const int nbs = (HW + NBLK - 1) / NBLK;
    const int b = blockIdx.x / nbs, blk = blockIdx.x % nbs;
    const int i = blk * NBLK + threadIdx.x;
    double v = i < HW ? (double)x[(size_t)b * HW + i] : 0.0;
    __shared__ double sh[NBLK];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = NBLK / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(NBLK) void k_sample_mean(const double* __restrict__ part, int nbs,
                                                      int HW, double* __restrict__ mean)
{
    const int b = blockIdx.x;
    __shared__ double sh[NBLK];
    double a = 0.0;
    for (int i = threadIdx.x; i < nbs; i += NBLK) a += part[(size_t)b * nbs + i];
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int s = NBLK / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) mean[b] = sh[0] / (double)HW;
}

// c_hat = c + d - mean(d); with a target also g = 2 (c_hat - t)/HW and the squared error r2
__global__ __launch_bounds__(NBLK) void k_project(const float* __restrict__ c, const float* __restrict__ d,
                                                  const double* __restrict__ mean, const float* __restrict__ tgt,
                                                  float* __restrict__ chat, float* __restrict__ g,
                                                  float* __restrict__ r2, int B, int HW)
{
    const size_t p = (size_t)blockIdx.x * NBLK + threadIdx.x;
    if (p >= (size_t)B * HW) return;
    const int b = (int)(p / HW);
    const float ch = c[p] + (float)((double)d[p] - mean[b]);
    chat[p] = ch;
    if (tgt) {
        const float r = ch - tgt[p];
        g[p] = 2.0f * r / (float)HW;
        r2[p] = r * r;
    }
}

// Inference: c_hat = c + d - mean(d), the mean reduced by every block from the sample's
// partials exactly as k_sample_mean does (so bitwise its value); 4 pixels per thread,
// blockIdx.y = sample.  Needs HW % 4 == 0 and 16-byte aligned c, d, c_hat.
__global__ __launch_bounds__(NBLK) void k_project_mean(const float* __restrict__ c, const float* __restrict__ d,
                                                       const double* __restrict__ part, int nbs,
                                                       float* __restrict__ chat, int HW)
{
    const int b = blockIdx.y;
    __shared__ double sh[NBLK];
    double a = 0.0;
    for (int i = threadIdx.x; i < nbs; i += NBLK) a += part[(size_t)b * nbs + i];
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int s = NBLK / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    const double mean = sh[0] / (double)HW;
    const int i4 = (blockIdx.x * NBLK + threadIdx.x) * 4;
    if (i4 >= HW) return;
    const size_t p = (size_t)b * HW + i4;
    const float4 cv = *reinterpret_cast<const float4*>(c + p), dv = *reinterpret_cast<const float4*>(d + p);
    float4 o;
    o.x = cv.x + (float)((double)dv.x - mean);
    o.y = cv.y + (float)((double)dv.y - mean);
    o.z = cv.z + (float)((double)dv.z - mean);
    o.w = cv.w + (float)((double)dv.w - mean);
    *reinterpret_cast<float4*>(chat + p) = o;
}

// g <- g - mean(g) (backward of the mass projection)
__global__ __launch_bounds__(NBLK) void k_center(float* __restrict__ g, const double* __restrict__ mean,
                                                 int B, int HW)
{
    const size_t p = (size_t)blockIdx.x * NBLK + threadIdx.x;
    if (p >= (size_t)B * HW) return;
    g[p] = (float)((double)g[p] - mean[p / HW]);
}

// output layer dgrad: ga3[p][ci] = bf16( (a3[p][ci] > 0) * sum_tap W4[tap][ci] g[p - off(tap)] )
__global__ __launch_bounds__(NBLK) void k_out_dgrad(const u16* __restrict__ a3, const u16* __restrict__ w4,
                                                    const float* __restrict__ g, u16* __restrict__ ga3,
                                                    int B, int H, int W)
{
    __shared__ float sw[9 * 32];
    for (int i = threadIdx.x; i < 9 * 32; i += NBLK) sw[i] = bf16_val(w4[i]);
    __syncthreads();
    const size_t p = (size_t)blockIdx.x * NBLK + threadIdx.x;
    const size_t HW = (size_t)H * W;
    if (p >= (size_t)B * HW) return;
    const int b = (int)(p / HW), r = (int)(p % HW), y = r / W, x = r % W;
    float gin[9];
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
        const int yy = wrapi(y - (tap / 3 - 1), H), xx = wrapi(x - (tap % 3 - 1), W);
        gin[tap] = g[((size_t)b * H + yy) * W + xx];
    }
    const u16* ap = a3 + p * 32;
    u16 outv[32];
#pragma unroll
    for (int ci = 0; ci < 32; ++ci) {
        float sum = 0.0f;
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) sum = fmaf(sw[tap * 32 + ci], gin[tap], sum);
        outv[ci] = bf16_bits(bf16_val(ap[ci]) > 0.0f ? sum : 0.0f);
    }
    uint4* dst = reinterpret_cast<uint4*>(ga3 + p * 32);
#pragma unroll
    for (int q = 0; q < 4; ++q) dst[q] = *reinterpret_cast<uint4*>(&outv[8 * q]);
}

// Output layer's weight gradient: part[block][tap * 32 + ci] = sum over this block's
// pixels p of a3(p + tap)[ci] g(p), part[block][288] = sum g(p).  Written per pixel q
// of a3 instead: a3(q)[ci] times g at the 3 x 3 neighbourhood of q, an outer product
// of 32 channels and 9 taps.  A block walks tiles of OWR rows x 32 pixels (a fixed
// stride of them: split-K over pixels); thread (pixel px, channel group cg) reads its
// 4 channels of a3 (8 bytes, 64 contiguous bytes per pixel, one coalesced read of
// a3 per launch) and keeps 9 x 4 FP32 sums; g's (OWR + 2) x 34 neighbourhood tile
// sits in LDS.  The sums are reduced over the block's 32 pixel lanes at the end.
constexpr int OWR = 8;  // rows per tile of k_out_wgrad
__global__ __launch_bounds__(NBLK) void k_out_wgrad(const u16* __restrict__ a3, const float* __restrict__ g,
                                                    float* __restrict__ part, int B, int H, int W)
{
    __shared__ float gl[OWR + 2][TW + 2];
    __shared__ float red[NBLK / 64][8][37];
    const int tiles_x = W / TW, tiles_y = (H + OWR - 1) / OWR;
    const int ntiles = tiles_x * tiles_y * B;
    const int px = threadIdx.x >> 3, cg = threadIdx.x & 7;
    float acc[9][4];
#pragma unroll
    for (int tap = 0; tap < 9; ++tap)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[tap][c] = 0.0f;
    float db = 0.0f;
    for (int t0 = blockIdx.x; t0 < ntiles; t0 += gridDim.x) {
        int t = t0;
        const int tx = t % tiles_x;
        t /= tiles_x;
        const int ty = t % tiles_y;
        const int b = t / tiles_y;
        const int x0 = tx * TW, y0 = ty * OWR;
        __syncthreads();  // the previous tile's reads of gl are done
        for (int q = threadIdx.x; q < (OWR + 2) * (TW + 2); q += NBLK) {
            const int r = q / (TW + 2), cx = q % (TW + 2);
            const int gy = ((y0 - 1 + r) % H + H) % H, gx = wrapi(x0 - 1 + cx, W);  // H may be < OWR
            gl[r][cx] = g[((size_t)b * H + gy) * W + gx];
        }
        __syncthreads();
        const int rows = min(OWR, H - y0);
        for (int r = 0; r < rows; ++r) {
            const uint2 av = *reinterpret_cast<const uint2*>(
                a3 + (((size_t)b * H + y0 + r) * W + x0 + px) * 32 + cg * 4);
            const float a[4] = {bf16_val((u16)(av.x & 0xffffu)), bf16_val((u16)(av.x >> 16)),
                                bf16_val((u16)(av.y & 0xffffu)), bf16_val((u16)(av.y >> 16))};
            // tap (dy, dx) pairs a3(p + (dy - 1, dx - 1)) with g(p): for a3 at q that is
            // g(q + (1 - dy, 1 - dx)), tile entry (r + 2 - dy, px + 2 - dx)
#pragma unroll
            for (int tap = 0; tap < 9; ++tap) {
                const float gv = gl[r + 2 - tap / 3][px + 2 - tap % 3];
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[tap][c] = fmaf(a[c], gv, acc[tap][c]);
            }
            if (cg == 0) db += gl[r + 1][px + 1];
        }
    }
    // sum over the 8 pixel lanes of each wave (lane = 8 p + cg), then over the waves
#pragma unroll
    for (int off = 8; off < 64; off <<= 1) {
#pragma unroll
        for (int tap = 0; tap < 9; ++tap)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[tap][c] += __shfl_xor(acc[tap][c], off, 64);
        db += __shfl_xor(db, off, 64);
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane < 8) {
#pragma unroll
        for (int tap = 0; tap < 9; ++tap)
#pragma unroll
            for (int c = 0; c < 4; ++c) red[wv][lane][tap * 4 + c] = acc[tap][c];
        red[wv][lane][36] = db;
    }
    __syncthreads();
    for (int o = threadIdx.x; o < 289; o += NBLK) {
        float v = 0.0f;
        if (o < 288) {
            const int tap = o / 32, ci = o % 32;
            for (int w = 0; w < NBLK / 64; ++w) v += red[w][ci / 4][tap * 4 + ci % 4];
        } else {
            for (int w = 0; w < NBLK / 64; ++w) v += red[w][0][36];
        }
        part[(size_t)blockIdx.x * 289 + o] = v;
    }
}

// Adam on FP32 masters (bias-corrected; Kingma & Ba)
__global__ __launch_bounds__(NBLK) void k_adam(float* __restrict__ p, float* __restrict__ m,
                                               float* __restrict__ v, const float* __restrict__ g, int n,
                                               float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int i = blockIdx.x * NBLK + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Residual check of a surrogate jump (per sample, [B, HW] arrays, FP64 sums):
//   part[3 (b nbs + blk) + 0] += sum ((c_hat - c_prev)/(K dt) + (c_hat - c_step)/dt)^2
//   part[... + 1]             += sum ((c_hat - c_prev)/(K dt))^2
//   part[... + 2]             += sum (c_hat - c_prev)
// where c_step is one explicit step of c_hat, so (c_hat - c_step)/dt = M K mu(c_hat)/m and
// the first sum is the squared backward-Euler residual of the jump divided by m.
__global__ __launch_bounds__(NBLK) void k_check_sums(const float* __restrict__ chat,
                                                     const float* __restrict__ cprev,
                                                     const float* __restrict__ cstep, int HW,
                                                     double inv_kdt, double inv_dt,
                                                     double* __restrict__ part)
{
    const int nbs = (HW + NBLK - 1) / NBLK;
    const int b = blockIdx.x / nbs, blk = blockIdx.x % nbs;
    const int i = blk * NBLK + threadIdx.x;
    double v0 = 0.0, v1 = 0.0, v2 = 0.0;
    if (i < HW) {
        const size_t p = (size_t)b * HW + i;
        const double dj = (double)chat[p] - (double)cprev[p];
        const double rt = dj * inv_kdt + ((double)chat[p] - (double)cstep[p]) * inv_dt;
        v0 = rt * rt;
        v1 = dj * inv_kdt * dj * inv_kdt;
        v2 = dj;
    }
    __shared__ double sh[3][NBLK];
    sh[0][threadIdx.x] = v0;
    sh[1][threadIdx.x] = v1;
    sh[2][threadIdx.x] = v2;
    __syncthreads();
    for (int s = NBLK / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int q = 0; q < 3; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int q = 0; q < 3; ++q) part[3 * (size_t)blockIdx.x + q] = sh[q][0];
}

__global__ __launch_bounds__(NBLK) void k_check_final(const double* __restrict__ part, int nbs,
                                                      double* __restrict__ out)
{
    const int b = blockIdx.x;
    __shared__ double sh[3][NBLK];
    for (int q = 0; q < 3; ++q) {
        double a = 0.0;
        for (int i = threadIdx.x; i < nbs; i += NBLK) a += part[3 * ((size_t)b * nbs + i) + q];
        sh[q][threadIdx.x] = a;
    }
    __syncthreads();
    for (int s = NBLK / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int q = 0; q < 3; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[3 * b + 0] = sqrt(sh[0][0]) / fmax(sqrt(sh[1][0]), 1e-300);  // rho
        out[3 * b + 1] = sh[2][0];                                        // sum (c_hat - c_prev)
        out[3 * b + 2] = sqrt(sh[1][0]);                                  // ||jump|| / (K dt)
    }
}

// first-layer weight gradient: dW1[tap][ci][co] = tile[tap][ci][co] for ci < 3
__global__ __launch_bounds__(NBLK) void k_extract_w1(const float* __restrict__ tile, float* __restrict__ dw1)
{
    const int i = blockIdx.x * NBLK + threadIdx.x;
    if (i >= 9 * 3 * 32) return;
    const int co = i % 32, ci = (i / 32) % 3, tap = i / 96;
    dw1[i] = tile[(tap * 32 + ci) * 32 + co];
}

}  // namespace

// ---------------------------------------------------------------------------
void nn_check(const float* chat, const float* cprev, const float* cstep, int B, int HW, double kdt,
              double dt, double* part, double* out, hipStream_t s)
{
    const int nbs = (HW + NBLK - 1) / NBLK;
    k_check_sums<<<B * nbs, NBLK, 0, s>>>(chat, cprev, cstep, HW, 1.0 / kdt, 1.0 / dt, part);
    k_check_final<<<B, NBLK, 0, s>>>(part, nbs, out);
}

void nn_extract_w1(const float* tile, float* dw1, hipStream_t s)
{
    k_extract_w1<<<(9 * 3 * 32 + NBLK - 1) / NBLK, NBLK, 0, s>>>(tile, dw1);
}

NNOffsets nn_offsets()
{
    NNOffsets o{};
    int k = 0;
    o.w1 = k; k += 9 * 3 * 32;
    o.b1 = k; k += 32;
    o.w2 = k; k += 9 * 32 * 32;
    o.b2 = k; k += 32;
    o.w3 = k; k += 9 * 32 * 32;
    o.b3 = k; k += 32;
    o.w4 = k; k += 9 * 32;
    o.b4 = k; k += 1;
    o.total = k;
    return o;
}

NNFragOffsets nn_frag_offsets()
{
    NNFragOffsets f{};
    const int n1 = 9 * 64 * 8, n2 = 9 * 2 * 64 * 8;
    f.f1 = 0;
    f.f2 = n1;
    f.f3 = n1 + n2;
    f.d2 = n1 + 2 * n2;
    f.d3 = n1 + 3 * n2;
    f.total = n1 + 4 * n2;
    return f;
}

int nn_wgrad_blocks(int B, int H, int W)
{
    const long long tiles = (long long)B * ((H + TR - 1) / TR) * (W / TW);
    return (int)(tiles < 1024 ? tiles : 1024);
}

int nn_conv_blocks(int B, int H, int W) { return B * ((H + CR - 1) / CR) * (W / TW); }

// resident blocks of a conv kernel on the current device (queried once per kernel)
template <int CIN, int MODE>
int conv_resident_blocks()
{
    static const int n = [] {
        int dev = 0, cus = 0, per = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_conv_mfma<CIN, MODE>, NBLK, 0) != hipSuccess)
            return 1024;
        return std::max(1, cus * per);
    }();
    return n;
}

void nn_prep_weights(const float* params, u16* frag, u16* w4, hipStream_t s)
{
    const NNFragOffsets fo = nn_frag_offsets();
    const int n = fo.total + 9 * 32;
    k_prep_weights<<<(n + NBLK - 1) / NBLK, NBLK, 0, s>>>(params, nn_offsets(), frag, fo, w4);
}

void nn_pack_input(const float* c, const float* M, const float* kappa, u16* a0, int B, int HW,
                   hipStream_t s)
{
    const size_t n = (size_t)B * HW;
    k_pack_input<<<(unsigned)((n + NBLK - 1) / NBLK), NBLK, 0, s>>>(c, M, kappa, a0, B, HW);
}

void nn_conv(int layer, int mode, const u16* in, const u16* frag, const float* bias, const u16* mask,
             u16* out, int B, int H, int W, hipStream_t s)
{
    const int nt = nn_conv_blocks(B, H, W);
    auto grid = [&](int resident) { return (unsigned)std::max(1, std::min(nt, resident)); };
    const InPlanes none{nullptr, nullptr, nullptr, nullptr, nullptr};
    const TapPlanes np{nullptr, nullptr, 0};
    if (layer == 1)
        k_conv_mfma<16, 0><<<grid(conv_resident_blocks<16, 0>()), NBLK, 0, s>>>(in, frag, bias, mask, out, B, H,
                                                                               W, nt, none, np);
    else if (mode == 0)
        k_conv_mfma<32, 0><<<grid(conv_resident_blocks<32, 0>()), NBLK, 0, s>>>(in, frag, bias, mask, out, B, H,
                                                                               W, nt, none, np);
    else
        k_conv_mfma<32, 1><<<grid(conv_resident_blocks<32, 1>()), NBLK, 0, s>>>(in, frag, bias, mask, out, B, H,
                                                                               W, nt, none, np);
}

void nn_conv12_planes(const float* c, const float* M, const float* kappa, const float* w1, const float* b1,
                      const u16* frag2, const float* bias2, u16* out, int B, int H, int W, hipStream_t s)
{
    const int nt = nn_conv_blocks(B, H, W);
    const unsigned g = (unsigned)std::max(1, std::min(nt, conv_resident_blocks<32, 4>()));
    k_conv_mfma<32, 4><<<g, NBLK, 0, s>>>(nullptr, frag2, bias2, nullptr, out, B, H, W, nt,
                                          InPlanes{c, M, kappa, w1, b1}, TapPlanes{nullptr, nullptr, 0});
}

void nn_conv3_taps(const u16* in, const u16* frag, const float* bias, const u16* w4, float* P, int B, int H, int W,
                   hipStream_t s)
{
    const int nt = nn_conv_blocks(B, H, W);
    const unsigned g = (unsigned)std::max(1, std::min(nt, conv_resident_blocks<32, 3>()));
    k_conv_mfma<32, 3><<<g, NBLK, 0, s>>>(in, frag, bias, nullptr, nullptr, B, H, W, nt,
                                          InPlanes{nullptr, nullptr, nullptr, nullptr, nullptr},
                                          TapPlanes{w4, P, (long long)B * H * W});
}

void nn_out_taps_project(const float* P, const float* params, const float* c, float* d, double* part,
                         double* mean, float* chat, int B, int H, int W, hipStream_t s)
{
    const int HW = H * W, nbs = (HW + NBLK - 1) / NBLK;
    k_out_taps<<<(unsigned)(B * nbs), NBLK, 0, s>>>(P, (long long)B * HW, params, nn_offsets(), d, part, H, W);
    const bool vec = HW % 4 == 0 && ((reinterpret_cast<uintptr_t>(c) | reinterpret_cast<uintptr_t>(d) |
                                      reinterpret_cast<uintptr_t>(chat)) & 15) == 0;
    if (vec) {
        k_project_mean<<<dim3((unsigned)((HW / 4 + NBLK - 1) / NBLK), (unsigned)B), NBLK, 0, s>>>(c, d, part, nbs,
                                                                                                chat, HW);
    } else {
        k_sample_mean<<<B, NBLK, 0, s>>>(part, nbs, HW, mean);
        nn_project(c, d, mean, nullptr, chat, nullptr, nullptr, B, HW, s);
    }
}

void nn_wgrad(int layer, const u16* ain, const u16* g, float* part, float* partb, int B, int H, int W,
              hipStream_t s)
{
    const int nb = nn_wgrad_blocks(B, H, W);
    if (layer == 1)
        k_wgrad_mfma<16><<<nb, NBLK, 0, s>>>(ain, g, part, partb, B, H, W);
    else
        k_wgrad_mfma<32><<<nb, NBLK, 0, s>>>(ain, g, part, partb, B, H, W);
}

void nn_sum_partials(const float* part, int nb, int n, float* out, hipStream_t s)
{
    k_sum_partials<<<(n + 31) / 32, NBLK, 0, s>>>(part, nb, n, out);
}

void nn_out_fwd(const u16* a3, const u16* w4, const float* params, float* d, int B, int H, int W,
                hipStream_t s)
{
    const unsigned nb = (unsigned)B * (unsigned)((H + OR - 1) / OR) * (unsigned)(W / TW);
    k_out_fwd<<<nb, NBLK, 0, s>>>(a3, w4, params, nn_offsets(), d, B, H, W);
}

void nn_sample_mean(const float* x, double* part, double* mean, int B, int HW, hipStream_t s)
{
    const int nbs = (HW + NBLK - 1) / NBLK;
    k_sample_sum<<<B * nbs, NBLK, 0, s>>>(x, HW, part);
    k_sample_mean<<<B, NBLK, 0, s>>>(part, nbs, HW, mean);
}

void nn_project(const float* c, const float* d, const double* mean, const float* tgt, float* chat,
                float* g, float* r2, int B, int HW, hipStream_t s)
{
    const size_t n = (size_t)B * HW;
    k_project<<<(unsigned)((n + NBLK - 1) / NBLK), NBLK, 0, s>>>(c, d, mean, tgt, chat, g, r2, B, HW);
}

void nn_center(float* g, const double* mean, int B, int HW, hipStream_t s)
{
    const size_t n = (size_t)B * HW;
    k_center<<<(unsigned)((n + NBLK - 1) / NBLK), NBLK, 0, s>>>(g, mean, B, HW);
}

int nn_out_wgrad_blocks(int B, int H, int W)
{
    const long long tiles = (long long)B * ((H + OWR - 1) / OWR) * (W / TW);
    return (int)(tiles < 1024 ? tiles : 1024);
}

void nn_out_bwd(const u16* a3, const u16* w4, const float* g, u16* ga3, float* part, int B, int H,
                int W, hipStream_t s)
{
    const size_t n = (size_t)B * H * W;
    k_out_dgrad<<<(unsigned)((n + NBLK - 1) / NBLK), NBLK, 0, s>>>(a3, w4, g, ga3, B, H, W);
    k_out_wgrad<<<nn_out_wgrad_blocks(B, H, W), NBLK, 0, s>>>(a3, g, part, B, H, W);
}

void nn_adam(float* p, float* m, float* v, const float* g, int n, int t, double lr, double b1,
             double b2, double eps, hipStream_t s)
{
    const double c1 = 1.0 - std::pow(b1, t), c2 = 1.0 - std::pow(b2, t);
    k_adam<<<(n + NBLK - 1) / NBLK, NBLK, 0, s>>>(p, m, v, g, n, (float)lr, (float)b1, (float)b2,
                                                  (float)eps, (float)c1, (float)c2);
}

}  // namespace pfk
