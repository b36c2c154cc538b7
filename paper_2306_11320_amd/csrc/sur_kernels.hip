// gfx950 kernels of the learned surrogate: a residual network of 3x3
// convolutions over (phi, u_x, u_y, T) frames that advances the lattice state
// by a fixed number of time steps.  Activations and weights are BF16, all
// products accumulate in FP32 on the matrix cores (v_mfma_f32_32x32x16_bf16).
//
// Layouts: activations NHWC with C = 32 channels (the 4-channel network input
// is padded to C = 8), weights [co = 32][tap = 9][ci] (rows beyond the layer's
// real output channels are zero), taps ordered (dy, dx) = (-1..1, -1..1) with
// tap = 3 (dy + 1) + (dx + 1).  Frames are periodic in x and zero-padded in y
// (x is the periodic direction of the lattices the surrogate stands in for).
//
// Convolution as an implicit GEMM: one wave computes a 32-pixel x 32-channel
// output block; the reduction runs over K = 9 Cin in blocks of 16, where each
// lane's 8 consecutive K entries are 8 consecutive channels of one tap, i.e.
// one 16-byte load from NHWC memory and one from the weights.
// MFMA 32x32x16 operand layout (checked on the device): lane l holds
// A[l % 32][8 (l / 32) + j] and B[8 (l / 32) + j][l % 32], j = 0..7; the
// accumulator element i of lane l is C[8 (i / 4) + 4 (l / 32) + i % 4][l % 32].
#include "sur_internal.hpp"
#include <mutex>

namespace sur {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ inline bf16x8 load8(const bf16* p)
{
    return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(p));
}

typedef short s16x8 __attribute__((ext_vector_type(8)));

// max(v, 0) of 8 BF16 values as packed 16-bit integer maxima: a BF16 value
// with its sign bit set is a negative 16-bit integer and a positive one a
// positive integer, so the integer maximum with 0 is the ReLU (-0 becomes +0)
// at four packed instructions instead of eight conversions and selects.
__device__ inline bf16x8 relu8(bf16x8 v)
{
    const s16x8 s = __builtin_bit_cast(s16x8, v);
    return __builtin_bit_cast(bf16x8, __builtin_elementwise_max(s, (s16x8)(short)0));
}

__device__ inline float to_f(bf16 v) { return (float)v; }

// Epilogue of one segment: element i of the accumulator is pixel
// x0 + 4 kh + 8 (i / 4) + i % 4 of the row (offset o_row of its first pixel,
// channel 0), channel co.  A segment inside the row (every segment of a row
// whose width is a multiple of 32) stores without per-pixel tests.
template <bool OUTF32, bool RES, bool MASK>
__device__ inline void conv_store(const f32x16& acc, float bv, const void* __restrict__ res,
                                  const bf16* __restrict__ mask, void* __restrict__ out, long long o_row, int x0, int W,
                                  int kh, int co)
{
    const long long o0 = o_row + (4 * kh) * 32 + co;
    auto one = [&](int i) {
        const long long idx = o0 + (8 * (i / 4) + (i % 4)) * 32;
        float v = acc[i] + bv;
        if (MASK) v = to_f(mask[idx]) > 0.f ? v : 0.f;
        if (OUTF32) {
            if (RES) v += static_cast<const float*>(res)[idx];
            static_cast<float*>(out)[idx] = v;
        } else {
            if (RES) v += to_f(static_cast<const bf16*>(res)[idx]);
            static_cast<bf16*>(out)[idx] = (bf16)v;
        }
    };
    if (x0 + 32 <= W) {
#pragma unroll
        for (int i = 0; i < 16; ++i) one(i);
    } else {
#pragma unroll
        for (int i = 0; i < 16; ++i)
            if (x0 + 4 * kh + 8 * (i / 4) + (i % 4) < W) one(i);
    }
}

// Per-wave LDS tile of the output layer's transposed epilogue: half a segment
// (16 pixels) of the accumulator, 32 channels in FP32, rows of kTP floats (the
// two halves of a wave's write, 4 rows apart, fall on disjoint banks).  The
// same transposition for the hidden layers' BF16 stores and residual loads
// (16-byte accesses, 4 memory instructions per segment instead of 32) was
// measured without gain: their cost is the bytes moved, not the instructions.
constexpr int kTP = 40;
typedef float TTile[16][kTP];

// Orders a wave's LDS writes before its lanes read what other lanes wrote.
__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Writes half h (pixels 16 h .. 16 h + 15 of the segment) of acc + bias to
// the tile: element i of the accumulator is pixel 8 (i / 4) + 4 kh + i % 4,
// channel co.
__device__ inline void tile_half(TTile& T, const f32x16& acc, float bv, int h, int kh, int co)
{
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int i = 8 * h + j;
        T[8 * (i / 4) + 4 * kh + i % 4 - 16 * h][co] = acc[i] + bv;
    }
}

// One 32-pixel segment of a 32-channel layer (row y of frame n, pixels x0 ..
// x0 + 31).  K block q is tap q / 2, channels 16 (q % 2) + 8 kh ... + 7: the
// three tap rows (clamped to the frame) and the three tap columns (periodic)
// are computed once per segment, and all 18 operands are loaded before the
// first matrix-core op.  A tap row outside the frame contributes nothing: its
// K blocks take their weight operands from the all-zero block sB[18] (a
// scalar choice of LDS address per block; the clamped row's activations are
// finite, so the products are exact zeros, as if the inputs were zeroed by a
// select per operand register).
template <bool RELU>
__device__ __forceinline__ f32x16 conv_seg32(const bf16* __restrict__ in, const bf16x8 (*__restrict__ sB)[64], int lz,
                                             int dil, int H, int W, int n, int y, int x0, int m, int kh)
{
    constexpr int CIN = 32, NKB = 18;
    const int xm = x0 + m < W ? x0 + m : W - 1;
    const bf16* rowp[3];
    bool rok[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const int yy = y + (r - 1) * dil;
        rok[r] = yy >= 0 && yy < H;
        rowp[r] = in + ((long long)n * H + (rok[r] ? yy : y)) * W * CIN + 8 * kh;
    }
    int xc[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int xx = xm + (c - 1) * dil;  // |offset| <= W, so one wrap suffices
        xc[c] = (xx < 0 ? xx + W : (xx >= W ? xx - W : xx)) * CIN;
    }
    bf16x8 a[NKB];
#pragma unroll
    for (int q = 0; q < NKB; ++q) {
        const int tap = q >> 1;
        a[q] = load8(rowp[tap / 3] + xc[tap % 3] + 16 * (q & 1));
    }
    f32x16 acc = {};
#pragma unroll
    for (int q = 0; q < NKB; ++q)
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(RELU ? relu8(a[q]) : a[q], sB[rok[(q >> 1) / 3] ? q : NKB][lz],
                                                      acc, 0, 0, 0);
    return acc;
}

// Stages the weight operands of a 32-channel layer in LDS, in the order the
// lanes read them, followed by an all-zero block (every work-item calls it).
template <int CIN>
__device__ inline void stage_weights(const bf16* __restrict__ w, bf16x8 (*sB)[64])
{
    constexpr int K = 9 * CIN, NKB = (K + 15) / 16;
    for (int e = threadIdx.x; e < (NKB + 1) * 64; e += blockDim.x) {
        const int q = e / 64, l = e % 64;
        const int kk = q * 16 + 8 * (l / 32);
        bf16x8 v = bf16x8{};
        if (kk < K) v = load8(w + ((long long)(l % 32) * 9 + kk / CIN) * CIN + kk % CIN);  // column co = l % 32
        sB[q][l] = v;
    }
    __syncthreads();
}

// out[n][y][x][co] = epilogue( sum_{tap, ci} A(n, y + d dy, x + d dx, ci) W[co][tap][ci] )
// with dilation d; A = relu(in) if RELU.  Epilogue: + bias[co] (if bias);
// then, if MASK, zero where mask <= 0; then, if RES, + res.  The output is
// FP32 if OUTF32, else BF16.  Per 32-pixel segment all K / 16 input operands
// are loaded before the first matrix-core op (rows outside the frame load a
// clamped row and are zeroed), so the loads of a wave are in flight together.
// A row of W pixels takes ceil(W / 32) segments; in the last one the pixels
// beyond the row repeat its last pixel and are not stored.  Segment indices
// are 32-bit (the host keeps N H ceil(W / 32) below 2^31): 64-bit divisions
// took ~250 scalar instructions per segment.
template <int CIN, bool RELU, bool OUTF32, bool RES, bool MASK>
__global__ __launch_bounds__(256) void k_conv(const bf16* __restrict__ in, const bf16* __restrict__ w,
                                              const float* __restrict__ bias, const void* __restrict__ res,
                                              const bf16* __restrict__ mask, void* __restrict__ out, int dil, int N,
                                              int H, int W)
{
    constexpr int K = 9 * CIN, NKB = (K + 15) / 16;
    const int lane = threadIdx.x % 64;
    const int segs_per_row = (W + 31) / 32;
    const int nseg = N * H * segs_per_row;
    // the segment index is the same for every lane of a wave: kept scalar, so
    // that everything derived from it (row, frame, validity of tap rows) is
    // scalar too
    const int wave0 = (int)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane((int)(threadIdx.x / 64));
    const int nwaves = (int)gridDim.x * 4;
    const int m = lane % 32, kh = lane / 32;
    // the weight operands of the whole K loop are staged once per workgroup
    __shared__ bf16x8 sB[NKB + 1][64];
    stage_weights<CIN>(w, sB);
    const int co = lane % 32;
    const float bv = bias ? bias[co] : 0.f;
    for (int seg = wave0; seg < nseg; seg += nwaves) {
        // an index the compiler cannot hoist: the weight operands are read from
        // LDS per segment instead of being held in 72 registers
        const int lz = lane + 64 * __builtin_amdgcn_readfirstlane((int)((unsigned)seg >> 31));
        const int x0 = (seg % segs_per_row) * 32;
        const int ny = seg / segs_per_row;
        const int y = ny % H, n = ny / H;
        if constexpr (CIN == 32) {
            const f32x16 acc = conv_seg32<RELU>(in, sB, lz, dil, H, W, n, y, x0, m, kh);
            conv_store<OUTF32, RES, MASK>(acc, bv, res, mask, out, (((long long)n * H + y) * W + x0) * 32, x0, W, kh,
                                          co);
        } else {
            const int xm = x0 + m < W ? x0 + m : W - 1;
            bf16x8 a[NKB];
#pragma unroll
            for (int q = 0; q < NKB; ++q) {
                const int kk = q * 16 + 8 * kh;
                const bool kv = kk < K;
                const int kc = kv ? kk : 0;
                const int tap = kc / CIN, ci = kc % CIN;
                const int yy = y + (tap / 3 - 1) * dil;
                int xx = xm + (tap % 3 - 1) * dil;  // |offset| <= W, so one wrap suffices
                xx = xx < 0 ? xx + W : (xx >= W ? xx - W : xx);
                const bool ok = kv && yy >= 0 && yy < H;
                const int yc = ok ? yy : y;
                a[q] = load8(in + (((long long)n * H + yc) * W + xx) * CIN + ci);
                if (!ok) a[q] = bf16x8{};
            }
            f32x16 acc = {};
#pragma unroll
            for (int q = 0; q < NKB; ++q)
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(RELU ? relu8(a[q]) : a[q], sB[q][lz], acc, 0, 0, 0);
            conv_store<OUTF32, RES, MASK>(acc, bv, res, mask, out, (((long long)n * H + y) * W + x0) * 32, x0, W, kh,
                                          co);
        }
    }
}

// A 32-channel layer with dilation d <= 16 by columns: a workgroup of kColRW
// waves computes the output rows y0, y0 + d, ..., y0 + (kColRW - 1) d of one
// 32-pixel column (wave k: row y0 + k d).  The kColRW + 2 input rows they read
// (y0 - d ... y0 + kColRW d; rows outside the frame clamped into it, their
// taps then take the zero weight block) are staged once in LDS over the
// column's window of 32 + 2d pixels (periodic in x), with the ReLU applied as
// they are staged, and the 18 operands of each segment are read from there:
// each input pixel is loaded ~1.25 times per segment instead of 9 times.
// Pixels are padded to 80 bytes, so a wave's operand reads meet distinct
// banks.  The products and their order are those of k_conv.
// The staged window holds up to kColPix pixels (dilation <= 16), or
// kColPixNarrow for dilation <= 4: 51 KB of LDS instead of 70 KB, so three
// workgroups fit a CU (6 waves per SIMD where the kernel holds <= 80 VGPRs).
// Measured at 256 x 1024: the hidden layers with dilation 1, 2 and 4 take
// 4-8% less time with the narrow window and a grid of three workgroups per CU
// (768, unevenly loaded: 1024 column groups); a grid of 512 that loads every
// workgroup evenly takes the wide window's time.
constexpr int kColPix = 64, kColPixNarrow = 40, kColPS = 40;
// Output rows (waves) per workgroup: eight (ten staged rows, 70 KB of LDS, two
// workgroups and 4 waves per SIMD) measured 12-14% faster per network block
// than four (six staged rows, 50 KB, three workgroups, 3 waves per SIMD).
constexpr int kColRW = 8;
constexpr int kColRows = kColRW + 2;

// ADV: the output layer of inference, whose epilogue adds the increment to the
// five state fields f (as k_conv_advance; N = 1).  VOL (with ADV): the
// epilogue also sums the light-phase volume (1 - phi) / 2 of the updated phi
// in FP64, per workgroup in a fixed order, into vpart[8 blockIdx.x] (the
// partials layout of k_frame_sums, which k_frame_final sums).  A last
// workgroup that sums the partials after an atomic ticket needs agent-scope
// fences (an L2 write-back per workgroup): measured slower than the separate
// final kernel.
constexpr int kVolParts = kVolPartsApi;  // at least the column kernel's grid (<= 256 * 2)
template <bool RELU, bool OUTF32, bool RES, bool MASK, bool ADV = false, int PIX = kColPix, bool VOL = false>
__global__ __launch_bounds__(64 * kColRW) void k_conv_col(const bf16* __restrict__ in, const bf16* __restrict__ w,
                                                          const float* __restrict__ bias, const void* __restrict__ res,
                                                          const bf16* __restrict__ mask, void* __restrict__ out,
                                                          int dil, int N, int H, int W, State5 f, Scales sc,
                                                          double* __restrict__ vpart = nullptr,
                                                          double* __restrict__ vout = nullptr)
{
    static_assert(!VOL || ADV, "the volume is summed in the state update's epilogue");
    constexpr int NKB = 18, RW = kColRW;
    const int lane = threadIdx.x % 64;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / 64));
    const int m = lane % 32, kh = lane / 32, co = lane % 32;
    __shared__ bf16x8 sB[NKB + 1][64];
    __shared__ __attribute__((aligned(16))) bf16 sX[kColRows][PIX][kColPS];
    // ADV: per-wave transposition tile of the five state channels (16 pixels)
    __shared__ float sT[ADV ? RW : 1][16][5];
    // With the wide window the weight operands (NKB + 1 blocks of 64 16-byte
    // entries, the last one zero) are loaded here and written to LDS with the
    // first item's rows, so the two loads are in flight together: measured
    // ~4% faster at dilation 8 and 2-3% for the output layer at 256 x 1024,
    // but 5-12% slower with the narrow window (three workgroups per CU), which
    // stages them first.
    constexpr bool EARLYW = PIX == kColPix;
    constexpr int WE = (NKB + 1) * 64, WPT = EARLYW ? (WE + 64 * RW - 1) / (64 * RW) : 1;
    bf16x8 wv[WPT];
    bool wpending = EARLYW;
    double vacc = 0.0;  // VOL: this lane's share of the light-phase volume
    if constexpr (EARLYW) {
#pragma unroll
        for (int i = 0; i < WPT; ++i) {
            const int e = threadIdx.x + i * 64 * RW, q = e / 64, l = e % 64;
            const int kk = q * 16 + 8 * (l / 32);
            wv[i] = bf16x8{};
            if (e < WE && kk < 9 * 32) wv[i] = load8(w + ((l % 32) * 9 + kk / 32) * 32 + kk % 32);
        }
    } else {
        stage_weights<32>(w, sB);
    }
    const float bv = bias ? bias[co] : 0.f;
    const int SC = (W + 31) / 32;
    const int G = ((H + dil - 1) / dil + RW - 1) / RW;  // groups of RW rows per residue class of y mod d
    const int nitems = N * dil * G * SC;
    const int win = 32 + 2 * dil;
    for (int t = blockIdx.x; t < nitems; t += gridDim.x) {
        const int sx = t % SC;
        const int u = t / SC;
        const int g = u % G, r = (u / G) % dil, n = u / G / dil;
        const int y0 = r + RW * g * dil;
        if (y0 >= H) continue;  // the same for the whole workgroup
        const int x0 = sx * 32;
        __syncthreads();  // every wave is done with the previous item's rows
        // RW / 4 rows per pass: work-item t takes row t / 256 of the pass and
        // channels 8c .. 8c + 7 of window pixel i, (i, c) = ((t % 256) / 4, t % 4)
        // (win <= PIX <= 64 pixels of 4 chunks; work-items beyond the window
        // load its last pixel and store nothing)
        constexpr int RP = RW / 4, NPASS = (kColRows + RP - 1) / RP;
        const int c = threadIdx.x % 4, i = (threadIdx.x % 256) / 4, jr = threadIdx.x / 256;
        int xx = x0 - dil + (i < win ? i : win - 1);
        if (xx < 0 || xx >= W) xx = ((xx % W) + W) % W;
        const int off = xx * 32 + 8 * c;
        bf16x8 v[NPASS];
#pragma unroll
        for (int k = 0; k < NPASS; ++k) {
            const int j = k * RP + jr;
            int yy = y0 + (j - 1) * dil;
            yy = yy < 0 ? 0 : (yy >= H ? H - 1 : yy);
            const bf16* rowp = in + ((long long)n * H + yy) * W * 32;
            if (j < kColRows) v[k] = load8(rowp + off);
        }
        if (EARLYW && wpending) {  // the same for the whole workgroup
#pragma unroll
            for (int q = 0; q < WPT; ++q) {
                const int e = threadIdx.x + q * 64 * RW;
                if (e < WE) sB[e / 64][e % 64] = wv[q];
            }
            wpending = false;
        }
        if (i < win) {
#pragma unroll
            for (int k = 0; k < NPASS; ++k) {
                const int j = k * RP + jr;
                if (j < kColRows) *reinterpret_cast<bf16x8*>(&sX[j][i][8 * c]) = RELU ? relu8(v[k]) : v[k];
            }
        }
        __syncthreads();
        const int y = y0 + wave * dil;
        if (y < H) {
            bool rok[3];
#pragma unroll
            for (int q3 = 0; q3 < 3; ++q3) {
                const int yy = y + (q3 - 1) * dil;
                rok[q3] = yy >= 0 && yy < H;
            }
            f32x16 acc = {};
#pragma unroll
            for (int q = 0; q < NKB; ++q) {
                const int tap = q >> 1, tr = tap / 3, tc = tap % 3;
                const bf16x8 a = *reinterpret_cast<const bf16x8*>(&sX[wave + tr][m + tc * dil][16 * (q & 1) + 8 * kh]);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, sB[rok[tr] ? q : NKB][lane], acc, 0, 0, 0);
            }
            if constexpr (ADV) {
                // lane l < 32 takes pixel x0 + l of the five state channels
                float (*T)[5] = sT[wave];
                float v[5];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    if (co < 5) {
#pragma unroll
                        for (int jj = 0; jj < 8; ++jj) {
                            const int ii = 8 * h + jj;
                            T[8 * (ii / 4) + 4 * kh + ii % 4 - 16 * h][co] = acc[ii] + bv;
                        }
                    }
                    wave_sync();
                    if (lane / 16 == h) {
#pragma unroll
                        for (int cc = 0; cc < 5; ++cc) v[cc] = T[lane % 16][cc];
                    }
                    wave_sync();
                }
                if (lane < 32 && x0 + lane < W) {
                    const long long p = (long long)y * W + x0 + lane;
#pragma unroll
                    for (int cc = 0; cc < 5; ++cc) {
                        float* fc = const_cast<float*>(f.v[cc]);
                        const float nv = fc[p] + v[cc] * sc.inc[cc];
                        fc[p] = nv;
                        if (VOL && cc == 0) vacc += 0.5 * (1.0 - (double)nv);
                    }
                }
            } else {
                conv_store<OUTF32, RES, MASK>(acc, bv, res, mask, out, (((long long)n * H + y) * W + x0) * 32, x0, W,
                                              kh, co);
            }
        }
    }
    if constexpr (VOL) {
        // the wave's sum (butterfly: every lane ends with the same value), then the
        // workgroup's in wave order into vpart[8 blockIdx.x]
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) vacc += __shfl_xor(vacc, o);
        __shared__ double sV[RW];
        if (lane == 0) sV[wave] = vacc;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int k = 0; k < RW; ++k) t += sV[k];
            vpart[8 * blockIdx.x] = t;
        }
    }
}

// The network's last layer with the state update fused into its epilogue,
// on one frame: f_c += (conv(A, w) + bias)_c inc[c] for the five state fields
// c < 5 (A = relu(in) if RELU; 32 input channels).  Equal to k_conv with an
// FP32 output followed by k_advance (the same sums, the same roundings), but
// the 32 FP32 channels of the increment are never written or read back.
template <bool RELU>
__global__ __launch_bounds__(256) void k_conv_advance(const bf16* __restrict__ in, const bf16* __restrict__ w,
                                                      const float* __restrict__ bias, State5 f, Scales sc, int dil,
                                                      int H, int W)
{
    constexpr int NKB = 18;
    const int lane = threadIdx.x % 64;
    const int segs_per_row = (W + 31) / 32;
    const int nseg = H * segs_per_row;
    const int wave0 = (int)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane((int)(threadIdx.x / 64));
    const int nwaves = (int)gridDim.x * 4;
    const int m = lane % 32, kh = lane / 32, co = lane % 32;
    __shared__ bf16x8 sB[NKB + 1][64];
    __shared__ TTile sT[4];
    stage_weights<32>(w, sB);
    TTile& T = sT[threadIdx.x / 64];
    const float bv = bias ? bias[co] : 0.f;
    for (int seg = wave0; seg < nseg; seg += nwaves) {
        const int lz = lane + 64 * __builtin_amdgcn_readfirstlane((int)((unsigned)seg >> 31));
        const int x0 = (seg % segs_per_row) * 32;
        const int y = seg / segs_per_row;
        const f32x16 acc = conv_seg32<RELU>(in, sB, lz, dil, H, W, 0, y, x0, m, kh);
        // through the transposition tile, lane l < 32 takes pixel x0 + l of the
        // five state channels: five coalesced 128-byte rows per segment
        float v[5];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            tile_half(T, acc, bv, h, kh, co);
            wave_sync();
            if (lane / 16 == h) {
#pragma unroll
                for (int c = 0; c < 5; ++c) v[c] = T[lane % 16][c];
            }
            wave_sync();
        }
        if (lane < 32 && x0 + lane < W) {
            const long long p = (long long)y * W + x0 + lane;
#pragma unroll
            for (int c = 0; c < 5; ++c) {
                float* fc = const_cast<float*>(f.v[c]);
                fc[p] = fc[p] + v[c] * sc.inc[c];
            }
        }
    }
}

// Weights of the adjoint convolution: wt[ci][8 - tap][co] = w[co][tap][ci]
// (channels swapped, taps mirrored).  wt has cin_t = 32 input channels and
// cout rows; rows ci >= cin of w stay zero.
__global__ void k_adjoint_weights(const bf16* __restrict__ w, int cin, bf16* __restrict__ wt)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;  // over 32 x 9 x 32
    if (i >= 32 * 9 * 32) return;
    const int co = i % 32, tap = (i / 32) % 9, ci = i / (32 * 9);
    wt[((long long)ci * 9 + (8 - tap)) * 32 + co] = ci < cin ? w[((long long)co * 9 + tap) * cin + ci] : (bf16)0.f;
}

// Weight gradient partials: part[g][co][kk] = sum over the workgroup's pixels of
// dy[p][co] * A(p + d off(tap))[ci], kk = tap * cin + ci, A = relu(in) if
// relu_in, dilation d.  Each workgroup walks whole 32-pixel segments; LDS
// holds dy of the segment and the nine shifted 32-pixel input windows it meets.
// Pixels of a row's last segment beyond the row contribute zero.
__global__ __launch_bounds__(256) void k_wgrad(const bf16* __restrict__ dy, const bf16* __restrict__ in, int cin,
                                               int relu_in, int dil, int N, int H, int W, float* __restrict__ part,
                                               int ntiles_n)
{
    __shared__ bf16 sdy[32][33];          // [pixel][co] (+1 pad)
    __shared__ bf16 sa[9][32][33];        // [tap][pixel][ci] (+1 pad), cin <= 32
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    const int segs_per_row = (W + 31) / 32;
    const long long nseg = (long long)N * H * segs_per_row;
    const long long s0 = (long long)blockIdx.x * nseg / gridDim.x, s1 = (long long)(blockIdx.x + 1) * nseg / gridDim.x;
    const int K = 9 * cin;
    f32x16 acc[3] = {};
    for (long long seg = s0; seg < s1; ++seg) {
        const int x0 = (int)(seg % segs_per_row) * 32;
        const long long nyy = seg / segs_per_row;
        const int y = (int)(nyy % H), n = (int)(nyy / H);
        __syncthreads();
        for (int q = threadIdx.x; q < 32 * 32; q += 256) {
            const int p = q / 32, c = q % 32;
            sdy[p][c] = x0 + p < W ? dy[(((long long)n * H + y) * W + x0 + p) * 32 + c] : (bf16)0.f;
        }
        for (int q = threadIdx.x; q < 9 * 32 * 32; q += 256) {
            const int c = q % 32, p = (q / 32) % 32, tap = q / (32 * 32);
            const int yy = y + (tap / 3 - 1) * dil;
            int xx = (x0 + p < W ? x0 + p : W - 1) + (tap % 3 - 1) * dil;
            xx = xx < 0 ? xx + W : (xx >= W ? xx - W : xx);
            bf16 v = (bf16)0.f;
            if (c < cin && yy >= 0 && yy < H && x0 + p < W) {
                v = in[(((long long)n * H + yy) * W + xx) * cin + c];
                if (relu_in && !(to_f(v) > 0.f)) v = (bf16)0.f;
            }
            sa[tap][p][c] = v;
        }
        __syncthreads();
        // GEMM: M = co (32), N = kk (tiles of 32), K = 32 pixels in two blocks of 16
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            const int tile = wave + 4 * t;
            if (tile >= ntiles_n) break;
            for (int kb = 0; kb < 32; kb += 16) {
                bf16x8 a, b;
                const int p0 = kb + 8 * (lane / 32);
                const int kk = tile * 32 + lane % 32;
                const bool valid = kk < K;
                const int tap = valid ? kk / cin : 0, ci = valid ? kk % cin : 0;
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    a[j] = sdy[p0 + j][lane % 32];
                    b[j] = valid ? sa[tap][p0 + j][ci] : (bf16)0.f;
                }
                acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[t], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        const int tile = wave + 4 * t;
        if (tile >= ntiles_n) break;
        const int kk = tile * 32 + lane % 32;
        if (kk >= K) continue;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int co = 8 * (i / 4) + 4 * (lane / 32) + (i % 4);
            part[((long long)blockIdx.x * 32 + co) * K + kk] = acc[t][i];
        }
    }
}

// Bias gradient partials: part[g][co] = sum over the workgroup's pixels of dy[p][co].
__global__ __launch_bounds__(256) void k_bgrad(const bf16* __restrict__ dy, long long npix, float* __restrict__ part)
{
    __shared__ float red[8][32];
    const int co = threadIdx.x % 32, r = threadIdx.x / 32;
    const long long p0 = (long long)blockIdx.x * npix / gridDim.x, p1 = (long long)(blockIdx.x + 1) * npix / gridDim.x;
    float s = 0.f;
    for (long long p = p0 + r; p < p1; p += 8) s += to_f(dy[p * 32 + co]);
    red[r][co] = s;
    __syncthreads();
    if (threadIdx.x < 32) {
        float t = 0.f;
        for (int q = 0; q < 8; ++q) t += red[q][threadIdx.x];
        part[(long long)blockIdx.x * 32 + threadIdx.x] = t;
    }
}

// out[j] = sum_g part[g][j] in the order g = 0, 1, ... (deterministic).
__global__ void k_reduce(const float* __restrict__ part, int ngroups, long long width, float* __restrict__ out)
{
    const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= width) return;
    float s = 0.f;
    for (int g = 0; g < ngroups; ++g) s += part[(long long)g * width + j];
    out[j] = s;
}

// Adam on FP32 master weights; writes the BF16 copy used by the convolutions.
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ gr, float* __restrict__ m1,
                       float* __restrict__ m2, bf16* __restrict__ pb, long long n, float lr, float b1, float b2,
                       float eps, float c1, float c2)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float g = gr[i];
    const float a = b1 * m1[i] + (1.f - b1) * g;
    const float b = b2 * m2[i] + (1.f - b2) * g * g;
    m1[i] = a;
    m2[i] = b;
    const float v = p[i] - lr * (a / c1) / (sqrtf(b / c2) + eps);
    p[i] = v;
    pb[i] = (bf16)v;
}

// Squared error of the predicted increment delta (channels 0..nout-1) against
// the target increment (nout channels): per-workgroup partial sums, and the
// gradient 2 (delta - target) * scale as BF16 (channels >= nout zero).
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ delta /*C=32*/,
                                             const float* __restrict__ target /*C=nout*/, long long npix, int nout,
                                             float scale, bf16* __restrict__ grad /*C=32*/, float* __restrict__ part)
{
    __shared__ float red[256];
    float s = 0.f;
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < npix * 32;
         q += (long long)gridDim.x * blockDim.x) {
        const long long p = q / 32;
        const int c = (int)(q % 32);
        float g = 0.f;
        if (c < nout) {
            const float e = delta[q] - target[p * nout + c];
            s += e * e;
            g = 2.f * e * scale;
        }
        grad[q] = (bf16)g;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Network input from the five FP32 state fields of one frame (x fastest):
// channels (phi, ux / U, uy / U, (T - T_rest(y)) / dT, c4, c5,
// (p - P (1 - phi) / 2) / P, 0), BF16: the pressure enters less its
// Young-Laplace part, so the small dynamic pressure keeps BF16's relative precision.
__global__ void k_pack(State5 f, long long npix, int w, Scales sc, bf16* __restrict__ x)
{
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npix) return;
    const float y = (float)(p / w);
    bf16* o = x + p * 8;
    o[0] = (bf16)f.v[0][p];
    o[1] = (bf16)(f.v[1][p] / sc.u);
    o[2] = (bf16)(f.v[2][p] / sc.u);
    o[3] = (bf16)((f.v[3][p] - (sc.t_a + sc.t_b * y)) / sc.dT);
    o[4] = (bf16)sc.c4;
    o[5] = (bf16)sc.c5;
    o[6] = (bf16)((f.v[4][p] - sc.P * 0.5f * (1.f - f.v[0][p])) / sc.P);
    o[7] = (bf16)0.f;
}

// Target increment between two states, channel c in units of inc[c]: FP32, C = 5.
__global__ void k_pack_target(State5 f0, State5 f1, long long npix, Scales sc, float* __restrict__ t)
{
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npix) return;
#pragma unroll
    for (int c = 0; c < 5; ++c) t[p * 5 + c] = (f1.v[c][p] - f0.v[c][p]) / sc.inc[c];
}

// Advances the five FP32 state fields in place: f_c += delta_c inc[c].
__global__ void k_advance(const float* __restrict__ delta, long long npix, Scales sc, State5 f)
{
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npix) return;
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        float* v = const_cast<float*>(f.v[c]);
        v[p] = v[p] + delta[p * 32 + c] * sc.inc[c];
    }
}

// Per-workgroup FP64 partial sums over one frame: the light-phase volume
// sum (1 - phi) / 2 if b is null, else, for the channels phi, ux, uy, T,
// sum (a - b)^2 and sum (b - rest)^2 with rest = (1, 0, 0, T_rest(y)).
__global__ __launch_bounds__(256) void k_frame_sums(State5 a, State5 b, int has_b, long long npix, int w, Scales sc,
                                                    double* __restrict__ part)
{
    __shared__ double red[8][256];
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < npix;
         p += (long long)gridDim.x * blockDim.x) {
        if (!has_b) {
            acc[0] += 0.5 * (1.0 - (double)a.v[0][p]);
            continue;
        }
        const double rest[4] = {1.0, 0.0, 0.0, (double)sc.t_a + (double)sc.t_b * (double)(p / w)};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const double bv = b.v[c][p];
            const double d = (double)a.v[c][p] - bv, r = bv - rest[c];
            acc[2 * c] += d * d;
            acc[2 * c + 1] += r * r;
        }
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o)
#pragma unroll
            for (int k = 0; k < 8; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x < 8) part[blockIdx.x * 8 + threadIdx.x] = red[threadIdx.x][0];
}

// Sums the partials of k_frame_sums over workgroups in a fixed order: each
// of 256 threads adds the groups g = t, t + 256, ... in turn, then a tree over
// the threads; one pass for each of the first nout quantities.
__global__ __launch_bounds__(256) void k_frame_final(const double* __restrict__ part, int groups, int nout,
                                                     double* __restrict__ out)
{
    __shared__ double red[256];
    const int t = threadIdx.x;
    for (int k = 0; k < nout; ++k) {
        double s = 0.0;
        for (int g = t; g < groups; g += 256) s += part[g * 8 + k];
        red[t] = s;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if (t < o) red[t] += red[t + o];
            __syncthreads();
        }
        if (t == 0) out[k] = red[0];
        __syncthreads();
    }
}

// ---- launchers ----

// Workgroups of a column-kernel launch: every column's group of kColRW rows of
// one residue class of y mod dil is one work item.
// per_cu: resident workgroups per CU (bound by LDS).
static unsigned col_groups(int dil, int N, int H, int W, int per_cu)
{
    const long long items = (long long)N * dil * (((H + dil - 1) / dil + kColRW - 1) / kColRW) * ((W + 31) / 32);
    const long long cap = 256LL * per_cu;
    return (unsigned)(items < cap ? items : cap);
}

template <int CIN, bool RELU, bool OUTF32, bool RES, bool MASK>
static void conv_t(const bf16* in, const bf16* w, const float* bias, const void* res, const bf16* mask, void* out,
                   int dil, int N, int H, int W, hipStream_t s)
{
    if (CIN == 32 && dil <= 4) {
        // by columns: a resident grid (three workgroups per CU) walks the
        // columns' groups of rows
        hipLaunchKernelGGL((k_conv_col<RELU, OUTF32, RES, MASK, false, kColPixNarrow>), dim3(col_groups(dil, N, H, W, 3)),
                           dim3(64 * kColRW), 0, s, in, w, bias, res, mask, out, dil, N, H, W, State5{}, Scales{});
        return;
    }
    if (CIN == 32 && dil <= 16) {
        // the same with the wide window (two workgroups per CU)
        hipLaunchKernelGGL((k_conv_col<RELU, OUTF32, RES, MASK>), dim3(col_groups(dil, N, H, W, 2)), dim3(64 * kColRW), 0, s,
                           in, w, bias, res, mask, out, dil, N, H, W, State5{}, Scales{});
        return;
    }
    // a resident grid (6 waves per SIMD on 256 CUs) walks the segments, so
    // each workgroup stages the weights once
    const long long segs = (long long)N * H * ((W + 31) / 32);
    long long groups = (segs + 3) / 4;
    if (groups > 1536) groups = 1536;
    hipLaunchKernelGGL((k_conv<CIN, RELU, OUTF32, RES, MASK>), dim3((unsigned)groups), dim3(256), 0, s, in, w, bias, res,
                       mask, out, dil, N, H, W);
}

template <int CIN, bool RELU, bool OUTF32>
static void conv_rm(const bf16* in, const bf16* w, const float* bias, const void* res, const bf16* mask, void* out,
                    int dil, int N, int H, int W, hipStream_t s)
{
    if (res && mask) conv_t<CIN, RELU, OUTF32, true, true>(in, w, bias, res, mask, out, dil, N, H, W, s);
    else if (res) conv_t<CIN, RELU, OUTF32, true, false>(in, w, bias, res, mask, out, dil, N, H, W, s);
    else if (mask) conv_t<CIN, RELU, OUTF32, false, true>(in, w, bias, res, mask, out, dil, N, H, W, s);
    else conv_t<CIN, RELU, OUTF32, false, false>(in, w, bias, res, mask, out, dil, N, H, W, s);
}

template <int CIN>
static void conv_c(const bf16* in, const bf16* w, const float* bias, const void* res, const bf16* mask, void* out,
                   int out_f32, int relu_in, int dil, int N, int H, int W, hipStream_t s)
{
    if (relu_in && out_f32) conv_rm<CIN, true, true>(in, w, bias, res, mask, out, dil, N, H, W, s);
    else if (relu_in) conv_rm<CIN, true, false>(in, w, bias, res, mask, out, dil, N, H, W, s);
    else if (out_f32) conv_rm<CIN, false, true>(in, w, bias, res, mask, out, dil, N, H, W, s);
    else conv_rm<CIN, false, false>(in, w, bias, res, mask, out, dil, N, H, W, s);
}

hipError_t conv(const bf16* in, int cin, const bf16* w, const float* bias, const void* res, const bf16* mask,
                void* out, int out_f32, int relu_in, int dil, int N, int H, int W, hipStream_t s)
{
    if (cin == 8) conv_c<8>(in, w, bias, res, mask, out, out_f32, relu_in, dil, N, H, W, s);
    else conv_c<32>(in, w, bias, res, mask, out, out_f32, relu_in, dil, N, H, W, s);
    return hipGetLastError();
}

// The output layer by columns (dilation <= 16) keeps the wide window and two
// workgroups per CU: with the narrow one and three per CU it was slower
// (11.6 against 10.2 us at 256 x 1024, dilation 1).
template <bool RELU, bool VOL>
static void col_advance(const bf16* in, const bf16* w, const float* bias, int dil, int H, int W, const Scales& sc,
                        const State5& f, double* vpart, double* vout, hipStream_t s)
{
    hipLaunchKernelGGL((k_conv_col<RELU, false, false, false, true, kColPix, VOL>), dim3(col_groups(dil, 1, H, W, 2)),
                       dim3(64 * kColRW), 0, s, in, w, bias, nullptr, nullptr, nullptr, dil, 1, H, W, f, sc, vpart, vout);
}

hipError_t conv_advance_volume(const bf16* in, const bf16* w, const float* bias, int relu_in, int dil, int H, int W,
                               const Scales& sc, const State5& f, double* vpart, double* vout, hipStream_t s)
{
    if (dil > 16 || col_groups(dil, 1, H, W, 2) > (unsigned)kVolParts) return hipErrorInvalidValue;
    if (relu_in) col_advance<true, true>(in, w, bias, dil, H, W, sc, f, vpart, vout, s);
    else col_advance<false, true>(in, w, bias, dil, H, W, sc, f, vpart, vout, s);
    hipLaunchKernelGGL(k_frame_final, dim3(1), dim3(256), 0, s, vpart, (int)col_groups(dil, 1, H, W, 2), 1, vout);
    return hipGetLastError();
}

hipError_t conv_advance(const bf16* in, const bf16* w, const float* bias, int relu_in, int dil, int H, int W,
                        const Scales& sc, const State5& f, hipStream_t s)
{
    if (dil <= 16) {
        if (relu_in) col_advance<true, false>(in, w, bias, dil, H, W, sc, f, nullptr, nullptr, s);
        else col_advance<false, false>(in, w, bias, dil, H, W, sc, f, nullptr, nullptr, s);
        return hipGetLastError();
    }
    const long long segs = (long long)H * ((W + 31) / 32);
    long long groups = (segs + 3) / 4;
    if (groups > 1536) groups = 1536;
    if (relu_in)
        hipLaunchKernelGGL(k_conv_advance<true>, dim3((unsigned)groups), dim3(256), 0, s, in, w, bias, f, sc, dil, H, W);
    else
        hipLaunchKernelGGL(k_conv_advance<false>, dim3((unsigned)groups), dim3(256), 0, s, in, w, bias, f, sc, dil, H,
                           W);
    return hipGetLastError();
}

hipError_t adjoint_weights(const bf16* w, int cin, bf16* wt, hipStream_t s)
{
    hipLaunchKernelGGL(k_adjoint_weights, dim3((32 * 9 * 32 + 255) / 256), dim3(256), 0, s, w, cin, wt);
    return hipGetLastError();
}

hipError_t wgrad(const bf16* dy, const bf16* in, int cin, int relu_in, int dil, int N, int H, int W, float* part,
                 int groups, float* out, hipStream_t s)
{
    const int ntiles_n = (9 * cin + 31) / 32;
    hipLaunchKernelGGL(k_wgrad, dim3(groups), dim3(256), 0, s, dy, in, cin, relu_in, dil, N, H, W, part, ntiles_n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const long long width = 32LL * 9 * cin;
    hipLaunchKernelGGL(k_reduce, dim3((unsigned)((width + 255) / 256)), dim3(256), 0, s, part, groups, width, out);
    return hipGetLastError();
}

hipError_t bgrad(const bf16* dy, long long npix, float* part, int groups, float* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_bgrad, dim3(groups), dim3(256), 0, s, dy, npix, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(32), 0, s, part, groups, 32LL, out);
    return hipGetLastError();
}

hipError_t adam(float* p, const float* g, float* m1, float* m2, bf16* pb, long long n, float lr, float b1, float b2,
                float eps, int t, hipStream_t s)
{
    const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, g, m1, m2, pb, n, lr, b1, b2,
                       eps, c1, c2);
    return hipGetLastError();
}

hipError_t mse(const float* delta, const float* target, long long npix, int nout, float scale, bf16* grad,
               float* part, int groups, hipStream_t s)
{
    hipLaunchKernelGGL(k_mse, dim3(groups), dim3(256), 0, s, delta, target, npix, nout, scale, grad, part);
    return hipGetLastError();
}

static dim3 pix_grid(long long npix) { return dim3((unsigned)((npix + 255) / 256)); }

hipError_t pack(const State5& f, long long npix, int w, const Scales& sc, bf16* x, hipStream_t s)
{
    hipLaunchKernelGGL(k_pack, pix_grid(npix), dim3(256), 0, s, f, npix, w, sc, x);
    return hipGetLastError();
}

hipError_t pack_target(const State5& f0, const State5& f1, long long npix, const Scales& sc, float* t, hipStream_t s)
{
    hipLaunchKernelGGL(k_pack_target, pix_grid(npix), dim3(256), 0, s, f0, f1, npix, sc, t);
    return hipGetLastError();
}

hipError_t advance(const float* delta, long long npix, const Scales& sc, const State5& f, hipStream_t s)
{
    hipLaunchKernelGGL(k_advance, pix_grid(npix), dim3(256), 0, s, delta, npix, sc, f);
    return hipGetLastError();
}

// Partial sums of the judge for callers that cannot allocate device memory:
// a file-scope array of kJudgeMaxGroups * 8 doubles per GPU, held until the
// process ends.  In host code `scratch` names a host-side stand-in, not
// device memory: its device address is taken once per device with
// hipGetSymbolAddress (the device current at that call) and only that address
// is passed to kernels.
static __device__ __align__(256) double scratch[kJudgeMaxGroups * 8];

namespace {
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t judge_scratch_ptr(double** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

hipError_t frame_sums(const State5& a, const State5* b, long long npix, int w, const Scales& sc, double* part,
                      int groups, double* out, hipStream_t s)
{
    const State5 bb = b ? *b : a;
    hipLaunchKernelGGL(k_frame_sums, dim3(groups), dim3(256), 0, s, a, bb, b != nullptr, npix, w, sc, part);
    hipLaunchKernelGGL(k_frame_final, dim3(1), dim3(256), 0, s, part, groups, b ? 8 : 1, out);
    return hipGetLastError();
}

}  // namespace sur
