// cnn.hip -- the U-Net's layers on gfx950: bf16 operands, fp32 accumulation
// on the matrix cores (v_mfma_f32_16x16x32_bf16).
//
// Every convolution is one implicit GEMM, out[p][n] = sum_k A(p, k) W[n][k],
// p an output pixel, n an output channel, k a (tap, input channel) pair, with
// A gathered from the input on the fly (no im2col buffer):
//   kConv3  3x3 cross-correlation, zero padding 1: k = tap * C_in + c,
//           A(p, k) = X[y + dy(tap)][x + dx(tap)][c]
//   kPoint  1x1: A(p, k) = X[p][k]
//   kUp     stride-2 2x2 transposed convolution, one GEMM per output parity
//           q = (a, c): A(p, k) = X[p][k], written to (2y + a, 2x + c)
//   kUpBack its backward data pass: k = q * C_out + o,
//           A(p, k) = dY[2y + a][2x + c][o]
// Tensors are NHWC bf16 with a channel stride, so a layer can read or write a
// channel slice of a wider tensor (the decoder's concatenation of skip and
// upsampled features is never copied).  Weights are packed [n][k] (k
// contiguous, K and N padded to multiples of 64 with zeros).
//
// MFMA 16x16x32 bf16 operand layout (lane l of 64): A holds row l % 16,
// columns 8 (l / 16) .. +7; B holds column l % 16, rows 8 (l / 16) .. +7;
// the 4 accumulators hold rows 4 (l / 16) .. +3 of column l % 16.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "cnn.h"

namespace eptv {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// fp32 -> bf16, round to nearest even (gfx950's v_cvt_pk_bf16_f32)
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

// two values in one conversion: a in the low half, b in the high half
__device__ __forceinline__ uint32_t pack_bf16x2(float a, float b)
{
    const bf16x2 v = {(__bf16)a, (__bf16)b};
    return __builtin_bit_cast(uint32_t, v);
}

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

union Frag {
    bf16x8 v;
    uint4 u;
    uint16_t h[8];
};

__device__ __forceinline__ Frag zero_frag()
{
    Frag f;
    f.u = make_uint4(0u, 0u, 0u, 0u);
    return f;
}

// 8 consecutive k of A(p, k) for one pixel p = (img, y, x) of the GEMM grid.
template <int MODE>
__device__ __forceinline__ Frag gather_a(const ConvArgs& a, int img, int y, int x, int k)
{
    Frag f = zero_frag();
    if (MODE == kConv3) {
        if (a.cin % 8 == 0) {
            if (k >= 9 * a.cin) return f;
            const int tap = k / a.cin, c = k - tap * a.cin;
            const int ys = y + tap / 3 - 1, xs = x + tap % 3 - 1;
            if ((unsigned)ys >= (unsigned)a.h || (unsigned)xs >= (unsigned)a.w) return f;
            f.u = *reinterpret_cast<const uint4*>(a.x + (((size_t)img * a.h + ys) * a.w + xs) * a.x_cs + a.x_co + c);
        } else {
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int kk = k + i;
                const int tap = kk / a.cin, c = kk - tap * a.cin;
                const int ys = y + tap / 3 - 1, xs = x + tap % 3 - 1;
                if (kk < 9 * a.cin && (unsigned)ys < (unsigned)a.h && (unsigned)xs < (unsigned)a.w)
                    f.h[i] = a.x[(((size_t)img * a.h + ys) * a.w + xs) * a.x_cs + a.x_co + c];
            }
        }
    } else if (MODE == kPoint || MODE == kUp) {
        if (a.cin % 8 == 0) {
            if (k >= a.cin) return f;
            f.u = *reinterpret_cast<const uint4*>(a.x + (((size_t)img * a.h + y) * a.w + x) * a.x_cs + a.x_co + k);
        } else {
#pragma unroll
            for (int i = 0; i < 8; ++i)
                if (k + i < a.cin) f.h[i] = a.x[(((size_t)img * a.h + y) * a.w + x) * a.x_cs + a.x_co + k + i];
        }
    } else {  // kUpBack: the input is the 2h x 2w gradient with cin channels per parity
        if (k >= 4 * a.cin) return f;
        const int q = k / a.cin, o = k - q * a.cin;
        const int ys = 2 * y + (q >> 1), xs = 2 * x + (q & 1);
        f.u = *reinterpret_cast<const uint4*>(a.x + (((size_t)img * 2 * a.h + ys) * 2 * a.w + xs) * a.x_cs + a.x_co +
                                              o);
    }
    return f;
}

// Epilogue of one 16 x 16 output tile formed as D[n][pixel] (the weights as
// the MFMA's A operand, so that lane l holds 4 consecutive channels
// n .. n + 3, n = 16 j + 4 (l / 16), of pixel l % 16): bias, ReLU, the fused
// ReLU mask, then one 8-byte (bf16) or 16-byte (fp32) store.  `vec`: the
// output and mask slices are 4-channel aligned.
__device__ __forceinline__ uint2 epi_mask4(const ConvArgs& a, size_t pix, int n, bool ok, bool vec)
{
    if (!ok || !a.mask) return make_uint2(0u, 0u);
    const uint16_t* src = a.mask + pix * a.m_cs + a.m_co + n;
    if (vec && n + 3 < a.cout) return *reinterpret_cast<const uint2*>(src);
    uint32_t h[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int r = 0; r < 4; ++r)
        if (n + r < a.cout) h[r] = src[r];
    return make_uint2(h[0] | (h[1] << 16), h[2] | (h[3] << 16));
}

// the bias of channels n .. n + 3 (zero past cout or without a bias)
__device__ __forceinline__ floatx4 epi_bias4(const ConvArgs& a, int n)
{
    floatx4 b = {0.0f, 0.0f, 0.0f, 0.0f};
    if (a.bias) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (n + r < a.cout) b[r] = a.bias[n + r];
    }
    return b;
}

__device__ __forceinline__ void epi_store4(const ConvArgs& a, size_t pix, int n, const floatx4& acc, uint2 m,
                                           bool vec, const floatx4& bias)
{
    float v[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        v[r] = acc[r] + bias[r];
        if (a.relu) v[r] = fmaxf(v[r], 0.0f);
        if (a.mask) {
            const uint32_t w = r < 2 ? m.x : m.y;
            if (!(bf2f((uint16_t)(w >> (16 * (r & 1)))) > 0.0f)) v[r] = 0.0f;
        }
    }
    const bool full = vec && n + 3 < a.cout;
    if (a.y32) {
        float* dst = a.y32 + pix * a.y_cs + a.y_co + n;
        if (full) {
            *reinterpret_cast<float4*>(dst) = make_float4(v[0], v[1], v[2], v[3]);
        } else {
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (n + r < a.cout) dst[r] = v[r];
        }
    } else {
        uint16_t* dst = a.y + pix * a.y_cs + a.y_co + n;
        if (full) {
            *reinterpret_cast<uint2*>(dst) = make_uint2(pack_bf16x2(v[0], v[1]), pack_bf16x2(v[2], v[3]));
        } else {
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (n + r < a.cout) dst[r] = f2bf(v[r]);
        }
    }
}

__device__ __forceinline__ bool epi_vec(const ConvArgs& a)
{
    return a.y_cs % 4 == 0 && a.y_co % 4 == 0 && (!a.mask || (a.m_cs % 4 == 0 && a.m_co % 4 == 0));
}

// Block: 4 waves, each RT x 16 consecutive pixels of the flattened (image, y,
// x) order of the GEMM grid, x 64 output channels; grid (pixel groups,
// channel blocks, parity q for kUp).  The block's 64 weight rows are staged in
// LDS a K-chunk at a time and shared by the 4 waves; the A operand is gathered
// straight from the input (each lane decodes its own pixels, so any image size
// works), one K-step ahead of the matrix instructions that use it.
constexpr int kConvKC = 256;           // K-chunk of staged weights
constexpr int kConvLd = kConvKC + 8;   // LDS row pitch (bf16), 16 B of padding

// Workgroups are handed to the 8 XCDs round robin; renumber the pixel tiles
// so that each XCD walks one contiguous band of them and the rows above and
// below a tile (the 3x3 taps) sit in the same L2.  A bijection on
// [0, 8 floor(G/8)), the identity on the tail.
__device__ __forceinline__ int xcd_band(int b, int G)
{
    const int per = G >> 3;
    if (b >= per * 8) return b;
    return (b & 7) * per + (b >> 3);
}

// The A operand when every 32-wide K-step lies inside one tap (C_in a
// multiple of 32, 16-byte aligned channel slices): the tap, its offset and the
// channel base are uniform over the wave, so a lane only adds its own pixel's
// base address and checks its row / column.
template <int MODE>
__device__ __forceinline__ Frag gather_fast(const ConvArgs& a, const uint16_t* base, int y, int x, bool v, int k)
{
    Frag f = zero_frag();
    if (MODE == kConv3) {
        const int tap = k / a.cin, c0 = k - tap * a.cin;
        const int dy = tap / 3 - 1, dx = tap - (tap / 3) * 3 - 1;
        if (v && tap < 9 && (unsigned)(y + dy) < (unsigned)a.h && (unsigned)(x + dx) < (unsigned)a.w)
            f.u = *reinterpret_cast<const uint4*>(base + ((long)dy * a.w + dx) * a.x_cs + c0);
    } else {  // kPoint, kUp
        if (v && k < a.cin) f.u = *reinterpret_cast<const uint4*>(base + k);
    }
    return f;
}

template <int MODE, int RT, int NT>
__global__ __launch_bounds__(256) void k_conv(ConvArgs a)
{
    constexpr int BN = 16 * NT;  // output channels per block
    // LDS: the weight chunks; then (modes with contiguous output pixels) the
    // block's outputs, [pixel][BN + 8] bf16, on their way to memory
    constexpr int OLD = BN + 8, WL = BN * kConvLd, OL = 64 * RT * OLD;
    __shared__ __attribute__((aligned(16))) uint16_t wlds[WL > OL ? WL : OL];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int hw = a.h * a.w, npix = a.n_img * hw;
    const int tile = xcd_band((int)blockIdx.x, (int)gridDim.x);
    const int p0 = (tile * 4 + wave) * (16 * RT);
    const int n0 = blockIdx.y * BN;
    const int q = MODE == kUp ? (int)blockIdx.z : 0;
    const uint16_t* wq = a.wt + (size_t)q * a.n_pad * a.k_pad;
    const int mrow = lane & 15, kq = (lane >> 4) * 8;
    const bool fast = MODE != kUpBack && a.cin % 32 == 0 && a.x_cs % 8 == 0 && a.x_co % 8 == 0;
    // With the image width a multiple of 16, a 16-pixel row tile lies in one
    // image row: its (image, row, first column) is decoded once, uniformly
    // over the wave, and a lane only adds its column offset.
    const bool row16 = a.w % 16 == 0;
    int ia[RT], ya[RT], xa[RT], xt[RT];
    bool va[RT];
    const uint16_t* base[RT];
#pragma unroll
    for (int i = 0; i < RT; ++i) {
        const int p = p0 + 16 * i + mrow;
        va[i] = p < npix;
        const int pd = row16 ? p0 + 16 * i : p;
        ia[i] = pd / hw;
        const int r = pd - ia[i] * hw;
        ya[i] = r / a.w;
        xt[i] = r - ya[i] * a.w;
        xa[i] = row16 ? xt[i] + mrow : xt[i];
        base[i] = a.x + (size_t)(va[i] ? p : 0) * a.x_cs + a.x_co + kq;
    }
    auto gather = [&](int i, int k) -> Frag {
        if (fast) return gather_fast<MODE == kUpBack ? kPoint : MODE>(a, base[i], ya[i], xa[i], va[i], k);
        return (va[i] && k < a.k_pad) ? gather_a<MODE>(a, ia[i], ya[i], xa[i], k + kq) : zero_frag();
    };
    floatx4 acc[RT][NT];
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[i][j] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    // A operand two K-steps ahead of its use: fa (this step), f1 (the next)
    Frag fa[RT], f1[RT];
#pragma unroll
    for (int i = 0; i < RT; ++i) {
        fa[i] = gather(i, 0);
        f1[i] = gather(i, 32);
    }
    for (int kc = 0; kc < a.k_pad; kc += kConvKC) {
        const int kn = min(kConvKC, a.k_pad - kc);  // a multiple of 64
        __syncthreads();                             // the previous chunk is consumed
        const int per_row = kn / 8;
        for (int idx = threadIdx.x; idx < BN * per_row; idx += 256) {
            const int row = idx / per_row, c8 = idx - row * per_row;
            *reinterpret_cast<uint4*>(wlds + row * kConvLd + c8 * 8) =
                *reinterpret_cast<const uint4*>(wq + (size_t)(n0 + row) * a.k_pad + kc + c8 * 8);
        }
        __syncthreads();
        for (int k0 = 0; k0 < kn; k0 += 32) {
            Frag fn[RT];
#pragma unroll
            for (int i = 0; i < RT; ++i) fn[i] = gather(i, kc + k0 + 64);  // two K-steps ahead
            Frag fb[NT];
#pragma unroll
            for (int j = 0; j < NT; ++j)
                fb[j].u = *reinterpret_cast<const uint4*>(wlds + (16 * j + mrow) * kConvLd + k0 + kq);
#pragma unroll
            for (int i = 0; i < RT; ++i)
#pragma unroll
                for (int j = 0; j < NT; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fb[j].v, fa[i].v, acc[i][j], 0, 0, 0);
#pragma unroll
            for (int i = 0; i < RT; ++i) {
                fa[i] = f1[i];
                f1[i] = fn[i];
            }
        }
    }
    // epilogue: accumulator r of lane l, row tile i, column tile j is pixel
    // p0 + 16 i + l % 16 (the lane's own pixel of the gather), channel
    // n0 + 16 j + 4 (l / 16) + r.  A row tile's mask values are loaded before
    // its first store (the compiler cannot move loads across stores that
    // might alias them).
    const bool staged = MODE != kUp && !a.y32 && a.cout % 8 == 0 && a.y_cs % 8 == 0 && a.y_co % 8 == 0 &&
                        (!a.mask || (a.m_cs % 8 == 0 && a.m_co % 8 == 0));
    if (staged) {
        // the block's pixels are p0_block .. + 64 RT - 1: stage bf16 outputs
        // (bias, ReLU) in LDS, then move 16-byte pieces (8 channels of one
        // pixel) to memory with the mask applied there
        const int pb = tile * 64 * RT;
        __syncthreads();  // every wave is done with the weights
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const floatx4 bias = epi_bias4(a, n0 + 16 * j + kq / 2);
#pragma unroll
            for (int i = 0; i < RT; ++i) {
                float v[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    v[r] = acc[i][j][r] + bias[r];
                    if (a.relu) v[r] = fmaxf(v[r], 0.0f);
                }
                *reinterpret_cast<uint2*>(wlds + (wave * 16 * RT + 16 * i + mrow) * OLD + 16 * j + kq / 2) =
                    make_uint2(pack_bf16x2(v[0], v[1]), pack_bf16x2(v[2], v[3]));
            }
        }
        __syncthreads();
        constexpr int C8 = BN / 8, PIECES = 64 * RT * C8, PPT_OUT = PIECES / 256, QB = PPT_OUT < 4 ? PPT_OUT : 4;
        static_assert(PIECES % 256 == 0 && PPT_OUT % QB == 0, "whole pieces per thread");
#pragma unroll
        for (int q0 = 0; q0 < PPT_OUT; q0 += QB) {
            Frag mv[QB];
            if (a.mask) {
#pragma unroll
                for (int qq = 0; qq < QB; ++qq) {
                    const int pc_ = threadIdx.x + 256 * (q0 + qq), px = pc_ / C8, n = n0 + (pc_ - px * C8) * 8;
                    mv[qq] = zero_frag();
                    if (pb + px < npix && n < a.cout)
                        mv[qq].u = *reinterpret_cast<const uint4*>(a.mask + (size_t)(pb + px) * a.m_cs + a.m_co + n);
                }
            }
#pragma unroll
            for (int qq = 0; qq < QB; ++qq) {
                const int pc_ = threadIdx.x + 256 * (q0 + qq), px = pc_ / C8, c8 = pc_ - px * C8, n = n0 + c8 * 8;
                if (pb + px >= npix || n >= a.cout) continue;
                Frag o;
                o.u = *reinterpret_cast<const uint4*>(wlds + px * OLD + c8 * 8);
                if (a.mask) {
#pragma unroll
                    for (int e = 0; e < 8; ++e)
                        if (!(bf2f(mv[qq].h[e]) > 0.0f)) o.h[e] = 0;
                }
                *reinterpret_cast<uint4*>(a.y + (size_t)(pb + px) * a.y_cs + a.y_co + n) = o.u;
            }
        }
        return;
    }
    const bool vec = epi_vec(a);
    floatx4 bias[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) bias[j] = epi_bias4(a, n0 + 16 * j + kq / 2);
#pragma unroll
    for (int i = 0; i < RT; ++i) {
        size_t pix;
        if (MODE == kUp)
            pix = ((size_t)ia[i] * 2 * a.h + 2 * ya[i] + (q >> 1)) * 2 * a.w + 2 * xa[i] + (q & 1);
        else
            pix = (size_t)(p0 + 16 * i + mrow);
        uint2 mk[NT];
#pragma unroll
        for (int j = 0; j < NT; ++j) mk[j] = epi_mask4(a, pix, n0 + 16 * j + kq / 2, va[i], vec);
        if (!va[i]) continue;
#pragma unroll
        for (int j = 0; j < NT; ++j) epi_store4(a, pix, n0 + 16 * j + kq / 2, acc[i][j], mk[j], vec, bias[j]);
    }
}

template <int MODE, int NT>
static void conv_launch_rt(const ConvArgs& a, int rt, dim3 grid, hipStream_t s)
{
    if (rt == 4)
        hipLaunchKernelGGL((k_conv<MODE, 4, NT>), grid, dim3(256), 0, s, a);
    else if (rt == 2)
        hipLaunchKernelGGL((k_conv<MODE, 2, NT>), grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((k_conv<MODE, 1, NT>), grid, dim3(256), 0, s, a);
}

template <int MODE>
static void conv_launch(const ConvArgs& a, int rt, int nt, dim3 grid, hipStream_t s)
{
    if (nt == 2)
        conv_launch_rt<MODE, 2>(a, rt, grid, s);
    else
        conv_launch_rt<MODE, 4>(a, rt, grid, s);
}

// ------------------------------------------------------------------ 3x3 convolutions from LDS tiles
// The block's output is a TH x 32 rectangle of one image; per chunk of 32
// input channels it stages the (TH + 2) x 34 input patch (zero outside the
// image) and the 9 taps' weights of its output channels in LDS, then every
// tap's A operand is an LDS read at a fixed offset from the lane's own pixel:
// the 9-fold reuse of each input value comes from LDS, not from global
// memory, and the inner loop is LDS reads and matrix instructions only.
constexpr int kPatchW = 34;             // 32 columns + halo
// LDS pitches: 96 B per patch pixel and 608 B per weight row (measured: far
// fewer bank conflicts than 80 B / 592 B or 112 B / 624 B)
constexpr int kPatchPS = 48;            // bf16 per patch pixel (32 channels + 32 B)
constexpr int kTapLd = 9 * 32 + 16;     // bf16 per weight row (9 taps x 32 channels + 32 B)
constexpr int kTileBlocksPerCu = 2;     // persistent blocks per CU
constexpr int kThin = 4;                // the thin side of a 1x1 layer done on the vector ALUs (the head)

// STAGED: the epilogue goes through LDS (16-byte stores, masks, pooling);
// otherwise each lane stores its 4 channels directly (no mask or pooling).
// KC: input channels staged per round trip (32, or 64 for layers with many
// chunks and few tiles: half the round trips per tile).  HEAD (STAGED, one
// 32-channel block): the thin 1x1 head of a.head_* from the staged outputs.
template <int TH, int NT, bool STAGED, int KC = 32, bool HEAD = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_conv3_tile(ConvArgs a, int ntiles)
{
    constexpr int BN = 16 * NT;       // output channels per block
    static_assert(!HEAD || STAGED, "the head reads the staged outputs");
    static_assert(TH == 8 || TH == 4, "8- or 4-row tiles");
    constexpr int RT = TH / 2;        // 16-pixel row tiles per wave
    constexpr int P8 = KC / 8;                                           // 16-byte pieces per pixel
    constexpr int PPS = KC == 32 ? kPatchPS : KC + 16;                   // bf16 per patch pixel
    constexpr int TLD = KC == 32 ? kTapLd : 9 * KC + 16;                 // bf16 per weight row
    constexpr int PN = (TH + 2) * kPatchW * P8, PPT = (PN + 255) / 256;  // patch uint4s, per thread
    constexpr int WN = BN * 9 * P8, WPT = (WN + 255) / 256;              // weight uint4s, per thread
    // LDS: the patch region, then the weights; a finished tile's outputs are
    // staged in the patch region ([pixel][BN + 8] bf16, the region grown to
    // fit) on their way to memory, so the weights stay in place
    constexpr int PATCH = (TH + 2) * kPatchW * PPS, OLD = BN + 8;
    constexpr int STAGE = !STAGED || PATCH > TH * 32 * OLD ? PATCH : TH * 32 * OLD;
    __shared__ __attribute__((aligned(16))) uint16_t lds[STAGE + BN * TLD];
    __shared__ float hwt[HEAD ? kThin * BN + kThin : 1];  // the head's weights [n][k], then its bias
    uint16_t* patch = lds;
    uint16_t* wts = lds + STAGE;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int tiles_x = (a.w + 31) / 32, tiles_y = (a.h + TH - 1) / TH;
    const int n0 = blockIdx.y * BN;
    const int nch = a.cin / KC;
    // persistent blocks: block b walks tiles of one contiguous band per XCD
    // (workgroups go to the 8 XCDs round robin), so neighbouring tiles share
    // an L2; without a multiple of 8 blocks, a plain stride
    const int G = (int)gridDim.x, b = (int)blockIdx.x;
    int t_first, t_step, t_end;
    if (G % 8 == 0) {
        const int band = (ntiles + 7) / 8, xcd = b & 7;
        t_first = xcd * band + (b >> 3);
        t_step = G >> 3;
        t_end = min(ntiles, (xcd + 1) * band);
    } else {
        t_first = b;
        t_step = G;
        t_end = ntiles;
    }
    if (t_first >= t_end) return;  // whole block, before any barrier
    const int mrow = lane & 15, kq = (lane >> 4) * 8;
    // a wave owns two image rows of the tile (so that a 2x2 pooling window
    // stays inside it): with 8-row tiles rows 2 w, 2 w + 1, both 16-column
    // halves (row tile i: row 2 w + i / 2, half i % 2); with 4-row tiles
    // rows 2 (w / 2) + i of half w % 2
    auto row_of = [&](int i) { return TH == 8 ? 2 * wave + (i >> 1) : 2 * (wave >> 1) + i; };
    auto col_of = [&](int i) { return 16 * (TH == 8 ? (i & 1) : (wave & 1)); };
    int lbase[RT];
#pragma unroll
    for (int i = 0; i < RT; ++i) lbase[i] = ((row_of(i) + 1) * kPatchW + col_of(i) + mrow + 1) * PPS + kq;
    auto tile_origin = [&](int t, int& img, int& y0, int& x0) __attribute__((always_inline)) {
        img = t / (tiles_x * tiles_y);
        const int r = t - img * tiles_x * tiles_y;
        const int ty = r / tiles_x;
        y0 = ty * TH;
        x0 = (r - ty * tiles_x) * 32;
    };
    // Staging through range-checked buffer loads: a piece outside the image
    // (or past the patch) gets offset -1, which the hardware's range check
    // turns into zeros, so no load sits behind a branch.  Byte offsets fit
    // 31 bits (checked at launch).
    const __amdgpu_buffer_rsrc_t rx =
        __builtin_amdgcn_make_buffer_rsrc((void*)a.x, (short)0, (int)((size_t)a.n_img * a.h * a.w * a.x_cs * 2), 0x00020000);
    const __amdgpu_buffer_rsrc_t rw =
        __builtin_amdgcn_make_buffer_rsrc((void*)a.wt, (short)0, (int)((size_t)a.n_pad * a.k_pad * 2), 0x00020000);
    u32x4 pr[PPT], wr[WPT];
    auto fetch_patch = [&](int t, int c0) __attribute__((always_inline)) {
        int img, y0, x0;
        tile_origin(t, img, y0, x0);
        // element offset of patch pixel (0, 0), image pixel (y0 - 1, x0 - 1)
        const int base = ((img * a.h + y0 - 1) * a.w + x0 - 1) * a.x_cs + a.x_co + c0;
#pragma unroll
        for (int u = 0; u < PPT; ++u) {
            const int idx = threadIdx.x + 256 * u;
            const int px = idx / P8, part = idx - px * P8;
            const int pr_ = px / kPatchW, pc = px - pr_ * kPatchW;
            const bool ok = idx < PN && (unsigned)(y0 - 1 + pr_) < (unsigned)a.h && (unsigned)(x0 - 1 + pc) < (unsigned)a.w;
            const int off = ok ? 2 * (base + (pr_ * a.w + pc) * a.x_cs + part * 8) : -1;
            pr[u] = __builtin_amdgcn_raw_buffer_load_b128(rx, off, 0, 0);
        }
    };
    auto fetch_w = [&](int c0) __attribute__((always_inline)) {
#pragma unroll
        for (int u = 0; u < WPT; ++u) {
            const int idx = threadIdx.x + 256 * u;
            const int row = idx / (9 * P8), rem = idx - row * (9 * P8), tap = rem / P8, part = rem - tap * P8;
            const int off = idx < WN ? 2 * ((n0 + row) * a.k_pad + tap * a.cin + c0 + part * 8) : -1;
            wr[u] = __builtin_amdgcn_raw_buffer_load_b128(rw, off, 0, 0);
        }
    };
    floatx4 acc[RT][NT];
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[i][j] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    int t = t_first, c = 0;
    bool w_staged = false;
    fetch_patch(t, 0);
    fetch_w(0);
    if constexpr (HEAD) {
        // behind the first item's loads; read after the main loop's first barrier
        for (int i = threadIdx.x; i < kThin * BN; i += 256) {
            const int n = i / BN, k = i - n * BN;
            hwt[i] = n < a.head_n && k < a.cout ? bf2f(a.head_wt[(size_t)n * a.head_kpad + k]) : 0.0f;
        }
        if (threadIdx.x < kThin)
            hwt[kThin * BN + threadIdx.x] = (int)threadIdx.x < a.head_n && a.head_bias ? a.head_bias[threadIdx.x] : 0.0f;
    }
    while (true) {
        __syncthreads();  // the previous item is consumed
#pragma unroll
        for (int u = 0; u < PPT; ++u) {
            const int idx = threadIdx.x + 256 * u;
            if (idx < PN) *reinterpret_cast<u32x4*>(patch + (idx / P8) * PPS + (idx % P8) * 8) = pr[u];
        }
        if (nch > 1 || !w_staged) {
#pragma unroll
            for (int u = 0; u < WPT; ++u) {
                const int idx = threadIdx.x + 256 * u;
                const int row = idx / (9 * P8), rem = idx - row * (9 * P8);  // tap KC + part 8 = rem 8
                if (idx < WN) *reinterpret_cast<u32x4*>(wts + row * TLD + rem * 8) = wr[u];
            }
            w_staged = true;
        }
        __syncthreads();
        // the next (tile, chunk) item is fetched while this one is computed
        int tn = t, cn = c + 1;
        if (cn == nch) {
            cn = 0;
            tn = t + t_step;
        }
        const bool more = tn < t_end;
        if (more) {
            fetch_patch(tn, cn * KC);
            if (nch > 1) fetch_w(cn * KC);
        }
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
#pragma unroll
            for (int ks = 0; ks < KC; ks += 32) {
                const int toff = ((tap / 3 - 1) * kPatchW + (tap % 3 - 1)) * PPS + ks;
                Frag fb[NT];
#pragma unroll
                for (int j = 0; j < NT; ++j)
                    fb[j].u = *reinterpret_cast<const uint4*>(wts + (16 * j + mrow) * TLD + tap * KC + ks + kq);
#pragma unroll
                for (int i = 0; i < RT; ++i) {
                    Frag fa;
                    fa.u = *reinterpret_cast<const uint4*>(patch + lbase[i] + toff);
#pragma unroll
                    for (int j = 0; j < NT; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fb[j].v, fa.v, acc[i][j], 0, 0, 0);
                }
            }
        }
        if (STAGED && c == nch - 1) {
            // epilogue through LDS: accumulator r of lane l, row tile i,
            // column tile j is the pixel at local row row_of(i), column
            // col_of(i) + l % 16, channel n0 + 16 j + 4 (l / 16) + r; each
            // wave writes its bf16 outputs (bias, ReLU) to the staging
            // region, then every thread moves whole 16-byte pieces (8
            // channels of one pixel) to memory, applying the mask there, and
            // forms the pooled pieces from the staged values
            int img, y0, x0;
            tile_origin(t, img, y0, x0);
            __syncthreads();  // every wave is done with the patch and the weights
#pragma unroll
            for (int j = 0; j < NT; ++j) {
                const floatx4 bias = epi_bias4(a, n0 + 16 * j + kq / 2);
#pragma unroll
                for (int i = 0; i < RT; ++i) {
                    float v[4];
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        v[r] = acc[i][j][r] + bias[r];
                        if (a.relu) v[r] = fmaxf(v[r], 0.0f);
                    }
                    const int px = row_of(i) * 32 + col_of(i) + mrow;
                    *reinterpret_cast<uint2*>(lds + px * OLD + 16 * j + kq / 2) =
                        make_uint2(pack_bf16x2(v[0], v[1]), pack_bf16x2(v[2], v[3]));
                }
            }
            __syncthreads();
            constexpr int C8 = BN / 8, PIECES = TH * 32 * C8, PPT_OUT = PIECES / 256, QB = PPT_OUT < 4 ? PPT_OUT : 4;
            static_assert(PIECES % 256 == 0 && PPT_OUT % QB == 0, "whole pieces per thread");
#pragma unroll
            for (int q0 = 0; q0 < PPT_OUT; q0 += QB) {
                // QB pieces at a time, their mask values loaded before the first store
                Frag mv[QB];
                if (a.mask) {
#pragma unroll
                    for (int qq = 0; qq < QB; ++qq) {
                        const int pc_ = threadIdx.x + 256 * (q0 + qq), px = pc_ / C8, n = n0 + (pc_ - px * C8) * 8;
                        const int y = y0 + (px >> 5), x = x0 + (px & 31);
                        mv[qq] = zero_frag();
                        if (y < a.h && x < a.w && n < a.cout)
                            mv[qq].u = *reinterpret_cast<const uint4*>(
                                a.mask + (((size_t)img * a.h + y) * a.w + x) * a.m_cs + a.m_co + n);
                    }
                }
#pragma unroll
                for (int qq = 0; qq < QB; ++qq) {
                    const int pc_ = threadIdx.x + 256 * (q0 + qq), px = pc_ / C8, c8 = pc_ - px * C8, n = n0 + c8 * 8;
                    const int y = y0 + (px >> 5), x = x0 + (px & 31);
                    if (y >= a.h || x >= a.w || n >= a.cout) continue;
                    Frag o;
                    o.u = *reinterpret_cast<const uint4*>(lds + px * OLD + c8 * 8);
                    if (a.mask) {
#pragma unroll
                        for (int e = 0; e < 8; ++e)
                            if (!(bf2f(mv[qq].h[e]) > 0.0f)) o.h[e] = 0;
                    }
                    *reinterpret_cast<uint4*>(a.y + (((size_t)img * a.h + y) * a.w + x) * a.y_cs + a.y_co + n) = o.u;
                }
            }
            if (a.pool) {
                // 2x2 average of the stored values, summed in the order of
                // the pooling kernel: (0,0) + (0,1) + (1,0) + (1,1)
                constexpr int PP = (TH / 2) * 16 * C8;
                for (int pc_ = threadIdx.x; pc_ < PP; pc_ += 256) {
                    const int pp = pc_ / C8, c8 = pc_ - pp * C8, n = n0 + c8 * 8;
                    const int ly = 2 * (pp >> 4), lx = 2 * (pp & 15);
                    const int y = y0 + ly, x = x0 + lx;
                    if (y + 1 >= a.h || x + 1 >= a.w || n >= a.cout) continue;
                    Frag f[4], o;
#pragma unroll
                    for (int d = 0; d < 4; ++d)
                        f[d].u = *reinterpret_cast<const uint4*>(lds + ((ly + (d >> 1)) * 32 + lx + (d & 1)) * OLD + c8 * 8);
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        float sum = 0.0f;
#pragma unroll
                        for (int d = 0; d < 4; ++d) sum += bf2f(f[d].h[e]);
                        o.h[e] = f2bf(0.25f * sum);
                    }
                    *reinterpret_cast<uint4*>(a.pool + (((size_t)img * (a.h / 2) + y / 2) * (a.w / 2) + x / 2) * a.p_cs +
                                              n) = o.u;
                }
            }
            if constexpr (HEAD) {
                // the head, one thread per pixel, in k_point_thin's order:
                // partial sum q over channels 8 q + 32 k + j (k, then j
                // ascending), then (s0 + s1) + (s2 + s3), then the bias; one
                // output at a time, so that few registers are added to those
                // the next tile's prefetch holds
                for (int px = threadIdx.x; px < TH * 32; px += 256) {
                    const int y = y0 + (px >> 5), x = x0 + (px & 31);
                    if (y >= a.h || x >= a.w) continue;
                    Frag xr[BN / 8];
#pragma unroll
                    for (int i = 0; i < BN / 8; ++i) xr[i].u = *reinterpret_cast<const uint4*>(lds + px * OLD + 8 * i);
                    float* yo = a.head_y32 + (((size_t)img * a.h + y) * a.w + x) * a.head_n;
#pragma unroll 1
                    for (int n = 0; n < a.head_n; ++n) {
                        const float* wn = hwt + n * BN;
                        float sq[4];
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            sq[q] = 0.0f;
#pragma unroll
                            for (int i = q; i < BN / 8; i += 4)
#pragma unroll
                                for (int j = 0; j < 8; ++j) sq[q] += bf2f(xr[i].h[j]) * wn[8 * i + j];
                        }
                        yo[n] = ((sq[0] + sq[1]) + (sq[2] + sq[3])) + hwt[kThin * BN + n];
                    }
                }
            }
        } else if (!STAGED && c == nch - 1) {
            // direct epilogue: accumulator r of lane l, row tile i, column
            // tile j is the pixel at local row row_of(i), column
            // col_of(i) + l % 16, channel n0 + 16 j + 4 (l / 16) + r
            int img, y0, x0;
            tile_origin(t, img, y0, x0);
            const bool vec = epi_vec(a);
#pragma unroll
            for (int j = 0; j < NT; ++j) {
                const floatx4 bias = epi_bias4(a, n0 + 16 * j + kq / 2);
#pragma unroll
                for (int i = 0; i < RT; ++i) {
                    const int y = y0 + row_of(i), x = x0 + col_of(i) + mrow;
                    if (y < a.h && x < a.w)
                        epi_store4(a, ((size_t)img * a.h + y) * a.w + x, n0 + 16 * j + kq / 2, acc[i][j],
                                   make_uint2(0u, 0u), vec, bias);
                }
            }
        }
        if (c == nch - 1) {
#pragma unroll
            for (int i = 0; i < RT; ++i)
#pragma unroll
                for (int j = 0; j < NT; ++j) acc[i][j] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
        }
        if (!more) break;
        t = tn;
        c = cn;
    }
}

// A 3x3 convolution of a one-channel input (the first layer): K = 9 is too
// thin for the matrix cores, so one thread per (output pixel, 8 channels)
// forms them with fp32 products of the bf16 operands (exact) and fp32 sums
// over the taps in order, then the bias.
constexpr int kC1MaxOut = 64;

__global__ __launch_bounds__(256) void k_conv3_c1(ConvArgs a, int seg_per_block)
{
    // weights as fp32 [tap][n] (4 channels per LDS read), bias [n], and the
    // three input rows around the block's pixels (zero outside the image)
    __shared__ __attribute__((aligned(16))) float wt[9 * kC1MaxOut];
    __shared__ __attribute__((aligned(16))) float bs[kC1MaxOut];
    __shared__ float rows[3][256 + 2];
    // block: segments blockIdx.y seg_per_block .. + seg_per_block - 1 (pb
    // pixels each, seg_per_block pb <= 256) of image row blockIdx.x
    // (img h + y), one thread per (pixel, 8 output channels)
    const int c8n = a.cout / 8, pb = 256 / c8n;
    const int row = blockIdx.x, img = row / a.h, y = row - img * a.h;
    for (int i = threadIdx.x; i < a.cout * 9; i += 256) {
        const int t = i / a.cout, n = i - t * a.cout;
        wt[i] = bf2f(a.wt[(size_t)n * a.k_pad + t]);
    }
    for (int i = threadIdx.x; i < a.cout; i += 256) bs[i] = a.bias ? a.bias[i] : 0.0f;
    const int lp = threadIdx.x / c8n, n0 = (threadIdx.x - lp * c8n) * 8;
    // the block's columns [x_beg, x_end) (at most 256) and one on each side
    // are staged once: element i = t + 256 k (k < 4) of the 3 x (W + 2) <= 774
    // values, row i / (W + 2), column i % (W + 2)
    const uint16_t* xin = a.x + (size_t)img * a.h * a.w * a.x_cs + a.x_co;
    const int x_beg = blockIdx.y * seg_per_block * pb, x_end = min(a.w, x_beg + seg_per_block * pb);
    const int W2 = x_end - x_beg + 2;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int i = threadIdx.x + 256 * k;
        if (i >= 3 * W2) continue;
        const int sr = i / W2, sc = i - sr * W2;
        const int ys = y + sr - 1, xs = x_beg + sc - 1;
        const bool in = (unsigned)ys < (unsigned)a.h && (unsigned)xs < (unsigned)a.w;
        float v = 0.0f;
        if (in && a.x32) {
            // fp32 input: round to bf16 here; the centre row's own pixels
            // are also stored (the layer's bf16 input)
            const uint16_t hv = f2bf(a.x32[((size_t)img * a.h + ys) * a.w + xs]);
            v = bf2f(hv);
            if (sr == 1 && sc >= 1 && sc < W2 - 1) const_cast<uint16_t*>(a.x)[((size_t)img * a.h + ys) * a.w + xs] = hv;
        } else if (in) {
            v = bf2f(xin[((size_t)ys * a.w + xs) * a.x_cs]);
        }
        rows[sr][sc] = v;
    }
    __syncthreads();  // the rows and the weights are staged
    for (int x0 = x_beg; x0 < x_end; x0 += pb) {
        const int x = x0 + lp, lx = x - x_beg;  // rows' column lx + 1 is pixel x
        if (lp >= pb || x >= x_end) continue;
        float acc[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const float v = rows[t / 3][lx + t % 3];
            const float4 w0 = *reinterpret_cast<const float4*>(wt + t * a.cout + n0);
            const float4 w1 = *reinterpret_cast<const float4*>(wt + t * a.cout + n0 + 4);
            acc[0] += v * w0.x;
            acc[1] += v * w0.y;
            acc[2] += v * w0.z;
            acc[3] += v * w0.w;
            acc[4] += v * w1.x;
            acc[5] += v * w1.y;
            acc[6] += v * w1.z;
            acc[7] += v * w1.w;
        }
        const float4 b0 = *reinterpret_cast<const float4*>(bs + n0), b1 = *reinterpret_cast<const float4*>(bs + n0 + 4);
        acc[0] += b0.x;
        acc[1] += b0.y;
        acc[2] += b0.z;
        acc[3] += b0.w;
        acc[4] += b1.x;
        acc[5] += b1.y;
        acc[6] += b1.z;
        acc[7] += b1.w;
        if (a.relu) {
#pragma unroll
            for (int j = 0; j < 8; ++j) acc[j] = fmaxf(acc[j], 0.0f);
        }
        uint4 o;
        o.x = pack_bf16x2(acc[0], acc[1]);
        o.y = pack_bf16x2(acc[2], acc[3]);
        o.z = pack_bf16x2(acc[4], acc[5]);
        o.w = pack_bf16x2(acc[6], acc[7]);
        *reinterpret_cast<uint4*>(a.y + (((size_t)row * a.w) + x) * a.y_cs + a.y_co + n0) = o;
    }
}

// 1x1 layers with a thin side (the head, C_in -> 3, and its backward data,
// 3 -> C_in): a 16 x 16 matrix tile would be mostly padding, so the vector
// ALUs form the outputs with fp32 products of the bf16 operands (exact) and
// fp32 sums, with lanes laid over channels so that each wave reads or
// writes contiguous memory.
constexpr int kThinWide = 256;  // the other side (kThin: the thin side)

__global__ __launch_bounds__(256) void k_point_thin(ConvArgs a)
{
    __shared__ float wt[kThin * kThinWide];  // [n][k]
    __shared__ float bs[kThinWide];
    for (int i = threadIdx.x; i < a.cout * a.cin; i += 256)
        wt[i] = bf2f(a.wt[(size_t)(i / a.cin) * a.k_pad + i % a.cin]);
    for (int i = threadIdx.x; i < a.cout; i += 256) bs[i] = a.bias ? a.bias[i] : 0.0f;
    __syncthreads();
    const int npix = a.n_img * a.h * a.w;
    if (a.cout <= kThin) {
        // thin output: a quad of lanes per pixel, lane j of the quad summing
        // input channels 8 j, 8 j + 32, ... (16-byte loads, consecutive lanes
        // contiguous); the quad's partial sums are added in lane order
        const int sub = threadIdx.x & 3;
        for (int p = (blockIdx.x * 256 + threadIdx.x) >> 2; p < (npix + 63) / 64 * 64; p += gridDim.x * 64) {
            const bool ok = p < npix;
            const uint16_t* xp = a.x + (size_t)(ok ? p : 0) * a.x_cs + a.x_co;
            float sum[kThin] = {0.0f, 0.0f, 0.0f, 0.0f};
            for (int k0 = 8 * sub; k0 < a.cin; k0 += 32) {
                Frag f;
                f.u = *reinterpret_cast<const uint4*>(xp + k0);
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const float xv = bf2f(f.h[j]);
#pragma unroll
                    for (int n = 0; n < kThin; ++n)
                        if (n < a.cout) sum[n] += xv * wt[n * a.cin + k0 + j];
                }
            }
            const int base = (threadIdx.x & 63) & ~3;
#pragma unroll
            for (int n = 0; n < kThin; ++n) {
                const float s0 = __shfl(sum[n], base), s1 = __shfl(sum[n], base + 1);
                const float s2 = __shfl(sum[n], base + 2), s3 = __shfl(sum[n], base + 3);
                sum[n] = (s0 + s1) + (s2 + s3);
            }
            if (!ok || sub != 0) continue;
#pragma unroll
            for (int n = 0; n < kThin; ++n) {
                if (n >= a.cout) continue;
                float v = sum[n] + bs[n];
                if (a.relu) v = fmaxf(v, 0.0f);
                if (a.mask && !(bf2f(a.mask[(size_t)p * a.m_cs + a.m_co + n]) > 0.0f)) v = 0.0f;
                if (a.y32)
                    a.y32[(size_t)p * a.y_cs + a.y_co + n] = v;
                else
                    a.y[(size_t)p * a.y_cs + a.y_co + n] = f2bf(v);
            }
        }
        return;
    }
    // thin input: one thread per (pixel, 8 output channels), consecutive
    // threads writing consecutive 16-byte pieces
    const int c8n = a.cout / 8;
    const long long work = (long long)npix * c8n;
    for (long long idx = (long long)blockIdx.x * 256 + threadIdx.x; idx < work; idx += (long long)gridDim.x * 256) {
        const int p = (int)(idx / c8n), n0 = (int)(idx - (long long)p * c8n) * 8;
        const uint16_t* xp = a.x + (size_t)p * a.x_cs + a.x_co;
        Frag m, o;
        if (a.mask) m.u = *reinterpret_cast<const uint4*>(a.mask + (size_t)p * a.m_cs + a.m_co + n0);
        float xv[kThin];
#pragma unroll
        for (int k = 0; k < kThin; ++k) xv[k] = k < a.cin ? bf2f(xp[k]) : 0.0f;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            float v = 0.0f;
#pragma unroll
            for (int k = 0; k < kThin; ++k)
                if (k < a.cin) v += xv[k] * wt[(n0 + j) * a.cin + k];
            v += bs[n0 + j];
            if (a.relu) v = fmaxf(v, 0.0f);
            if (a.mask && !(bf2f(m.h[j]) > 0.0f)) v = 0.0f;
            o.h[j] = f2bf(v);
        }
        *reinterpret_cast<uint4*>(a.y + (size_t)p * a.y_cs + a.y_co + n0) = o.u;
    }
}

static bool point_thin_fits(const ConvArgs& a, int mode)
{
    if (mode != kPoint) return false;
    if (a.cout <= kThin && a.cin <= kThinWide && a.cin % 8 == 0 && a.x_cs % 8 == 0 && a.x_co % 8 == 0) return true;
    return a.cin <= kThin && a.cout <= kThinWide && a.cout % 8 == 0 && !a.y32 && a.y_cs % 8 == 0 && a.y_co % 8 == 0 &&
           (!a.mask || (a.m_cs % 8 == 0 && a.m_co % 8 == 0));
}

// ------------------------------------------------------------------ stride-2 2x2 transposed convolution
// out[2y + a][2x + c][n] = act(b[n] + sum_k X[y][x][k] W[q][n][k]), q = 2a + c.
// Block = 32 input pixels of one row (x0 .. x0 + 31) x BN output channels;
// wave w forms parity q = w with the weights as the MFMA's A operand
// (D[n][pixel]), both operands read straight from memory as 16-byte rows.
// The 2 x 64 output pixels of the block are staged in LDS and leave as whole
// 16-byte pieces, so every output row is written contiguously.
template <int NT>
__global__ __launch_bounds__(256) void k_up2x2(ConvArgs a)
{
    constexpr int BN = 16 * NT, OLD = BN + 8;
    __shared__ __attribute__((aligned(16))) uint16_t out[2 * 64 * OLD];
    const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int mrow = lane & 15, kq = (lane >> 4) * 8;
    const int tiles_x = (a.w + 31) / 32;
    const int t = blockIdx.x, row = t / tiles_x;  // row = img * h + y
    const int x0 = (t - row * tiles_x) * 32, n0 = blockIdx.y * BN;
    const int img = row / a.h, y = row - img * a.h;
    const uint16_t* wq = a.wt + (size_t)q * a.n_pad * a.k_pad;
    const uint16_t* xr = a.x + ((size_t)row * a.w) * a.x_cs + a.x_co;
    floatx4 acc[2][NT];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[i][j] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    // operands of K-step k0 (zero past C_in; packed weight rows are zero
    // there already, k < k_pad)
    auto load = [&](int k0, Frag* fx, Frag* fw) __attribute__((always_inline)) {
        const int k = k0 + kq;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int x = x0 + 16 * i + mrow;
            fx[i] = zero_frag();
            if (x < a.w && k < a.cin) fx[i].u = *reinterpret_cast<const uint4*>(xr + (size_t)x * a.x_cs + k);
        }
#pragma unroll
        for (int j = 0; j < NT; ++j)
            fw[j].u = *reinterpret_cast<const uint4*>(wq + (size_t)(n0 + 16 * j + mrow) * a.k_pad + min(k, a.k_pad - 8));
    };
    Frag fx[2], fw[NT];
    load(0, fx, fw);
    for (int k0 = 0; k0 < a.cin; k0 += 32) {
        Frag gx[2], gw[NT];  // the next K-step, loaded while this one is multiplied
        if (k0 + 32 < a.cin) load(k0 + 32, gx, gw);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < NT; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fw[j].v, fx[i].v, acc[i][j], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 2; ++i) fx[i] = gx[i];
#pragma unroll
        for (int j = 0; j < NT; ++j) fw[j] = gw[j];
    }
    // accumulator r of lane l, pixel tile i, channel tile j: input pixel
    // x0 + 16 i + l % 16, channel n0 + 16 j + 4 (l / 16) + r -> staged at
    // output row q / 2, column 2 (16 i + l % 16) + q % 2
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        const floatx4 bias = epi_bias4(a, n0 + 16 * j + kq / 2);
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            float v[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                v[r] = acc[i][j][r] + bias[r];
                if (a.relu) v[r] = fmaxf(v[r], 0.0f);
            }
            const int px = (q >> 1) * 64 + 2 * (16 * i + mrow) + (q & 1);
            *reinterpret_cast<uint2*>(out + px * OLD + 16 * j + kq / 2) =
                make_uint2(pack_bf16x2(v[0], v[1]), pack_bf16x2(v[2], v[3]));
        }
    }
    __syncthreads();
    constexpr int C8 = BN / 8, PIECES = 128 * C8;
    const int W2 = 2 * a.w;
    for (int pc_ = threadIdx.x; pc_ < PIECES; pc_ += 256) {
        const int px = pc_ / C8, c8 = pc_ - px * C8, n = n0 + c8 * 8;
        const int fr = px >> 6, fc = 2 * x0 + (px & 63);
        if (fc >= W2 || n >= a.cout) continue;
        const size_t pix = ((size_t)img * 2 * a.h + 2 * y + fr) * W2 + fc;
        *reinterpret_cast<uint4*>(a.y + pix * a.y_cs + a.y_co + n) = *reinterpret_cast<const uint4*>(out + px * OLD + c8 * 8);
    }
}

static bool up2x2_fits(const ConvArgs& a, int mode)
{
    return mode == kUp && !a.y32 && !a.mask && a.cin % 8 == 0 && a.cout % 8 == 0 && a.x_cs % 8 == 0 &&
           a.x_co % 8 == 0 && a.y_cs % 8 == 0 && a.y_co % 8 == 0;
}

// The LDS-tile kernel's shape for a layer (false where it does not apply:
// C_in a multiple of 32, bf16 output, every slice 16-byte aligned, byte
// offsets within 31 bits): the largest tile that still gives enough blocks
// (8 rows and 64 channels preferred; smaller layers fall back to 4 rows, then
// to 32-channel tiles; 32 output channels or fewer: a 32-wide channel tile).
static bool conv3_tile_shape(const ConvArgs& a, int mode, int& th, int& tn)
{
    if (!(mode == kConv3 && a.cin % 32 == 0 && a.x_cs % 8 == 0 && a.x_co % 8 == 0 && !a.y32 && a.cout % 8 == 0 &&
          a.y_cs % 8 == 0 && a.y_co % 8 == 0 && (!a.mask || (a.m_cs % 8 == 0 && a.m_co % 8 == 0)) &&
          (!a.pool || a.p_cs % 8 == 0) && (size_t)a.n_img * a.h * a.w * a.x_cs * 2 < (size_t(1) << 31) &&
          (size_t)a.n_pad * a.k_pad * 2 < (size_t(1) << 31)))
        return false;
    const int nt = a.cout <= 32 ? 2 : 4;
    const long long t8 = (long long)a.n_img * ((a.h + 7) / 8) * ((a.w + 31) / 32);
    const long long t4 = (long long)a.n_img * ((a.h + 3) / 4) * ((a.w + 31) / 32);
    const long long c4 = (a.cout + 63) / 64, c2 = (a.cout + 31) / 32;
    if (t8 * (nt == 4 ? c4 : c2) >= 512) th = 8, tn = nt;
    else if (t4 * (nt == 4 ? c4 : c2) >= 512) th = 4, tn = nt;
    else if (t4 * c2 >= 512) th = 4, tn = 2;  // more blocks for the small layers
    else if (t4 * (nt == 4 ? c4 : c2) >= 256) th = 4, tn = nt;
    else th = 4, tn = 2;  // small layers: the most blocks
    return true;
}

bool conv3_head_fits(const ConvArgs& a, int head_n)
{
    ConvArgs b = a;
    b.head_y32 = nullptr;
    int th = 0, tn = 0;
    return head_n >= 1 && head_n <= kThin && !a.mask && !a.x32 && conv3_tile_shape(b, kConv3, th, tn) && th == 8 &&
           tn == 2 && a.cout <= 32;
}

static hipError_t launch_conv_impl(const ConvArgs& a, int mode, hipStream_t s, bool* pooled)
{
    *pooled = false;
    const int npix = a.n_img * a.h * a.w;
    if (mode == kConv3 && a.cin == 1 && !a.y32 && a.cout % 8 == 0 && a.cout <= kC1MaxOut && a.y_cs % 8 == 0 &&
        a.y_co % 8 == 0 && (!a.x32 || (a.x_cs == 1 && a.x_co == 0))) {
        // row segments per block: the per-block set-up spread over several
        // segments, while keeping about 2048 blocks
        const int pb = 256 / (a.cout / 8), nseg = (a.w + pb - 1) / pb;
        // (a block stages at most 256 columns of its row)
        const int spb = std::max(1, std::min({nseg, a.n_img * a.h * nseg / 2048, 256 / pb}));
        hipLaunchKernelGGL(k_conv3_c1, dim3((unsigned)(a.n_img * a.h), (unsigned)((nseg + spb - 1) / spb)), dim3(256),
                           0, s, a, spb);
        return hipGetLastError();
    }
    if (up2x2_fits(a, mode)) {
        const int nt = a.cout <= 32 ? 2 : 4, bn = 16 * nt;
        dim3 g((unsigned)(a.n_img * a.h * ((a.w + 31) / 32)), (unsigned)((a.cout + bn - 1) / bn));
        if (nt == 2) hipLaunchKernelGGL(k_up2x2<2>, g, dim3(256), 0, s, a);
        else hipLaunchKernelGGL(k_up2x2<4>, g, dim3(256), 0, s, a);
        return hipGetLastError();
    }
    if (point_thin_fits(a, mode)) {
        const long long work = a.cout <= kThin ? (long long)npix * 4 : (long long)npix * (a.cout / 8);
        const unsigned g = (unsigned)std::min<long long>((work + 255) / 256, 4096);
        hipLaunchKernelGGL(k_point_thin, dim3(g), dim3(256), 0, s, a);
        return hipGetLastError();
    }
    const int nt = a.cout <= 32 ? 2 : 4;
    int th = 0, tn = 0;
    if (conv3_tile_shape(a, mode, th, tn)) {
        const long long t8 = (long long)a.n_img * ((a.h + 7) / 8) * ((a.w + 31) / 32);
        const long long t4 = (long long)a.n_img * ((a.h + 3) / 4) * ((a.w + 31) / 32);
        const long long c4 = (a.cout + 63) / 64, c2 = (a.cout + 31) / 32;
        {
            // persistent blocks: about kTileBlocksPerCu per CU over all channel blocks
            const long long nt_ = th == 8 ? t8 : t4, cbn = tn == 4 ? c4 : c2;
            const long long want = std::max(8LL, (long long)kTileBlocksPerCu * 256 / cbn / 8 * 8);
            const int G = (int)std::min(nt_, want);
            dim3 g((unsigned)G, (unsigned)cbn);
            const int ntl = (int)nt_;
            ConvArgs b = a;
            // the kernel pools in its epilogue (even image sides)
            *pooled = a.pool && a.h % 2 == 0 && a.w % 2 == 0;
            if (!*pooled) b.pool = nullptr;
            if (a.head_y32) {  // conv3_head_fits: 8 x 32 tiles, one channel block
                hipLaunchKernelGGL((k_conv3_tile<8, 2, true, 32, true>), g, dim3(256), 0, s, b, ntl);
                return hipGetLastError();
            }
            // measured on MI355X: the LDS-staged epilogue pays off except for
            // 8 x 64 tiles without a mask or pooling (many input chunks per
            // tile, and the staging adds registers there)
            if (th == 8 && tn == 4) {
                if (b.mask || b.pool) hipLaunchKernelGGL((k_conv3_tile<8, 4, true>), g, dim3(256), 0, s, b, ntl);
                else hipLaunchKernelGGL((k_conv3_tile<8, 4, false>), g, dim3(256), 0, s, b, ntl);
            } else if (th == 8) {
                hipLaunchKernelGGL((k_conv3_tile<8, 2, true>), g, dim3(256), 0, s, b, ntl);
            } else if (tn == 4) {
                hipLaunchKernelGGL((k_conv3_tile<4, 4, true>), g, dim3(256), 0, s, b, ntl);
            } else if (a.cin % 64 == 0) {  // 64 input channels per round trip
                hipLaunchKernelGGL((k_conv3_tile<4, 2, true, 64>), g, dim3(256), 0, s, b, ntl);
            } else {
                hipLaunchKernelGGL((k_conv3_tile<4, 2, true>), g, dim3(256), 0, s, b, ntl);
            }
            return hipGetLastError();
        }
    }
    const int cblk = (a.cout + 16 * nt - 1) / (16 * nt), par = mode == kUp ? 4 : 1;
    // the largest row-tile count that still gives about two blocks per CU
    int rt = 4;
    while (rt > 1 && (long long)((npix + 64 * rt - 1) / (64 * rt)) * cblk * par < 512) rt /= 2;
    dim3 grid((unsigned)((npix + 64 * rt - 1) / (64 * rt)), (unsigned)cblk, (unsigned)par);
    switch (mode) {
    case kConv3: conv_launch<kConv3>(a, rt, nt, grid, s); break;
    case kPoint: conv_launch<kPoint>(a, rt, nt, grid, s); break;
    case kUp: conv_launch<kUp>(a, rt, nt, grid, s); break;
    default: conv_launch<kUpBack>(a, rt, nt, grid, s); break;
    }
    return hipGetLastError();
}

static bool conv3_c1_takes_fp32(const ConvArgs& a, int mode)
{
    return mode == kConv3 && a.cin == 1 && !a.y32 && a.cout % 8 == 0 && a.cout <= kC1MaxOut && a.y_cs % 8 == 0 &&
           a.y_co % 8 == 0 && a.x_cs == 1 && a.x_co == 0;
}

hipError_t launch_conv(const ConvArgs& a, int mode, hipStream_t s)
{
    bool pooled = false;
    hipError_t e = hipSuccess;
    if (a.head_y32 && (mode != kConv3 || !conv3_head_fits(a, a.head_n) || !a.head_wt || a.head_kpad < a.cout))
        return hipErrorInvalidValue;
    if (a.x32 && !conv3_c1_takes_fp32(a, mode)) {  // the bf16 input first, as a pass of its own
        if (a.x_cs != a.cin || a.x_co != 0) return hipErrorInvalidValue;
        ConvArgs b = a;
        b.x32 = nullptr;
        e = launch_to_bf16(a.x32, const_cast<uint16_t*>(a.x), (size_t)a.n_img * a.h * a.w * a.cin, s);
        if (e == hipSuccess) e = launch_conv(b, mode, s);
        return e;
    }
    e = launch_conv_impl(a, mode, s, &pooled);
    if (e == hipSuccess && a.pool && !pooled) {  // the pooling as a pass of its own (dense output)
        if (a.p_cs != a.cout || a.y32) return hipErrorInvalidValue;
        e = launch_avgpool(a.y, a.y_cs, a.y_co, a.pool, a.n_img, a.h, a.w, a.cout, s);
    }
    return e;
}

// ------------------------------------------------------------------ weight gradients (3x3 fallback)
// For 3x3 layers whose C_in is neither a multiple of 32 nor 1 (the tiled
// kernels below take those): dW[n][k] = sum_p dY[p][n] A(p, k), split over
// chunks of pixels: block (chunk, n block, k block) writes its 64 x 64 fp32
// partial; k_wgrad_finish sums the chunks in order.  The reduction runs over
// pixels, which are not contiguous in NHWC, so each 64-pixel step stages dY
// and A transposed in LDS ([channel][pixel], four pixels per 8-byte store);
// then each wave (2 x 2 arrangement) forms a 32 n x 32 k tile with MFMA rows
// n (A' = dY^T) and columns k, 32 pixels per instruction.
constexpr int kWgLd = 72;  // LDS pitch in bf16 (64 pixels + 16 B)

__global__ __launch_bounds__(256) void k_wgrad(ConvArgs a, const uint16_t* __restrict__ dy, int dy_cs, int dy_co,
                                               int chunk_px, float* part, float* bpart)
{
    __shared__ __attribute__((aligned(16))) uint16_t t_dy[64 * kWgLd];
    __shared__ __attribute__((aligned(16))) uint16_t t_a[64 * kWgLd];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int chunk = blockIdx.x;
    const int n0 = blockIdx.y * 64;
    const int k0 = blockIdx.z * 64;
    const int kb = k0;
    const int hw = a.h * a.w, npix = a.n_img * hw;
    const int p_beg = chunk * chunk_px, p_end = min(npix, p_beg + chunk_px);
    // loader role: threads 0-127 stage dY, 128-255 stage A; 4 pixels x 8 channels each
    const int lt = threadIdx.x & 127, lg = lt >> 3, lc = (lt & 7) * 8;
    const bool load_dy = threadIdx.x < 128;
    const bool dy_vec = (dy_cs % 8 == 0) && (dy_co % 8 == 0) && (n0 + lc + 8 <= a.cout);
    // compute role
    const int wn = wave >> 1, wk = wave & 1, row = lane & 15, pq = (lane >> 4) * 8;
    floatx4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    // the bias gradient sum_p dY[p][n] rides along in the first k block of
    // each parity: thread t sums channel t % 64 over pixels 16 (t / 64) .. +15
    // of every staged step
    const bool do_bias = bpart && kb == 0;
    float bsum = 0.0f;
    for (int ps = p_beg; ps < p_end; ps += 64) {
        Frag v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            v[u] = zero_frag();
            const int p = ps + lg * 4 + u;
            if (p >= p_end) continue;
            const int img = p / hw, r = p - img * hw, yy = r / a.w, xx = r - yy * a.w;
            if (load_dy) {
                const uint16_t* src = dy + (size_t)p * dy_cs + dy_co + n0 + lc;
                if (dy_vec) {
                    v[u].u = *reinterpret_cast<const uint4*>(src);
                } else {
#pragma unroll
                    for (int i = 0; i < 8; ++i)
                        if (n0 + lc + i < a.cout) v[u].h[i] = src[i];
                }
            } else {
                v[u] = gather_a<kConv3>(a, img, yy, xx, kb + lc);
            }
        }
        __syncthreads();  // the previous step's tiles are consumed
        uint16_t* dst = load_dy ? t_dy : t_a;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            uint2 w;
            w.x = (uint32_t)v[0].h[i] | ((uint32_t)v[1].h[i] << 16);
            w.y = (uint32_t)v[2].h[i] | ((uint32_t)v[3].h[i] << 16);
            *reinterpret_cast<uint2*>(dst + (lc + i) * kWgLd + lg * 4) = w;
        }
        __syncthreads();
        if (do_bias) {
            Frag b0, b1;
            b0.u = *reinterpret_cast<const uint4*>(t_dy + (threadIdx.x & 63) * kWgLd + (threadIdx.x >> 6) * 16);
            b1.u = *reinterpret_cast<const uint4*>(t_dy + (threadIdx.x & 63) * kWgLd + (threadIdx.x >> 6) * 16 + 8);
#pragma unroll
            for (int i = 0; i < 8; ++i) bsum += bf2f(b0.h[i]);
#pragma unroll
            for (int i = 0; i < 8; ++i) bsum += bf2f(b1.h[i]);
        }
#pragma unroll
        for (int s2 = 0; s2 < 64; s2 += 32) {
            Frag fa[2], fb[2];
#pragma unroll
            for (int i = 0; i < 2; ++i)
                fa[i].u = *reinterpret_cast<const uint4*>(t_dy + (32 * wn + 16 * i + row) * kWgLd + s2 + pq);
#pragma unroll
            for (int j = 0; j < 2; ++j)
                fb[j].u = *reinterpret_cast<const uint4*>(t_a + (32 * wk + 16 * j + row) * kWgLd + s2 + pq);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i].v, fb[j].v, acc[i][j], 0, 0, 0);
        }
    }
    // partial[chunk][n][k] over the padded n x k_pad grid
    const int kw = a.k_pad;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int n = n0 + 32 * wn + 16 * i + (lane >> 4) * 4 + r, k = k0 + 32 * wk + 16 * j + row;
                part[((size_t)chunk * a.n_pad + n) * kw + k] = acc[i][j][r];
            }
    if (do_bias) {
        __syncthreads();  // every wave is done with the tiles
        float* red = reinterpret_cast<float*>(t_a);
        red[threadIdx.x] = bsum;
        __syncthreads();
        if (threadIdx.x < 64) {
            const int t = threadIdx.x;
            const float v = (red[t] + red[64 + t]) + (red[128 + t] + red[192 + t]);
            bpart[(size_t)chunk * a.n_pad + n0 + t] = v;
        }
    }
}

// ------------------------------------------------------------------ 3x3 weight gradients from LDS tiles
// For C_in a multiple of 32 (and 16-byte aligned slices): block = (pixel
// chunk, 32 output channels from n0, 32 input channels from c0), all 9 taps,
// i.e. a 32 x 288 slice of dW held in the waves' accumulators while the
// block walks its chunk's tiles (4 RPW rows x 32 columns of one image).  Per
// tile it stages dY [pixel][n] and the (4 RPW + 2) x 34 input patch
// [pixel][c] in LDS exactly as they lie in NHWC memory.  The matrix
// instructions reduce over pixels: A = dY^T (row n, 32 pixels of one image
// row), B = the input shifted by the tap (32 pixels x 16 channels).  gfx950's
// transposing LDS read (ds_read_b64_tr_b16: within each 16-lane group, lane
// j receives column j of the 4 x 16 block that the group's lanes address,
// four rows of 4 consecutive columns each) hands a lane 4 consecutive pixels
// of one channel, so neither tile is ever transposed in registers, and a
// tap's shift is only a different pixel address.
//
// Wave w owns tile rows w RPW .. w RPW + RPW - 1.  It loads the A operands of
// its rows once per tile and walks the RPW + 2 patch rows: each patch row's
// three column shifts are loaded once and serve every (output row, tap) pair
// that reads that patch row (up to three).  The bias gradient sum_p dY[p][n]
// rides along in the blocks of the first channel chunk as a product with a
// B operand of ones.  At the end the 4 waves' accumulators are summed in LDS
// and the block writes its partial[chunk][n][tap C_in + c].
constexpr int kWg3Ld = 40;  // bf16 per staged pixel (32 channels + 16 B)

typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) bf16x4 lds_bf16x4;

// the MFMA operand of 8 consecutive pixels (two transposing reads of 4)
__device__ __forceinline__ bf16x8 tr_frag(const uint16_t* lo, const uint16_t* hi)
{
    const bf16x4 a = __builtin_amdgcn_ds_read_tr16_b64_v4bf16((lds_bf16x4*)lo);
    const bf16x4 b = __builtin_amdgcn_ds_read_tr16_b64_v4bf16((lds_bf16x4*)hi);
    return __builtin_shufflevector(a, b, 0, 1, 2, 3, 4, 5, 6, 7);
}

template <int RPW>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_wgrad3(
    ConvArgs a, const uint16_t* __restrict__ dy, int dy_cs, int dy_co, int tiles_per_chunk, int nbn, int nbc,
    float* part, float* bpart)
{
    constexpr int TH = 4 * RPW, PR = TH + 2;
    constexpr int DN = TH * 32 * 4, DPT = (DN + 255) / 256;        // dY uint4s, per thread
    constexpr int PN = PR * kPatchW * 4, PPT = (PN + 255) / 256;   // patch uint4s, per thread
    __shared__ __attribute__((aligned(16))) uint16_t lds[(TH * 32 + PR * kPatchW) * kWg3Ld];
    static_assert(sizeof(lds) >= 4 * 16 * 64 * sizeof(float), "the wave reduction reuses the tiles");
    uint16_t* t_dy = lds;
    uint16_t* t_x = lds + TH * 32 * kWg3Ld;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // work item: consecutive items share a chunk (and so its tiles) and land
    // on one XCD's L2
    const int item = xcd_band((int)blockIdx.x, (int)gridDim.x);
    const int cb = item % nbc, nb = (item / nbc) % nbn, chunk = item / (nbc * nbn);
    const int n0 = nb * 32, c0 = cb * 32;
    const int tiles_x = (a.w + 31) / 32, tiles_y = (a.h + TH - 1) / TH;
    const int ntiles = a.n_img * tiles_x * tiles_y;
    const int t_beg = chunk * tiles_per_chunk, t_end = min(ntiles, t_beg + tiles_per_chunk);
    const bool do_bias = bpart && cb == 0;
    // lane roles in the transposing reads: group g = lane / 16 covers pixels
    // 8 g .. 8 g + 7 of a 32-pixel row; lane i of the group addresses pixel
    // 8 g + 4 h + i / 4 (h: first or second read) and channels 4 (i % 4) .. +3
    const int px_lane = 8 * (lane >> 4) + ((lane & 15) >> 2), ch_lane = 4 * (lane & 3);
    floatx4 acc[9][2][2];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[t][i][j] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    floatx4 accb[2] = {floatx4{0.0f, 0.0f, 0.0f, 0.0f}, floatx4{0.0f, 0.0f, 0.0f, 0.0f}};
    Frag ones;
#pragma unroll
    for (int i = 0; i < 8; ++i) ones.h[i] = 0x3f80;  // bf16 1.0
    for (int t = t_beg; t < t_end; ++t) {
        const int img = t / (tiles_x * tiles_y), r = t - img * tiles_x * tiles_y;
        const int ty = r / tiles_x, y0 = ty * TH, x0 = (r - ty * tiles_x) * 32;
        u32x4 dv[DPT], pv[PPT];
#pragma unroll
        for (int u = 0; u < DPT; ++u) {
            const int idx = threadIdx.x + 256 * u, px = idx >> 2, part8 = (idx & 3) * 8;
            const int y = y0 + (px >> 5), x = x0 + (px & 31);
            dv[u] = u32x4{0u, 0u, 0u, 0u};
            if (idx < DN && y < a.h && x < a.w && n0 + part8 < a.cout)
                dv[u] = *reinterpret_cast<const u32x4*>(dy + (((size_t)img * a.h + y) * a.w + x) * dy_cs + dy_co + n0 +
                                                        part8);
        }
#pragma unroll
        for (int u = 0; u < PPT; ++u) {
            const int idx = threadIdx.x + 256 * u, px = idx >> 2, part8 = (idx & 3) * 8;
            const int pr = px / kPatchW, pc = px - pr * kPatchW;
            const int y = y0 - 1 + pr, x = x0 - 1 + pc;
            pv[u] = u32x4{0u, 0u, 0u, 0u};
            if (idx < PN && (unsigned)y < (unsigned)a.h && (unsigned)x < (unsigned)a.w)
                pv[u] = *reinterpret_cast<const u32x4*>(a.x + (((size_t)img * a.h + y) * a.w + x) * a.x_cs + a.x_co +
                                                        c0 + part8);
        }
        __syncthreads();  // the previous tile is consumed
#pragma unroll
        for (int u = 0; u < DPT; ++u) {
            const int idx = threadIdx.x + 256 * u;
            if (idx < DN) *reinterpret_cast<u32x4*>(t_dy + (idx >> 2) * kWg3Ld + (idx & 3) * 8) = dv[u];
        }
#pragma unroll
        for (int u = 0; u < PPT; ++u) {
            const int idx = threadIdx.x + 256 * u;
            if (idx < PN) *reinterpret_cast<u32x4*>(t_x + (idx >> 2) * kWg3Ld + (idx & 3) * 8) = pv[u];
        }
        __syncthreads();
        // A operands of the wave's rows: dY^T, channels 16 i + lane % 16
        bf16x8 fa[RPW][2];
#pragma unroll
        for (int rr = 0; rr < RPW; ++rr)
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const uint16_t* p = t_dy + ((wave * RPW + rr) * 32 + px_lane) * kWg3Ld + 16 * i + ch_lane;
                fa[rr][i] = tr_frag(p, p + 4 * kWg3Ld);
            }
        if (do_bias) {
#pragma unroll
            for (int rr = 0; rr < RPW; ++rr)
#pragma unroll
                for (int i = 0; i < 2; ++i)
                    accb[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[rr][i], ones.v, accb[i], 0, 0, 0);
        }
        // patch row wave RPW + pr serves output row rr through tap row
        // dy = pr - rr - 1 (dy in -1..1)
#pragma unroll
        for (int pr = 0; pr < RPW + 2; ++pr) {
            bf16x8 fb[3][2];
#pragma unroll
            for (int dx = 0; dx < 3; ++dx)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const uint16_t* p = t_x + ((wave * RPW + pr) * kPatchW + px_lane + dx) * kWg3Ld + 16 * j + ch_lane;
                    fb[dx][j] = tr_frag(p, p + 4 * kWg3Ld);
                }
#pragma unroll
            for (int rr = 0; rr < RPW; ++rr) {
                const int dyi = pr - rr;  // tap row index dy + 1
                if (dyi < 0 || dyi > 2) continue;
#pragma unroll
                for (int dx = 0; dx < 3; ++dx)
#pragma unroll
                    for (int i = 0; i < 2; ++i)
#pragma unroll
                        for (int j = 0; j < 2; ++j)
                            acc[dyi * 3 + dx][i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                fa[rr][i], fb[dx][j], acc[dyi * 3 + dx][i][j], 0, 0, 0);
            }
        }
    }
    // sum the 4 waves' accumulators through LDS, one tap at a time; lane l's
    // accumulator r of (i, j) is n = n0 + 16 i + 4 (l / 16) + r,
    // c = c0 + 16 j + l % 16
    __syncthreads();
    float* red = reinterpret_cast<float*>(lds);
    const size_t kw = a.k_pad;
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
#pragma unroll
        for (int q = 0; q < 16; ++q) red[(wave * 16 + q) * 64 + lane] = acc[tap][q >> 3][(q >> 2) & 1][q & 3];
        __syncthreads();
        for (int e = threadIdx.x; e < 1024; e += 256) {
            const int q = e >> 6, l = e & 63;
            const float s = (red[e] + red[1024 + e]) + (red[2048 + e] + red[3072 + e]);
            const int n = n0 + 16 * (q >> 3) + 4 * (l >> 4) + (q & 3), c = c0 + 16 * ((q >> 2) & 1) + (l & 15);
            if (n < a.cout) part[((size_t)chunk * a.n_pad + n) * kw + tap * a.cin + c] = s;
        }
        __syncthreads();
    }
    if (do_bias) {
        // column 0 (lanes 0, 16, 32, 48) of the ones-product holds the sums
#pragma unroll
        for (int q = 0; q < 8; ++q) red[(wave * 8 + q) * 64 + lane] = accb[q >> 2][q & 3];
        __syncthreads();
        if (threadIdx.x < 32) {
            const int t = threadIdx.x, q = (t >> 4) * 4 + (t & 3), l = ((t & 15) >> 2) * 16;
            const float s = (red[q * 64 + l] + red[(8 + q) * 64 + l]) + (red[(16 + q) * 64 + l] + red[(24 + q) * 64 + l]);
            if (n0 + t < a.cout) bpart[(size_t)chunk * a.n_pad + n0 + t] = s;
        }
    }
}

// ------------------------------------------------------------------ pointwise weight gradients
// The 1x1 layer and the stride-2 2x2 transposed convolution (one GEMM per
// output parity q): dW[q][n][c] = sum_p dY(p, q)[n] X[p][c] over the GEMM's
// pixels p, dY(p, q) being the output pixel that p writes for parity q.
// Block = (chunk of 256-pixel tiles, parity, 32 output channels from n0, 32
// input channels from c0); per tile it stages dY [pixel][n] and X [pixel][c]
// in LDS as they lie in memory (16-byte loads where the slices allow, else
// element loads, zero past the channel counts), and wave w reduces pixels
// 64 w .. 64 w + 63 of the tile with the transposing LDS reads, as in the
// 3x3 kernel (without taps).  The bias gradient rides along in the blocks of
// the first channel chunk.
template <int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_wgrad_pt(
    ConvArgs a, const uint16_t* __restrict__ dy, int dy_cs, int dy_co, int tiles_per_chunk, int nbn, int nbc,
    float* part, float* bpart)
{
    constexpr int NQ = MODE == kUp ? 4 : 1;
    __shared__ __attribute__((aligned(16))) uint16_t lds[2 * 256 * kWg3Ld];
    static_assert(sizeof(lds) >= 4 * 16 * 64 * sizeof(float), "the wave reduction reuses the tiles");
    uint16_t* t_dy = lds;
    uint16_t* t_x = lds + 256 * kWg3Ld;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int item = xcd_band((int)blockIdx.x, (int)gridDim.x);
    const int cb = item % nbc, nb = (item / nbc) % nbn, q = (item / (nbc * nbn)) % NQ;
    const int chunk = item / (nbc * nbn * NQ);
    const int n0 = nb * 32, c0 = cb * 32;
    const int hw = a.h * a.w, npix = a.n_img * hw, ntiles = (npix + 255) / 256;
    const int t_beg = chunk * tiles_per_chunk, t_end = min(ntiles, t_beg + tiles_per_chunk);
    const bool do_bias = bpart && cb == 0;
    const bool dy_vec = dy_cs % 8 == 0 && dy_co % 8 == 0;
    const bool x_vec = a.x_cs % 8 == 0 && a.x_co % 8 == 0;
    const double inv_w = 1.0 / (double)a.w;
    const int px_lane = 8 * (lane >> 4) + ((lane & 15) >> 2), ch_lane = 4 * (lane & 3);
    floatx4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    floatx4 accb[2] = {floatx4{0.0f, 0.0f, 0.0f, 0.0f}, floatx4{0.0f, 0.0f, 0.0f, 0.0f}};
    Frag ones;
#pragma unroll
    for (int i = 0; i < 8; ++i) ones.h[i] = 0x3f80;  // bf16 1.0
    // a tile's 16-byte pieces (4 per thread of dY and of X) into registers;
    // the next tile's are loaded while this one is multiplied
    u32x4 dv[4], xv[4];
    auto fetch = [&](int t) __attribute__((always_inline)) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int idx = threadIdx.x + 256 * u, px = idx >> 2, s8 = (idx & 3) * 8;
            const int p = t * 256 + px;
            Frag fd = zero_frag(), fx = zero_frag();
            if (p < npix) {
                size_t pd = (size_t)p;
                if (MODE == kUp) {
                    // row R = img h + y of the GEMM grid; its output rows are
                    // 2 R and 2 R + 1 (img 2h + 2y = 2 R).  R = p / w through
                    // a double reciprocal, corrected to the exact quotient
                    int R = (int)((double)p * inv_w);
                    if (R * a.w > p) --R;
                    if ((R + 1) * a.w <= p) ++R;
                    const int x = p - R * a.w;
                    pd = ((size_t)(2 * R + (q >> 1))) * 2 * a.w + 2 * x + (q & 1);
                }
                const uint16_t* sd = dy + pd * dy_cs + dy_co + n0 + s8;
                if (dy_vec && n0 + s8 + 8 <= a.cout) {
                    fd.u = *reinterpret_cast<const uint4*>(sd);
                } else {
#pragma unroll
                    for (int i = 0; i < 8; ++i)
                        if (n0 + s8 + i < a.cout) fd.h[i] = sd[i];
                }
                const uint16_t* sx = a.x + (size_t)p * a.x_cs + a.x_co + c0 + s8;
                if (x_vec && c0 + s8 + 8 <= a.cin) {
                    fx.u = *reinterpret_cast<const uint4*>(sx);
                } else {
#pragma unroll
                    for (int i = 0; i < 8; ++i)
                        if (c0 + s8 + i < a.cin) fx.h[i] = sx[i];
                }
            }
            dv[u] = u32x4{fd.u.x, fd.u.y, fd.u.z, fd.u.w};
            xv[u] = u32x4{fx.u.x, fx.u.y, fx.u.z, fx.u.w};
        }
    };
    if (t_beg < t_end) fetch(t_beg);
    for (int t = t_beg; t < t_end; ++t) {
        __syncthreads();  // the previous tile is consumed
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int idx = threadIdx.x + 256 * u;
            *reinterpret_cast<u32x4*>(t_dy + (idx >> 2) * kWg3Ld + (idx & 3) * 8) = dv[u];
            *reinterpret_cast<u32x4*>(t_x + (idx >> 2) * kWg3Ld + (idx & 3) * 8) = xv[u];
        }
        __syncthreads();
        if (t + 1 < t_end) fetch(t + 1);
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int pr = 64 * wave + 32 * s + px_lane;
            bf16x8 fa[2], fb[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const uint16_t* p = t_dy + pr * kWg3Ld + 16 * i + ch_lane;
                fa[i] = tr_frag(p, p + 4 * kWg3Ld);
                const uint16_t* px = t_x + pr * kWg3Ld + 16 * i + ch_lane;
                fb[i] = tr_frag(px, px + 4 * kWg3Ld);
            }
#pragma unroll
            for (int i = 0; i < 2; ++i) {
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
                if (do_bias) accb[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], ones.v, accb[i], 0, 0, 0);
            }
        }
    }
    // the 4 waves' sums through LDS; lane l's accumulator r of (i, j) is
    // n = n0 + 16 i + 4 (l / 16) + r, c = c0 + 16 j + l % 16
    __syncthreads();
    float* red = reinterpret_cast<float*>(lds);
    const size_t kw = (size_t)NQ * a.k_pad;
#pragma unroll
    for (int e = 0; e < 16; ++e) red[(wave * 16 + e) * 64 + lane] = acc[e >> 3][(e >> 2) & 1][e & 3];
    __syncthreads();
    for (int e = threadIdx.x; e < 1024; e += 256) {
        const int qq = e >> 6, l = e & 63;
        const float s = (red[e] + red[1024 + e]) + (red[2048 + e] + red[3072 + e]);
        const int n = n0 + 16 * (qq >> 3) + 4 * (l >> 4) + (qq & 3), c = c0 + 16 * ((qq >> 2) & 1) + (l & 15);
        if (n < a.cout && c < a.cin) part[((size_t)chunk * a.n_pad + n) * kw + (size_t)q * a.k_pad + c] = s;
    }
    if (do_bias) {
        __syncthreads();
#pragma unroll
        for (int e = 0; e < 8; ++e) red[(wave * 8 + e) * 64 + lane] = accb[e >> 2][e & 3];
        __syncthreads();
        if (threadIdx.x < 32) {
            const int t = threadIdx.x, e = (t >> 4) * 4 + (t & 3), l = ((t & 15) >> 2) * 16;
            const float s = (red[e * 64 + l] + red[(8 + e) * 64 + l]) + (red[(16 + e) * 64 + l] + red[(24 + e) * 64 + l]);
            if (n0 + t < a.cout) bpart[((size_t)chunk * NQ + q) * a.n_pad + n0 + t] = s;
        }
    }
}

// ------------------------------------------------------------------ 3x3 weight gradients of a one-channel input
// The first layer (C_in = 1): K = 9 taps, so per 32-pixel row a lane builds
// its B operand itself, 8 pixels of one tap read from the staged input patch
// (column 9 of B is all ones: the bias gradient; columns 10-15 zero), and the
// A operand (dY^T) comes from the transposing reads as in the other kernels.
// Block = (chunk of 8 x 32 tiles, 32 output channels from n0).
__global__ __launch_bounds__(256) void k_wgrad3_c1(ConvArgs a, const uint16_t* __restrict__ dy, int dy_cs, int dy_co,
                                                   int tiles_per_chunk, int nbn, float* part, float* bpart)
{
    constexpr int TH = 8, PR = TH + 2, DN = TH * 32 * 4;
    __shared__ __attribute__((aligned(16))) uint16_t t_dy[TH * 32 * kWg3Ld];
    __shared__ uint16_t t_x[PR * kPatchW];
    static_assert(sizeof(t_dy) >= 4 * 8 * 64 * sizeof(float), "the wave reduction reuses the tile");
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int item = xcd_band((int)blockIdx.x, (int)gridDim.x);
    const int nb = item % nbn, chunk = item / nbn, n0 = nb * 32;
    const int tiles_x = (a.w + 31) / 32, tiles_y = (a.h + TH - 1) / TH;
    const int ntiles = a.n_img * tiles_x * tiles_y;
    const int t_beg = chunk * tiles_per_chunk, t_end = min(ntiles, t_beg + tiles_per_chunk);
    const int px_lane = 8 * (lane >> 4) + ((lane & 15) >> 2), ch_lane = 4 * (lane & 3);
    const int tap = lane & 15, g = lane >> 4;
    const int tdy = tap / 3, tdx = tap - 3 * (tap / 3);
    floatx4 acc[2] = {floatx4{0.0f, 0.0f, 0.0f, 0.0f}, floatx4{0.0f, 0.0f, 0.0f, 0.0f}};
    for (int t = t_beg; t < t_end; ++t) {
        const int img = t / (tiles_x * tiles_y), r = t - img * tiles_x * tiles_y;
        const int ty = r / tiles_x, y0 = ty * TH, x0 = (r - ty * tiles_x) * 32;
        u32x4 dv[DN / 256];
#pragma unroll
        for (int u = 0; u < DN / 256; ++u) {
            const int idx = threadIdx.x + 256 * u, px = idx >> 2, part8 = (idx & 3) * 8;
            const int y = y0 + (px >> 5), x = x0 + (px & 31);
            dv[u] = u32x4{0u, 0u, 0u, 0u};
            if (y < a.h && x < a.w && n0 + part8 < a.cout)
                dv[u] = *reinterpret_cast<const u32x4*>(dy + (((size_t)img * a.h + y) * a.w + x) * dy_cs + dy_co + n0 +
                                                        part8);
        }
        uint16_t xv[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int idx = threadIdx.x + 256 * u, pr = idx / kPatchW, pc = idx - pr * kPatchW;
            const int y = y0 - 1 + pr, x = x0 - 1 + pc;
            xv[u] = 0;
            if (idx < PR * kPatchW && (unsigned)y < (unsigned)a.h && (unsigned)x < (unsigned)a.w)
                xv[u] = a.x[(((size_t)img * a.h + y) * a.w + x) * a.x_cs + a.x_co];
        }
        __syncthreads();  // the previous tile is consumed
#pragma unroll
        for (int u = 0; u < DN / 256; ++u) {
            const int idx = threadIdx.x + 256 * u;
            *reinterpret_cast<u32x4*>(t_dy + (idx >> 2) * kWg3Ld + (idx & 3) * 8) = dv[u];
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int idx = threadIdx.x + 256 * u;
            if (idx < PR * kPatchW) t_x[idx] = xv[u];
        }
        __syncthreads();
#pragma unroll
        for (int rr = 0; rr < 2; ++rr) {
            const int row = wave * 2 + rr;
            Frag fb = zero_frag();
            if (tap < 9) {
                const uint16_t* src = t_x + (row + tdy) * kPatchW + 8 * g + tdx;
#pragma unroll
                for (int k = 0; k < 8; ++k) fb.h[k] = src[k];
            } else if (tap == 9) {
#pragma unroll
                for (int k = 0; k < 8; ++k) fb.h[k] = 0x3f80;  // bf16 1.0
            }
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const uint16_t* p = t_dy + (row * 32 + px_lane) * kWg3Ld + 16 * i + ch_lane;
                acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(tr_frag(p, p + 4 * kWg3Ld), fb.v, acc[i], 0, 0, 0);
            }
        }
    }
    // lane l's accumulator r of n-tile i: n = n0 + 16 i + 4 (l / 16) + r, tap l % 16
    __syncthreads();
    float* red = reinterpret_cast<float*>(t_dy);
#pragma unroll
    for (int e = 0; e < 8; ++e) red[(wave * 8 + e) * 64 + lane] = acc[e >> 2][e & 3];
    __syncthreads();
    for (int e = threadIdx.x; e < 512; e += 256) {
        const int qq = e >> 6, l = e & 63;
        const float s = (red[e] + red[512 + e]) + (red[1024 + e] + red[1536 + e]);
        const int n = n0 + 16 * (qq >> 2) + 4 * (l >> 4) + (qq & 3), k = l & 15;
        if (n >= a.cout) continue;
        if (k < 9) part[((size_t)chunk * a.n_pad + n) * a.k_pad + k] = s;
        else if (k == 9 && bpart) bpart[(size_t)chunk * a.n_pad + n] = s;
    }
}

// The weight and bias gradients from the blocks' partials, written straight
// into the parameter layout: element i < co kw of the packed [n][kw] grid
// (n = i / kw, k = i % kw) sums part[c stride + i] over the chunks c and goes
// to the weight array ([3][3][C_in][C_out], [C_in][C_out] or
// [2][2][C_in][C_out], i.e. index (k-row) C_out + n); the co elements after
// them sum the bias partials bpart[c n_pad + n] over bchunks.  A block covers
// 32 elements with 8 slices: slice s adds chunks s, s + 8, ... in order, then
// the 8 slice sums are added in order of s (a fixed order, so the result does
// not depend on the launch).
constexpr int kRedSlices = 8;

__global__ __launch_bounds__(256) void k_wgrad_finish(const float* __restrict__ part, int chunks, size_t stride,
                                                      int kw, int mode, int ci, int co, int k_pad,
                                                      const float* __restrict__ bpart, int bchunks, int n_pad,
                                                      float* gw, float* gb)
{
    __shared__ float red[kRedSlices][32];
    const int e = threadIdx.x & 31, sl = threadIdx.x >> 5;
    const size_t count = (size_t)co * kw, total = count + (gb ? co : 0);
    const size_t i = (size_t)blockIdx.x * 32 + e;
    const float* src = i < count ? part + i : bpart + (i - count);
    const size_t st = i < count ? stride : (size_t)n_pad;
    const int nc = i < count ? chunks : bchunks;
    float s = 0.0f;
    if (i < total) {
        int c = sl;
        for (; c + 3 * kRedSlices < nc; c += 4 * kRedSlices) {  // 4 loads in flight
            float v[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) v[j] = src[(size_t)(c + j * kRedSlices) * st];
#pragma unroll
            for (int j = 0; j < 4; ++j) s += v[j];
        }
        for (; c < nc; c += kRedSlices) s += src[(size_t)c * st];
    }
    red[sl][e] = s;
    __syncthreads();
    if (sl == 0 && i < total) {
        float t = red[0][e];
#pragma unroll
        for (int j = 1; j < kRedSlices; ++j) t += red[j][e];
        if (i >= count) {
            gb[i - count] = t;
        } else {
            const int n = (int)(i / kw), k = (int)(i - (size_t)n * kw);
            if (mode == kUp) {
                const int q = k / k_pad, c = k - q * k_pad;
                if (c < ci) gw[((size_t)q * ci + c) * co + n] = t;
            } else if (k < (mode == kConv3 ? 9 * ci : ci)) {
                gw[(size_t)k * co + n] = t;
            }
        }
    }
}

int wgrad_chunks(const ConvArgs& a, int chunk_px)
{
    const int npix = a.n_img * a.h * a.w;
    return (npix + chunk_px - 1) / chunk_px;
}

int wgrad_max_chunks(int npix, int n_pad, int kw)
{
    // about 1024 blocks in all (4 per CU), but no chunk under 1024 pixels;
    // fewer chunks also keep the ordered chunk sum short.  Non-decreasing in
    // npix, so the largest batch bounds every smaller one.
    const int per_chunk = (n_pad / 64) * (kw / 64);
    return std::max(1, std::min((1024 + per_chunk - 1) / per_chunk, (npix + 1023) / 1024));
}

int wgrad_chunk_px(int npix, int n_pad, int kw)
{
    const int chunks = wgrad_max_chunks(npix, n_pad, kw);
    const int px = (npix + chunks - 1) / chunks;
    return (px + 63) / 64 * 64;  // ceil(npix / px) <= chunks
}

// k_wgrad3 applies: a 3x3 layer with C_in a multiple of 32 and 16-byte
// aligned slices; k_wgrad3_c1: a 3x3 layer with one input channel
static bool wgrad3_fits(const ConvArgs& a, int mode, int dy_cs, int dy_co)
{
    return mode == kConv3 && a.cin % 32 == 0 && a.cout % 8 == 0 && a.x_cs % 8 == 0 && a.x_co % 8 == 0 &&
           dy_cs % 8 == 0 && dy_co % 8 == 0;
}

static bool wgrad3_c1_fits(const ConvArgs& a, int mode, int dy_cs, int dy_co)
{
    return mode == kConv3 && a.cin == 1 && a.cout % 8 == 0 && dy_cs % 8 == 0 && dy_co % 8 == 0;
}

constexpr int kWg3Rpw = 2;       // rows per wave: 8-row tiles
constexpr int kWg3Blocks = 512;   // about two blocks per CU
constexpr int kWgPtBlocks = 1024; // the pointwise kernel: about four per CU

static long long wgrad3_tiles(int n_img, int h, int w)
{
    return (long long)n_img * ((h + 4 * kWg3Rpw - 1) / (4 * kWg3Rpw)) * ((w + 31) / 32);
}

static long long wgrad_pt_tiles(int n_img, int h, int w) { return ((long long)n_img * h * w + 255) / 256; }

// chunks over nt tiles for m blocks per chunk: about kWg3Blocks blocks in
// all, every chunk non-empty
static int tile_chunks(long long nt, long long m, int* tiles_per_chunk, int blocks = kWg3Blocks)
{
    const long long t = std::max(1LL, (nt * m + blocks - 1) / blocks);
    *tiles_per_chunk = (int)t;
    return (int)((nt + t - 1) / t);
}

// chunks of the LDS-tiled kernels (0 where none applies); an upper bound over
// every batch up to n_img: ceil(nt / ceil(nt m / B)) <= min(nt, ceil(B / m))
int wgrad_tiled_max_chunks(int mode, int n_img, int h, int w, int ci, int co)
{
    const long long nbn = (co + 31) / 32;
    long long nt, m;
    if (mode == kConv3 && (ci % 32 == 0 || ci == 1)) {
        nt = wgrad3_tiles(n_img, h, w);
        m = nbn * std::max(1, ci / 32);
    } else if (mode == kPoint || mode == kUp) {
        nt = wgrad_pt_tiles(n_img, h, w);
        m = nbn * ((ci + 31) / 32) * (mode == kUp ? 4 : 1);
        return (int)std::min(nt, (kWgPtBlocks + m - 1) / m);
    } else {
        return 0;
    }
    return (int)std::min(nt, (kWg3Blocks + m - 1) / m);
}

hipError_t launch_wgrad(const ConvArgs& a, int mode, const uint16_t* dy, int dy_cs, int dy_co, int chunk_px,
                        float* part, float* out, float* bpart, float* bias_out, hipStream_t s)
{
    const int kw = mode == kUp ? 4 * a.k_pad : a.k_pad;
    float* bp = bias_out ? bpart : nullptr;
    int chunks, tpc = 1;
    const int nbn = (a.cout + 31) / 32;
    if (wgrad3_fits(a, mode, dy_cs, dy_co)) {
        const int nbc = a.cin / 32;
        chunks = tile_chunks(wgrad3_tiles(a.n_img, a.h, a.w), (long long)nbn * nbc, &tpc);
        hipLaunchKernelGGL(k_wgrad3<kWg3Rpw>, dim3((unsigned)(chunks * nbn * nbc)), dim3(256), 0, s, a, dy, dy_cs,
                           dy_co, tpc, nbn, nbc, part, bp);
    } else if (wgrad3_c1_fits(a, mode, dy_cs, dy_co)) {
        chunks = tile_chunks(wgrad3_tiles(a.n_img, a.h, a.w), nbn, &tpc);
        hipLaunchKernelGGL(k_wgrad3_c1, dim3((unsigned)(chunks * nbn)), dim3(256), 0, s, a, dy, dy_cs, dy_co, tpc,
                           nbn, part, bp);
    } else if (mode == kPoint || mode == kUp) {
        const int nbc = (a.cin + 31) / 32, nq = mode == kUp ? 4 : 1;
        chunks = tile_chunks(wgrad_pt_tiles(a.n_img, a.h, a.w), (long long)nbn * nbc * nq, &tpc, kWgPtBlocks);
        const dim3 g((unsigned)(chunks * nbn * nbc * nq));
        if (mode == kUp)
            hipLaunchKernelGGL(k_wgrad_pt<kUp>, g, dim3(256), 0, s, a, dy, dy_cs, dy_co, tpc, nbn, nbc, part, bp);
        else
            hipLaunchKernelGGL(k_wgrad_pt<kPoint>, g, dim3(256), 0, s, a, dy, dy_cs, dy_co, tpc, nbn, nbc, part, bp);
    } else {
        chunks = wgrad_chunks(a, chunk_px);
        dim3 grid((unsigned)chunks, (unsigned)(a.n_pad / 64), (unsigned)(kw / 64));
        hipLaunchKernelGGL(k_wgrad, grid, dim3(256), 0, s, a, dy, dy_cs, dy_co, chunk_px, part, bp);
    }
    const size_t total = (size_t)a.cout * kw + (bias_out ? a.cout : 0);
    hipLaunchKernelGGL(k_wgrad_finish, dim3((unsigned)((total + 31) / 32)), dim3(256), 0, s, part, chunks,
                       (size_t)a.n_pad * kw, kw, mode, a.cin, a.cout, a.k_pad, bpart, chunks * (mode == kUp ? 4 : 1),
                       a.n_pad, out, bias_out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ elementwise
// 2x2 average pooling and its adjoint (channel slices)
__global__ void k_avgpool(const uint16_t* x, int xcs, int xco, uint16_t* y, int n_img, int h, int w, int c)
{
    const size_t n = (size_t)n_img * (h / 2) * (w / 2) * c;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int k = (int)(i % c);
        size_t t = i / c;
        const int xo = (int)(t % (w / 2));
        t /= (w / 2);
        const int yo = (int)(t % (h / 2));
        const int img = (int)(t / (h / 2));
        float s = 0.0f;
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx)
                s += bf2f(x[(((size_t)img * h + 2 * yo + dy) * w + 2 * xo + dx) * xcs + xco + k]);
        y[i] = f2bf(0.25f * s);
    }
}

__global__ void k_avgpool_back(const uint16_t* dy, uint16_t* dx, int dxcs, int dxco, int n_img, int h, int w, int c,
                               int accumulate, const uint16_t* mask, int mcs, int mco)
{
    // dx has h x w pixels; dy has h/2 x w/2 with c channels (dense)
    const size_t n = (size_t)n_img * h * w * c;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int k = (int)(i % c);
        size_t t = i / c;
        const int x = (int)(t % w);
        t /= w;
        const int y = (int)(t % h);
        const int img = (int)(t / h);
        float v = 0.25f * bf2f(dy[(((size_t)img * (h / 2) + y / 2) * (w / 2) + x / 2) * c + k]);
        const size_t px = ((size_t)img * h + y) * w + x;
        uint16_t* d = dx + px * dxcs + dxco + k;
        if (accumulate) v += bf2f(*d);
        if (mask && !(bf2f(mask[px * mcs + mco + k]) > 0.0f)) v = 0.0f;
        *d = f2bf(v);
    }
}

// The same two, 8 channels (16 bytes) per thread for 16-byte aligned slices
// (the same sums in the same order).
__global__ void k_avgpool8(const uint16_t* x, int xcs, int xco, uint16_t* y, int n_img, int h, int w, int c8)
{
    const size_t n = (size_t)n_img * (h / 2) * (w / 2) * c8;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int k = (int)(i % c8) * 8;
        const size_t t = i / c8;
        const int xo = (int)(t % (w / 2));
        const size_t t2 = t / (w / 2);
        const int yo = (int)(t2 % (h / 2));
        const int img = (int)(t2 / (h / 2));
        Frag v[4];
#pragma unroll
        for (int d = 0; d < 4; ++d)
            v[d].u = *reinterpret_cast<const uint4*>(
                x + (((size_t)img * h + 2 * yo + (d >> 1)) * w + 2 * xo + (d & 1)) * xcs + xco + k);
        Frag o;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            float sum = 0.0f;
#pragma unroll
            for (int d = 0; d < 4; ++d) sum += bf2f(v[d].h[j]);
            o.h[j] = f2bf(0.25f * sum);
        }
        *reinterpret_cast<uint4*>(y + t * (size_t)c8 * 8 + k) = o.u;
    }
}

__global__ void k_avgpool_back8(const uint16_t* dy, uint16_t* dx, int dxcs, int dxco, int n_img, int h, int w, int c8,
                                int accumulate, const uint16_t* mask, int mcs, int mco)
{
    const size_t n = (size_t)n_img * h * w * c8;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int k = (int)(i % c8) * 8;
        const size_t t = i / c8;
        const int x = (int)(t % w);
        const size_t t2 = t / w;
        const int y = (int)(t2 % h);
        const int img = (int)(t2 / h);
        Frag g, o;
        g.u = *reinterpret_cast<const uint4*>(dy + (((size_t)img * (h / 2) + y / 2) * (w / 2) + x / 2) * c8 * 8 + k);
        uint4* d = reinterpret_cast<uint4*>(dx + t * dxcs + dxco + k);
        if (accumulate) o.u = *d;
        Frag m;
        if (mask) m.u = *reinterpret_cast<const uint4*>(mask + t * mcs + mco + k);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            float v = 0.25f * bf2f(g.h[j]);
            if (accumulate) v += bf2f(o.h[j]);
            if (mask && !(bf2f(m.h[j]) > 0.0f)) v = 0.0f;
            o.h[j] = f2bf(v);
        }
        *d = o.u;
    }
}

hipError_t launch_avgpool(const uint16_t* x, int xcs, int xco, uint16_t* y, int n_img, int h, int w, int c,
                          hipStream_t s)
{
    if (c % 8 == 0 && xcs % 8 == 0 && xco % 8 == 0) {
        const size_t n8 = (size_t)n_img * (h / 2) * (w / 2) * (c / 8);
        hipLaunchKernelGGL(k_avgpool8, dim3((unsigned)std::min<size_t>((n8 + 255) / 256, 8192)), dim3(256), 0, s, x,
                           xcs, xco, y, n_img, h, w, c / 8);
        return hipGetLastError();
    }
    const size_t n = (size_t)n_img * (h / 2) * (w / 2) * c;
    hipLaunchKernelGGL(k_avgpool, dim3((unsigned)std::min<size_t>((n + 255) / 256, 8192)), dim3(256), 0, s, x, xcs, xco,
                       y, n_img, h, w, c);
    return hipGetLastError();
}

hipError_t launch_avgpool_back(const uint16_t* dy, uint16_t* dx, int dxcs, int dxco, int n_img, int h, int w, int c,
                               int accumulate, const uint16_t* mask, int mcs, int mco, hipStream_t s)
{
    if (c % 8 == 0 && dxcs % 8 == 0 && dxco % 8 == 0 && (!mask || (mcs % 8 == 0 && mco % 8 == 0))) {
        const size_t n8 = (size_t)n_img * h * w * (c / 8);
        hipLaunchKernelGGL(k_avgpool_back8, dim3((unsigned)std::min<size_t>((n8 + 255) / 256, 8192)), dim3(256), 0, s,
                           dy, dx, dxcs, dxco, n_img, h, w, c / 8, accumulate, mask, mcs, mco);
        return hipGetLastError();
    }
    const size_t n = (size_t)n_img * h * w * c;
    hipLaunchKernelGGL(k_avgpool_back, dim3((unsigned)std::min<size_t>((n + 255) / 256, 8192)), dim3(256), 0, s, dy, dx,
                       dxcs, dxco, n_img, h, w, c, accumulate, mask, mcs, mco);
    return hipGetLastError();
}

// fp32 <-> bf16 (dense)
__global__ void k_to_bf16(const float* x, uint16_t* y, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        y[i] = f2bf(x[i]);
}

hipError_t launch_to_bf16(const float* x, uint16_t* y, size_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)std::min<size_t>((n + 255) / 256, 8192)), dim3(256), 0, s, x, y, n);
    return hipGetLastError();
}

__global__ void k_to_f32(const uint16_t* x, float* y, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        y[i] = bf2f(x[i]);
}

hipError_t launch_to_f32(const uint16_t* x, float* y, size_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_to_f32, dim3((unsigned)std::min<size_t>((n + 255) / 256, 8192)), dim3(256), 0, s, x, y, n);
    return hipGetLastError();
}

// ------------------------------------------------------------------ weights
// fp32 master (oracle layout) -> packed bf16 GEMM operands
//   conv3 forward: W[a][c][i][o] -> P[o][(3a+c) Ci + i]
//   conv3 backward data: P[i][(8 - tap) Co + o] (flipped taps, in/out swapped)
//   1x1: W[i][o] -> P[o][i];  backward data: P[i][o]
//   up (2x2, stride 2) forward: W[a][c][i][o] -> P[q = 2a + c][o][i]
//   up backward data: P[i][q Co + o]
// One launch packs every table entry: blockIdx.y selects the entry, the
// x blocks stride over its elements.
__global__ __launch_bounds__(256) void k_pack(const PackDesc* __restrict__ tab)
{
    const PackDesc d = tab[blockIdx.y];
    const int nq = (d.mode == kUp && !d.back) ? 4 : 1;
    const int ci = d.ci, co = d.co, k_pad = d.k_pad;
    const size_t plane = (size_t)d.n_pad * k_pad, total = (size_t)nq * plane;
    const float* w = d.w;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const int q = (int)(e / plane);
        const size_t r = e - (size_t)q * plane;
        const int n = (int)(r / k_pad), k = (int)(r - (size_t)n * k_pad);
        float v = 0.0f;
        if (d.mode == kConv3 && !d.back) {
            if (n < co && k < 9 * ci) v = w[(size_t)k * co + n];
        } else if (d.mode == kConv3) {
            if (n < ci && k < 9 * co) {
                const int tap = 8 - k / co, o = k % co;
                v = w[((size_t)tap * ci + n) * co + o];
            }
        } else if (d.mode == kPoint && !d.back) {
            if (n < co && k < ci) v = w[(size_t)k * co + n];
        } else if (d.mode == kPoint) {
            if (n < ci && k < co) v = w[(size_t)n * co + k];
        } else if (!d.back) {  // up forward, parity q
            if (n < co && k < ci) v = w[((size_t)q * ci + k) * co + n];
        } else {  // up backward data
            if (n < ci && k < 4 * co) {
                const int qq = k / co, o = k % co;
                v = w[((size_t)qq * ci + n) * co + o];
            }
        }
        d.out[e] = f2bf(v);
    }
}

hipError_t launch_pack(const PackDesc* tab, int entries, hipStream_t s)
{
    if (entries <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pack, dim3(64, (unsigned)entries), dim3(256), 0, s, tab);
    return hipGetLastError();
}

// Adam (Kingma & Ba, Algorithm 1) on the fp32 masters
__global__ void k_adam(float* p, const float* g, float* m, float* v, size_t n, float lr, float b1, float b2, float eps,
                       float c1, float c2)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, size_t n, float lr, float b1, float b2, float eps,
                       int step, hipStream_t s)
{
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((unsigned)std::min<size_t>((n + 255) / 256, 4096)), dim3(256), 0, s, p, g, m, v, n,
                       lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

// mean squared error and its gradient (fp32 NHWC, dense)
__global__ __launch_bounds__(256) void k_mse(const float* y, const float* t, size_t n, float* dy, double* part)
{
    __shared__ double red[256];
    double s = 0.0;
    const float sc = 2.0f / (float)n;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        const float d = y[i] - t[i];
        s += (double)d * d;
        if (dy) dy[i] = sc * d;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// out = scale * sum of part[0 .. n): thread t adds t, t + 256, ... in order,
// then a fixed-order tree over the 256 sums
__global__ __launch_bounds__(256) void k_sum_parts(const double* part, int n, double scale, float* out)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = (float)(red[0] * scale);
}

hipError_t launch_mse(const float* y, const float* t, size_t n, float* dy, double* part, int nblocks, float* loss,
                      hipStream_t s)
{
    hipLaunchKernelGGL(k_mse, dim3((unsigned)nblocks), dim3(256), 0, s, y, t, n, dy, part);
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, s, part, nblocks, 1.0 / (double)n, loss);
    return hipGetLastError();
}

// ------------------------------------------------------------------ EPTV <-> network tensors
// Network tensors are NHWC fp32 on the pixel grid.  With weights, channel 0 is
// the weight of the half-edge right of pixel (i, j) (wx[j][i+1]), channel 1 of
// the half-edge above it (wy[j+1][i]), channel 2 the image, minus an optional
// base image, times `scale`; without weights, that image channel alone.
__global__ void k_eptv_to_maps(const float* f, const float* f_base, const float* wx, const float* wy, int n_img,
                               int ny, int nx, float scale, float* y)
{
    const size_t per = (size_t)ny * nx, n = (size_t)n_img * per;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        const float v = (f_base ? f[e] - f_base[e] : f[e]) * scale;
        if (!wx) {
            y[e] = v;
            continue;
        }
        const size_t img = e / per, pix = e - img * per;
        const int j = (int)(pix / nx), i = (int)(pix - (size_t)j * nx);
        y[e * 3 + 0] = wx[img * (size_t)ny * (nx + 1) + (size_t)j * (nx + 1) + i + 1];
        y[e * 3 + 1] = wy[img * (size_t)(ny + 1) * nx + (size_t)(j + 1) * nx + i];
        y[e * 3 + 2] = v;
    }
}

// The inverse for a 3-channel tensor: the image is channel 2 divided by
// `scale`, plus the optional base image, truncated at zero; the weights are
// clamped to [0, 1]; the half-edges on the left and bottom border, which no
// pixel's channels hold, take the weight of the adjacent half-edge of the
// same row / column.
__global__ void k_maps_to_eptv(const float* y, const float* f_base, int n_img, int ny, int nx, float inv_scale,
                               float* f, float* wx, float* wy)
{
    const size_t per = (size_t)ny * nx, n = (size_t)n_img * per;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        const size_t img = e / per, pix = e - img * per;
        const int j = (int)(pix / nx), i = (int)(pix - (size_t)j * nx);
        const float* yy = y + e * 3;
        const float w0 = fminf(fmaxf(yy[0], 0.0f), 1.0f), w1 = fminf(fmaxf(yy[1], 0.0f), 1.0f);
        const float v = yy[2] * inv_scale;
        f[e] = fmaxf(f_base ? v + f_base[e] : v, 0.0f);
        float* wxi = wx + img * (size_t)ny * (nx + 1);
        float* wyi = wy + img * (size_t)(ny + 1) * nx;
        wxi[(size_t)j * (nx + 1) + i + 1] = w0;
        if (i == 0) wxi[(size_t)j * (nx + 1)] = w0;
        wyi[(size_t)(j + 1) * nx + i] = w1;
        if (j == 0) wyi[i] = w1;
    }
}

static unsigned grid_for(size_t n) { return (unsigned)std::min<size_t>(std::max<size_t>((n + 255) / 256, 1), 4096); }

hipError_t launch_eptv_to_maps(const float* f, const float* f_base, const float* wx, const float* wy, int n_img,
                               int ny, int nx, float scale, float* y, hipStream_t s)
{
    const size_t n = (size_t)n_img * ny * nx;
    hipLaunchKernelGGL(k_eptv_to_maps, dim3(grid_for(n)), dim3(256), 0, s, f, f_base, wx, wy, n_img, ny, nx, scale,
                       y);
    return hipGetLastError();
}

hipError_t launch_maps_to_eptv(const float* y, const float* f_base, int n_img, int ny, int nx, float scale, float* f,
                               float* wx, float* wy, hipStream_t s)
{
    const size_t n = (size_t)n_img * ny * nx;
    hipLaunchKernelGGL(k_maps_to_eptv, dim3(grid_for(n)), dim3(256), 0, s, y, f_base, n_img, ny, nx, 1.0f / scale, f,
                       wx, wy);
    return hipGetLastError();
}

}  // namespace eptv
