// cnn.h -- the U-Net layer kernels (cnn.hip) and the network (unet.cpp).
// Internal to the library.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstdint>

namespace eptv {

enum ConvMode : int { kConv3 = 0, kPoint = 1, kUp = 2, kUpBack = 3 };

// One implicit-GEMM convolution.  x / y are NHWC bf16 (uint16 bit patterns)
// with channel stride *_cs and channel offset *_co (a slice of a wider
// tensor); y32, if set, receives fp32 output instead of y.  h, w: the GEMM's
// pixel grid (the input grid; kUp writes 2h x 2w, kUpBack reads 2h x 2w).
struct ConvArgs {
    const uint16_t* x = nullptr;
    int x_cs = 0, x_co = 0;
    uint16_t* y = nullptr;
    float* y32 = nullptr;
    int y_cs = 0, y_co = 0;
    const uint16_t* wt = nullptr;  // packed [q][n_pad][k_pad]
    const float* bias = nullptr;   // [cout] or null
    int n_img = 0, h = 0, w = 0;
    int cin = 0;   // GEMM input channels (per parity for kUpBack)
    int cout = 0;  // GEMM output channels
    int n_pad = 0, k_pad = 0;
    int relu = 0;
    // mask, if set: zero every output whose element of this tensor (same
    // pixel, channel n at m_co + n, stride m_cs) is not positive -- the
    // backward of a ReLU whose output it is, fused into the epilogue
    const uint16_t* mask = nullptr;
    int m_cs = 0, m_co = 0;
    // pool, if set (3x3 layers, even h and w): also write the 2x2 average
    // pooling of the (bf16) output, [n_img][h/2][w/2] with channel stride p_cs
    uint16_t* pool = nullptr;
    int p_cs = 0;
    // x32, if set: the input as dense fp32 (channel stride cin); it is rounded
    // to bf16, the values also written to x (dense, the layer's stored input)
    const float* x32 = nullptr;
    // head_y32, if set (3x3 layers that conv3_head_fits): also the 1x1
    // convolution of the layer's bf16 output with head_wt (packed
    // [head_n][head_kpad]) plus head_bias, written to head_y32 as dense fp32
    // [pixel][head_n] (head_n <= 4), summed in the thin pointwise kernel's order
    const uint16_t* head_wt = nullptr;
    const float* head_bias = nullptr;
    float* head_y32 = nullptr;
    int head_n = 0, head_kpad = 0;
};

inline int pad64(int n) { return (n + 63) / 64 * 64; }

hipError_t launch_conv(const ConvArgs& a, int mode, hipStream_t s);
// whether a 3x3 layer's launch can also form a thin 1x1 head of head_n
// outputs from its output (one block holds every channel of its pixels)
bool conv3_head_fits(const ConvArgs& a, int head_n);
int wgrad_chunks(const ConvArgs& a, int chunk_px);
// pixels per weight-gradient chunk for a layer with npix GEMM pixels and an
// n_pad x kw partial tile grid (also sizes the partial buffers)
int wgrad_chunk_px(int npix, int n_pad, int kw);
int wgrad_max_chunks(int npix, int n_pad, int kw);
// chunks of the LDS-tiled weight-gradient kernels (0 where none applies): an
// upper bound for every batch up to n_img
int wgrad_tiled_max_chunks(int mode, int n_img, int h, int w, int ci, int co);
// dW into out (the parameter layout: [3][3][C_in][C_out], [C_in][C_out] or
// [2][2][C_in][C_out]) and, if bias_out is given, the bias gradient
// sum_p dY[p][n] into bias_out[cout]; part and bpart are partial-sum scratch
hipError_t launch_wgrad(const ConvArgs& a, int mode, const uint16_t* dy, int dy_cs, int dy_co, int chunk_px,
                        float* part, float* out, float* bpart, float* bias_out, hipStream_t s);

hipError_t launch_avgpool(const uint16_t* x, int xcs, int xco, uint16_t* y, int n_img, int h, int w, int c,
                          hipStream_t s);
// dx (+)= the adjoint of 2x2 average pooling of dy; with mask (same layout
// as dx), elements whose mask value is not positive are set to zero
hipError_t launch_avgpool_back(const uint16_t* dy, uint16_t* dx, int dxcs, int dxco, int n_img, int h, int w, int c,
                               int accumulate, const uint16_t* mask, int mcs, int mco, hipStream_t s);
hipError_t launch_to_bf16(const float* x, uint16_t* y, size_t n, hipStream_t s);
hipError_t launch_eptv_to_maps(const float* f, const float* f_base, const float* wx, const float* wy, int n_img,
                               int ny, int nx, float scale, float* y, hipStream_t s);
hipError_t launch_maps_to_eptv(const float* y, const float* f_base, int n_img, int ny, int nx, float scale, float* f,
                               float* wx, float* wy, hipStream_t s);
hipError_t launch_to_f32(const uint16_t* x, float* y, size_t n, hipStream_t s);
// fp32 master weights (parameter layout) -> packed bf16 GEMM operands
//   conv3 forward: W[a][c][i][o] -> P[o][(3a+c) Ci + i]
//   conv3 backward data: P[i][(8 - tap) Co + o] (flipped taps, in/out swapped)
//   1x1: W[i][o] -> P[o][i];  backward data: P[i][o]
//   up (2x2, stride 2) forward: W[a][c][i][o] -> P[q = 2a + c][o][i]
//   up backward data: P[i][q Co + o]
struct PackDesc {
    const float* w;
    uint16_t* out;
    int mode, back, ci, co, n_pad, k_pad;
};
// every entry of a device-resident table, one launch
hipError_t launch_pack(const PackDesc* tab, int entries, hipStream_t s);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, size_t n, float lr, float b1, float b2, float eps,
                       int step, hipStream_t s);
hipError_t launch_mse(const float* y, const float* t, size_t n, float* dy, double* part, int nblocks, float* loss,
                      hipStream_t s);

}  // namespace eptv
