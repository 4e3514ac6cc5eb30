// unet.cpp -- the U-Net that proposes EPTV edge weights and a warm start:
// layer graph, buffers, forward and backward passes, Adam, and the
// eptv_unet_* C ABI.  Every layer runs on the kernels of cnn.hip.
//
// Architecture (levels L, base channels C): encoder level l has two 3x3
// convolutions with C 2^l channels and ReLU, levels joined by 2x2 average
// pooling; the decoder goes back up with a stride-2 2x2 transposed
// convolution (ReLU), concatenates the encoder's output of that level (the
// skip), and applies two 3x3 convolutions with ReLU; a 1x1 convolution gives
// the output channels.  Parameters are ordered and laid out as in the FP64
// reference (per layer: weights [3][3][C_in][C_out], [2][2][C_in][C_out] or
// [C_in][C_out], then the bias).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "cnn.h"
#include "host_internal.h"

namespace eptv {

struct Layer {
    int mode = kConv3;
    int ci = 0, co = 0;
    int lev = 0;                             // level of the GEMM's pixel grid
    size_t w_off = 0, b_off = 0, w_len = 0;  // into the flat parameter arrays
    int n_pad = 0, k_pad = 0;                // forward GEMM
    int nb_pad = 0, kb_pad = 0;              // backward-data GEMM
    uint16_t* wf = nullptr;                  // packed forward weights
    uint16_t* wb = nullptr;                  // packed backward-data weights
};

struct Tensor {
    uint16_t* p = nullptr;
    int c = 0;  // channels (stride)
};

}  // namespace eptv

struct eptv_unet_s {
    int c_in = 0, c_out = 0, base = 0, levels = 0, max_batch = 0, h = 0, w = 0;
    int n = 0;  // batch of the last forward
    std::vector<eptv::Layer> layers;
    size_t n_params = 0;
    float *params = nullptr, *grads = nullptr, *adam_m = nullptr, *adam_v = nullptr;
    // activations per level
    eptv::Tensor xin;                                 // input, bf16
    std::vector<eptv::Tensor> in, a, cat, da, db;     // level inputs, e?a outputs, [skip | up], decoder outputs
    eptv::Tensor bout;                                // bottleneck output
    // gradients
    eptv::Tensor g_head;                              // dY of the head, bf16
    std::vector<eptv::Tensor> g_in, g_a, g_cat, g_da, g_db;
    eptv::Tensor g_bout;
    float* part = nullptr;                            // weight-gradient partials
    size_t part_floats = 0;
    float* bpart = nullptr;                           // bias-gradient partials
    double* mse_part = nullptr;
    eptv::PackDesc* pack_tab = nullptr;               // device: forward and backward packing of every layer
    int pack_n = 0;
    std::vector<void*> allocs;
};

namespace eptv {

static constexpr int kMseBlocks = 1024;

static int layer_index(const eptv_unet_s& u, const char kind, int level, char sub)
{
    // order: e0a e0b e1a e1b ... e(L-1)b, then u(L-2) d(L-2)a d(L-2)b ... u0 d0a d0b, head
    const int L = u.levels;
    if (kind == 'e') return 2 * level + (sub == 'b');
    if (kind == 'h') return 2 * L + 3 * (L - 1);
    const int pos = (L - 2 - level) * 3;  // decoder position
    return 2 * L + pos + (kind == 'u' ? 0 : (sub == 'a' ? 1 : 2));
}

static ConvArgs conv_args(const eptv_unet_s& u, const Layer& L, int n, int h, int w, bool back)
{
    ConvArgs a;
    a.n_img = n;
    a.h = h;
    a.w = w;
    a.cin = back ? (L.mode == kUp ? L.co : L.co) : L.ci;
    a.cout = back ? L.ci : L.co;
    a.n_pad = back ? L.nb_pad : L.n_pad;
    a.k_pad = back ? L.kb_pad : L.k_pad;
    a.wt = back ? L.wb : L.wf;
    a.bias = back ? nullptr : u.params + L.b_off;
    return a;
}

static hipError_t repack(eptv_unet_s& u, hipStream_t s) { return launch_pack(u.pack_tab, u.pack_n, s); }

static hipError_t forward(eptv_unet_s& u, const float* x, int n, float* y, hipStream_t s)
{
    hipError_t e;
    const int L = u.levels;
    // the head (1x1, c_out outputs in fp32) is formed by the last decoder
    // layer's epilogue where its launch allows (one block holds all of a
    // pixel's channels), else by a launch of its own
    const int hl = layer_index(u, 'h', 0, 0);
    bool head_fused = false;
    auto conv = [&](int li, int mode, const uint16_t* xp, int xcs, int xco, int h, int w, uint16_t* yp, int ycs,
                    int yco, float* y32, int relu, const Tensor* pool = nullptr, const float* x32 = nullptr,
                    bool try_head = false) {
        const Layer& Ly = u.layers[li];
        ConvArgs a = conv_args(u, Ly, n, h, w, false);
        a.x = xp;
        a.x_cs = xcs;
        a.x_co = xco;
        a.y = yp;
        a.y32 = y32;
        a.y_cs = ycs;
        a.y_co = yco;
        a.relu = relu;
        if (pool) {
            a.pool = pool->p;
            a.p_cs = pool->c;
        }
        a.x32 = x32;
        if (try_head && conv3_head_fits(a, u.c_out)) {
            const ConvArgs hd = conv_args(u, u.layers[hl], n, h, w, false);
            a.head_wt = hd.wt;
            a.head_bias = hd.bias;
            a.head_kpad = hd.k_pad;
            a.head_n = u.c_out;
            a.head_y32 = y;
            head_fused = true;
        }
        return launch_conv(a, mode, s);
    };
    for (int l = 0; l < L; ++l) {
        const int h = u.h >> l, w = u.w >> l, C = u.base << l;
        const Tensor& inp = l == 0 ? u.xin : u.in[l];
        // the first layer reads the fp32 input and stores its bf16 rounding
        // (xin, kept for the backward pass) on the way
        if ((e = conv(layer_index(u, 'e', l, 'a'), kConv3, inp.p, inp.c, 0, h, w, u.a[l].p, C, 0, nullptr, 1, nullptr,
                      l == 0 ? x : nullptr)) != hipSuccess)
            return e;
        // the level output (the skip half of the concatenation, or the
        // bottleneck), and below the bottom level its 2x2 average pooling, the
        // next level's input, from the same epilogue
        const Tensor& out = l < L - 1 ? u.cat[l] : u.bout;
        if ((e = conv(layer_index(u, 'e', l, 'b'), kConv3, u.a[l].p, C, 0, h, w, out.p, out.c, 0, nullptr, 1,
                      l < L - 1 ? &u.in[l + 1] : nullptr)) != hipSuccess)
            return e;
    }
    for (int l = L - 2; l >= 0; --l) {
        const int h = u.h >> l, w = u.w >> l, C = u.base << l;
        const Tensor& up_in = l == L - 2 ? u.bout : u.db[l + 1];
        // transposed conv from level l+1 into the upper half of the concatenation
        if ((e = conv(layer_index(u, 'u', l, 0), kUp, up_in.p, up_in.c, 0, h / 2, w / 2, u.cat[l].p, 2 * C, C,
                      nullptr, 1)) != hipSuccess)
            return e;
        if ((e = conv(layer_index(u, 'd', l, 'a'), kConv3, u.cat[l].p, 2 * C, 0, h, w, u.da[l].p, C, 0, nullptr, 1)) !=
            hipSuccess)
            return e;
        if ((e = conv(layer_index(u, 'd', l, 'b'), kConv3, u.da[l].p, C, 0, h, w, u.db[l].p, C, 0, nullptr, 1,
                      nullptr, nullptr, l == 0)) != hipSuccess)
            return e;
    }
    if (head_fused) return hipSuccess;
    const Tensor& last = L > 1 ? u.db[0] : u.bout;
    return conv(hl, kPoint, last.p, last.c, 0, u.h, u.w, nullptr, u.c_out, 0, y, 0);
}

// weight and bias gradients of layer li from its input x (slice) and its
// output gradient dy (slice, already masked by the ReLU)
static hipError_t layer_grads(eptv_unet_s& u, int li, int n, int h, int w, const uint16_t* xp, int xcs, int xco,
                              const uint16_t* dy, int dycs, int dyco, hipStream_t s)
{
    Layer& Ly = u.layers[li];
    ConvArgs a = conv_args(u, Ly, n, h, w, false);
    a.x = xp;
    a.x_cs = xcs;
    a.x_co = xco;
    const int cpx = wgrad_chunk_px(n * h * w, Ly.n_pad, (Ly.mode == kUp ? 4 : 1) * Ly.k_pad);
    return launch_wgrad(a, Ly.mode, dy, dycs, dyco, cpx, u.part, u.grads + Ly.w_off, u.bpart, u.grads + Ly.b_off, s);
}

// backward data of layer li: gradient of its input from its output gradient;
// with mask (the input, where it is a ReLU's output), the ReLU's backward is
// applied in the same epilogue
static hipError_t layer_back(eptv_unet_s& u, int li, int n, int h, int w, const uint16_t* dy, int dycs, int dyco,
                             uint16_t* dx, int dxcs, int dxco, const Tensor* mask, hipStream_t s)
{
    const Layer& Ly = u.layers[li];
    ConvArgs a = conv_args(u, Ly, n, h, w, true);
    a.x = dy;
    a.x_cs = dycs;
    a.x_co = dyco;
    a.y = dx;
    a.y_cs = dxcs;
    a.y_co = dxco;
    if (mask) {
        a.mask = mask->p;
        a.m_cs = mask->c;
        a.m_co = dxco;
    }
    return launch_conv(a, Ly.mode == kUp ? kUpBack : Ly.mode, s);
}

// Every gradient that flows into a ReLU's output is masked where it is
// produced: by the backward-data epilogue of the layer that consumed the
// ReLU's output, or (the encoder outputs, which also feed the pooling) by the
// pooling adjoint that adds the second contribution.  Masking is a product
// with 0 / 1, so masking each contribution equals masking their sum.
static hipError_t backward(eptv_unet_s& u, const float* dy, float* dx, hipStream_t s)
{
    hipError_t e;
    const int L = u.levels, n = u.n;
    // head
    const int hl = layer_index(u, 'h', 0, 0);
    const Tensor& last = L > 1 ? u.db[0] : u.bout;
    if ((e = launch_to_bf16(dy, u.g_head.p, (size_t)n * u.h * u.w * u.c_out, s)) != hipSuccess) return e;
    if ((e = layer_grads(u, hl, n, u.h, u.w, last.p, last.c, 0, u.g_head.p, u.c_out, 0, s)) != hipSuccess)
        return e;
    Tensor g_last = L > 1 ? u.g_db[0] : u.g_bout;
    if ((e = layer_back(u, hl, n, u.h, u.w, u.g_head.p, u.c_out, 0, g_last.p, g_last.c, 0, &last, s)) != hipSuccess)
        return e;
    // decoder, from the top level down the U
    for (int l = 0; l <= L - 2; ++l) {
        const int h = u.h >> l, w = u.w >> l, C = u.base << l;
        const int lb = layer_index(u, 'd', l, 'b'), la = layer_index(u, 'd', l, 'a'), lu = layer_index(u, 'u', l, 0);
        if ((e = layer_grads(u, lb, n, h, w, u.da[l].p, C, 0, u.g_db[l].p, C, 0, s)) != hipSuccess) return e;
        if ((e = layer_back(u, lb, n, h, w, u.g_db[l].p, C, 0, u.g_da[l].p, C, 0, &u.da[l], s)) != hipSuccess)
            return e;
        if ((e = layer_grads(u, la, n, h, w, u.cat[l].p, 2 * C, 0, u.g_da[l].p, C, 0, s)) != hipSuccess)
            return e;
        // both halves of the concatenation are ReLU outputs (the skip: the
        // encoder's; the upper half: the transposed convolution's)
        if ((e = layer_back(u, la, n, h, w, u.g_da[l].p, C, 0, u.g_cat[l].p, 2 * C, 0, &u.cat[l], s)) != hipSuccess)
            return e;
        const Tensor& up_in = l == L - 2 ? u.bout : u.db[l + 1];
        Tensor& g_up_in = l == L - 2 ? u.g_bout : u.g_db[l + 1];
        if ((e = layer_grads(u, lu, n, h / 2, w / 2, up_in.p, up_in.c, 0, u.g_cat[l].p, 2 * C, C, s)) !=
            hipSuccess)
            return e;
        if ((e = layer_back(u, lu, n, h / 2, w / 2, u.g_cat[l].p, 2 * C, C, g_up_in.p, g_up_in.c, 0, &up_in, s)) !=
            hipSuccess)
            return e;
    }
    // encoder, from the bottleneck up
    for (int l = L - 1; l >= 0; --l) {
        const int h = u.h >> l, w = u.w >> l, C = u.base << l;
        const int lb = layer_index(u, 'e', l, 'b'), la = layer_index(u, 'e', l, 'a');
        // gradient of the level output: the skip half of the concatenation (or
        // the bottleneck's), plus the pooling path into level l+1
        Tensor gout = l < L - 1 ? u.g_cat[l] : u.g_bout;
        const Tensor& out = l < L - 1 ? u.cat[l] : u.bout;
        if (l < L - 1) {
            if ((e = launch_avgpool_back(u.g_in[l + 1].p, gout.p, gout.c, 0, n, h, w, C, 1, out.p, out.c, 0, s)) !=
                hipSuccess)
                return e;
        }
        if ((e = layer_grads(u, lb, n, h, w, u.a[l].p, C, 0, gout.p, gout.c, 0, s)) != hipSuccess) return e;
        if ((e = layer_back(u, lb, n, h, w, gout.p, gout.c, 0, u.g_a[l].p, C, 0, &u.a[l], s)) != hipSuccess)
            return e;
        const Tensor& inp = l == 0 ? u.xin : u.in[l];
        if ((e = layer_grads(u, la, n, h, w, inp.p, inp.c, 0, u.g_a[l].p, C, 0, s)) != hipSuccess) return e;
        if (l > 0) {
            if ((e = layer_back(u, la, n, h, w, u.g_a[l].p, C, 0, u.g_in[l].p, u.g_in[l].c, 0, nullptr, s)) !=
                hipSuccess)
                return e;
        } else if (dx) {
            // input gradient (bf16 through g_in[0]) to fp32: via the head-gradient buffer's width is not
            // enough in general, so g_in[0] holds it and the caller reads it converted below
            if ((e = layer_back(u, la, n, h, w, u.g_a[l].p, C, 0, u.g_in[0].p, u.g_in[0].c, 0, nullptr, s)) !=
                hipSuccess)
                return e;
        }
    }
    return hipSuccess;
}

}  // namespace eptv

using namespace eptv;

namespace {

template <class T>
hipError_t dalloc(eptv_unet_s& u, T** p, size_t count)
{
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T));
    if (e == hipSuccess) {
        u.allocs.push_back(q);
        e = hipMemset(q, 0, std::max<size_t>(count, 1) * sizeof(T));
    }
    *p = (T*)q;
    return e;
}

}  // namespace

extern "C" {

int eptv_unet_destroy(eptv_unet u)
{
    if (!u) return EPTV_ERR_ARG;
    for (void* p : u->allocs) hipFree(p);
    delete u;
    return EPTV_OK;
}

int eptv_unet_create(int c_in, int c_out, int base, int levels, int max_batch, int height, int width, eptv_unet* out)
{
    if (!out) return EPTV_ERR_ARG;
    *out = nullptr;
    if (c_in < 1 || c_in > 256 || c_out < 1 || c_out > 256 || base < 1 || base > 256 || levels < 1 || levels > 6 ||
        max_batch < 1 || height < 1 || width < 1)
        return EPTV_ERR_ARG;
    if (height % (1 << (levels - 1)) || width % (1 << (levels - 1))) return EPTV_ERR_ARG;
    if (levels > 1 && (base % 8)) return EPTV_ERR_ARG;  // channel slices must stay 16-byte aligned
    eptv_unet u = new (std::nothrow) eptv_unet_s();
    if (!u) return EPTV_ERR_ARG;
    u->c_in = c_in;
    u->c_out = c_out;
    u->base = base;
    u->levels = levels;
    u->max_batch = max_batch;
    u->h = height;
    u->w = width;
    const int L = levels;
    // layers in parameter order
    auto add = [&](int mode, int ci, int co, int lev) {
        Layer Ly;
        Ly.mode = mode;
        Ly.lev = lev;
        Ly.ci = ci;
        Ly.co = co;
        Ly.w_len = (size_t)(mode == kConv3 ? 9 : (mode == kUp ? 4 : 1)) * ci * co;
        Ly.w_off = u->n_params;
        Ly.b_off = Ly.w_off + Ly.w_len;
        u->n_params = Ly.b_off + co;
        Ly.n_pad = pad64(co);
        Ly.k_pad = pad64(mode == kConv3 ? 9 * ci : ci);
        Ly.nb_pad = pad64(ci);
        Ly.kb_pad = pad64(mode == kConv3 ? 9 * co : (mode == kUp ? 4 * co : co));
        u->layers.push_back(Ly);
    };
    int c = c_in;
    for (int l = 0; l < L; ++l) {
        add(kConv3, c, base << l, l);
        add(kConv3, base << l, base << l, l);
        c = base << l;
    }
    for (int l = L - 2; l >= 0; --l) {
        add(kUp, c, base << l, l + 1);  // its GEMM runs over the coarser input grid
        add(kConv3, 2 * (base << l), base << l, l);
        add(kConv3, base << l, base << l, l);
        c = base << l;
    }
    add(kPoint, c, c_out, 0);
    hipError_t e = hipSuccess;
    for (float** p : {&u->params, &u->grads, &u->adam_m, &u->adam_v})
        if (e == hipSuccess) e = dalloc(*u, p, u->n_params);
    size_t part = 0, bpart = 0;
    for (Layer& Ly : u->layers) {
        const int q = Ly.mode == kUp ? 4 : 1;
        if (e == hipSuccess) e = dalloc(*u, &Ly.wf, (size_t)q * Ly.n_pad * Ly.k_pad);
        if (e == hipSuccess) e = dalloc(*u, &Ly.wb, (size_t)Ly.nb_pad * Ly.kb_pad);
    }
    // activations and gradients
    const size_t B = (size_t)max_batch;
    auto tensor = [&](Tensor& t, int ch, int lev) {
        t.c = ch;
        if (e == hipSuccess) e = dalloc(*u, &t.p, B * (height >> lev) * (width >> lev) * ch);
    };
    tensor(u->xin, c_in, 0);
    u->in.resize(L);
    u->a.resize(L);
    u->cat.resize(L);
    u->da.resize(L);
    u->db.resize(L);
    u->g_in.resize(L);
    u->g_a.resize(L);
    u->g_cat.resize(L);
    u->g_da.resize(L);
    u->g_db.resize(L);
    for (int l = 0; l < L; ++l) {
        const int C = base << l;
        if (l > 0) tensor(u->in[l], base << (l - 1), l);
        if (l > 0) tensor(u->g_in[l], base << (l - 1), l);
        tensor(u->a[l], C, l);
        tensor(u->g_a[l], C, l);
        if (l < L - 1) {
            tensor(u->cat[l], 2 * C, l);
            tensor(u->g_cat[l], 2 * C, l);
            tensor(u->da[l], C, l);
            tensor(u->db[l], C, l);
            tensor(u->g_da[l], C, l);
            tensor(u->g_db[l], C, l);
        }
    }
    tensor(u->g_in[0], c_in, 0);
    tensor(u->bout, base << (L - 1), L - 1);
    tensor(u->g_bout, base << (L - 1), L - 1);
    tensor(u->g_head, c_out, 0);
    // weight-gradient partials: the largest layer
    for (const Layer& Ly : u->layers) {
        const size_t npix = B * (height >> Ly.lev) * (width >> Ly.lev);
        size_t chunks = wgrad_max_chunks((int)npix, Ly.n_pad, (Ly.mode == kUp ? 4 : 1) * Ly.k_pad);
        chunks = std::max(chunks, (size_t)wgrad_tiled_max_chunks(Ly.mode, (int)B, height >> Ly.lev, width >> Ly.lev,
                                                                 Ly.ci, Ly.co));
        part = std::max(part, chunks * Ly.n_pad * (Ly.mode == kUp ? 4 : 1) * Ly.k_pad);
        bpart = std::max(bpart, chunks * (Ly.mode == kUp ? 4 : 1) * Ly.n_pad);  // one row per chunk and parity
    }
    u->part_floats = part;
    if (e == hipSuccess) e = dalloc(*u, &u->part, part);
    if (e == hipSuccess) e = dalloc(*u, &u->bpart, bpart);
    if (e == hipSuccess) e = dalloc(*u, &u->mse_part, (size_t)kMseBlocks);
    // the packing table (fixed pointers from here on)
    std::vector<PackDesc> tab;
    for (const Layer& Ly : u->layers) {
        tab.push_back({u->params + Ly.w_off, Ly.wf, Ly.mode, 0, Ly.ci, Ly.co, Ly.n_pad, Ly.k_pad});
        tab.push_back({u->params + Ly.w_off, Ly.wb, Ly.mode, 1, Ly.ci, Ly.co, Ly.nb_pad, Ly.kb_pad});
    }
    u->pack_n = (int)tab.size();
    if (e == hipSuccess) e = dalloc(*u, &u->pack_tab, tab.size());
    if (e == hipSuccess) e = hipMemcpy(u->pack_tab, tab.data(), tab.size() * sizeof(PackDesc), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        const int rc = hip_fail(e, "eptv_unet_create");
        eptv_unet_destroy(u);
        return rc;
    }
    *out = u;
    return EPTV_OK;
}

int eptv_unet_param_count(eptv_unet u, long long* n)
{
    if (!u || !n) return EPTV_ERR_ARG;
    *n = (long long)u->n_params;
    return EPTV_OK;
}

int eptv_unet_set_params(eptv_unet u, const float* params, void* stream)
{
    if (!u || !params) return EPTV_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    EPTV_HIP(hipMemcpyAsync(u->params, params, u->n_params * 4, hipMemcpyHostToDevice, s));
    EPTV_HIP(hipMemsetAsync(u->adam_m, 0, u->n_params * 4, s));
    EPTV_HIP(hipMemsetAsync(u->adam_v, 0, u->n_params * 4, s));
    EPTV_HIP(repack(*u, s));
    EPTV_HIP(hipStreamSynchronize(s));
    return EPTV_OK;
}

int eptv_unet_get_params(eptv_unet u, float* params, void* stream)
{
    if (!u || !params) return EPTV_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    EPTV_HIP(hipMemcpyAsync(params, u->params, u->n_params * 4, hipMemcpyDeviceToHost, s));
    EPTV_HIP(hipStreamSynchronize(s));
    return EPTV_OK;
}

int eptv_unet_get_grads(eptv_unet u, float* grads, void* stream)
{
    if (!u || !grads) return EPTV_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    EPTV_HIP(hipMemcpyAsync(grads, u->grads, u->n_params * 4, hipMemcpyDeviceToHost, s));
    EPTV_HIP(hipStreamSynchronize(s));
    return EPTV_OK;
}

int eptv_unet_forward(eptv_unet u, const float* x, int n, float* y, void* stream)
{
    if (!u || !x || !y || n < 1 || n > u->max_batch) return EPTV_ERR_ARG;
    u->n = n;
    EPTV_HIP(forward(*u, x, n, y, (hipStream_t)stream));
    return EPTV_OK;
}

int eptv_unet_backward(eptv_unet u, const float* dy, float* dx, void* stream)
{
    if (!u || !dy || u->n < 1) return EPTV_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    EPTV_HIP(backward(*u, dy, dx, s));
    if (dx) {
        const size_t n = (size_t)u->n * u->h * u->w * u->c_in;
        EPTV_HIP(launch_to_f32(u->g_in[0].p, dx, n, s));
    }
    return EPTV_OK;
}

int eptv_unet_adam(eptv_unet u, float lr, float beta1, float beta2, float eps, int step, void* stream)
{
    if (!u || step < 1 || !(lr >= 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
        return EPTV_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    EPTV_HIP(launch_adam(u->params, u->grads, u->adam_m, u->adam_v, u->n_params, lr, beta1, beta2, eps, step, s));
    EPTV_HIP(repack(*u, s));
    return EPTV_OK;
}

int eptv_unet_mse(eptv_unet u, const float* y, const float* target, size_t n, float* dy, float* loss, void* stream)
{
    if (!u || !y || !target || !loss || n == 0) return EPTV_ERR_ARG;
    EPTV_HIP(launch_mse(y, target, n, dy, u->mse_part, kMseBlocks, loss, (hipStream_t)stream));
    return EPTV_OK;
}

int eptv_maps_from_eptv(int n_img, int ny, int nx, const float* f, const float* f_base, const float* wx,
                        const float* wy, float scale, float* maps, void* stream)
{
    if (n_img < 1 || ny < 1 || nx < 1 || !f || !maps || (!wx) != (!wy) || !(scale > 0) || !std::isfinite(scale))
        return EPTV_ERR_ARG;
    EPTV_HIP(launch_eptv_to_maps(f, f_base, wx, wy, n_img, ny, nx, scale, maps, (hipStream_t)stream));
    return EPTV_OK;
}

int eptv_maps_to_eptv(int n_img, int ny, int nx, const float* maps, float scale, const float* f_base, float* f,
                      float* wx, float* wy, void* stream)
{
    if (n_img < 1 || ny < 1 || nx < 1 || !maps || !f || !wx || !wy || !(scale > 0) || !std::isfinite(scale))
        return EPTV_ERR_ARG;
    EPTV_HIP(launch_maps_to_eptv(maps, f_base, n_img, ny, nx, scale, f, wx, wy, (hipStream_t)stream));
    return EPTV_OK;
}

}  // extern "C"
