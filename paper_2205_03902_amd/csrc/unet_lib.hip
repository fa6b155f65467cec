// libimsp host side of the learned-initialisation network: layer table, workspace
// layout, forward / backward / Adam sequences behind the C ABI of include/unet.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <new>
#include <string>
#include <vector>

#include "unet.h"
#include "unet_kernels.hpp"

using namespace unet;

namespace {

thread_local std::string u_err;

un_status ufail(un_status st, const std::string &msg)
{
    u_err = msg;
    return st;
}

constexpr size_t kAlign = 256;
constexpr int kWgradTarget = 2048;   // workgroups a weight-gradient launch aims for
constexpr int kMaxSplits = 256;      // pixel splits of one weight gradient
constexpr size_t kMaxPartialFloats = (size_t)8 << 20;   // FP32 partials of one weight gradient (32 MiB)
constexpr int kMaxColSplits = 512;   // pixel splits of one bias gradient

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
bool pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }
int ilog2(int x)
{
    int l = 0;
    while ((1 << l) < x) ++l;
    return l;
}
int r8(int x) { return (x + 7) / 8 * 8; }
int r32(int x) { return (x + 31) / 32 * 32; }
long long cdiv(long long a, long long b) { return (a + b - 1) / b; }

struct Layer {
    un_layer info;
    int G;             // output-gradient channels the data gradient gathers (cout rounded to 8)
    int d_rows, d_k;   // data-gradient weight matrix: input channels x r32(taps G)
    size_t wb, wd;     // offsets (elements) of the bf16 forward / data-gradient copies
    int splits;        // weight-gradient pixel splits at max_batch
};

struct Layout {
    size_t params, grads, adam_m, adam_v, wbf, wdf, gout, gx, gy, stats, mse_part, wpart, bpart, total;
    std::vector<size_t> enc_a0, enc_a1, pool, dec_up, dec_a0, dec_a1, dskip;
};

}  // namespace

struct un_net {
    un_config cfg{};
    int L = 0, in_pad = 0, hl = 0, wl = 0;
    std::vector<Layer> layers;
    int64_t n_params = 0;
    size_t wbf_count = 0, wdf_count = 0, wpart_count = 0;
    Layout lay{};
    char *ws = nullptr;
    int step = 0;
    int last_batch = 0;

    template <class T>
    T *at(size_t off) const { return reinterpret_cast<T *>(ws + off); }
    int width(int l) const { return cfg.base << l; }
    long long pixels(int batch, int l) const { return (long long)batch << (hl + wl - 2 * l); }
    int enc(int l, int j) const { return 2 * l + j; }
    int dec(int l, int j) const { return 2 * L + 3 * (L - 2 - l) + j; }
    int head() const { return 2 * L + 3 * (L - 1); }
};

namespace {

un_status check_config(const un_config *c)
{
    if (!c) return ufail(UN_ERR_INVALID_ARG, "config is NULL");
    if (c->in_ch < 1 || c->in_ch > 16 || c->out_ch < 1 || c->out_ch > 16)
        return ufail(UN_ERR_INVALID_ARG, "in_ch and out_ch must be in [1, 16]");
    if (c->levels < 1 || c->levels > 5) return ufail(UN_ERR_INVALID_ARG, "levels must be in [1, 5]");
    if (c->base < 8 || c->base % 8 || (c->base << (c->levels - 1)) > 256)
        return ufail(UN_ERR_INVALID_ARG, "base must be a multiple of 8 with base << (levels - 1) <= 256");
    if (!pow2(c->height) || !pow2(c->width) || c->height < 8 || c->width < 8 || c->height > 4096 || c->width > 4096)
        return ufail(UN_ERR_INVALID_ARG, "height and width must be powers of two in [8, 4096]");
    if ((c->height >> (c->levels - 1)) < 1 || (c->width >> (c->levels - 1)) < 1)
        return ufail(UN_ERR_INVALID_ARG, "height and width must be divisible by 2^(levels - 1)");
    if (c->max_batch < 1) return ufail(UN_ERR_INVALID_ARG, "max_batch must be >= 1");
    const long long px = (long long)c->max_batch * c->height * c->width;
    if (px * c->base > ((long long)1 << 31) - 1)
        return ufail(UN_ERR_INVALID_ARG, "max_batch x height x width x base must stay below 2^31");
    return UN_OK;
}

int wgrad_tiles(const un_layer &li)
{
    const int bm = li.n_rows <= 32 ? 32 : li.n_rows <= 64 && li.kpad >= 128 ? 64 : 128;
    const int bn = (li.n_rows <= 32 || li.kpad >= 128) ? 128 : 32;
    return (int)(cdiv(li.n_rows, bm) * cdiv(li.kpad, bn));
}

// Builds the layer table and workspace layout (host only).
void plan(un_net &n)
{
    const un_config &c = n.cfg;
    n.L = c.levels;
    n.in_pad = r8(c.in_ch);
    n.hl = ilog2(c.height);
    n.wl = ilog2(c.width);
    n.layers.clear();
    int64_t off = 0;
    auto add = [&](int kind, int cin, int cout) {
        Layer ly{};
        un_layer &li = ly.info;
        li.kind = kind;
        li.cin = cin;
        li.cout = cout;
        li.taps = kind == UN_CONV3X3 ? 9 : kind == UN_UPCONV2X2 ? 4 : 1;
        li.n_rows = kind == UN_UPCONV2X2 ? 4 * cout : cout;
        li.kpad = kind == UN_UPCONV2X2 ? r32(cin) : r32(li.taps * cin);
        li.w_offset = off;
        off += (int64_t)li.n_rows * li.kpad;
        li.b_offset = off;
        off += cout;
        off = (off + 63) / 64 * 64;
        ly.G = r8(cout);
        ly.d_rows = cin;
        ly.d_k = r32(li.taps * ly.G);
        n.layers.push_back(ly);
    };
    int cin = n.in_pad;
    for (int l = 0; l < n.L; ++l) {
        add(UN_CONV3X3, cin, n.width(l));
        add(UN_CONV3X3, n.width(l), n.width(l));
        cin = n.width(l);
    }
    for (int l = n.L - 2; l >= 0; --l) {
        add(UN_UPCONV2X2, n.width(l + 1), n.width(l));
        add(UN_CONV3X3, 2 * n.width(l), n.width(l));
        add(UN_CONV3X3, n.width(l), n.width(l));
    }
    add(UN_CONV1X1, c.base, c.out_ch);
    n.n_params = off;

    size_t wb = 0, wd = 0, wp = 0;
    for (Layer &ly : n.layers) {
        ly.wb = wb;
        wb += (size_t)ly.info.n_rows * ly.info.kpad;
        wb = (wb + 127) / 128 * 128;
        ly.wd = wd;
        wd += (size_t)ly.d_rows * ly.d_k;
        wd = (wd + 127) / 128 * 128;
        const long long per_split = (long long)ly.info.n_rows * ly.info.kpad;
        ly.splits = (int)std::min<long long>({(long long)kMaxSplits, cdiv(kWgradTarget, wgrad_tiles(ly.info)),
                                              std::max<long long>(1, (long long)kMaxPartialFloats / per_split)});
        ly.splits = std::max(ly.splits, 1);
        wp = std::max(wp, (size_t)ly.splits * ly.info.n_rows * ly.info.kpad);
    }
    n.wbf_count = wb;
    n.wdf_count = wd;
    n.wpart_count = wp;

    Layout &y = n.lay;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t r = o;
        o = align_up(o + bytes);
        return r;
    };
    const size_t np = (size_t)n.n_params * sizeof(float);
    y.params = take(np);
    y.grads = take(np);
    y.adam_m = take(np);
    y.adam_v = take(np);
    y.wbf = take(wb * 2);
    y.wdf = take(wd * 2);
    const int B = c.max_batch;
    y.enc_a0.assign(n.L, 0);
    y.enc_a1.assign(n.L, 0);
    y.pool.assign(n.L, 0);
    y.dec_up.assign(n.L, 0);
    y.dec_a0.assign(n.L, 0);
    y.dec_a1.assign(n.L, 0);
    y.dskip.assign(n.L, 0);
    for (int l = 0; l < n.L; ++l) {
        const size_t img = (size_t)n.pixels(B, l) * n.width(l) * 2;
        y.enc_a0[l] = take(img);
        y.enc_a1[l] = take(img);
        if (l < n.L - 1) {
            y.pool[l] = take((size_t)n.pixels(B, l + 1) * n.width(l) * 2);
            y.dec_up[l] = take(img);
            y.dec_a0[l] = take(img);
            y.dec_a1[l] = take(img);
            y.dskip[l] = take(img);
        }
    }
    const size_t gmax = (size_t)n.pixels(B, 0) * c.base * 2;
    y.gout = take((size_t)n.pixels(B, 0) * r8(c.out_ch) * 2);
    y.gx = take(gmax);
    y.gy = take(gmax);
    y.stats = take((size_t)B * c.out_ch * 2 * sizeof(double));
    y.mse_part = take((size_t)B * c.out_ch * kMseChunks * 2 * sizeof(double));
    y.wpart = take(wp * sizeof(float));
    y.bpart = take((size_t)kMaxColSplits * 256 * sizeof(float));
    y.total = o;
}

bool launch_ok(const char *what)
{
    const hipError_t e = hipGetLastError();
    if (e == hipSuccess) return true;
    u_err = std::string(what) + ": " + hipGetErrorString(e);
    return false;
}

void gemm(const GemmArgs &a, hipStream_t st)
{
    const long long M = a.r.m_total;
    const int N = a.o.n_total;
    const long long g128 = cdiv(M, 128) * cdiv(N, 128), g64 = cdiv(M, 128) * cdiv(N, 64);
    // K steps of 64 give each barrier twice the matrix-core work of 32 (the same products in the
    // same order) but hold 55-74 KB of LDS, two workgroups a CU: they pay where the grid fits in
    // one round of those (the 64^2 and 32^2 levels at batch 16: forward 0.855 -> 0.815 ms), not
    // where it takes several (the 128^2 GEMM: 0.815 -> 0.828 ms)
    const bool k64 = a.kpad % 64 == 0 && a.o.ostride == 1;
    const dim3 grid64((unsigned)cdiv(M, 128), (unsigned)cdiv(N, 64)), grid128((unsigned)cdiv(M, 128), (unsigned)cdiv(N, 128));
    if (N <= 32) {
        gemm_kernel<128, 32, 4, 1><<<dim3((unsigned)cdiv(M, 128), (unsigned)cdiv(N, 32)), kThreads, 0, st>>>(a);
    } else if (N <= 64) {
        gemm_kernel<128, 64, 2, 2><<<grid64, kThreads, 0, st>>>(a);
    } else if (k64 && g128 > 256 && g128 <= 512) {
        gemm_kernel<128, 128, 2, 2, 64><<<grid128, kThreads, 0, st>>>(a);
    } else if (k64 && g64 <= 512) {
        gemm_kernel<128, 64, 2, 2, 64><<<grid64, kThreads, 0, st>>>(a);
    } else if (g128 < 1024 || a.o.ostride > 1) {
        // the coarse levels: 128 x 64 tiles double the workgroups of a grid that would leave CUs
        // with one or two (the same sums: each output's K order does not depend on the tiling);
        // the transposed convolutions (K of 64 to 256, a few steps a tile) likewise: 1 % of the
        // forward at batch 16
        gemm_kernel<128, 64, 2, 2><<<grid64, kThreads, 0, st>>>(a);
    } else {
        gemm_kernel<128, 128, 2, 2><<<grid128, kThreads, 0, st>>>(a);
    }
}

void wgrad(const WgradArgs &a, int splits, hipStream_t st)
{
    const int R = a.n_rows, K = a.kpad;
    if (R <= 32) {
        wgrad_kernel<32, 128, 1, 4><<<dim3((unsigned)cdiv(K, 128), (unsigned)cdiv(R, 32), splits), kThreads, 0, st>>>(a);
    } else if (R <= 64 && K >= 128) {
        wgrad_kernel<64, 128, 2, 2><<<dim3((unsigned)cdiv(K, 128), (unsigned)cdiv(R, 64), splits), kThreads, 0, st>>>(a);
    } else if (K >= 128) {
        wgrad_kernel<128, 128, 2, 2><<<dim3((unsigned)cdiv(K, 128), (unsigned)cdiv(R, 128), splits), kThreads, 0, st>>>(a);
    } else {
        wgrad_kernel<128, 32, 4, 1><<<dim3((unsigned)cdiv(K, 32), (unsigned)cdiv(R, 128), splits), kThreads, 0, st>>>(a);
    }
}

Gather gather_of(const uint16_t *s0, int c0, const uint16_t *s1, int c1, int h_log, int w_log, int kind_taps,
                 int stride)
{
    Gather g{};
    g.src0 = s0;
    g.src1 = s1;
    g.c0 = c0;
    g.c1 = c1;
    g.hs_log = h_log;
    g.ws_log = w_log;
    g.stride = stride;
    g.taps = kind_taps;
    g.kw = kind_taps == 9 ? 3 : kind_taps == 4 ? 2 : 1;
    g.pad = kind_taps == 9 ? 1 : 0;
    return g;
}

RowGrid rows_of(int batch, int h_log, int w_log)
{
    RowGrid r{};
    r.ho_log = h_log;
    r.wo_log = w_log;
    r.m_total = (int)((long long)batch << (h_log + w_log));
    return r;
}

OutMap plain_map(int nout, int n_total, int h_log, int w_log)
{
    OutMap o{};
    o.nout = nout;
    o.n_total = n_total;
    o.ostride = 1;
    o.okw = 1;
    o.hd_log = h_log;
    o.wd_log = w_log;
    return o;
}

OutMap up_map(int cout, int h_log_in, int w_log_in)
{
    OutMap o{};
    o.nout = cout;
    o.n_total = 4 * cout;
    o.ostride = 2;
    o.okw = 2;
    o.hd_log = h_log_in + 1;
    o.wd_log = w_log_in + 1;
    return o;
}

// Whether a 3x3 convolution to `cout` channels from c0 (+ c1) input channels on a 2^hl x 2^wl
// image runs as the direct convolution (conv3x3_kernel, 32 output channels a launch). Four launches
// (128 channels) pay only from 128 x 128 up: at 64 x 64 each launch has too few workgroups to fill
// the chip and the implicit GEMM is faster.
bool direct_conv_fits(int cout, int c0, int c1, int hl, int wl)
{
    const int cin = c0 + c1;
    const bool wide = (cin == 32 || cin == 64) && c0 % 16 == 0 && c1 % 16 == 0;
    const bool narrow = cin == 8 && c1 == 0;   // the input layer: up to 8 channels, two taps a step
    return cout % 32 == 0 && (cout <= 64 || (cout <= 128 && hl >= 7)) && (wide || narrow) && hl >= 6 && wl >= 4;
}

// Output channels [0, d0c) go to out0 (d0c a pixel, masked by mask if given), the rest to out1
// (cout - d0c a pixel): the split of a concatenation's gradient.
void direct_conv(const uint16_t *in0, int c0, const uint16_t *in1, int c1, int hl, int wl, int batch, int cout,
                 const uint16_t *w, int kpad, const float *bias, int relu, const uint16_t *mask, uint16_t *out0,
                 int d0c, uint16_t *out1, hipStream_t st)
{
    for (int h = 0; h < cout / 32; ++h) {   // 32 output channels a launch
        const bool first = h * 32 < d0c;
        Conv3Args c{};
        c.src0 = in0; c.src1 = in1; c.c0 = c0; c.c1 = c1;
        c.h_log = hl; c.w_log = wl;
        c.w = w + (size_t)h * 32 * kpad; c.kpad = kpad;
        c.bias = bias ? bias + h * 32 : nullptr; c.relu = relu;
        c.mask = (mask && first) ? mask + h * 32 : nullptr;
        c.dst = first ? out0 + h * 32 : out1 + (h * 32 - d0c);
        c.ldd = first ? d0c : cout - d0c;
        if (c0 + c1 == 8) {    // 16-row tiles, four per workgroup
            const dim3 grid(1u << (wl - 4), 1u << (hl - 6), (unsigned)batch);
            conv3x3_kernel<16, 8, 4><<<grid, kThreads, 0, st>>>(c);
        } else if (c0 + c1 == 32) {   // 16-row tiles, four per workgroup
            const dim3 grid(1u << (wl - 4), 1u << (hl - 6), (unsigned)batch);
            conv3x3_kernel<16, 32, 4><<<grid, kThreads, 0, st>>>(c);
        } else {               // 8-row tiles, four per workgroup
            const dim3 grid(1u << (wl - 4), 1u << (hl - 5), (unsigned)batch);
            conv3x3_kernel<8, 64, 4><<<grid, kThreads, 0, st>>>(c);
        }
    }
}

// Forward of one layer.  in0 / in1: inputs (in1 the skip of a concatenation); level: image
// level of the input (for the transposed convolution, the coarser one).
void layer_forward(const un_net &n, int li, int batch, int level, const uint16_t *in0, int c0, const uint16_t *in1,
                   int c1, void *out, hipStream_t st)
{
    const Layer &ly = n.layers[li];
    const int hlg = n.hl - level, wlg = n.wl - level;
    GemmArgs a{};
    a.r = rows_of(batch, hlg, wlg);
    a.w = n.at<uint16_t>(n.lay.wbf) + ly.wb;
    a.kpad = ly.info.kpad;
    a.bias = n.at<float>(n.lay.params) + ly.info.b_offset;
    a.dst0 = out;
    a.d0c = ly.info.cout;
    if (ly.info.kind == UN_UPCONV2X2) {
        a.g = gather_of(in0, c0, nullptr, 0, hlg, wlg, 1, 1);
        a.o = up_map(ly.info.cout, hlg, wlg);
    } else {
        if (ly.info.kind == UN_CONV1X1 && !in1 && ly.info.cout <= kHeadMax && c0 > 0 && c0 % 8 == 0 && c0 <= kHeadC) {
            // the head: a per-pixel kernel (a GEMM of a few columns is all pipeline start-up)
            const long long px = n.pixels(batch, level);
            const unsigned blocks = (unsigned)((px + 255) / 256);
            float *y = static_cast<float *>(out);
            switch (c0 / 8) {
            case 1: head_kernel<1><<<blocks, 256, 0, st>>>(in0, a.w, a.kpad, a.bias, ly.info.cout, y, px); break;
            case 2: head_kernel<2><<<blocks, 256, 0, st>>>(in0, a.w, a.kpad, a.bias, ly.info.cout, y, px); break;
            case 3: head_kernel<3><<<blocks, 256, 0, st>>>(in0, a.w, a.kpad, a.bias, ly.info.cout, y, px); break;
            case 4: head_kernel<4><<<blocks, 256, 0, st>>>(in0, a.w, a.kpad, a.bias, ly.info.cout, y, px); break;
            case 5: head_kernel<5><<<blocks, 256, 0, st>>>(in0, a.w, a.kpad, a.bias, ly.info.cout, y, px); break;
            case 6: head_kernel<6><<<blocks, 256, 0, st>>>(in0, a.w, a.kpad, a.bias, ly.info.cout, y, px); break;
            case 7: head_kernel<7><<<blocks, 256, 0, st>>>(in0, a.w, a.kpad, a.bias, ly.info.cout, y, px); break;
            default: head_kernel<8><<<blocks, 256, 0, st>>>(in0, a.w, a.kpad, a.bias, ly.info.cout, y, px); break;
            }
            return;
        }
        if (ly.info.kind == UN_CONV3X3 && direct_conv_fits(ly.info.cout, c0, in1 ? c1 : 0, hlg, wlg)) {
            direct_conv(in0, c0, in1, in1 ? c1 : 0, hlg, wlg, batch, ly.info.cout, a.w, a.kpad, a.bias, 1, nullptr,
                        static_cast<uint16_t *>(out), ly.info.cout, nullptr, st);
            return;
        }
        a.g = gather_of(in0, c0, in1, c1, hlg, wlg, ly.info.taps, 1);
        a.o = plain_map(ly.info.cout, ly.info.cout, hlg, wlg);
        a.relu = ly.info.kind == UN_CONV3X3;
        a.out_f32 = ly.info.kind == UN_CONV1X1;
    }
    gemm(a, st);
}

// Weight and bias gradients of one layer from its output gradient gy (gyc channels per pixel).
void layer_weight_grad(un_net &n, int li, int batch, int level, const uint16_t *in0, int c0, const uint16_t *in1,
                       int c1, const uint16_t *gy, int gyc, hipStream_t st)
{
    const Layer &ly = n.layers[li];
    const int hlg = n.hl - level, wlg = n.wl - level;
    WgradArgs a{};
    a.r = rows_of(batch, hlg, wlg);
    a.gy = gy;
    a.gyc = gyc;
    a.n_rows = ly.info.n_rows;
    a.kpad = ly.info.kpad;
    long long out_pixels;
    if (ly.info.kind == UN_UPCONV2X2) {
        a.g = gather_of(in0, c0, nullptr, 0, hlg, wlg, 1, 1);
        a.o = up_map(ly.info.cout, hlg, wlg);
        out_pixels = n.pixels(batch, level - 1);
    } else {
        a.g = gather_of(in0, c0, in1, c1, hlg, wlg, ly.info.taps, 1);
        a.o = plain_map(gyc, gyc, hlg, wlg);
        out_pixels = n.pixels(batch, level);
    }
    const long long M = a.r.m_total;
    const long long chunk = std::max<long long>(64, r32((int)cdiv(M, ly.splits)));
    a.m_chunk = (int)chunk;
    const int splits = (int)cdiv(M, chunk);
    a.part = n.at<float>(n.lay.wpart);
    wgrad(a, splits, st);
    float *grads = n.at<float>(n.lay.grads);
    const long long wcount = (long long)a.n_rows * a.kpad;
    sum_splits_kernel<<<(unsigned)cdiv(cdiv(wcount, 4), 256), 256, 0, st>>>(a.part, splits, wcount,
                                                                           grads + ly.info.w_offset);

    const int cout = ly.info.cout;
    const long long cchunk = std::max<long long>(256, cdiv(out_pixels, kMaxColSplits));
    const int csplits = (int)cdiv(out_pixels, cchunk);
    float *bpart = n.at<float>(n.lay.bpart);
    colsum_partial_kernel<<<csplits, kThreads, 0, st>>>(gy, gyc, cout, out_pixels, (int)cchunk, bpart);
    sum_splits_kernel<<<(unsigned)cdiv(cout, 256), 256, 0, st>>>(bpart, csplits, cout, grads + ly.info.b_offset);
}

// Input gradient of one layer: gy (G channels at the layer's output level) -> dst0 [, dst1],
// optionally multiplied by (mask > 0).
void layer_data_grad(const un_net &n, int li, int batch, int level, const uint16_t *gy, void *dst0, int d0c,
                     void *dst1, int d1c, const uint16_t *mask, hipStream_t st)
{
    const Layer &ly = n.layers[li];
    const int hlg = n.hl - level, wlg = n.wl - level;   // input level of the layer
    GemmArgs a{};
    a.r = rows_of(batch, hlg, wlg);
    a.w = n.at<uint16_t>(n.lay.wdf) + ly.wd;
    a.kpad = ly.d_k;
    if (ly.info.kind == UN_UPCONV2X2) a.g = gather_of(gy, ly.G, nullptr, 0, hlg + 1, wlg + 1, 4, 2);
    else a.g = gather_of(gy, ly.G, nullptr, 0, hlg, wlg, ly.info.taps, 1);
    if (ly.info.kind == UN_CONV3X3 && d0c % 32 == 0 && d0c + (dst1 ? d1c : 0) == ly.d_rows &&
        direct_conv_fits(ly.d_rows, ly.G, 0, hlg, wlg)) {
        // the same convolution of the output gradient with the flipped weights, masked, the
        // channels of a concatenation split over its two sources
        direct_conv(gy, ly.G, nullptr, 0, hlg, wlg, batch, ly.d_rows, a.w, a.kpad, nullptr, 0, mask,
                    static_cast<uint16_t *>(dst0), d0c, static_cast<uint16_t *>(dst1), st);
        return;
    }
    a.o = plain_map(ly.d_rows, ly.d_rows, hlg, wlg);
    a.mask = mask;
    a.dst0 = dst0;
    a.d0c = d0c;
    a.dst1 = dst1;
    a.d1c = d1c;
    gemm(a, st);
}

void run_forward(un_net &n, int batch, const uint16_t *x, float *y, hipStream_t st)
{
    const Layout &L = n.lay;
    const uint16_t *h = x;
    int hc = n.in_pad;
    for (int l = 0; l < n.L; ++l) {
        uint16_t *a0 = n.at<uint16_t>(L.enc_a0[l]), *a1 = n.at<uint16_t>(L.enc_a1[l]);
        layer_forward(n, n.enc(l, 0), batch, l, h, hc, nullptr, 0, a0, st);
        layer_forward(n, n.enc(l, 1), batch, l, a0, n.width(l), nullptr, 0, a1, st);
        if (l < n.L - 1) {
            uint16_t *p = n.at<uint16_t>(L.pool[l]);
            const long long cnt = n.pixels(batch, l + 1) * (n.width(l) / 8);
            maxpool_kernel<<<(unsigned)cdiv(cnt, 256), 256, 0, st>>>(a1, n.width(l), n.hl - l, n.wl - l, cnt, p);
            h = p;
            hc = n.width(l);
        } else {
            h = a1;
            hc = n.width(l);
        }
    }
    for (int l = n.L - 2; l >= 0; --l) {
        uint16_t *up = n.at<uint16_t>(L.dec_up[l]), *a0 = n.at<uint16_t>(L.dec_a0[l]);
        uint16_t *a1 = n.at<uint16_t>(L.dec_a1[l]);
        layer_forward(n, n.dec(l, 0), batch, l + 1, h, hc, nullptr, 0, up, st);
        layer_forward(n, n.dec(l, 1), batch, l, up, n.width(l), n.at<uint16_t>(L.enc_a1[l]), n.width(l), a0, st);
        layer_forward(n, n.dec(l, 2), batch, l, a0, n.width(l), nullptr, 0, a1, st);
        h = a1;
        hc = n.width(l);
    }
    layer_forward(n, n.head(), batch, 0, h, hc, nullptr, 0, y, st);
    n.last_batch = batch;
}

void run_backward(un_net &n, int batch, const uint16_t *x, const float *target, const float *y, double *loss,
                  hipStream_t st)
{
    const Layout &L = n.lay;
    const int oc = n.cfg.out_ch;
    const long long P = n.pixels(batch, 0);
    const long long hw = n.pixels(1, 0);
    double *stats = n.at<double>(L.stats);
    uint16_t *gout = n.at<uint16_t>(L.gout);
    double *mpart = n.at<double>(L.mse_part);
    mse_partial_kernel<<<dim3(kMseChunks, batch), kThreads, 0, st>>>(y, target, oc, hw, mpart);
    mse_stats_kernel<<<(unsigned)cdiv(batch * oc, 64), 64, 0, st>>>(mpart, batch * oc, stats);
    const int gc = n.layers[n.head()].G;    // the output gradient's channels: out_ch rounded up to 8
    mse_grad_kernel<<<(unsigned)cdiv(P, 256), 256, 0, st>>>(y, target, stats, oc, gc, hw, P, gout, loss);

    uint16_t *X = n.at<uint16_t>(L.gx), *Y = n.at<uint16_t>(L.gy);
    const uint16_t *last = n.L > 1 ? n.at<uint16_t>(L.dec_a1[0]) : n.at<uint16_t>(L.enc_a1[0]);
    layer_weight_grad(n, n.head(), batch, 0, last, n.cfg.base, nullptr, 0, gout, gc, st);
    layer_data_grad(n, n.head(), batch, 0, gout, X, n.cfg.base, nullptr, 0, last, st);

    for (int l = 0; l <= n.L - 2; ++l) {
        const int w = n.width(l);
        uint16_t *a0 = n.at<uint16_t>(L.dec_a0[l]), *up = n.at<uint16_t>(L.dec_up[l]);
        uint16_t *skip = n.at<uint16_t>(L.enc_a1[l]), *dskip = n.at<uint16_t>(L.dskip[l]);
        layer_weight_grad(n, n.dec(l, 2), batch, l, a0, w, nullptr, 0, X, w, st);
        layer_data_grad(n, n.dec(l, 2), batch, l, X, Y, w, nullptr, 0, a0, st);
        layer_weight_grad(n, n.dec(l, 1), batch, l, up, w, skip, w, Y, w, st);
        layer_data_grad(n, n.dec(l, 1), batch, l, Y, X, w, dskip, w, nullptr, st);
        const uint16_t *hin = (l == n.L - 2) ? n.at<uint16_t>(L.enc_a1[n.L - 1]) : n.at<uint16_t>(L.dec_a1[l + 1]);
        layer_weight_grad(n, n.dec(l, 0), batch, l + 1, hin, n.width(l + 1), nullptr, 0, X, w, st);
        layer_data_grad(n, n.dec(l, 0), batch, l + 1, X, Y, n.width(l + 1), nullptr, 0, hin, st);
        std::swap(X, Y);
    }
    for (int l = n.L - 1; l >= 0; --l) {
        const int w = n.width(l);
        uint16_t *a0 = n.at<uint16_t>(L.enc_a0[l]);
        layer_weight_grad(n, n.enc(l, 1), batch, l, a0, w, nullptr, 0, X, w, st);
        layer_data_grad(n, n.enc(l, 1), batch, l, X, Y, w, nullptr, 0, a0, st);
        const uint16_t *in0 = l == 0 ? x : n.at<uint16_t>(L.pool[l - 1]);
        const int c0 = l == 0 ? n.in_pad : n.width(l - 1);
        layer_weight_grad(n, n.enc(l, 0), batch, l, in0, c0, nullptr, 0, Y, w, st);
        if (l > 0) {
            const int wp = n.width(l - 1);
            layer_data_grad(n, n.enc(l, 0), batch, l, Y, X, wp, nullptr, 0, nullptr, st);
            const long long cnt = n.pixels(batch, l) * (wp / 8);
            maxpool_backward_kernel<<<(unsigned)cdiv(cnt, 256), 256, 0, st>>>(
                n.at<uint16_t>(L.enc_a1[l - 1]), X, n.at<uint16_t>(L.dskip[l - 1]), wp, n.hl - l + 1, n.wl - l + 1,
                cnt, Y);
            std::swap(X, Y);
        }
    }
}

__global__ void zero_kernel(float *p, long long count)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0.0f;
}

void refresh_bf16(un_net &n, hipStream_t st)
{
    const float *p = n.at<float>(n.lay.params);
    for (const Layer &ly : n.layers) {
        const long long cnt = (long long)ly.info.n_rows * ly.info.kpad;
        to_bf16_kernel<<<(unsigned)cdiv(cnt, 256), 256, 0, st>>>(p + ly.info.w_offset, cnt,
                                                                 n.at<uint16_t>(n.lay.wbf) + ly.wb);
        const long long dc = (long long)ly.d_rows * ly.d_k;
        dgrad_weights_kernel<<<(unsigned)cdiv(dc, 256), 256, 0, st>>>(
            p + ly.info.w_offset, ly.info.kind == UN_UPCONV2X2, ly.info.taps, ly.info.cin, ly.info.cout, ly.G,
            ly.info.kpad, ly.d_rows, ly.d_k, n.at<uint16_t>(n.lay.wdf) + ly.wd);
    }
}

un_status check_net(const un_net *n)
{
    if (!n || !n->ws) return ufail(UN_ERR_INVALID_ARG, "network is NULL");
    return UN_OK;
}

}  // namespace

extern "C" {

un_status un_workspace_size(const un_config *cfg, size_t *ws_bytes)
{
    un_status s = check_config(cfg);
    if (s != UN_OK) return s;
    if (!ws_bytes) return ufail(UN_ERR_INVALID_ARG, "ws_bytes is NULL");
    un_net n;
    n.cfg = *cfg;
    plan(n);
    *ws_bytes = n.lay.total;
    return UN_OK;
}

un_status un_net_create(const un_config *cfg, void *workspace, size_t ws_bytes, un_net **out)
{
    un_status s = check_config(cfg);
    if (s != UN_OK) return s;
    if (!out) return ufail(UN_ERR_INVALID_ARG, "out is NULL");
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) % kAlign))
        return ufail(UN_ERR_INVALID_ARG, "workspace must be a non-NULL, 256-byte aligned device pointer");
    un_net *n = new (std::nothrow) un_net;
    if (!n) return ufail(UN_ERR_INVALID_ARG, "out of host memory");
    n->cfg = *cfg;
    plan(*n);
    if (ws_bytes < n->lay.total) {
        const size_t need = n->lay.total;
        delete n;
        return ufail(UN_ERR_BUDGET, "workspace too small: " + std::to_string(need) + " bytes needed");
    }
    n->ws = static_cast<char *>(workspace);
    *out = n;
    return UN_OK;
}

void un_net_destroy(un_net *net) { delete net; }

int32_t un_layer_count(const un_net *net) { return net ? (int32_t)net->layers.size() : 0; }

un_status un_layer_info(const un_net *net, int32_t index, un_layer *out)
{
    un_status s = check_net(net);
    if (s != UN_OK) return s;
    if (!out || index < 0 || index >= (int32_t)net->layers.size())
        return ufail(UN_ERR_INVALID_ARG, "layer index out of range or out is NULL");
    *out = net->layers[index].info;
    return UN_OK;
}

un_status un_params(un_net *net, float **params, float **grads, int64_t *count)
{
    un_status s = check_net(net);
    if (s != UN_OK) return s;
    if (params) *params = net->at<float>(net->lay.params);
    if (grads) *grads = net->at<float>(net->lay.grads);
    if (count) *count = net->n_params;
    return UN_OK;
}

un_status un_sync_weights(un_net *net, hipStream_t stream)
{
    un_status s = check_net(net);
    if (s != UN_OK) return s;
    const long long np = net->n_params;
    zero_kernel<<<(unsigned)cdiv(np, 256), 256, 0, stream>>>(net->at<float>(net->lay.adam_m), np);
    zero_kernel<<<(unsigned)cdiv(np, 256), 256, 0, stream>>>(net->at<float>(net->lay.adam_v), np);
    zero_kernel<<<(unsigned)cdiv(np, 256), 256, 0, stream>>>(net->at<float>(net->lay.grads), np);
    refresh_bf16(*net, stream);
    net->step = 0;
    return launch_ok("un_sync_weights") ? UN_OK : UN_ERR_HIP;
}

un_status un_forward(un_net *net, hipStream_t stream, int32_t batch, const uint16_t *x, float *y)
{
    un_status s = check_net(net);
    if (s != UN_OK) return s;
    if (batch < 1 || batch > net->cfg.max_batch) return ufail(UN_ERR_INVALID_ARG, "batch must be in [1, max_batch]");
    if (!x || !y) return ufail(UN_ERR_INVALID_ARG, "x and y must be device pointers");
    run_forward(*net, batch, x, y, stream);
    return launch_ok("un_forward") ? UN_OK : UN_ERR_HIP;
}

un_status un_backward(un_net *net, hipStream_t stream, int32_t batch, const uint16_t *x, const float *target,
                      float *y, double *loss_out)
{
    un_status s = check_net(net);
    if (s != UN_OK) return s;
    if (batch < 1 || batch > net->cfg.max_batch) return ufail(UN_ERR_INVALID_ARG, "batch must be in [1, max_batch]");
    if (!x || !y || !target) return ufail(UN_ERR_INVALID_ARG, "x, target and y must be device pointers");
    run_forward(*net, batch, x, y, stream);
    run_backward(*net, batch, x, target, y, loss_out, stream);
    return launch_ok("un_backward") ? UN_OK : UN_ERR_HIP;
}

un_status un_adam_step(un_net *net, hipStream_t stream, float lr, float beta1, float beta2, float eps)
{
    un_status s = check_net(net);
    if (s != UN_OK) return s;
    if (!(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
        return ufail(UN_ERR_INVALID_ARG, "need lr >= 0, beta1 and beta2 in [0, 1), eps > 0");
    const int t = ++net->step;
    const float c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, t)));
    const float c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, t)));
    const long long np = net->n_params;
    adam_kernel<<<(unsigned)cdiv(np, 256), 256, 0, stream>>>(
        net->at<float>(net->lay.params), net->at<float>(net->lay.grads), net->at<float>(net->lay.adam_m),
        net->at<float>(net->lay.adam_v), np, lr, beta1, beta2, eps, c1, c2);
    refresh_bf16(*net, stream);
    return launch_ok("un_adam_step") ? UN_OK : UN_ERR_HIP;
}

un_status un_activation(const un_net *net, int32_t index, const uint16_t **data, int32_t *height, int32_t *width,
                        int32_t *channels)
{
    un_status s = check_net(net);
    if (s != UN_OK) return s;
    if (!data || index < 0 || index >= 6 * net->L) return ufail(UN_ERR_INVALID_ARG, "activation index out of range");
    const int L = net->L;
    const bool decoder = index >= 3 * L;
    const int lvl = (index % (3 * L)) / 3, j = index % 3;
    if ((decoder && lvl > L - 2) || (!decoder && j == 2 && lvl == L - 1))
        return ufail(UN_ERR_INVALID_ARG, "no such activation at this level");
    size_t off;
    int lv = lvl;
    if (!decoder) {
        off = j == 0 ? net->lay.enc_a0[lvl] : j == 1 ? net->lay.enc_a1[lvl] : net->lay.pool[lvl];
        if (j == 2) lv = lvl + 1;
    } else {
        off = j == 0 ? net->lay.dec_up[lvl] : j == 1 ? net->lay.dec_a0[lvl] : net->lay.dec_a1[lvl];
    }
    *data = net->at<const uint16_t>(off);
    if (height) *height = net->cfg.height >> lv;
    if (width) *width = net->cfg.width >> lv;
    if (channels) *channels = net->width(lvl);
    return UN_OK;
}

const char *un_last_error(void) { return u_err.c_str(); }

}  // extern "C"
