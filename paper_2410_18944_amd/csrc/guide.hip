// Guide handle, parameter initialisation, fp16 shadow / MFMA fragment
// swizzle, and the standalone inference and direction-sampling entry points.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "guide_device.h"
#include "guide_internal.h"
#include "walk_common.h"

using namespace wost;

namespace wost {

int guide_prepare(const wost_guide* g, int dim, GuideDev& out)
{
    if (!g) { set_error("guide: NULL handle"); return WOST_EINVAL; }
    if (g->cfg.dim != dim) { set_error("guide: dimension %d does not match geometry %d", g->cfg.dim, dim); return WOST_EINVAL; }
    if (!g->shadow) { set_error("guide: parameters not bound"); return WOST_ESTATE; }
    out = g->dev;
    out.grid = (const uint32_t*)g->shadow;
    out.frags = (const half4_t*)((const _Float16*)g->shadow + g->frag_base);
    return WOST_OK;
}

// ---------------------------------------------------------------- kernels

__global__ void zero_f32(float* p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.f;
}

template <int D>
__global__ __launch_bounds__(64) void guide_infer_kernel(const GuideDev g, const float* pts, int64_t n, float* out_raw)
{
    extern __shared__ float s_out[];
    const int lane = threadIdx.x;
    const int stride = guide_out_stride(g);
    const int64_t i = (int64_t)blockIdx.x * 64 + lane;
    float x[D];
#pragma unroll
    for (int c = 0; c < D; ++c) x[c] = i < n ? pts[i * D + c] : 0.f;
    guide_forward_wave<D>(g, x, s_out, lane, stride);
    __syncthreads();
    if (i < n)
        for (int j = 0; j < g.n_out; ++j) out_raw[i * g.n_out + j] = s_out[lane * stride + j];
}

template <int D>
__global__ __launch_bounds__(64) void guide_sample_kernel(const GuideDev g, const float* pts, const float* normals,
                                                          int64_t n, uint32_t k0, uint32_t k1, uint32_t jw,
                                                          float* out_nu, float* out_pdf)
{
    extern __shared__ float s_out[];
    const int lane = threadIdx.x;
    const int stride = guide_out_stride(g);
    const int64_t i = (int64_t)blockIdx.x * 64 + lane;
    float x[D], nin[D];
    bool onN = false;
#pragma unroll
    for (int c = 0; c < D; ++c) {
        x[c] = i < n ? pts[i * D + c] : 0.f;
        nin[c] = (i < n && normals) ? normals[i * D + c] : 0.f;
        onN = onN || nin[c] != 0.f;
    }
    guide_forward_wave<D>(g, x, s_out, lane, stride);
    __syncthreads();
    if (i >= n) return;
    Stream rs;
    rs.p = (uint32_t)i; rs.j = jw; rs.k0 = k0; rs.k1 = k1;
    const uint4 wd = rs.block(0u, kBlkDir);
    float nu[D], pm;
    guided_draw<D>(g, s_out + lane * stride, rs, 0u, wd, onN, nin, nu, &pm);
#pragma unroll
    for (int c = 0; c < D; ++c) out_nu[i * D + c] = nu[c];
    out_pdf[i] = pm;
}

}  // namespace wost

// ---------------------------------------------------------------- C ABI

extern "C" int wost_guide_create(const wost_guide_config* c, wost_guide** out)
{
    if (!c || !out) { set_error("wost_guide_create: NULL argument"); return WOST_EINVAL; }
    *out = nullptr;
    if (c->dim != 2 && c->dim != 3) { set_error("wost_guide_create: dim must be 2 or 3"); return WOST_EINVAL; }
    if (c->feats != 2) { set_error("wost_guide_create: feats must be 2"); return WOST_EUNSUPPORTED; }
    if (c->hidden != kHidden) { set_error("wost_guide_create: hidden width must be 64"); return WOST_EUNSUPPORTED; }
    if (c->levels < 1 || c->levels > kMaxLevels || (c->levels * c->feats) % 16 != 0) {
        set_error("wost_guide_create: levels*feats must be a multiple of 16 with levels <= %d", kMaxLevels);
        return WOST_EUNSUPPORTED;
    }
    if (c->n_hidden < 1 || c->n_hidden > kMaxLayers - 1) { set_error("wost_guide_create: n_hidden in [1, %d]", kMaxLayers - 1); return WOST_EINVAL; }
    const int n_out = c->K * (c->dim + 2) + 1;
    const int out_pad = (n_out + 15) / 16 * 16;
    if (c->K < 1 || c->K > 16 || out_pad > kMaxOutPad) { set_error("wost_guide_create: K in [1, 16]"); return WOST_EINVAL; }
    if (c->log2_table < 2 || c->log2_table > 24) { set_error("wost_guide_create: log2_table in [2, 24]"); return WOST_EINVAL; }
    if (c->n_min < 1 || c->n_max < c->n_min) { set_error("wost_guide_create: need 1 <= n_min <= n_max"); return WOST_EINVAL; }
    for (int i = 0; i < c->dim; ++i)
        if (!(c->aabb_hi[i] > c->aabb_lo[i])) { set_error("wost_guide_create: empty AABB"); return WOST_EINVAL; }
    wost_guide* g = new wost_guide();
    g->cfg = *c;
    GuideDev& d = g->dev;
    memset(&d, 0, sizeof(d));
    d.dim = c->dim;
    d.L = c->levels;
    d.log2T = c->log2_table;
    d.K = c->K;
    d.n_out = n_out;
    d.out_pad = out_pad;
    const double T = std::ldexp(1.0, c->log2_table);
    const double b = c->levels > 1 ? std::exp((std::log((double)c->n_max) - std::log((double)c->n_min)) / (c->levels - 1)) : 1.0;
    for (int l = 0; l < c->levels; ++l) {
        const int N = (int)std::floor(c->n_min * std::pow(b, (double)l));
        d.res[l] = N;
        d.dense[l] = std::pow((double)(N + 1), (double)c->dim) <= T ? 1 : 0;
    }
    for (int i = 0; i < 3; ++i) {
        d.lo[i] = i < c->dim ? c->aabb_lo[i] : 0.f;
        d.inv_ext[i] = i < c->dim ? 1.f / (c->aabb_hi[i] - c->aabb_lo[i]) : 0.f;
    }
    g->n_grid = (int64_t)c->levels * (1ll << c->log2_table) * c->feats;
    // fragments start on a 16-byte boundary (paired fragments are read as one 16-byte load)
    g->frag_base = (g->n_grid + 7) & ~(int64_t)7;
    // layers
    const int n_layers = c->n_hidden + 1;
    d.n_layers = n_layers;
    int64_t off = g->n_grid;
    int32_t frag = 0;
    for (int l = 0; l < n_layers; ++l) {
        const int in = l == 0 ? c->levels * c->feats : kHidden;
        const int outd = l == n_layers - 1 ? n_out : kHidden;
        g->layer_in[l] = in;
        g->layer_out[l] = outd;
        g->layer_off[l] = off;
        off += (int64_t)in * outd;
        d.kb[l] = in / 16;
        d.mb[l] = (outd + 15) / 16;
        d.frag_off[l] = frag;
        frag += d.mb[l] * d.kb[l] * 64;
    }
    // backward fragments follow: same block count per layer (in blocks x out blocks)
    for (int l = 0; l < n_layers; ++l) d.bfrag_off[l] = frag + d.frag_off[l];
    g->n_params = off;
    g->n_frag_halves = (int64_t)frag * 4 * 2;
    d.sampling = WOST_SAMPLING_MIS_LEARNED;
    d.c_fixed = 0.5f;
    d.reflect = 1;
    *out = g;
    return WOST_OK;
}

extern "C" int64_t wost_guide_param_count(const wost_guide* g) { return g ? g->n_params : -1; }

extern "C" int wost_guide_set_reflect(wost_guide* g, int32_t reflect)
{
    if (!g) { set_error("wost_guide_set_reflect: NULL handle"); return WOST_EINVAL; }
    if (reflect != 0 && reflect != 1) { set_error("wost_guide_set_reflect: reflect must be 0 or 1"); return WOST_EINVAL; }
    g->dev.reflect = reflect;
    return WOST_OK;
}

extern "C" int32_t wost_guide_get_reflect(const wost_guide* g) { return g ? g->dev.reflect : -1; }

extern "C" int64_t wost_guide_shadow_bytes(const wost_guide* g)
{
    return g ? 2 * (g->frag_base + g->n_frag_halves) : -1;
}

extern "C" int wost_guide_bind(wost_guide* g, float* master, void* shadow, float* m, float* v, float* grad)
{
    if (!g || !master || !shadow) { set_error("wost_guide_bind: master and shadow are required"); return WOST_EINVAL; }
    if (((uintptr_t)shadow) & 15) { set_error("wost_guide_bind: shadow must be 16-byte aligned"); return WOST_EINVAL; }
    g->master = master;
    g->shadow = shadow;
    g->adam_m = m;
    g->adam_v = v;
    g->grad = grad;
    return WOST_OK;
}

// small per-guide device tables (layer offsets) are passed through kernel
// arguments; copy them into a constant-size struct
struct LayerTabs {
    int64_t off[kMaxLayers];
    int32_t in[kMaxLayers];
    int32_t out[kMaxLayers];
};

__global__ void init_params_kernel2(float* master, int64_t n_grid, int64_t n_total, LayerTabs t, int n_layers,
                                    uint32_t k0, uint32_t k1)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_total) return;
    const uint4 w = philox(make_uint4((uint32_t)i, (uint32_t)(i >> 32), 0x6D1u, 0u), k0, k1);
    const float u = 2.f * u01(w.x) - 1.f;
    if (i < n_grid) {
        master[i] = 1e-4f * u;
        return;
    }
    int l = 0;
    while (l + 1 < n_layers && i >= t.off[l + 1]) ++l;
    master[i] = u * sqrtf(6.f / (float)t.in[l]);
}

__global__ void sync_shadow_kernel2(const float* master, _Float16* shadow, int64_t n_grid, int64_t frag_base,
                                    GuideDev g, LayerTabs t, int64_t n_frag_halves)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_grid) {
        shadow[i] = (_Float16)master[i];
        return;
    }
    if (i < frag_base) {
        shadow[i] = (_Float16)0.f;  // alignment padding
        return;
    }
    const int64_t f = i - frag_base;
    if (f >= n_frag_halves) return;
    int64_t frag = f >> 2;
    const int e = (int)(f & 3);
    const int64_t n_fwd = g.bfrag_off[0];
    const bool bwd = frag >= n_fwd;
    if (bwd) frag -= n_fwd;
    int l = 0;
    while (l + 1 < g.n_layers && frag >= g.frag_off[l + 1]) ++l;
    const int rel = (int)(frag - g.frag_off[l]);
    // forward blocks run along the input features, backward blocks along the
    // output features; invert frag_index for this layer's block count
    const int KB = bwd ? g.mb[l] : g.kb[l];
    const int blk = rel >> 6;
    const int mb = blk / KB;
    int kb = blk - mb * KB, lane;
    if ((kb | 1) < KB) {
        const int q = rel - (mb * KB + (kb & ~1)) * 64;
        kb = (kb & ~1) + (q & 1);
        lane = q >> 1;
    } else {
        lane = rel & 63;
    }
    int row, colo;
    if (!bwd) {
        // forward A = W^T: m = output feature (16 mb + lane%16), k = input feature
        row = 16 * kb + 4 * (lane >> 4) + e;
        colo = 16 * mb + (lane & 15);
    } else {
        // backward A = W: m = input feature (16 mb + lane%16), k = output feature
        row = 16 * mb + (lane & 15);
        colo = 16 * kb + 4 * (lane >> 4) + e;
    }
    float v = 0.f;
    if (row < t.in[l] && colo < t.out[l]) v = master[t.off[l] + (int64_t)row * t.out[l] + colo];
    shadow[i] = (_Float16)v;
}

static LayerTabs tabs_of(const wost_guide* g)
{
    LayerTabs t;
    memset(&t, 0, sizeof(t));
    for (int l = 0; l < g->dev.n_layers; ++l) {
        t.off[l] = g->layer_off[l];
        t.in[l] = g->layer_in[l];
        t.out[l] = g->layer_out[l];
    }
    return t;
}

extern "C" int wost_guide_sync_shadow(wost_guide* g, void* stream)
{
    if (!g || !g->master || !g->shadow) { set_error("wost_guide_sync_shadow: guide not bound"); return WOST_ESTATE; }
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = g->frag_base + g->n_frag_halves;
    hipLaunchKernelGGL(sync_shadow_kernel2, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g->master,
                       (_Float16*)g->shadow, g->n_grid, g->frag_base, g->dev, tabs_of(g), g->n_frag_halves);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error("wost_guide_sync_shadow: %s", hipGetErrorString(e)); return WOST_EHIP; }
    return WOST_OK;
}

extern "C" int wost_guide_init(wost_guide* g, uint64_t seed, void* stream)
{
    if (!g || !g->master || !g->shadow) { set_error("wost_guide_init: guide not bound"); return WOST_ESTATE; }
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = g->n_params;
    const unsigned grid = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(init_params_kernel2, dim3(grid), dim3(256), 0, s, g->master, g->n_grid, n, tabs_of(g),
                       g->dev.n_layers, (uint32_t)seed, (uint32_t)(seed >> 32));
    float* zs[3] = {g->adam_m, g->adam_v, g->grad};
    for (float* z : zs)
        if (z) hipLaunchKernelGGL(zero_f32, dim3(grid), dim3(256), 0, s, z, n);
    g->adam_step = 0;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error("wost_guide_init: %s", hipGetErrorString(e)); return WOST_EHIP; }
    return wost_guide_sync_shadow(g, stream);
}

extern "C" int wost_guide_infer(const wost_guide* g, const float* pts, int64_t n, float* out_raw, void* stream)
{
    if (!g || !pts || !out_raw) { set_error("wost_guide_infer: NULL argument"); return WOST_EINVAL; }
    GuideDev d;
    int rc = guide_prepare(g, g->cfg.dim, d);
    if (rc != WOST_OK) return rc;
    if (n <= 0) return n == 0 ? WOST_OK : WOST_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const unsigned grid = (unsigned)((n + 63) / 64);
    const size_t lds = sizeof(float) * 64 * guide_out_stride(d);
    if (d.dim == 2) hipLaunchKernelGGL(guide_infer_kernel<2>, dim3(grid), dim3(64), lds, s, d, pts, n, out_raw);
    else hipLaunchKernelGGL(guide_infer_kernel<3>, dim3(grid), dim3(64), lds, s, d, pts, n, out_raw);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error("wost_guide_infer: %s", hipGetErrorString(e)); return WOST_EHIP; }
    return WOST_OK;
}

extern "C" int wost_guide_sample(const wost_guide* g, int32_t sampling, float c_fixed, const float* pts,
                                 const float* normals, int64_t n, uint64_t seed, uint32_t walk_index, float* out_nu,
                                 float* out_pdf, void* stream)
{
    if (!g || !pts || !out_nu || !out_pdf) { set_error("wost_guide_sample: NULL argument"); return WOST_EINVAL; }
    if (sampling < WOST_SAMPLING_MIS_LEARNED || sampling > WOST_SAMPLING_GUIDED_ONLY) {
        set_error("wost_guide_sample: sampling must be a guided mode");
        return WOST_EINVAL;
    }
    GuideDev d;
    int rc = guide_prepare(g, g->cfg.dim, d);
    if (rc != WOST_OK) return rc;
    d.sampling = sampling;
    d.c_fixed = c_fixed;
    if (n <= 0) return n == 0 ? WOST_OK : WOST_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const unsigned grid = (unsigned)((n + 63) / 64);
    const size_t lds = sizeof(float) * 64 * guide_out_stride(d);
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    if (d.dim == 2)
        hipLaunchKernelGGL(guide_sample_kernel<2>, dim3(grid), dim3(64), lds, s, d, pts, normals, n, k0, k1, walk_index, out_nu, out_pdf);
    else
        hipLaunchKernelGGL(guide_sample_kernel<3>, dim3(grid), dim3(64), lds, s, d, pts, normals, n, k0, k1, walk_index, out_nu, out_pdf);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error("wost_guide_sample: %s", hipGetErrorString(e)); return WOST_EHIP; }
    return WOST_OK;
}

extern "C" void wost_guide_free(wost_guide* g) { delete g; }
