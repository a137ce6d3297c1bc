// Online training of the guide (Sec. 4.2 KL objective, Sec. 4.4 selection
// probability loss, Sec. 5.2 online scheme) on gfx950.
//
// Per training record (x, nu, n, p_sample, p_t) the loss
//     l = -w [ log p_g(nu | Theta(x)) + e log( c sg(p_g) + (1 - c) p_u ) ],
//     w = p_t / p_sample,
// has exactly the paper's one-sample gradients: d l / d Theta is the
// "one_sample_kld" estimator -p_t grad p_g / (p~ p_g), and d l / d c is the
// "one_sample_sp" estimator -e p_t (p_g - p_u) / p~^2 (sg = stop-gradient).
//
// Kernel layout: one 64-wide wave per workgroup processes tiles of 64
// records.  Forward recomputes the grid encoding and runs the MLP on MFMA in
// the transposed form (see guide_device.h), storing every layer's input
// activations in LDS as [feature][walk] fp16.  The per-record output gradient
// is scaled by a power of two (per tile and per layer) before the fp16
// conversion.  Backward propagates dH = W dZ in registers with pre-swizzled
// W fragments; weight gradients dW^T = sum_walk dZ^T H contract over the tile
// from the LDS operands and accumulate in an fp32 LDS copy per workgroup,
// written once as a partial and reduced deterministically.  Grid gradients are
// scattered with fp32 atomics into the corners the forward pass read.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>

#include "guide_device.h"
#include "guide_internal.h"
#include "walk_common.h"

namespace wost {

struct TrainArgs {
    const float* rec;
    int64_t cap;
    int64_t begin, count;
    float e_mis;
    float scale;            // multiplies every record's gradient
    const float* dloss;     // per-record upstream gradient (or null = 1)
    float* loss_out;        // per-record loss (or null)
    float* loss_sum;        // device scalar += loss_scale * sum(loss) (or null)
    float loss_scale;
    float* grad;            // gradient vector (grid part first)
    float* partials;        // [gridDim.x][n_frag] weight gradients in MFMA fragment order
    int32_t n_frag;         // floats per workgroup row (= 256 x weight-gradient blocks)
    int32_t blk_off[kMaxLayers];   // first 16x16 block of each layer in a row
    float* gco;             // per-record feature gradients of every level [2 L][count]
    uint32_t* gmax;         // [L] largest |feature gradient| of each level (float bits)
    int32_t backward;
    int32_t p_mlp;
    int32_t off[kMaxLayers];   // layer weight offsets relative to the MLP start
    int32_t in[kMaxLayers];
    int32_t out[kMaxLayers];
};

// B(k) = d log v / d kappa + (1 - mu.nu): the kappa derivative of the vMF
// log-density is mu.nu - 1 + B(k), a small difference of O(1) terms near the
// mode, so B is computed without cancellation.
//  2D: B = 1 - I1(k)/I0(k).  For k >= 20 the asymptotic series of the ratio
//      (from r' = 1 - r/k - r^2, r = I1/I0): 1/(2k) + 1/(8k^2) + 1/(8k^3)
//      + 25/(128k^4) + 13/(32k^5) + 1073/(1024k^6); below, the polynomial
//      approximations of I0e and I1e.
//  3D: B = 1 + 1/k - coth(k) = 1/k - 2/(e^{2k} - 1) (series for small k).
__device__ __forceinline__ float vmf_dlog_offset2(float k)
{
    if (k >= 20.f) {
        const float u = 1.f / k;
        return u * (0.5f + u * (0.125f + u * (0.125f + u * (25.f / 128.f + u * (13.f / 32.f + u * (1073.f / 1024.f))))));
    }
    return 1.f - i1e_f(k) / i0e_f(k);
}

__device__ __forceinline__ float vmf_dlog_offset3(float k)
{
    if (k < 0.3f) {
        const float k2 = k * k;
        return 1.f + k * (-1.f / 3.f + k2 * (1.f / 45.f - k2 * (2.f / 945.f)));
    }
    return 1.f / k - 2.f / expm1f(2.f * k);
}

__device__ __forceinline__ float softplus(float z) { return fmaxf(z, 0.f) + log1pf(expf(-fabsf(z))); }

// Loss of one record and (optionally, in place) its gradient w.r.t. the raw
// outputs y (row in LDS; padded entries untouched).  dscale multiplies dy.
// On a Neumann record p_g is the reflected mixture (Sec. 4.3) when mirror is
// set, else the plain mixture (reflection off).
template <int D>
__device__ float record_loss_grad(float* y, int K, const float* nu, const float* n, bool onN, bool mirror, float ps,
                                  float pt, float e, bool want_grad, float dscale)
{
    const float area = D == 2 ? 2.f * kPi : 4.f * kPi;
    float nr[D];
    {
        const float cn = dot<D>(nu, n);
#pragma unroll
        for (int i = 0; i < D; ++i) nr[i] = fmaf(-2.f * cn, n[i], nu[i]);
    }
    // pass 1: log-softmax of lambda', mixture log-density (streaming LSE)
    float lmax = -INFINITY;
    for (int i = 0; i < K; ++i) lmax = fmaxf(lmax, y[i * (D + 2) + D + 1]);
    float lsum = 0.f;
    for (int i = 0; i < K; ++i) lsum += expf(y[i * (D + 2) + D + 1] - lmax);
    const float lse_lam = lmax + logf(lsum);
    float m = -INFINITY, s = 0.f;
    for (int i = 0; i < K; ++i) {
        const float* r = y + i * (D + 2);
        float n2 = 0.f;
#pragma unroll
        for (int d = 0; d < D; ++d) n2 = fmaf(r[d], r[d], n2);
        const float inv = rsqrtf(fmaxf(n2, 1e-30f));
        float mu[D];
#pragma unroll
        for (int d = 0; d < D; ++d) mu[d] = r[d] * inv;
        const float k = expf(fminf(fmaxf(r[D], kKappaLogMin), kKappaLogMax));
        const float base = r[D + 1] - lse_lam + vmf_lognorm<D>(k);
        const float t1 = fmaf(k, dot<D>(mu, nu) - 1.f, base);
        float mt = fmaxf(m, t1);
        s = s * expf(m - mt) + expf(t1 - mt);
        m = mt;
        if (mirror) {
            const float t2 = fmaf(k, dot<D>(mu, nr) - 1.f, base);
            mt = fmaxf(m, t2);
            s = s * expf(m - mt) + expf(t2 - mt);
            m = mt;
        }
    }
    const float log_pg = m + logf(s);
    // selection probability c = sigmoid(c'), c' clamped to [-15, 15]; the MIS
    // pdf c p_g + (1 - c) p_u is combined in log space
    const float craw = y[K * (D + 2)];
    const float cr = fminf(fmaxf(craw, -kCLogit), kCLogit);
    const float log_c = -softplus(-cr), log_1mc = -softplus(cr);
    const float c = expf(log_c);
    const float log_pu = logf((onN ? 2.f : 1.f) / area);
    const float la = log_c + log_pg, lb = log_1mc + log_pu;
    const float lmx = fmaxf(la, lb);
    const float log_pm = lmx + logf(expf(la - lmx) + expf(lb - lmx));
    const float w = ps > 0.f ? pt / ps : 0.f;
    const float loss = -w * (log_pg + e * log_pm);
    if (!want_grad) return loss;
    const float gw = -w * dscale;
    // pass 2: responsibilities and gradients, lobe by lobe (reads lobe i
    // before overwriting it)
    for (int i = 0; i < K; ++i) {
        float* r = y + i * (D + 2);
        float n2 = 0.f;
#pragma unroll
        for (int d = 0; d < D; ++d) n2 = fmaf(r[d], r[d], n2);
        const float inv = rsqrtf(fmaxf(n2, 1e-30f));
        float mu[D];
#pragma unroll
        for (int d = 0; d < D; ++d) mu[d] = r[d] * inv;
        const float kp = r[D];
        const bool clamped = kp < kKappaLogMin || kp > kKappaLogMax;
        const float k = expf(fminf(fmaxf(kp, kKappaLogMin), kKappaLogMax));
        const float lam = expf(r[D + 1] - lse_lam);
        const float base = r[D + 1] - lse_lam + vmf_lognorm<D>(k);
        const float B = D == 2 ? vmf_dlog_offset2(k) : vmf_dlog_offset3(k);
        const float c1 = dot<D>(mu, nu);
        const float g1 = expf(fmaf(k, c1 - 1.f, base) - log_pg);
        float c2 = 0.f, g2 = 0.f;
        if (mirror) {
            c2 = dot<D>(mu, nr);
            g2 = expf(fmaf(k, c2 - 1.f, base) - log_pg);
        }
        // d log p_g / d lambda'_i, kappa'_i, mu'_i
        const float dlam = g1 + g2 - lam;
        const float dkap = clamped ? 0.f : k * (g1 * (B - (1.f - c1)) + g2 * (B - (1.f - c2)));
        float dmu[D];
#pragma unroll
        for (int d = 0; d < D; ++d) {
            float v = g1 * (nu[d] - c1 * mu[d]);
            if (mirror) v += g2 * (nr[d] - c2 * mu[d]);
            dmu[d] = v * k * inv;
        }
#pragma unroll
        for (int d = 0; d < D; ++d) r[d] = gw * dmu[d];
        r[D] = gw * dkap;
        r[D + 1] = gw * dlam;
    }
    // d log(c p_g + (1 - c) p_u) / d c' = r_g - c, r_g = c p_g / p~
    const bool c_clamped = craw < -kCLogit || craw > kCLogit;
    y[K * (D + 2)] = c_clamped ? 0.f : gw * e * (expf(la - log_pm) - c);
    return loss;
}

__device__ __forceinline__ float wave_max(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}

__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// power-of-two factor bringing max |v| to about 2^10 (1 if max is 0)
__device__ __forceinline__ float pow2_scale(float maxabs)
{
    if (!(maxabs > 0.f) || !(maxabs < INFINITY)) return 1.f;
    return exp2f(floorf(log2f(1024.f / maxabs)));
}

__device__ __forceinline__ half4_t lds_h4(const _Float16* p)
{
    return *(const half4_t*)p;
}

template <int D>
__global__ __launch_bounds__(64) void train_kernel(const GuideDev g, const TrainArgs a)
{
    extern __shared__ float smem[];
    const int lane = threadIdx.x, g4 = lane >> 4, col = lane & 15;
    const int L = g.n_layers;
    const int K = g.K;
    const int out_pad = g.out_pad;
    const int ystride = out_pad + 1;
    const int kb0 = g.kb[0];
    const int rows_act = 16 * kb0 + 64 * (L - 1);
    const int rmax = out_pad > 64 ? out_pad : 64;
    // LDS: the raw outputs s_y share their space with one of the two dZ
    // buffers (s_y is dead once the output gradient has been staged in s_d1)
    const int ybytes = 64 * ystride * 4, dbytes = rmax * 64 * 2;
    float* s_y = smem;
    _Float16* s_d0 = (_Float16*)smem;
    _Float16* s_act = (_Float16*)((char*)smem + (ybytes > dbytes ? ybytes : dbytes));
    _Float16* s_d1 = s_act + rows_act * 64;
    const int64_t T = 1ll << g.log2T;
    // this workgroup's weight-gradient row, accumulated across its tiles in
    // the MFMA fragment layout (each lane owns a float4 of every block)
    float4* const prow = a.backward ? (float4*)(a.partials + (int64_t)blockIdx.x * a.n_frag) : nullptr;
    if (a.backward)
        for (int j = lane; j < a.n_frag / 4; j += 64) prow[j] = make_float4(0.f, 0.f, 0.f, 0.f);

    const int64_t n_tiles = (a.count + 63) / 64;
    float loss_acc = 0.f;
    float gmx[4][2] = {{0.f, 0.f}, {0.f, 0.f}, {0.f, 0.f}, {0.f, 0.f}};   // per owned level
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int64_t i = tile * 64 + lane;
        const bool valid = i < a.count;
        const int64_t r = a.begin + i;
        float x[D], nu[D], nn[D];
        float ps = 1.f, pt = 0.f;
        bool onN = false;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            x[d] = valid ? a.rec[(int64_t)d * a.cap + r] : 0.f;
            nu[d] = valid ? a.rec[(int64_t)(D + d) * a.cap + r] : 1.f / (float)D;
            nn[d] = valid ? a.rec[(int64_t)(2 * D + d) * a.cap + r] : 0.f;
            onN = onN || nn[d] != 0.f;
        }
        if (valid) {
            ps = a.rec[(int64_t)(3 * D) * a.cap + r];
            pt = a.rec[(int64_t)(3 * D + 4) * a.cap + r];
        }
        // ---------------- forward
        for (int cb = 0; cb < 4; ++cb) {
            const int w = 16 * cb + col;
            float xw[D], xh[D];
#pragma unroll
            for (int d = 0; d < D; ++d) xw[d] = __shfl(x[d], w);
            normalise_input<D>(g, xw, xh);
            half8_t act[2];
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) {
                if (kb >= kb0) break;
                const int l0 = 8 * kb + 2 * g4;
                const float2 f0 = grid_level<D>(g, l0, xh);
                const float2 f1 = grid_level<D>(g, l0 + 1, xh);
                half4_t h;
                h[0] = (_Float16)f0.x; h[1] = (_Float16)f0.y; h[2] = (_Float16)f1.x; h[3] = (_Float16)f1.y;
                put_half(act[kb >> 1], kb & 1, h);
#pragma unroll
                for (int e = 0; e < 4; ++e) s_act[(16 * kb + 4 * g4 + e) * 64 + w] = h[e];
            }
            int row_off = 16 * kb0;
            for (int layer = 0; layer + 1 < L; ++layer) {
                const half4_t* A = g.frags + g.frag_off[layer];
                const int KB = g.kb[layer];
                half8_t nxt[2];
#pragma unroll
                for (int mb = 0; mb < 4; ++mb) {
                    const float4_t c = mfma_row_block(A, mb, KB, lane, act, float4_t{0.f, 0.f, 0.f, 0.f});
                    half4_t h;
#pragma unroll
                    for (int e = 0; e < 4; ++e) h[e] = (_Float16)fmaxf(c[e], 0.f);
                    put_half(nxt[mb >> 1], mb & 1, h);
#pragma unroll
                    for (int e = 0; e < 4; ++e) s_act[(row_off + 16 * mb + 4 * g4 + e) * 64 + w] = h[e];
                }
                act[0] = nxt[0];
                act[1] = nxt[1];
                row_off += 64;
            }
            {
                const int layer = L - 1;
                const half4_t* A = g.frags + g.frag_off[layer];
                const int KB = g.kb[layer];
                for (int mb = 0; mb < g.mb[layer]; ++mb) {
                    const float4_t c = mfma_row_block(A, mb, KB, lane, act, float4_t{0.f, 0.f, 0.f, 0.f});
#pragma unroll
                    for (int e = 0; e < 4; ++e) s_y[w * ystride + 16 * mb + 4 * g4 + e] = c[e];
                }
            }
        }
        __syncthreads();
        // ---------------- per-record loss and output gradient (lane = record)
        float* yrow = s_y + lane * ystride;
        const float up = valid ? (a.dloss ? a.dloss[i] : 1.f) * a.scale : 0.f;
        const float loss = record_loss_grad<D>(yrow, K, nu, nn, onN, onN && g.reflect != 0, ps, pt, a.e_mis,
                                               a.backward != 0, up);
        if (valid) {
            if (a.loss_out) a.loss_out[i] = loss;
            loss_acc += loss;
        }
        if (!a.backward) {
            __syncthreads();
            continue;
        }
        // padded records and any non-finite gradient contribute exactly zero
        for (int j = 0; j < out_pad; ++j)
            if (!valid || j >= g.n_out || !(fabsf(yrow[j]) < INFINITY)) yrow[j] = 0.f;
        float mx = 0.f;
        for (int j = 0; j < out_pad; ++j) mx = fmaxf(mx, fabsf(yrow[j]));
        float Sc = pow2_scale(wave_max(mx));
        for (int j = 0; j < out_pad; ++j) s_d1[j * 64 + lane] = (_Float16)(yrow[j] * Sc);
        __syncthreads();
        // ---------------- backward
        _Float16* cur = s_d1;
        _Float16* nxt = s_d0;
        for (int layer = L - 1; layer >= 0; --layer) {
            const int rows_out = layer == L - 1 ? out_pad : 64;
            const int rows_in = layer == 0 ? 16 * kb0 : 64;
            const _Float16* act = s_act + (layer == 0 ? 0 : (16 * kb0 + 64 * (layer - 1))) * 64;
            const float inv_sc = 1.f / Sc;
            // weight gradient: dW^T[out][in] += sum_walk dZ^T[out][walk] H[walk][in]
            for (int mb = 0; mb < rows_out / 16; ++mb) {
                for (int nb = 0; nb < rows_in / 16; ++nb) {
                    float4_t c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int kk = 0; kk < 4; kk += 2) {
                        const _Float16* const ap = cur + (16 * mb + col) * 64 + 16 * kk + 4 * g4;
                        const _Float16* const bp = act + (16 * nb + col) * 64 + 16 * kk + 4 * g4;
                        half8_t av, bv;
                        put_half(av, 0, lds_h4(ap));
                        put_half(av, 1, lds_h4(ap + 16));
                        put_half(bv, 0, lds_h4(bp));
                        put_half(bv, 1, lds_h4(bp + 16));
                        c = mfma_k32(av, bv, c);
                    }
                    float4* const dst = prow + (a.blk_off[layer] + mb * (rows_in / 16) + nb) * 64 + lane;
                    float4 v = *dst;
                    v.x = fmaf(c[0], inv_sc, v.x);
                    v.y = fmaf(c[1], inv_sc, v.y);
                    v.z = fmaf(c[2], inv_sc, v.z);
                    v.w = fmaf(c[3], inv_sc, v.w);
                    *dst = v;
                }
            }
            // data gradient dH^T = W dZ^T (rows = input features of this layer)
            const half4_t* Bw = g.frags + g.bfrag_off[layer];
            const int KBo = rows_out / 16;
            const int MBi = rows_in / 16;
            float4_t dz[4][4];
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) {
#pragma unroll
                for (int mb = 0; mb < 4; ++mb) {
                    float4_t c = {0.f, 0.f, 0.f, 0.f};
                    if (mb < MBi) {
                        int kb = 0;
                        for (; kb + 1 < KBo; kb += 2) {
                            half8_t bv;
#pragma unroll
                            for (int e = 0; e < 4; ++e) {
                                bv[e] = cur[(16 * kb + 4 * g4 + e) * 64 + 16 * cb + col];
                                bv[4 + e] = cur[(16 * kb + 16 + 4 * g4 + e) * 64 + 16 * cb + col];
                            }
                            c = mfma_k32(*(const half8_t*)(Bw + frag_index(mb, kb, KBo, lane)), bv, c);
                        }
                        if (kb < KBo) {
                            half4_t bv;
#pragma unroll
                            for (int e = 0; e < 4; ++e) bv[e] = cur[(16 * kb + 4 * g4 + e) * 64 + 16 * cb + col];
                            c = mfma_k16(Bw[frag_index(mb, kb, KBo, lane)], bv, c);
                        }
                        if (layer > 0) {
#pragma unroll
                            for (int e = 0; e < 4; ++e)
                                if (!((float)act[(16 * mb + 4 * g4 + e) * 64 + 16 * cb + col] > 0.f)) c[e] = 0.f;
                        }
                    }
                    dz[cb][mb] = c;
                }
            }
            if (layer > 0) {
                float m2 = 0.f;
#pragma unroll
                for (int cb = 0; cb < 4; ++cb)
#pragma unroll
                    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
                        for (int e = 0; e < 4; ++e) m2 = fmaxf(m2, fabsf(dz[cb][mb][e]));
                const float s2 = pow2_scale(wave_max(m2));
#pragma unroll
                for (int cb = 0; cb < 4; ++cb)
#pragma unroll
                    for (int mb = 0; mb < 4; ++mb)
                        if (mb < MBi) {
#pragma unroll
                            for (int e = 0; e < 4; ++e)
                                nxt[(16 * mb + 4 * g4 + e) * 64 + 16 * cb + col] = (_Float16)(dz[cb][mb][e] * s2);
                        }
                Sc *= s2;
                __syncthreads();
                _Float16* t = cur; cur = nxt; nxt = t;
            } else {
                // feature gradients, staged per record for slice_scatter_kernel:
                // this lane owns levels 8 mb + 2 g4 + {0,1} of walk 16 cb + col
                const float inv = 1.f / Sc;
#pragma unroll
                for (int cb = 0; cb < 4; ++cb) {
                    const int w = 16 * cb + col;
                    float xw[D], xh[D];
#pragma unroll
                    for (int d = 0; d < D; ++d) xw[d] = __shfl(x[d], w);
                    normalise_input<D>(g, xw, xh);
                    const bool wvalid = __shfl((int)valid, w) != 0;
#pragma unroll
                    for (int mb = 0; mb < 4; ++mb) {
                        if (mb >= kb0) break;
#pragma unroll
                        for (int lv = 0; lv < 2; ++lv) {
                            const int l = 8 * mb + 2 * g4 + lv;
                            const float gf0 = dz[cb][mb][2 * lv] * inv, gf1 = dz[cb][mb][2 * lv + 1] * inv;
                            if (wvalid) {
                                const int64_t iw = tile * 64 + w;
                                a.gco[(int64_t)(2 * l) * a.count + iw] = gf0;
                                a.gco[(int64_t)(2 * l + 1) * a.count + iw] = gf1;
                                gmx[mb][lv] = fmaxf(gmx[mb][lv], fmaxf(fabsf(gf0), fabsf(gf1)));
                            }
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
    if (a.loss_sum) {
        const float s = wave_sum(loss_acc);
        if (lane == 0) atomicAdd(a.loss_sum, s * a.loss_scale);
    }
    if (a.backward) {
        // the 16 lanes of a group own the same levels: reduce, one atomic each
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
            if (mb >= kb0) break;
#pragma unroll
            for (int lv = 0; lv < 2; ++lv) {
                float m = gmx[mb][lv];
                for (int o = 8; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
                if (col == 0 && m > 0.f) atomicMax(&a.gmax[8 * mb + 2 * g4 + lv], __float_as_uint(m));
            }
        }
    }
}

// Feature gradients of the grid levels, without global atomics.  A workgroup
// owns a slice of kSliceEntries consecutive entries of one level's table and
// adds, over its share of the records, every corner contribution that falls
// in its slice.  It accumulates in LDS in 64-bit fixed point (integer LDS
// atomics run far faster than fp32 ones, and integer sums do not depend on
// their order): the scale 2^k keeps the share's largest possible sum, records
// x the level's largest |feature gradient|, below 2^62.  With one share per
// slice it then adds the slice to the gradient with plain loads and stores
// (no other workgroup writes those entries); with R shares it writes its
// partial slice and slice_reduce_kernel adds the R partials.  A workgroup
// reads its records four per thread in flight; dense levels skip records
// whose corners all miss the slice.
constexpr int kSliceEntries = 10240;   // 160 KB of LDS
constexpr int kSliceThreads = 1024;
constexpr int kSliceUnroll = 4;

struct SliceTab {
    int32_t n;                      // rows: one per level
    int32_t level[kMaxLevels];
    int32_t entries[kMaxLevels];    // table entries of the level
    int32_t shares[kMaxLevels];     // record shares R of each slice of the row
    int32_t first[kMaxLevels + 1];  // first workgroup of each row; first[n] = workgroups
    int64_t poff[kMaxLevels + 1];   // first float of each row's partials (R > 1 rows); poff[n] = floats
};

template <int D>
__global__ __launch_bounds__(kSliceThreads) void slice_scatter_kernel(const GuideDev g, const float* rec, int64_t cap,
                                                                      int64_t begin, int64_t count, const float* gco,
                                                                      const uint32_t* gmax, const SliceTab st,
                                                                      float* grad, float* partial)
{
    extern __shared__ unsigned long long s_q[];
    int k = 0;
    while (k + 1 < st.n && (int)blockIdx.x >= st.first[k + 1]) ++k;
    const int R = st.shares[k];
    const int wg = (int)blockIdx.x - st.first[k];
    const int slice = wg / R, share = wg % R;
    const int l = st.level[k];
    const uint32_t lo = (uint32_t)slice * (uint32_t)kSliceEntries;
    const uint32_t n_here = min((uint32_t)kSliceEntries, (uint32_t)st.entries[k] - lo);
    for (uint32_t j = threadIdx.x; j < 2 * n_here; j += blockDim.x) s_q[j] = 0ull;
    __syncthreads();
    const int64_t r_lo = count * share / R, r_hi = count * (share + 1) / R;
    // fixed-point scale: |sum| <= (r_hi - r_lo) * gm < 2^(e + cn) <= 2^61
    const float gm = __uint_as_float(gmax[l]);
    int e = 0;
    (void)frexpf(gm, &e);
    int cn = 0;
    while ((int64_t(1) << cn) < r_hi - r_lo) ++cn;
    const int ks = 61 - e - cn;
    const int N = g.res[l];
    const bool dense = g.dense[l] != 0;
    const uint32_t mask = (uint32_t)((1ll << g.log2T) - 1);
    const float* g0 = gco + (int64_t)(2 * l) * count;
    const float* g1 = gco + (int64_t)(2 * l + 1) * count;
    const int64_t step = (int64_t)blockDim.x * kSliceUnroll;
    // positions of the next group of records are fetched while the current
    // group is processed
    float xn[kSliceUnroll][D];
    auto fetch = [&](int64_t b0) {
#pragma unroll
        for (int u = 0; u < kSliceUnroll; ++u) {
            const int64_t i = max(r_lo, min(b0 + (int64_t)u * blockDim.x, r_hi - 1));
#pragma unroll
            for (int d = 0; d < D; ++d) xn[u][d] = rec[(int64_t)d * cap + begin + i];
        }
    };
    if (gm > 0.f) fetch(r_lo + threadIdx.x);
    for (int64_t base = r_lo + threadIdx.x; gm > 0.f && base < r_hi; base += step) {
        float x[kSliceUnroll][D];
#pragma unroll
        for (int u = 0; u < kSliceUnroll; ++u)
#pragma unroll
            for (int d = 0; d < D; ++d) x[u][d] = xn[u][d];
        if (base + step < r_hi) fetch(base + step);
        // corners of every record of the group, then the gradients of the
        // records with a corner in the slice (one round of loads), then the
        // LDS sums
        uint32_t rel[kSliceUnroll][1 << D];
        float fr[kSliceUnroll][D];
        bool hit[kSliceUnroll];
#pragma unroll
        for (int u = 0; u < kSliceUnroll; ++u) {
            float xh[D];
            normalise_input<D>(g, x[u], xh);
            int cc[D];
#pragma unroll
            for (int d = 0; d < D; ++d) {
                const float pos = xh[d] * (float)N;
                int ci = (int)floorf(pos);
                ci = min(max(ci, 0), N - 1);
                cc[d] = ci;
                fr[u][d] = pos - (float)ci;
            }
            // the corner indices (the forward gather's, grid_level)
            uint32_t part[D][2];
            uint32_t stride = 1;
#pragma unroll
            for (int d = 0; d < D; ++d) {
                const uint32_t prime = d == 0 ? 1u : (d == 1 ? 2654435761u : 805459861u);
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    part[d][b] = dense ? (uint32_t)(cc[d] + b) * stride : (uint32_t)(cc[d] + b) * prime;
                stride *= (uint32_t)(N + 1);
            }
            bool any = false;
#pragma unroll
            for (int corner = 0; corner < (1 << D); ++corner) {
                uint32_t idx = 0;
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    const uint32_t t = part[d][(corner >> d) & 1];
                    idx = dense ? idx + t : idx ^ t;
                }
                if (!dense) idx &= mask;
                rel[u][corner] = idx - lo;
                any = any || rel[u][corner] < n_here;
            }
            hit[u] = any && base + (int64_t)u * blockDim.x < r_hi;
        }
        float f0[kSliceUnroll], f1[kSliceUnroll];
#pragma unroll
        for (int u = 0; u < kSliceUnroll; ++u) {
            const int64_t i = base + (int64_t)u * blockDim.x;
            f0[u] = hit[u] ? ldexpf(g0[i], ks) : 0.f;
            f1[u] = hit[u] ? ldexpf(g1[i], ks) : 0.f;
        }
#pragma unroll
        for (int u = 0; u < kSliceUnroll; ++u) {
            if (f0[u] == 0.f && f1[u] == 0.f) continue;
#pragma unroll
            for (int corner = 0; corner < (1 << D); ++corner) {
                if (rel[u][corner] < n_here) {
                    float wt = 1.f;
#pragma unroll
                    for (int d = 0; d < D; ++d) wt *= (corner >> d) & 1 ? fr[u][d] : 1.f - fr[u][d];
                    atomicAdd(&s_q[2 * rel[u][corner]], (unsigned long long)(long long)(wt * f0[u]));
                    atomicAdd(&s_q[2 * rel[u][corner] + 1], (unsigned long long)(long long)(wt * f1[u]));
                }
            }
        }
    }
    __syncthreads();
    const double inv = ldexp(1.0, -ks);
    if (R == 1) {
        float* gl = grad + (int64_t)l * (1ll << g.log2T) * 2 + 2 * (int64_t)lo;
        for (uint32_t j = threadIdx.x; j < 2 * n_here; j += blockDim.x) {
            const long long q = (long long)s_q[j];
            if (q != 0) gl[j] += (float)((double)q * inv);
        }
    } else {
        float* pr = partial + st.poff[k] + (int64_t)share * 2 * st.entries[k] + 2 * (int64_t)lo;
        for (uint32_t j = threadIdx.x; j < 2 * n_here; j += blockDim.x) pr[j] = (float)((double)(long long)s_q[j] * inv);
    }
}

// grad += the sum of the R partial rows of every level with R > 1
__global__ __launch_bounds__(256) void slice_reduce_kernel(const GuideDev g, const SliceTab st, const float* partial,
                                                           float* grad)
{
    const int64_t f = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int k = -1;
    int64_t j = f;
    for (int r = 0; r < st.n; ++r) {
        if (st.shares[r] == 1) continue;
        const int64_t n2 = 2 * (int64_t)st.entries[r];
        if (j < n2) { k = r; break; }
        j -= n2;
    }
    if (k < 0) return;
    float v = 0.f;
    for (int r = 0; r < st.shares[k]; ++r) v += partial[st.poff[k] + (int64_t)r * 2 * st.entries[k] + j];
    if (v != 0.f) grad[(int64_t)st.level[k] * (1ll << g.log2T) * 2 + j] += v;
}

struct FragMap {
    int32_t n_layers;
    int32_t off[kMaxLayers], in[kMaxLayers], out[kMaxLayers], blk_off[kMaxLayers], nb[kMaxLayers];
};

// Sums the workgroups' weight-gradient rows into the MLP gradient.  Weight
// (layer l, input i, output o) sits at l's offset + i * out + o; in a row it
// is element 4 * lane + e of block blk_off[l] + (o / 16) * nb[l] + i / 16,
// with lane = 16 ((o / 4) % 4) + i % 16 and e = o % 4 (the 16x16x16 MFMA
// accumulator layout).  Thread t of block (x, y) sums float4 t of rows y,
// y + gridDim.y, ... (coalesced), then adds each of its four sums to its
// weight (padding outputs o >= out are dropped).
__global__ __launch_bounds__(256) void reduce_partials(const float* partials, int nrows, int n_frag, FragMap m,
                                                       float* grad_mlp)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;     // float4 index in a row
    if (4 * t >= n_frag) return;
    const float4* p = (const float4*)partials;
    const int n4 = n_frag / 4;
    float4 s0 = make_float4(0.f, 0.f, 0.f, 0.f), s1 = s0;
    int r = blockIdx.y;
    for (; r + (int)gridDim.y < nrows; r += 2 * gridDim.y) {
        const float4 a = p[(int64_t)r * n4 + t], b = p[(int64_t)(r + gridDim.y) * n4 + t];
        s0.x += a.x; s0.y += a.y; s0.z += a.z; s0.w += a.w;
        s1.x += b.x; s1.y += b.y; s1.z += b.z; s1.w += b.w;
    }
    if (r < nrows) {
        const float4 a = p[(int64_t)r * n4 + t];
        s0.x += a.x; s0.y += a.y; s0.z += a.z; s0.w += a.w;
    }
    const float sum[4] = {s0.x + s1.x, s0.y + s1.y, s0.z + s1.z, s0.w + s1.w};
    const int blk = t / 64, lane = t % 64;
    int l = 0;
    while (l + 1 < m.n_layers && blk >= m.blk_off[l + 1]) ++l;
    const int lb = blk - m.blk_off[l];
    const int mb = lb / m.nb[l], nb = lb % m.nb[l];
    const int i = 16 * nb + (lane & 15);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int o = 16 * mb + 4 * (lane >> 4) + e;
        if (o < m.out[l] && i < m.in[l]) atomicAdd(grad_mlp + m.off[l] + i * m.out[l] + o, sum[e]);
    }
}

__global__ void adam_kernel(float* p, float* m, float* v, float* gr, int64_t n, float lr_t, float b1, float b2,
                            float eps_t)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float g = gr[i];
    const float mi = fmaf(b1, m[i], (1.f - b1) * g);
    const float vi = fmaf(b2, v[i], (1.f - b2) * g * g);
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr_t * mi / (sqrtf(vi) + eps_t);
    gr[i] = 0.f;
}

__global__ void zero_f32_t(float* p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.f;
}

// training target of every record: |V_{k+1}| = |U - prefix_k| / T_{k+1}
__global__ void tail_pass_kernel(float* rec, int64_t cap, const unsigned long long* count, int dim,
                                 const float* walk_value, int64_t n_slots)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = (int64_t)min((unsigned long long)cap, *count);
    if (i >= n) return;
    const uint32_t slot = __float_as_uint(rec[(int64_t)(3 * dim + 3) * cap + i]);
    const float pre = rec[(int64_t)(3 * dim + 1) * cap + i];
    const float tn = rec[(int64_t)(3 * dim + 2) * cap + i];
    float pt = 0.f;
    if ((int64_t)slot < n_slots && tn > 0.f) pt = fabsf(walk_value[slot] - pre) / tn;
    if (!(pt < INFINITY)) pt = 0.f;
    rec[(int64_t)(3 * dim + 4) * cap + i] = pt;
}

// Training set of a batch: row i of dst is a copy of a row of src drawn
// uniformly (with replacement) by Philox4x32-10 word (i, 0, 0, 0) under the
// key (seed lo, seed hi), so minibatches mix records of every walk of the
// batch instead of the runs of records one wave appended together.
__global__ void records_sample_kernel(const float* __restrict__ src, int64_t src_cap,
                                      const unsigned long long* __restrict__ src_count, int nf, float* __restrict__ dst,
                                      int64_t dst_cap, int64_t m, uint32_t k0, uint32_t k1)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const int64_t n = (int64_t)min((unsigned long long)src_cap, *src_count);
    if (n <= 0) return;
    const uint4 w = philox(make_uint4((uint32_t)i, (uint32_t)(i >> 32), 0u, 0u), k0, k1);
    // index floor(u n) for the 64-bit fraction u of two words
    const uint64_t u64 = ((uint64_t)w.x << 32) | (uint64_t)w.y;
    const int64_t j = (int64_t)__umul64hi(u64, (uint64_t)n);
    for (int f = 0; f < nf; ++f) dst[(int64_t)f * dst_cap + i] = src[(int64_t)f * src_cap + j];
}

__global__ void set_count_kernel(unsigned long long* dst, const unsigned long long* src, unsigned long long m)
{
    if (threadIdx.x == 0) *dst = *src > 0 ? m : 0ull;
}

static int g_train_cu = 0;

static int train_grid_cap()
{
    if (g_train_cu == 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
            g_train_cu = v;
        else
            g_train_cu = 256;
    }
    return 4 * g_train_cu;
}

// one row per grid level (table: (res + 1)^dim cells when dense, 2^log2T
// entries when hashed).  Each slice of a row gets R record shares so that a
// workgroup meets about count x 2^dim / 16 corner contributions (uniformly
// spread records assumed), and all R scale up until the workgroups about
// fill the chip.
static SliceTab slice_table(const GuideDev& g, int64_t count)
{
    SliceTab st;
    memset(&st, 0, sizeof(st));
    int64_t slices[kMaxLevels];
    const double target = (double)(1 << g.dim) * (double)std::max<int64_t>(count, 1) / 16.0;
    int64_t total = 0;
    for (int l = 0; l < g.L; ++l) {
        int64_t e = 1ll << g.log2T;
        if (g.dense[l]) {
            e = 1;
            for (int d = 0; d < g.dim; ++d) e *= g.res[l] + 1;
        }
        st.level[l] = l;
        st.entries[l] = (int32_t)e;
        slices[l] = (e + kSliceEntries - 1) / kSliceEntries;
        const double hits = (double)(1 << g.dim) * (double)count * (double)std::min<int64_t>(e, kSliceEntries) / (double)e;
        st.shares[l] = (int32_t)std::max(1.0, std::min(64.0, std::ceil(hits / target)));
        total += slices[l] * st.shares[l];
    }
    st.n = g.L;
    const int64_t fill = train_grid_cap() / 4;
    if (total > 0 && total < fill) {
        const int64_t m = (fill + total - 1) / total;
        for (int l = 0; l < st.n; ++l) st.shares[l] = (int32_t)std::min<int64_t>(64, st.shares[l] * m);
    }
    // shares never exceed the records
    for (int l = 0; l < st.n; ++l) st.shares[l] = (int32_t)std::max<int64_t>(1, std::min<int64_t>(st.shares[l], count));
    int64_t wg = 0, floats = 0;
    for (int l = 0; l < st.n; ++l) {
        st.first[l] = (int32_t)wg;
        st.poff[l] = floats;
        wg += slices[l] * st.shares[l];
        if (st.shares[l] > 1) floats += (int64_t)st.shares[l] * 2 * st.entries[l];
    }
    st.first[st.n] = (int32_t)wg;
    st.poff[st.n] = floats;
    return st;
}

// the partial slices of rows with R > 1, 256-byte aligned
static int64_t slice_partial_bytes(const SliceTab& st)
{
    return (st.poff[st.n] * 4 + 255) / 256 * 256;
}

// floats of the reduction over rows with R > 1
static int64_t slice_reduce_floats(const SliceTab& st)
{
    int64_t f = 0;
    for (int l = 0; l < st.n; ++l)
        if (st.shares[l] > 1) f += 2 * (int64_t)st.entries[l];
    return f;
}

// floats per workgroup row of weight-gradient partials: one 16x16 block per
// (16 outputs, 16 inputs) of every layer, output rows padded to 16
static int64_t frag_floats(const GuideDev& g)
{
    int64_t blocks = 0;
    for (int l = 0; l < g.n_layers; ++l) {
        const int rows_out = l == g.n_layers - 1 ? g.out_pad : 64;
        const int rows_in = l == 0 ? 16 * g.kb[0] : 64;
        blocks += (rows_out / 16) * (rows_in / 16);
    }
    return blocks * 256;
}

static int64_t train_ws_partials(const wost_guide* gd, int64_t count)
{
    const int64_t n_tiles = (count + 63) / 64;
    const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(n_tiles, train_grid_cap()));
    return (grid * frag_floats(gd->dev) * 4 + 255) / 256 * 256;
}

static size_t train_lds_bytes(const wost_guide* gd, bool backward)
{
    (void)backward;
    const GuideDev& g = gd->dev;
    const int rows_act = 16 * g.kb[0] + 64 * (g.n_layers - 1);
    const int rmax = g.out_pad > 64 ? g.out_pad : 64;
    const size_t ybytes = sizeof(float) * 64 * (g.out_pad + 1), dbytes = 2 * (size_t)rmax * 64;
    return (ybytes > dbytes ? ybytes : dbytes) + 2 * (size_t)rows_act * 64 + dbytes;
}

static int launch_train(const wost_guide* gd, const wost_records* rec, int64_t begin, int64_t count, float e_mis,
                        float scale, const float* dloss, float* loss_out, float* loss_sum, float loss_scale,
                        float* grad, void* workspace, int64_t ws_bytes, bool backward, hipStream_t s)
{
    GuideDev g;
    int rc = guide_prepare(gd, gd->cfg.dim, g);
    if (rc != WOST_OK) return rc;
    if (!rec || !rec->data || begin < 0 || count < 0 || begin + count > rec->capacity) {
        set_error("guide training: record range out of bounds");
        return WOST_EINVAL;
    }
    if (count == 0) return WOST_OK;
    TrainArgs a;
    memset(&a, 0, sizeof(a));
    a.rec = rec->data;
    a.cap = rec->capacity;
    a.begin = begin;
    a.count = count;
    a.e_mis = e_mis;
    a.scale = scale;
    a.dloss = dloss;
    a.loss_out = loss_out;
    a.loss_sum = loss_sum;
    a.loss_scale = loss_scale;
    a.grad = grad;
    a.backward = backward ? 1 : 0;
    a.p_mlp = (int32_t)(gd->n_params - gd->n_grid);
    FragMap fm;
    memset(&fm, 0, sizeof(fm));
    fm.n_layers = g.n_layers;
    int blk = 0;
    for (int l = 0; l < g.n_layers; ++l) {
        a.off[l] = (int32_t)(gd->layer_off[l] - gd->n_grid);
        a.in[l] = gd->layer_in[l];
        a.out[l] = gd->layer_out[l];
        const int rows_out = l == g.n_layers - 1 ? g.out_pad : 64;
        const int rows_in = l == 0 ? 16 * g.kb[0] : 64;
        a.blk_off[l] = blk;
        fm.off[l] = a.off[l];
        fm.in[l] = a.in[l];
        fm.out[l] = a.out[l];
        fm.blk_off[l] = blk;
        fm.nb[l] = rows_in / 16;
        blk += (rows_out / 16) * (rows_in / 16);
    }
    a.n_frag = blk * 256;
    const int64_t n_tiles = (count + 63) / 64;
    const int grid = (int)std::min<int64_t>(n_tiles, train_grid_cap());
    SliceTab st;
    memset(&st, 0, sizeof(st));
    float* slice_part = nullptr;
    if (backward) {
        if (!grad) { set_error("guide training: no gradient buffer bound"); return WOST_ESTATE; }
        const int64_t part = train_ws_partials(gd, count);
        st = slice_table(g, count);
        const int64_t gco_bytes = ((int64_t)2 * g.L * count * 4 + 255) / 256 * 256;
        const int64_t need = part + gco_bytes + 256 + slice_partial_bytes(st);
        if (!workspace || ws_bytes < need) { set_error("guide training: workspace %lld < %lld", (long long)ws_bytes, (long long)need); return WOST_ESIZE; }
        a.partials = (float*)workspace;
        a.gco = (float*)((char*)workspace + part);
        a.gmax = (uint32_t*)((char*)workspace + part + gco_bytes);
        slice_part = (float*)((char*)workspace + part + gco_bytes + 256);
        hipLaunchKernelGGL(zero_f32_t, dim3(1), dim3(64), 0, s, (float*)a.gmax, (int64_t)g.L);
    }
    const size_t lds = train_lds_bytes(gd, backward);
    if (lds > 160 * 1024) { set_error("guide training: configuration needs %zu bytes of LDS", lds); return WOST_EUNSUPPORTED; }
    if (g.dim == 2) hipLaunchKernelGGL(train_kernel<2>, dim3(grid), dim3(64), lds, s, g, a);
    else hipLaunchKernelGGL(train_kernel<3>, dim3(grid), dim3(64), lds, s, g, a);
    if (backward) {
        // rows are summed in 32 interleaved groups, each group's sums added to
        // the gradient with atomics
        const int ry = std::min(grid, 32);
        hipLaunchKernelGGL(reduce_partials, dim3((a.n_frag / 4 + 255) / 256, ry), dim3(256), 0, s,
                           (const float*)a.partials, grid, a.n_frag, fm, grad + gd->n_grid);
        const size_t sl = sizeof(unsigned long long) * 2 * (size_t)kSliceEntries;
        const dim3 sg((unsigned)st.first[st.n]);
        if (g.dim == 2)
            hipLaunchKernelGGL(slice_scatter_kernel<2>, sg, dim3(kSliceThreads), sl, s, g, (const float*)a.rec, a.cap,
                               a.begin, a.count, (const float*)a.gco, (const uint32_t*)a.gmax, st, grad, slice_part);
        else
            hipLaunchKernelGGL(slice_scatter_kernel<3>, sg, dim3(kSliceThreads), sl, s, g, (const float*)a.rec, a.cap,
                               a.begin, a.count, (const float*)a.gco, (const uint32_t*)a.gmax, st, grad, slice_part);
        const int64_t rf = slice_reduce_floats(st);
        if (rf > 0)
            hipLaunchKernelGGL(slice_reduce_kernel, dim3((unsigned)((rf + 255) / 256)), dim3(256), 0, s, g, st,
                               (const float*)slice_part, grad);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error("guide training: launch failed: %s", hipGetErrorString(e)); return WOST_EHIP; }
    return WOST_OK;
}

}  // namespace wost

using namespace wost;

extern "C" int64_t wost_guide_train_workspace_bytes(const wost_guide* g, int64_t count)
{
    if (!g || count < 0) return -1;
    return train_ws_partials(g, count) + ((int64_t)2 * g->dev.L * count * 4 + 255) / 256 * 256 + 256 +
           slice_partial_bytes(slice_table(g->dev, count)) + 256;
}

extern "C" int wost_tail_pass(int32_t dim, const wost_records* rec, const float* walk_value, int64_t n_slots,
                              void* stream)
{
    if ((dim != 2 && dim != 3) || !rec || !rec->data || !rec->count || !walk_value) {
        set_error("wost_tail_pass: bad arguments");
        return WOST_EINVAL;
    }
    if (rec->capacity == 0) return WOST_OK;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(tail_pass_kernel, dim3((unsigned)((rec->capacity + 255) / 256)), dim3(256), 0, s, rec->data,
                       rec->capacity, (const unsigned long long*)rec->count, dim, walk_value, n_slots);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error("wost_tail_pass: %s", hipGetErrorString(e)); return WOST_EHIP; }
    return WOST_OK;
}

extern "C" int wost_records_sample(int32_t dim, const wost_records* src, uint64_t seed, int64_t m,
                                   const wost_records* dst, void* stream)
{
    if ((dim != 2 && dim != 3) || !src || !src->data || !src->count || !dst || !dst->data || !dst->count || m < 0) {
        set_error("wost_records_sample: bad arguments");
        return WOST_EINVAL;
    }
    if (m > dst->capacity) {
        set_error("wost_records_sample: %lld rows do not fit the destination (%lld)", (long long)m,
                  (long long)dst->capacity);
        return WOST_ESIZE;
    }
    hipStream_t s = (hipStream_t)stream;
    if (m > 0 && src->capacity > 0)
        hipLaunchKernelGGL(records_sample_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, src->data,
                           src->capacity, (const unsigned long long*)src->count, 3 * dim + 5, dst->data, dst->capacity,
                           m, (uint32_t)seed, (uint32_t)(seed >> 32));
    // the destination holds m rows (zero if the source is empty: the rows
    // are then left unwritten and must not be trained on)
    hipLaunchKernelGGL(set_count_kernel, dim3(1), dim3(64), 0, s, (unsigned long long*)dst->count,
                       (const unsigned long long*)src->count, (unsigned long long)m);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error("wost_records_sample: %s", hipGetErrorString(e)); return WOST_EHIP; }
    return WOST_OK;
}

extern "C" int wost_guide_loss_fwd(const wost_guide* g, const wost_records* rec, int64_t begin, int64_t count,
                                   float e_mis, float* loss_out, void* stream)
{
    if (!g || !loss_out) { set_error("wost_guide_loss_fwd: NULL argument"); return WOST_EINVAL; }
    return launch_train(g, rec, begin, count, e_mis, 1.f, nullptr, loss_out, nullptr, 0.f, nullptr, nullptr, 0, false,
                        (hipStream_t)stream);
}

extern "C" int wost_guide_loss_bwd(const wost_guide* g, const wost_records* rec, int64_t begin, int64_t count,
                                   float e_mis, float scale, const float* dloss, float* grad, void* workspace,
                                   int64_t ws_bytes, void* stream)
{
    if (!g) { set_error("wost_guide_loss_bwd: NULL guide"); return WOST_EINVAL; }
    float* gr = grad ? grad : g->grad;
    return launch_train(g, rec, begin, count, e_mis, scale, dloss, nullptr, nullptr, 0.f, gr, workspace, ws_bytes, true,
                        (hipStream_t)stream);
}

extern "C" int wost_guide_adam_step(wost_guide* g, const wost_adam* opt, void* stream)
{
    if (!g || !opt) { set_error("wost_guide_adam_step: NULL argument"); return WOST_EINVAL; }
    if (!g->master || !g->adam_m || !g->adam_v || !g->grad) { set_error("wost_guide_adam_step: Adam state not bound"); return WOST_ESTATE; }
    g->adam_step += 1;
    const double t = (double)g->adam_step;
    const double b1 = opt->beta1, b2 = opt->beta2;
    const double c1 = 1.0 - std::pow(b1, t), c2 = 1.0 - std::pow(b2, t);
    const float lr_t = (float)(opt->lr * std::sqrt(c2) / c1);
    const float eps_t = (float)(opt->eps * std::sqrt(c2));
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = g->n_params;
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g->master, g->adam_m,
                       g->adam_v, g->grad, n, lr_t, opt->beta1, opt->beta2, eps_t);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error("wost_guide_adam_step: %s", hipGetErrorString(e)); return WOST_EHIP; }
    return wost_guide_sync_shadow(g, stream);
}

extern "C" int wost_guide_train_step(wost_guide* g, const wost_records* rec, int64_t begin, int64_t count,
                                     const wost_adam* opt, float* loss_out, void* workspace, int64_t ws_bytes,
                                     void* stream)
{
    if (!g || !opt) { set_error("wost_guide_train_step: NULL argument"); return WOST_EINVAL; }
    if (!g->grad || !g->adam_m || !g->adam_v) { set_error("wost_guide_train_step: training state not bound"); return WOST_ESTATE; }
    if (count <= 0) return WOST_OK;
    hipStream_t s = (hipStream_t)stream;
    if (loss_out) hipLaunchKernelGGL(zero_f32_t, dim3(1), dim3(64), 0, s, loss_out, (int64_t)1);
    int rc = launch_train(g, rec, begin, count, opt->e_mis, 1.f / (float)count, nullptr, nullptr, loss_out,
                          1.f / (float)count, g->grad, workspace, ws_bytes, true, s);
    if (rc != WOST_OK) return rc;
    return wost_guide_adam_step(g, opt, stream);
}

// ---------------------------------------------------------------- allocation-free training step
namespace wost {

// Workspace of wost_guide_train_step_noalloc: the per-workgroup weight-gradient
// partials, the per-record feature-gradient staging, the per-level gradient
// maxima and the partial slices of one training step.  It is a device-side
// array; its name in host code is not a device address, so the host uses the
// address hipGetSymbolAddress returns for the current device.  Every device
// that loads the library holds its own copy until the process ends, and every
// call on a device reuses that device's copy (the kernels overwrite what they
// read: each workgroup clears its own partial row, every record writes its
// staging entries, the maxima are cleared before the step and every partial
// slice is written whole).
static __device__ __align__(256) unsigned char scratch[WOST_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxScratchDevices = 64;
static void* g_scratch_addr[kMaxScratchDevices];
static std::mutex g_scratch_mu;

// address of `scratch` on the current device, looked up once per device
static int scratch_address(void** out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxScratchDevices) {
        set_error("wost_guide_train_step_noalloc: no usable current device (%d)", dev);
        return WOST_EHIP;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error("wost_guide_train_step_noalloc: scratch address on device %d: %s", dev, hipGetErrorString(e));
            return WOST_EHIP;
        }
        g_scratch_addr[dev] = p;
    }
    *out = g_scratch_addr[dev];
    return WOST_OK;
}

}  // namespace wost

extern "C" int wost_guide_train_step_noalloc(wost_guide* g, const wost_records* rec, int64_t begin, int64_t count,
                                             const wost_adam* opt, float* loss_out, void* stream)
{
    if (!g || !opt) { set_error("wost_guide_train_step_noalloc: NULL argument"); return WOST_EINVAL; }
    if (count < 0) { set_error("wost_guide_train_step_noalloc: negative record count"); return WOST_EINVAL; }
    const int64_t need = wost_guide_train_workspace_bytes(g, count);
    if (need < 0 || need > (int64_t)WOST_NOALLOC_SCRATCH_BYTES) {
        set_error("wost_guide_train_step_noalloc: %lld records need %lld bytes of workspace, above the %lld-byte "
                  "library scratch; use fewer records per call or wost_guide_train_step",
                  (long long)count, (long long)need, (long long)WOST_NOALLOC_SCRATCH_BYTES);
        return WOST_ESIZE;
    }
    void* ws = nullptr;
    const int rc = scratch_address(&ws);
    if (rc != WOST_OK) return rc;
    return wost_guide_train_step(g, rec, begin, count, opt, loss_out, ws, (int64_t)WOST_NOALLOC_SCRATCH_BYTES, stream);
}
