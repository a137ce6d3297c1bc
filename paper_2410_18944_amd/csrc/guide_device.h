// Guide network and guided direction draw on gfx950.
//
// Network (Sec. 5.2): x -> multi-resolution grid G(x) (L levels x F=2 features,
// bilinear / trilinear interpolation; hashed levels where the dense lattice
// does not fit the table) -> bias-free ReLU MLP of width 64 -> K(d+2)+1 raw
// outputs, mapped by Tab. "reg_map": mu = mu'/|mu'|, kappa = exp(kappa'),
// lambda = softmax(lambda'), c = sigmoid(c').
//
// Evaluation is per wavefront on MFMA (v_mfma_f32_16x16x16_f16) in the
// transposed form H^T_{l+1} = relu(W_l^T H^T_l): the batch of 64 walks is the
// N dimension (four 16-column blocks).  With the 16x16x16 layouts
//   A[m][k]: lane l holds m = l%16, k = 4(l/16)+i
//   B[k][n]: lane l holds k = 4(l/16)+i, n = l%16
//   D[m][n]: lane l holds m = 4(l/16)+i, n = l%16
// the D fragment of one layer (rows = output features) is, after ReLU and the
// fp16 conversion, exactly the B fragment of the next layer's K block, so the
// activations never leave registers.  Weights are stored pre-swizzled as A
// fragments (8 contiguous bytes per lane).  The last layer's D fragments are
// transposed through LDS so each lane reads its own walk's outputs.
#pragma once

#include "geom_device.h"
#include "walk_common.h"

namespace wost {

typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));
typedef _Float16 half8_t __attribute__((ext_vector_type(8)));

// c += A B over two 16-deep blocks of K at once.  The 16x16x32 FP16 MFMA pairs
// element j of an A lane with element j of the B lanes of the same 16-lane
// group, like the 16x16x16 form does for its four elements; handing it the
// two 16-deep operand pairs of a lane side by side therefore adds exactly the
// two 16x16x16 products, in one instruction.
__device__ __forceinline__ float4_t mfma_k32(const half8_t& a, const half8_t& b, const float4_t& c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ float4_t mfma_k16(const half4_t& a, const half4_t& b, const float4_t& c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ half4_t half_lo(const half8_t& v) { return {v[0], v[1], v[2], v[3]}; }
__device__ __forceinline__ half4_t half_hi(const half8_t& v) { return {v[4], v[5], v[6], v[7]}; }

// writes h into the low (hi = 0) or high four elements of v
__device__ __forceinline__ void put_half(half8_t& v, int hi, const half4_t& h)
{
    if (hi) {
        v[4] = h[0]; v[5] = h[1]; v[6] = h[2]; v[7] = h[3];
    } else {
        v[0] = h[0]; v[1] = h[1]; v[2] = h[2]; v[3] = h[3];
    }
}

// Operand fragment layout of one layer (in units of one lane's four halves):
// block (mb, kb) of a layer with KB blocks along K.  The blocks 2j and 2j + 1
// of a row block are interleaved lane by lane, so a lane reads both with one
// 16-byte load; an unpaired last block keeps 64 consecutive fragments.
__host__ __device__ __forceinline__ int frag_index(int mb, int kb, int KB, int lane)
{
    return ((kb | 1) < KB) ? (mb * KB + (kb & ~1)) * 64 + 2 * lane + (kb & 1) : (mb * KB + kb) * 64 + lane;
}

// A x B over K = 16 KB for the 16x16 output block mb: B is held as pairs of
// 16-deep fragments (pair p = blocks 2p, 2p + 1), at most four blocks.
__device__ __forceinline__ float4_t mfma_row_block(const half4_t* A, int mb, int KB, int lane, const half8_t* b,
                                                   float4_t c)
{
#pragma unroll
    for (int kb = 0; kb < 4; kb += 2) {
        if (kb + 1 < KB)
            c = mfma_k32(*(const half8_t*)(A + frag_index(mb, kb, KB, lane)), b[kb >> 1], c);
        else if (kb < KB)
            c = mfma_k16(A[frag_index(mb, kb, KB, lane)], half_lo(b[kb >> 1]), c);
    }
    return c;
}

constexpr int kMaxLevels = 16;
constexpr int kMaxLayers = 6;
constexpr int kHidden = 64;
constexpr int kMaxOutPad = 96;
constexpr float kKappaLogMin = -10.f;
constexpr float kKappaLogMax = 9.f;
constexpr float kCLogit = 15.f;     // |c'| clamp: keeps 1 - c representable in FP32

struct GuideDev {
    const uint32_t* grid;       // fp16 pairs [L][T]
    const half4_t* frags;       // swizzled MLP A fragments
    int32_t frag_off[kMaxLayers];  // forward (W^T) fragment offset per layer, in half4 units
    int32_t bfrag_off[kMaxLayers]; // backward (W) fragment offset per layer, in half4 units
    int32_t kb[kMaxLayers];     // K blocks (in / 16)
    int32_t mb[kMaxLayers];     // M blocks (out_padded / 16)
    int32_t n_layers;
    int32_t dim, L, log2T, K, n_out, out_pad;
    int32_t res[kMaxLevels];
    int32_t dense[kMaxLevels];
    float lo[3], inv_ext[3];
    int32_t sampling;
    float c_fixed;
    int32_t reflect;
};

// row stride (floats) of the per-walk raw outputs in LDS: the outputs
// themselves, rounded up to an odd count so the 64 rows fall in distinct banks
__host__ __device__ inline int guide_out_stride(const GuideDev& g) { return g.n_out | 1; }

struct RecDev {
    float* data;
    int64_t capacity;
    unsigned long long* count;
};

// ---------------------------------------------------------------- encoding

__device__ __forceinline__ float2 unpack_h2(uint32_t w)
{
    union { uint32_t u; _Float16 h[2]; } c;
    c.u = w;
    return make_float2((float)c.h[0], (float)c.h[1]);
}

// F=2 features of level l at normalised position xh (in [0,1]^D)
template <int D>
__device__ __forceinline__ float2 grid_level(const GuideDev& g, int l, const float* xh)
{
    const int N = g.res[l];
    const uint32_t* tab = g.grid + ((size_t)l << g.log2T);
    const uint32_t mask = (1u << g.log2T) - 1u;
    int c[D];
    float fr[D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
        const float pos = xh[i] * (float)N;
        int ci = (int)floorf(pos);
        ci = min(max(ci, 0), N - 1);
        c[i] = ci;
        fr[i] = pos - (float)ci;
    }
    float2 acc = make_float2(0.f, 0.f);
    const bool dense = g.dense[l] != 0;
#pragma unroll
    for (int corner = 0; corner < (1 << D); ++corner) {
        float w = 1.f;
        uint32_t idx;
        if (dense) {
            uint32_t stride = 1;
            idx = 0;
#pragma unroll
            for (int i = 0; i < D; ++i) {
                const int b = (corner >> i) & 1;
                w *= b ? fr[i] : 1.f - fr[i];
                idx += (uint32_t)(c[i] + b) * stride;
                stride *= (uint32_t)(N + 1);
            }
        } else {
            const uint32_t primes[3] = {1u, 2654435761u, 805459861u};
            idx = 0;
#pragma unroll
            for (int i = 0; i < D; ++i) {
                const int b = (corner >> i) & 1;
                w *= b ? fr[i] : 1.f - fr[i];
                idx ^= (uint32_t)(c[i] + b) * primes[i];
            }
            idx &= mask;
        }
        const float2 f = unpack_h2(tab[idx]);
        acc.x = fmaf(w, f.x, acc.x);
        acc.y = fmaf(w, f.y, acc.y);
    }
    return acc;
}

template <int D>
__device__ __forceinline__ void normalise_input(const GuideDev& g, const float* x, float* xh)
{
#pragma unroll
    for (int i = 0; i < D; ++i) xh[i] = fminf(fmaxf((x[i] - g.lo[i]) * g.inv_ext[i], 0.f), 1.f);
}

// ---------------------------------------------------------------- MLP on MFMA

// Evaluates the network for the 64 walks of the wave (positions x per lane;
// every lane participates) and leaves raw outputs in LDS: out[lane][j].
template <int D>
__device__ void guide_forward_wave(const GuideDev& g, const float* x, float* lds_out, int lane, int stride)
{
    const int g4 = lane >> 4;       // 16-lane group
    const int col = lane & 15;      // column within a block
    for (int cb = 0; cb < 4; ++cb) {
        // this lane encodes walk w = 16 cb + col, features k = 16 kb + 4 g4 + i
        const int w = 16 * cb + col;
        float xw[D], xh[D];
#pragma unroll
        for (int i = 0; i < D; ++i) xw[i] = __shfl(x[i], w);
        normalise_input<D>(g, xw, xh);
        half8_t act[2];
        const int kb0 = g.kb[0];
        // every loop over the four 16-feature blocks is unrolled with a guard,
        // so the activation fragments stay in registers
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
            if (kb >= kb0) break;
            const int l0 = 8 * kb + 2 * g4;
            const float2 f0 = grid_level<D>(g, l0, xh);
            const float2 f1 = grid_level<D>(g, l0 + 1, xh);
            half4_t h;
            h[0] = (_Float16)f0.x; h[1] = (_Float16)f0.y; h[2] = (_Float16)f1.x; h[3] = (_Float16)f1.y;
            put_half(act[kb >> 1], kb & 1, h);
        }
        // hidden layers
        for (int layer = 0; layer + 1 < g.n_layers; ++layer) {
            const half4_t* A = g.frags + g.frag_off[layer];
            const int KB = g.kb[layer];
            half8_t nxt[2];
#pragma unroll
            for (int mb = 0; mb < 4; ++mb) {
                const float4_t c = mfma_row_block(A, mb, KB, lane, act, float4_t{0.f, 0.f, 0.f, 0.f});
                half4_t h;
#pragma unroll
                for (int i = 0; i < 4; ++i) h[i] = (_Float16)fmaxf(c[i], 0.f);
                put_half(nxt[mb >> 1], mb & 1, h);
            }
            act[0] = nxt[0];
            act[1] = nxt[1];
        }
        // output layer -> LDS, transposed to [walk][output]
        {
            const int layer = g.n_layers - 1;
            const half4_t* A = g.frags + g.frag_off[layer];
            const int KB = g.kb[layer];
            for (int mb = 0; mb < g.mb[layer]; ++mb) {
                const float4_t c = mfma_row_block(A, mb, KB, lane, act, float4_t{0.f, 0.f, 0.f, 0.f});
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int j = 16 * mb + 4 * g4 + i;
                    if (j < g.n_out) lds_out[w * stride + j] = c[i];
                }
            }
        }
    }
}

// ---------------------------------------------------------------- vMF pieces

// log of the vMF normaliser: v(nu) = exp(kappa (mu.nu - 1) + lognorm)
// 2D: -log(2 pi I0e(kappa)) with I0e by Abramowitz & Stegun 9.8.1-9.8.2
// 3D: log(kappa / (2 pi (1 - e^{-2 kappa})))
__device__ __forceinline__ float i0e_f(float k)
{
    if (k <= 3.75f) {
        const float t = (k / 3.75f) * (k / 3.75f);
        const float i0 = 1.f + t * (3.5156229f + t * (3.0899424f + t * (1.2067492f + t * (0.2659732f + t * (0.0360768f + t * 0.0045813f)))));
        return i0 * expf(-k);
    }
    const float t = 3.75f / k;
    const float p = 0.39894228f + t * (0.01328592f + t * (0.00225319f + t * (-0.00157565f + t * (0.00916281f + t * (-0.02057706f + t * (0.02635537f + t * (-0.01647633f + t * 0.00392377f)))))));
    return p * rsqrtf(k);
}

// I1e by Abramowitz & Stegun 9.8.3-9.8.4
__device__ __forceinline__ float i1e_f(float k)
{
    if (k <= 3.75f) {
        const float t = (k / 3.75f) * (k / 3.75f);
        const float i1 = k * (0.5f + t * (0.87890594f + t * (0.51498869f + t * (0.15084934f + t * (0.02658733f + t * (0.00301532f + t * 0.00032411f))))));
        return i1 * expf(-k);
    }
    const float t = 3.75f / k;
    const float p = 0.39894228f + t * (-0.03988024f + t * (-0.00362018f + t * (0.00163801f + t * (-0.01031555f + t * (0.02282967f + t * (-0.02895312f + t * (0.01787654f - t * 0.00420059f)))))));
    return p * rsqrtf(k);
}

template <int D>
__device__ __forceinline__ float vmf_lognorm(float k)
{
    if (D == 2) return -logf(2.f * kPi * i0e_f(k));
    return logf(k) - logf(2.f * kPi) - logf(-expm1f(-2.f * k));
}

// One lobe of a lane's raw-output row, mapped per Tab. reg_map: unit mean
// (mu' normalised), concentration exp(kappa') with kappa' clamped.  Lobes are
// read from the row one at a time, so no per-lane lobe arrays are kept.
template <int D>
struct Lobe {
    float mu[D];
    float kappa;
};

template <int D>
__device__ __forceinline__ Lobe<D> lobe_at(const float* y, int i)
{
    const float* r = y + i * (D + 2);
    Lobe<D> l;
    float n2 = 0.f;
#pragma unroll
    for (int d = 0; d < D; ++d) n2 = fmaf(r[d], r[d], n2);
    const float inv = n2 > 0.f ? rsqrtf(n2) : 0.f;
#pragma unroll
    for (int d = 0; d < D; ++d) l.mu[d] = n2 > 0.f ? r[d] * inv : (d == 0 ? 1.f : 0.f);
    l.kappa = expf(fminf(fmaxf(r[D], kKappaLogMin), kKappaLogMax));
    return l;
}

// raw mixture logit of lobe i
template <int D>
__device__ __forceinline__ float lobe_logit(const float* y, int i) { return y[i * (D + 2) + D + 1]; }

// Best & Fisher (1979) von Mises angle offset; iteration i uses block 4+i.
__device__ __forceinline__ float von_mises_offset(float k, const Stream& rs, uint32_t step)
{
    const float s4 = sqrtf(1.f + 4.f * k * k);
    const float tau = 1.f + s4;
    const float rho = 2.f * k * tau / ((s4 + 1.f) * (tau + sqrtf(2.f * tau)));
    const float r = (1.f + rho * rho) / (2.f * rho);
    for (uint32_t it = 0; it < 64; ++it) {
        const uint4 w = rs.block(step, kBlkVm + it);
        const float u1 = u01(w.x), u2 = u01(w.y), u3 = u01(w.z);
        const float z = cospif(u1);
        const float f = (1.f + r * z) / (r + z);
        const float cc = k * (r - f);
        if (cc * (2.f - cc) > u2 || (u2 > 0.f && logf(cc / u2) + 1.f - cc >= 0.f)) {
            const float psi = acosf(fminf(fmaxf(f, -1.f), 1.f));
            return u3 < 0.5f ? -psi : psi;
        }
    }
    return 0.f;   // not reached in practice (acceptance >= 0.66 per iteration)
}

// orthonormal tangent pair (Duff et al. 2017)
__device__ __forceinline__ void onb(const float* n, float* t1, float* t2)
{
    const float sgn = copysignf(1.f, n[2]);
    const float a = -1.f / (sgn + n[2]);
    const float b = n[0] * n[1] * a;
    t1[0] = 1.f + sgn * n[0] * n[0] * a; t1[1] = sgn * b; t1[2] = -sgn * n[0];
    t2[0] = b; t2[1] = sgn + n[1] * n[1] * a; t2[2] = -n[1];
}

// One MIS draw (Sec. 4.4): with probability c a lobe ~ lambda and a vMF
// sample from it, else uniform; invalid draws on a Neumann boundary are
// reflected about the tangent plane (Sec. 4.3).  Returns nu and the MIS pdf
// c p_g(nu) + (1 - c) p_u(nu) of the direction actually used.  With
// reflection off (g.reflect = 0, the ablation of Sec. 6) p_g on a Neumann
// point is the plain mixture on the valid half, and a guided draw into the
// wall (nu . n <= 0) returns *pmis = -1: its recursive term is zero.
template <int D>
__device__ __forceinline__ void guided_draw(const GuideDev& g, const float* y, const Stream& rs, uint32_t step,
                                            const uint4& wd, bool onN, const float* nin, float* nu, float* pmis)
{
    const int K = g.K;
    // softmax of the mixture logits: lambda_i = exp(l_i - lmax) / lsum
    float lmax = -INFINITY;
    for (int i = 0; i < K; ++i) lmax = fmaxf(lmax, lobe_logit<D>(y, i));
    float lsum = 0.f;
    for (int i = 0; i < K; ++i) lsum += expf(lobe_logit<D>(y, i) - lmax);
    const float il = 1.f / lsum;
    const float craw = y[K * (D + 2)];
    float c;
    if (g.sampling == WOST_SAMPLING_MIS_LEARNED) c = 1.f / (1.f + expf(-fminf(fmaxf(craw, -kCLogit), kCLogit)));
    else if (g.sampling == WOST_SAMPLING_MIS_FIXED) c = g.c_fixed;
    else c = 1.f;
    const bool guided = u01(wd.z) < c;
    if (guided) {
        const float target = u01(wd.w);
        int sel = K - 1;
        float cum = 0.f;
        for (int i = 0; i < K; ++i) {
            cum += expf(lobe_logit<D>(y, i) - lmax) * il;
            if (target < cum) { sel = i; break; }
        }
        const Lobe<D> L = lobe_at<D>(y, sel);
        if (D == 2) {
            const float psi = von_mises_offset(L.kappa, rs, step);
            float s, co;
            sincosf(psi, &s, &co);
            nu[0] = co * L.mu[0] - s * L.mu[1];
            nu[1] = s * L.mu[0] + co * L.mu[1];
        } else {
            const uint4 b3 = rs.block(step, kBlkSrc1);
            const float k = L.kappa;
            const float sm = -log1pf(u01(b3.y) * expm1f(-2.f * k)) / k;
            const float st = sqrtf(fmaxf(0.f, sm * (2.f - sm)));
            float t1[3], t2[3];
            onb(L.mu, t1, t2);
            float sp, cp;
            sincospif(2.f * u01(b3.z), &sp, &cp);
#pragma unroll
            for (int i = 0; i < D; ++i) nu[i] = (1.f - sm) * L.mu[i] + st * (cp * t1[i] + sp * t2[i]);
        }
    } else {
        uniform_dir<D>(u01(wd.x), u01(wd.y), nu);
    }
    const float area = D == 2 ? 2.f * kPi : 4.f * kPi;
    // reflection into the valid hemisphere on a Neumann boundary; the guided
    // density of the used direction then sums the lobes at nu and at its mirror
    float nr[D];
    const bool mirror = onN && g.reflect != 0;
    if (onN) {
        float cn = dot<D>(nu, nin);
        if (guided && !mirror && cn <= 0.f) {
            *pmis = -1.f;
            return;
        }
        if (cn < 0.f) {
#pragma unroll
            for (int i = 0; i < D; ++i) nu[i] = fmaf(-2.f * cn, nin[i], nu[i]);
            cn = -cn;
        }
#pragma unroll
        for (int i = 0; i < D; ++i) nr[i] = fmaf(-2.f * cn, nin[i], nu[i]);
    }
    float pg = 0.f, pr = 0.f;
    for (int i = 0; i < K; ++i) {
        const Lobe<D> L = lobe_at<D>(y, i);
        const float lam = expf(lobe_logit<D>(y, i) - lmax) * il;
        const float ln = vmf_lognorm<D>(L.kappa);
        pg = fmaf(lam, expf(fmaf(L.kappa, dot<D>(L.mu, nu) - 1.f, ln)), pg);
        if (mirror) pr = fmaf(lam, expf(fmaf(L.kappa, dot<D>(L.mu, nr) - 1.f, ln)), pr);
    }
    if (onN) *pmis = c * (pg + pr) + (1.f - c) * (2.f / area);
    else *pmis = c * pg + (1.f - c) * (1.f / area);
}

}  // namespace wost
