// Per-step device helpers of the walk: Philox stream, analytic fields, Green's
// function of the ball, uniform directions.
#pragma once

#include "wost_internal.h"

namespace wost {

constexpr float kPi = 3.14159265358979323846f;

// Philox4x32-10 (Salmon et al., SC'11), from its published definition.
__device__ __forceinline__ uint4 philox(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// 32-bit word -> uniform float in [0, 1) with 24 random bits (exact in FP32)
__device__ __forceinline__ float u01(uint32_t w) { return (float)(w >> 8) * 5.9604644775390625e-08f; }

// Per-walk stream: counter (point, walk-of-point, step, block), key = seed.
struct Stream {
    uint32_t p, j, k0, k1;
    __device__ __forceinline__ uint4 block(uint32_t step, uint32_t b) const
    {
        return philox(make_uint4(p, j, step, b), k0, k1);
    }
};

// Draw layout per step (shared with the oracle):
//   block 0: direction words (u0, u1), MIS selection, lobe selection
//   block 1: Neumann descent, point on primitive (2 words), roulette
//   block 2: source radius (3 words), source direction word 0
//   block 3: source direction word 1, 3D vMF eta, 3D vMF azimuth, unused
//   block 4+i: 2D von Mises rejection iteration i (U1, U2, U3)
enum : uint32_t { kBlkDir = 0, kBlkNeu = 1, kBlkSrc0 = 2, kBlkSrc1 = 3, kBlkVm = 4 };

template <int D>
__device__ __forceinline__ float field_value(const FieldDev& f, const float* x)
{
    switch (f.kind) {
    case WOST_FIELD_CONST: return f.p[0];
    case WOST_FIELD_EXP_SIN: return expf(x[0]) * sinf(x[1]);
    case WOST_FIELD_RE_Z3: return x[0] * (x[0] * x[0] - 3.f * x[1] * x[1]);
    case WOST_FIELD_X2_MINUS_Y2: return x[0] * x[0] - x[1] * x[1];
    case WOST_FIELD_R2: {
        float s = 0.f;
#pragma unroll
        for (int i = 0; i < D; ++i) s = fmaf(x[i], x[i], s);
        return s;
    }
    case WOST_FIELD_GAUSS_SUM: {
        float s = 0.f;
        for (int j = 0; j < f.n; ++j) {
            const float* row = f.p + j * (2 + D);
            float d2 = 0.f;
#pragma unroll
            for (int i = 0; i < D; ++i) { const float t = x[i] - row[2 + i]; d2 = fmaf(t, t, d2); }
            s = fmaf(row[0], expf(-d2 / (2.f * row[1] * row[1])), s);
        }
        return s;
    }
    default: return 0.f;
    }
}

// outward normal derivative for the Neumann data
template <int D>
__device__ __forceinline__ float neumann_value(const FieldDev& h, const float* z, const float* n_out)
{
    float g[3] = {0.f, 0.f, 0.f};
    switch (h.kind) {
    case WOST_FIELD_CONST: return h.p[0];
    case WOST_FIELD_EXP_SIN: { const float e = expf(z[0]); g[0] = e * sinf(z[1]); g[1] = e * cosf(z[1]); break; }
    case WOST_FIELD_RE_Z3: g[0] = 3.f * (z[0] * z[0] - z[1] * z[1]); g[1] = -6.f * z[0] * z[1]; break;
    case WOST_FIELD_X2_MINUS_Y2: g[0] = 2.f * z[0]; g[1] = -2.f * z[1]; break;
    case WOST_FIELD_R2:
#pragma unroll
        for (int i = 0; i < D; ++i) g[i] = 2.f * z[i];
        break;
    default: return 0.f;
    }
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < D; ++i) s = fmaf(g[i], n_out[i], s);
    return s;
}

// Green's function of the ball B(x, r) with zero boundary values, -Lap G = delta
template <int D>
__device__ __forceinline__ float green_ball(float r, float rho)
{
    if (D == 2) return logf(r / rho) * (1.f / (2.f * kPi));
    return (1.f / rho - 1.f / r) * (1.f / (4.f * kPi));
}

template <int D>
__device__ __forceinline__ void uniform_dir(float u0, float u1, float* nu)
{
    if (D == 2) {
        float s, c;
        sincospif(2.f * u0, &s, &c);
        nu[0] = c; nu[1] = s;
    } else {
        const float z = 1.f - 2.f * u0;
        const float rr = sqrtf(fmaxf(0.f, 1.f - z * z));
        float s, c;
        sincospif(2.f * u1, &s, &c);
        nu[0] = rr * c; nu[1] = rr * s; nu[2] = z;
    }
}

}  // namespace wost
