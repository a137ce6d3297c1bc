// Host-side guide handle.
#pragma once

#include "guide_device.h"

struct wost_guide {
    wost_guide_config cfg;
    wost::GuideDev dev;             // static part (pointers filled by guide_prepare)
    int64_t n_grid = 0;             // grid parameters (L * T * F)
    int64_t frag_base = 0;          // first MLP fragment half in the shadow (multiple of 8)
    int64_t n_params = 0;           // grid + MLP parameters
    int64_t n_frag_halves = 0;      // swizzled MLP fragment halves in the shadow
    int64_t layer_off[wost::kMaxLayers] = {};
    int32_t layer_in[wost::kMaxLayers] = {};
    int32_t layer_out[wost::kMaxLayers] = {};
    float* master = nullptr;
    void* shadow = nullptr;
    float* adam_m = nullptr;
    float* adam_v = nullptr;
    float* grad = nullptr;
    int64_t adam_step = 0;
};

namespace wost {
int guide_prepare(const wost_guide* g, int dim, GuideDev& out);
}  // namespace wost
