// Training loss of one ray and its seeds (the adjoints of the logit and of the distance),
// shared by every kernel that forms seeds so that they agree bit for bit.
//   kind 0 (DDF_LOSS_BCE_L1): binary cross-entropy with logits on the hit flag, mean over
//          the N rays, plus L1 on the distance over the n_hit rays with a label; weights 1:1.
//   kind 1 (DDF_LOSS_CLAMP): the clamp loss of Eq. 7 on the distance alone,
//          |c(t) - c(d)| / N with c the two-sided clamp at delta (a miss clamps to delta).
//   kind 2 (DDF_LOSS_SQUISH): the squish loss of Eq. 6 on the distance alone, with
//          sigma = tanh and the absolute value: |tanh(t) - tanh(d)| / N (tanh(+inf) = 1).
// Seeds of kinds 1 and 2: sign(c(d) - c(t)) c'(d) / N (c' = 1 strictly inside the clamp
// window, 0 outside and on its edges; 1 - tanh^2 for the squish), no logit gradient.
#pragma once
#include <cmath>

namespace ddf {

struct LossSpec {
    int kind;      // 0, 1, 2 as above
    float delta;   // clamp window (kind 1)
};

// Returns the ray's term of the loss and sets the seeds; inv_n = 1 / N, inv_nhit = 1 / n_hit.
__device__ inline float ray_loss(float z, float d, float t, float inv_n, float inv_nhit, LossSpec ls, float &gl,
                                 float &gd) {
    if (ls.kind == 0) {
        const float y = t < INFINITY ? 1.f : 0.f;
        const float sig = 1.f / (1.f + expf(-z));
        gl = (sig - y) * inv_n;
        const float diff = d - (y > 0.f ? t : 0.f);
        gd = y > 0.f ? (diff > 0.f ? inv_nhit : (diff < 0.f ? -inv_nhit : 0.f)) : 0.f;
        return (fmaxf(z, 0.f) - z * y + log1pf(expf(-fabsf(z)))) * inv_n + y * fabsf(diff) * inv_nhit;
    }
    float cd, ct, dc;
    if (ls.kind == 1) {
        cd = fminf(ls.delta, fmaxf(-ls.delta, d));
        ct = fminf(ls.delta, fmaxf(-ls.delta, t));
        dc = (d > -ls.delta && d < ls.delta) ? 1.f : 0.f;
    } else {
        cd = tanhf(d);
        ct = t < INFINITY ? tanhf(t) : 1.f;
        dc = 1.f - cd * cd;
    }
    const float diff = cd - ct;
    gl = 0.f;
    gd = (diff > 0.f ? inv_n : (diff < 0.f ? -inv_n : 0.f)) * dc;
    return fabsf(diff) * inv_n;
}

}  // namespace ddf
