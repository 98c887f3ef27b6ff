// Input t of the learned search range's network from the raw state after
// the probe expansions: distances as log(d + c) (c = 1e-3 for cosine, 1 for
// squared L2), all but the nearest seed's taken relative to it; the two
// counts (|S| and the distance computations) as log(1 + n).  One definition
// for the fused predictor of the search and the standalone transform kernel.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/onng.h"

namespace onng {

// f: raw feature t; f0: raw feature 0 (the nearest seed's distance)
__device__ __forceinline__ float feature_input(int t, float f, float f0, int metric) {
    if (t == 8 || t == 13) return log1pf(f);
    const float c = metric == ONNG_COSINE ? 1e-3f : 1.0f;
    const float lg = logf(fmaxf(f, 0.0f) + c);
    if (t == 0) return lg;
    return lg - logf(fmaxf(f0, 0.0f) + c);
}

}  // namespace onng
