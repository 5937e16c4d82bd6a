// Row sum of one lane over a column-major SELL chunk (64 ordered rows,
// entry k of lane l at base + k * 64): the products of entries k < len, in
// order k = 0, 1, ..., accumulated in AT.  Entries are fetched U at a time
// (all loads of a group before its products).  Padding (k >= len)
// contributes nothing, by a select, so a non-finite x entry never reaches
// another row.
#pragma once
#include "internal.h"

namespace xab {

template <class VT, class XT, class AT, int U>
__device__ __forceinline__ AT sell_lane_sum(const VT *__restrict__ val, const int32_t *__restrict__ cols,
                                            const XT *__restrict__ x, int64_t base, int32_t w, int32_t len) {
    constexpr int C = xab_plan::kSellC;
    AT acc = AT(0);
    int32_t k = 0;
    for (; k + U <= w; k += U) {
        VT v[U];
        int32_t c[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            v[u] = __builtin_nontemporal_load(val + base + (int64_t)(k + u) * C);
            c[u] = __builtin_nontemporal_load(cols + base + (int64_t)(k + u) * C);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const AT p = (AT)v[u] * (AT)x[c[u]];
            acc = k + u < len ? acc + p : acc;
        }
    }
    for (; k < w; ++k) {
        const VT v = __builtin_nontemporal_load(val + base + (int64_t)k * C);
        const int32_t c = __builtin_nontemporal_load(cols + base + (int64_t)k * C);
        const AT p = (AT)v * (AT)x[c];
        acc = k < len ? acc + p : acc;
    }
    return acc;
}

}  // namespace xab
