// Row-tile partition of the persistent plan (host code; no HIP dependency, so that the
// CPU tests compile it on its own).
#pragma once

#include <algorithm>
#include <cstdint>
#include <vector>

namespace qh {

// Contiguous partition of the row tiles into exactly `wpg` parts of 1..L row tiles each
// that minimises the largest part's work (cum = prefix sums of the per-row-tile work):
// binary search on that bound, each bound checked by greedy packing (extending a part as
// far as both limits allow needs the fewest parts); then the heaviest parts with two or
// more row tiles are split at their balance point until there are wpg parts (a split
// never raises the bound).  Returns the wpg + 1 cut points, or nothing when no such
// partition exists.
inline std::vector<int32_t> partition_rows(const std::vector<int64_t> &cum, int64_t n_rt, int wpg, int L) {
    if (wpg < 1 || n_rt < wpg || (n_rt + wpg - 1) / wpg > L) return {};
    std::vector<int32_t> cut;
    auto pack = [&](int64_t B) -> bool {
        cut.assign(1, 0);
        int64_t cur = 0;
        while (cur < n_rt) {
            int64_t e = cur + 1;
            if (cum[e] - cum[cur] > B) return false;
            while (e < n_rt && e - cur < L && cum[e + 1] - cum[cur] <= B) ++e;
            cut.push_back((int32_t)e);
            cur = e;
            if ((int64_t)cut.size() - 1 > wpg) return false;
        }
        return true;
    };
    int64_t lo = 0, hi = cum[n_rt];
    for (int64_t rt = 0; rt < n_rt; ++rt) lo = std::max(lo, cum[rt + 1] - cum[rt]);
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (pack(mid)) hi = mid;
        else lo = mid + 1;
    }
    if (!pack(lo)) return {};
    while ((int64_t)cut.size() - 1 < wpg) {
        int best = -1;
        int64_t bw = -1;
        for (int q = 0; q + 1 < (int)cut.size(); ++q)
            if (cut[q + 1] - cut[q] >= 2 && cum[cut[q + 1]] - cum[cut[q]] > bw) {
                bw = cum[cut[q + 1]] - cum[cut[q]];
                best = q;
            }
        if (best < 0) return {};
        const int64_t a = cut[best], b = cut[best + 1];
        int64_t at = a + 1, av = -1;
        for (int64_t m = a + 1; m < b; ++m) {
            const int64_t v = std::max(cum[m] - cum[a], cum[b] - cum[m]);
            if (av < 0 || v < av) { av = v; at = m; }
        }
        cut.insert(cut.begin() + best + 1, (int32_t)at);
    }
    return cut;
}

}  // namespace qh
