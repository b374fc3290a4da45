// Checks the persistent plan's row-tile partition against an exhaustive dynamic program:
// over random work profiles, partition counts and row-tile limits, the partition must
// cover the row tiles with exactly wpg contiguous parts of 1..L row tiles whose largest
// work equals the DP optimum, and must report "no partition" exactly when none exists.
#include <cstdio>
#include <random>

#include "partition.h"

static int64_t best_bound(const std::vector<int64_t> &cum, int n, int wpg, int L) {
    const int64_t inf = INT64_MAX / 4;
    std::vector<std::vector<int64_t>> dp(wpg + 1, std::vector<int64_t>(n + 1, inf));
    dp[0][0] = 0;
    for (int k = 1; k <= wpg; ++k)
        for (int e = 1; e <= n; ++e)
            for (int a = std::max(0, e - L); a < e; ++a)
                if (dp[k - 1][a] < inf) dp[k][e] = std::min(dp[k][e], std::max(dp[k - 1][a], cum[e] - cum[a]));
    return dp[wpg][n];
}

int main() {
    std::mt19937 rng(12345);
    const int Ls[3] = {2, 4, 8};
    int bad = 0, feasible = 0;
    for (int t = 0; t < 4000; ++t) {
        const int n = 1 + (int)(rng() % 48), wpg = 1 + (int)(rng() % n), L = Ls[rng() % 3];
        std::vector<int64_t> cum(n + 1, 0);
        for (int i = 0; i < n; ++i) cum[i + 1] = cum[i] + 1 + (int64_t)(rng() % 11);
        const std::vector<int32_t> cut = qh::partition_rows(cum, n, wpg, L);
        const int64_t b = best_bound(cum, n, wpg, L);
        if (cut.empty()) {
            if (b < INT64_MAX / 4) { ++bad; std::printf("missed n=%d wpg=%d L=%d\n", n, wpg, L); }
            continue;
        }
        ++feasible;
        if ((int)cut.size() != wpg + 1 || cut[0] != 0 || cut[wpg] != n) { ++bad; continue; }
        int64_t mb = 0;
        for (int w = 0; w < wpg; ++w) {
            const int len = cut[w + 1] - cut[w];
            if (len < 1 || len > L) ++bad;
            mb = std::max(mb, cum[cut[w + 1]] - cum[cut[w]]);
        }
        if (mb != b) { ++bad; std::printf("bound %lld, optimum %lld\n", (long long)mb, (long long)b); }
    }
    std::printf("feasible %d, bad %d\n", feasible, bad);
    return bad != 0 || feasible < 1000;
}
