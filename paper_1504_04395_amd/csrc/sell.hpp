// SELL-C-sigma storage of a CSR pattern, built on the host at matrix set-up.
//
// Rows are stably sorted by length, longest first, inside consecutive windows
// of sigma rows.  Consecutive sorted positions form chunks of C rows.  A chunk
// is stored column-major (slot k of its row r at cptr[ch] + k * C + r) and
// padded to its longest row.  `row` maps a sorted position back to its row of
// A.  `idx` is the CSR position of each slot (-1 for padding), through which
// the device copies the values; a padding slot has value 0 and points at the
// row's own column, so its product term is an exact zero.
//
// Plain C++: the library and the CPU test harness both build it.
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <vector>

namespace skr {

struct HostSell {
    std::vector<int> cptr, clen, row, ci, idx;
};

// false (and `out` unspecified) when the layout would need 2^31 or more
// slots, since slot offsets are int32 on the device
inline bool build_sell(int n, const std::vector<int>& rp, const std::vector<int>& ci, int C, int sigma,
                       HostSell& out) {
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    for (int w0 = 0; w0 < n; w0 += sigma) {
        const int w1 = std::min(n, w0 + sigma);
        std::stable_sort(order.begin() + w0, order.begin() + w1, [&](int a, int b) {
            return (rp[a + 1] - rp[a]) > (rp[b + 1] - rp[b]);
        });
    }
    const int nch = (n + C - 1) / C;
    out.cptr.assign(nch + 1, 0);
    out.clen.assign(nch, 0);
    out.row = order;
    size_t off = 0;
    for (int ch = 0; ch < nch; ++ch) {
        int w = 0;
        for (int r = 0; r < C && ch * C + r < n; ++r) {
            const int i = order[ch * C + r];
            w = std::max(w, rp[i + 1] - rp[i]);
        }
        out.clen[ch] = w;
        out.cptr[ch] = (int)off;
        off += (size_t)w * C;
        if (off > (size_t)INT32_MAX) return false;
    }
    out.cptr[nch] = (int)off;
    out.ci.assign(off, 0);
    out.idx.assign(off, -1);
    for (int ch = 0; ch < nch; ++ch) {
        for (int r = 0; r < C; ++r) {
            const int p = ch * C + r;
            const int i = p < n ? order[p] : 0;
            const int len = p < n ? rp[i + 1] - rp[i] : 0;
            for (int k = 0; k < out.clen[ch]; ++k) {
                const size_t e = (size_t)out.cptr[ch] + (size_t)k * C + r;
                if (k < len) {
                    out.ci[e] = ci[rp[i] + k];
                    out.idx[e] = rp[i] + k;
                } else {
                    out.ci[e] = i;
                }
            }
        }
    }
    return true;
}

}  // namespace skr
