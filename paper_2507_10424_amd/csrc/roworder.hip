// Row order of the streaming check kernel (host code, run once per graph at
// build time).
//
// The check kernel reads, for every row of a 64-frame tile, the posteriors of
// the row's bits: 256 bytes per bit (64 frames), 16.6 MB per tile on n = 64800,
// against 4 MB of L2 per XCD.  Rows run in launch order, so a posterior is
// read from the L2 again only if another row of the same bit comes soon
// after.  In the CSR order of an expander graph that is rare: a model of the
// L2 as the last 8,192 bits touched gives 12% hits on the n = 64800 code.
// This order is built greedily: after each row, the next one is, among the
// unplaced rows that share a bit with the last few rows placed, the one with
// the most bits among the recently touched ones (ties to the lower index; no
// candidate: the first unplaced row).  The same model then gives 36%.  The
// streaming path renumbers the rows in this order (so that the messages of
// rows launched together also lie together in memory), while each column's
// sum keeps ascending original check order: every message, syndrome and
// posterior is the same.
#include <cstdint>
#include <vector>

#include "ldpc_internal.h"

namespace ldpc {

std::vector<int32_t> stream_row_order(const std::vector<int32_t> &rowptr, const std::vector<int32_t> &col, int32_t m,
                                      int32_t n) {
    constexpr int64_t kWindow = 8192; // bits touched recently enough to count as cached
    constexpr int kRecent = 8;        // candidates: rows sharing a bit with the last kRecent rows placed
    std::vector<int32_t> cptr(n + 1, 0), crow(col.size());
    for (int32_t j : col) ++cptr[j + 1];
    for (int32_t j = 0; j < n; ++j) cptr[j + 1] += cptr[j];
    {
        std::vector<int32_t> fill(cptr.begin(), cptr.end() - 1);
        for (int32_t i = 0; i < m; ++i)
            for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) crow[fill[col[e]]++] = i;
    }
    std::vector<int64_t> last(n, -((int64_t)1 << 40));
    std::vector<char> placed(m, 0);
    std::vector<int32_t> seen(m, -1), order;
    order.reserve(m);
    int64_t now = 0;
    int32_t first_free = 0;
    for (int32_t step = 0; step < m; ++step) {
        int32_t best = -1, best_score = -1;
        const int32_t lo = step > kRecent ? step - kRecent : 0;
        for (int32_t p = lo; p < step; ++p) {
            const int32_t r = order[p];
            for (int32_t e = rowptr[r]; e < rowptr[r + 1]; ++e) {
                const int32_t j = col[e];
                for (int32_t q = cptr[j]; q < cptr[j + 1]; ++q) {
                    const int32_t i2 = crow[q];
                    if (placed[i2] || seen[i2] == step) continue;
                    seen[i2] = step;
                    int32_t sc = 0;
                    for (int32_t e2 = rowptr[i2]; e2 < rowptr[i2 + 1]; ++e2) sc += last[col[e2]] >= now - kWindow;
                    if (sc > best_score || (sc == best_score && i2 < best)) {
                        best = i2;
                        best_score = sc;
                    }
                }
            }
        }
        if (best < 0) {
            while (placed[first_free]) ++first_free;
            best = first_free;
        }
        placed[best] = 1;
        order.push_back(best);
        for (int32_t e = rowptr[best]; e < rowptr[best + 1]; ++e) last[col[e]] = now++;
    }
    return order;
}

} // namespace ldpc
