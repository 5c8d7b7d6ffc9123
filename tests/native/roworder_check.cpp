// Checks the streaming check kernel's row order (csrc/roworder.hip) on one
// graph read from stdin ("m n" then, per row, its degree and bits): it is a
// permutation of the rows, and under a model of the L2 as an LRU cache of the
// last C distinct bits touched (C on the command line, default 8192), rows
// visited in that order find their bits cached more often than in index
// order.  Prints "ok <hit rate in index order> <hit rate in the built order>".
#include <cstdio>
#include <cstdlib>
#include <list>
#include <unordered_map>
#include <vector>

#include "ldpc_internal.h"

static int fail(const char *what) {
    std::printf("FAIL %s\n", what);
    return 1;
}

static double lru_hits(const std::vector<int32_t> &order, const std::vector<int32_t> &rowptr,
                       const std::vector<int32_t> &col, size_t cap) {
    std::list<int32_t> lru;
    std::unordered_map<int32_t, std::list<int32_t>::iterator> where;
    size_t hits = 0, total = 0;
    for (int32_t i : order)
        for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            const int32_t j = col[e];
            ++total;
            auto it = where.find(j);
            if (it != where.end()) {
                ++hits;
                lru.erase(it->second);
            } else if (lru.size() == cap) {
                where.erase(lru.back());
                lru.pop_back();
            }
            lru.push_front(j);
            where[j] = lru.begin();
        }
    return total ? (double)hits / (double)total : 0.0;
}

int main(int argc, char **argv) {
    const size_t cap = argc > 1 ? (size_t)std::atol(argv[1]) : 8192;
    int m, n;
    if (std::scanf("%d %d", &m, &n) != 2) return fail("input");
    std::vector<int32_t> rowptr(m + 1, 0), col;
    for (int i = 0; i < m; ++i) {
        int d;
        if (std::scanf("%d", &d) != 1) return fail("input");
        for (int k = 0; k < d; ++k) {
            int x;
            if (std::scanf("%d", &x) != 1) return fail("input");
            col.push_back(x);
        }
        rowptr[i + 1] = (int32_t)col.size();
    }
    const std::vector<int32_t> ord = ldpc::stream_row_order(rowptr, col, m, n);
    if ((int)ord.size() != m) return fail("size");
    std::vector<char> seen(m, 0);
    for (int32_t i : ord) {
        if (i < 0 || i >= m || seen[i]) return fail("not a permutation");
        seen[i] = 1;
    }
    std::vector<int32_t> nat(m);
    for (int i = 0; i < m; ++i) nat[i] = i;
    std::printf("ok %.4f %.4f\n", lru_hits(nat, rowptr, col, cap), lru_hits(ord, rowptr, col, cap));
    return 0;
}
