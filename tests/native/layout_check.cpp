// Checks the on-chip decoder's bank-conflict-free layout (csrc/layout.hip)
// on one graph read from stdin ("m n" then, per row, its degree and bits),
// in the geometry given on the command line (rows and bits per thread,
// bit-side stride, column degree profile in hex; default 2 4, the largest
// column degree, no profile): every row slot below m holds a distinct row
// with its own edges, each bit sits in a slot of its own 64-slot block (with
// a profile: in a slot whose profile entry is at least its degree), every
// message has a position of its own,
// the bit-side table lists each bit's messages in ascending check order and
// zero positions past its degree, and no two lanes of a message access
// conflict on the LDS banks (writes: distinct positions modulo 16 per 16
// lanes; reads: distinct words modulo 32 per 32 lanes).  Prints "ok <mean
// max posterior-gather load>" or a failure.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "ldpc_internal.h"

static int fail(const char *what) {
    std::printf("FAIL %s\n", what);
    return 1;
}

int main(int argc, char **argv) {
    int m, n;
    if (std::scanf("%d %d", &m, &n) != 2) return fail("input");
    std::vector<int32_t> rowptr(m + 1, 0), col, rc(m, 0);
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
    std::vector<int> cdeg(n, 0);
    for (int j : col) ++cdeg[j];
    const int dmax = *std::max_element(cdeg.begin(), cdeg.end());
    const int rpt = argc > 1 ? std::atoi(argv[1]) : 2, cpt = argc > 2 ? std::atoi(argv[2]) : 4;
    const int dvs = argc > 3 ? std::atoi(argv[3]) : dmax;
    const uint32_t dvp = argc > 4 ? (uint32_t)std::strtoul(argv[4], nullptr, 16) : 0u;
    ldpc::OnchipLayout L;
    if (!ldpc::onchip_cf_layout(rowptr, col, rc, m, n, rpt, cpt, dvs, dvp, &L)) return fail("no layout");
    const int nt = L.nt, dc = L.dc, dv = L.dv, S = rpt * nt, P = cpt * nt;
    if (L.rpt != rpt || L.cpt != cpt || dv != dvs || S < m || P < n) return fail("geometry");
    if ((int)L.edge.size() != S * dc || (int)L.bitpos.size() != P * dv || (int)L.slot_bit.size() != n)
        return fail("table sizes");
    // messages bit slot p reads: its profile entry, or the stride
    auto cap = [&](int p) { return dvp ? (int)((dvp >> (4 * (p / nt))) & 15u) : dv; };
    // bits: a permutation of 0..n-1 inside 64-slot blocks, or into slots whose cap holds them
    std::vector<int> bit_slot(n, -1);
    for (int p = 0; p < n; ++p) {
        const int j = L.slot_bit[p];
        if (j < 0 || j >= n || bit_slot[j] >= 0) return fail("bit slots");
        if (dvp ? cap(p) < cdeg[j] : j / 64 != p / 64) return fail("bit slots");
        bit_slot[j] = p;
    }
    // rows: slots below m hold distinct rows with exactly their edges
    std::vector<int> seen_row(m, 0), used(L.npos, 0);
    std::vector<std::vector<int>> rows_of_bit(n);
    std::vector<int> pos_of(col.size(), -1);
    for (int s = 0; s < m; ++s) {
        std::vector<int> bits_here, pos_here;
        for (int k = 0; k < dc; ++k) {
            const uint32_t w = L.edge[(size_t)s * dc + k];
            bits_here.push_back((int)(w & 0xffff));
            pos_here.push_back((int)(w >> 16));
        }
        // find the row with this bit set (slots hold rows of degree dc)
        std::vector<int> gb;
        for (int b : bits_here) {
            if (b >= n) return fail("bit slot range");
            gb.push_back(L.slot_bit[b]);
        }
        std::vector<int> sorted = gb;
        std::sort(sorted.begin(), sorted.end());
        int row = -1;
        for (int i = 0; i < m && row < 0; ++i) {
            if (seen_row[i]) continue;
            std::vector<int> r(col.begin() + rowptr[i], col.begin() + rowptr[i + 1]);
            if (r == sorted) row = i;
        }
        if (row < 0) return fail("row edges");
        seen_row[row] = 1;
        for (int k = 0; k < dc; ++k) {
            const int p = pos_here[k];
            if (p < 0 || p >= L.npos - 1 || used[p]++) return fail("message positions");
            const int e = rowptr[row] + (int)(std::lower_bound(col.begin() + rowptr[row], col.begin() + rowptr[row + 1], gb[k]) -
                                              (col.begin() + rowptr[row]));
            pos_of[e] = p;
            rows_of_bit[gb[k]].push_back(row);
        }
    }
    // bit side: the u-th entry is the message of the u-th check in ascending
    // order, then zero positions (never a message's, never the rows-past-m one)
    int nmsg = 0;
    for (int p = 0; p < L.npos; ++p) nmsg += used[p];
    if (nmsg != (int)col.size()) return fail("message count");
    auto is_zero = [&](uint32_t p) { return (int)p < L.npos - 1 && !used[p]; };
    for (int p = n; p < P; ++p)
        for (int u = 0; u < dv; ++u)
            if (!is_zero(L.bitpos[(size_t)p * dv + u])) return fail("empty bit slot reads a message");
    for (int j = 0; j < n; ++j) {
        std::vector<int> r = rows_of_bit[j];
        std::sort(r.begin(), r.end());
        if ((int)r.size() != cdeg[j]) return fail("column degree");
        for (int u = 0; u < dv; ++u) {
            if (u >= (int)r.size()) {
                if (!is_zero(L.bitpos[(size_t)bit_slot[j] * dv + u])) return fail("padding entry");
                continue;
            }
            const int i = r[u];
            const int e = rowptr[i] + (int)(std::lower_bound(col.begin() + rowptr[i], col.begin() + rowptr[i + 1], j) -
                                            (col.begin() + rowptr[i]));
            if ((int)L.bitpos[(size_t)bit_slot[j] * dv + u] != pos_of[e]) return fail("bit-side positions");
        }
    }
    // banks: check instructions (wave, r, k): writes and message reads; posterior gathers
    double load = 0;
    int halves = 0;
    for (int w = 0; w < nt / 64; ++w)
        for (int r = 0; r < rpt; ++r)
            for (int k = 0; k < dc; ++k) {
                for (int q = 0; q < 4; ++q) {
                    int cnt[16] = {0};
                    for (int l = 16 * q; l < 16 * q + 16; ++l) {
                        const int s = r * nt + 64 * w + l;
                        if (s < m && ++cnt[(L.edge[(size_t)s * dc + k] >> 16) % 16] > 1) return fail("write conflict");
                    }
                }
                for (int h = 0; h < 2; ++h) {
                    int cnt[32] = {0}, sc[32] = {0};
                    std::vector<int> sb;
                    for (int l = 32 * h; l < 32 * h + 32; ++l) {
                        const int s = r * nt + 64 * w + l;
                        if (s >= m) continue;
                        const uint32_t v = L.edge[(size_t)s * dc + k];
                        if (++cnt[(v >> 16) % 32] > 1) return fail("message read conflict (check pass)");
                        if (std::find(sb.begin(), sb.end(), (int)(v & 0xffff)) == sb.end()) {
                            sb.push_back((int)(v & 0xffff));
                            ++sc[(v & 0xffff) % 32];
                        }
                    }
                    load += *std::max_element(sc, sc + 32);
                    ++halves;
                }
            }
    for (int c = 0; c < cpt; ++c)
        for (int w = 0; w < nt / 64; ++w)
            for (int u = 0; u < dv; ++u)
                for (int h = 0; h < 2; ++h) {
                    int cnt[32] = {0};
                    std::vector<uint32_t> words;
                    for (int l = 32 * h; l < 32 * h + 32; ++l) {
                        if (u >= cap(c * nt)) continue; // not read
                        const uint32_t v = L.bitpos[(size_t)(c * nt + 64 * w + l) * dv + u];
                        if (std::find(words.begin(), words.end(), v) != words.end()) continue; // same word
                        words.push_back(v);
                        if (++cnt[v % 32] > 1) return fail("message read conflict (bit pass)");
                    }
                }
    std::printf("ok %.4f\n", load / halves);
    return 0;
}
