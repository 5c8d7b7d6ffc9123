// Bank-conflict-free LDS layout for the on-chip decoder (host code, run once
// per graph at build time).
//
// gfx950 LDS serves an 8-byte read (ds_read_b64) of a wavefront 32 lanes at a
// time and an 8-byte write 16 lanes at a time.  A read is conflict-free when
// the 32 lanes of each half address distinct 8-byte words modulo 32 (or the
// same word); a write when the 16 lanes of each quarter address distinct words
// modulo 16.  Measured: ds_read_b64 2.5 cycles per wavefront instruction and CU
// conflict-free, 7.5 with random addresses; ds_write_b64 6.2 and 11.9.
//
// The on-chip decoder's LDS traffic per round (a geometry of rpt rows and cpt
// bits per thread) is: in the check pass, per own row and edge, a read of the bit's
// posterior s (a gather), a read of the edge's previous message and a write
// of its new one; in the bit pass, per own bit, reads of its column's
// messages (a gather) and a write of s.  The layout chooses
//   * which thread slot holds which check row (rows are interchangeable),
//   * the order of each row's edges (min, parity and the messages do not
//     depend on it),
//   * and a free LDS position for every edge's message,
// so that every message read and write is conflict-free and the posterior
// gathers nearly so.  Bits move only inside their 64-slot block (so frame I/O
// stays coalesced), or, with a column degree profile, are placed in ascending
// degree (bit slot index c then holds bits of degree at most the profile's
// entry c, and the kernel reads that many messages for it) and move only
// among the slots of their own degree.  Columns of lower degree than the table's stride, and bit
// slots past n, read zero messages from positions that nothing writes: their
// bit sums then take the same instructions as the others and stay exact.
//
// Message positions are exact by construction.  Give each edge a class c in
// 0..31 (its position is c modulo 32).  Its write (check pass) falls in one
// quarter of a check instruction, its read in the check pass in the half that
// contains that quarter, its read in the bit pass in one half of a bit
// instruction.  Write c = x + 16 h.  Quarters need distinct x; halves need
// distinct (x, h).  Split every bit half into two nodes of at most 16 edges:
// the multigraph between check quarters and those nodes has degree at most
// 16, so (Konig) its edges take 16 colours x with no two alike at a node.
// Then each check half and each bit half holds every x at most twice, and
// the h of the two must differ: each edge has at most one such partner of
// each kind, so these constraints form paths and even cycles, which a 2-
// colouring satisfies.
//
// Posterior gathers: a check instruction reads, in each half, s of the k-th
// edge of 32 rows, at the bit index modulo 32.  Rows are placed in thread
// slots so that every half-group of 32 rows has its edges spread evenly over
// the 32 classes (local search), then each half-group's edges are ordered by
// a proper edge colouring of its (rows x classes) multigraph, classes with
// more edges than the row degree split into nodes of at most that many.
#include <algorithm>
#include <cstdint>
#include <numeric>
#include <random>
#include <vector>

#include "ldpc_internal.h"

namespace ldpc {
namespace {

// Proper edge colouring of a bipartite multigraph with `ncol` colours, where
// every node has degree <= ncol (Konig's theorem guarantees one), by the
// alternating-path method.  Returns the colour of every edge.
std::vector<int32_t> bipartite_edge_colour(int32_t nleft, int32_t nright, const std::vector<int32_t> &ea,
                                           const std::vector<int32_t> &eb, int32_t ncol) {
    const size_t E = ea.size();
    std::vector<int32_t> at((size_t)nleft * ncol, -1), bt((size_t)nright * ncol, -1), colour(E, -1);
    std::vector<int32_t> path;
    for (size_t e = 0; e < E; ++e) {
        const int32_t a = ea[e], b = eb[e];
        int32_t al = 0, be = 0;
        while (at[(size_t)a * ncol + al] >= 0) ++al;
        while (bt[(size_t)b * ncol + be] >= 0) ++be;
        if (bt[(size_t)b * ncol + al] >= 0) {
            // alternating al / be path from b; swapping its colours frees al at b
            // (the path cannot end at a: al is free at a, and a path reaching a
            // would arrive by an al edge)
            path.clear();
            int32_t node = b, c = al;
            bool right = true;
            for (;;) {
                const int32_t f = right ? bt[(size_t)node * ncol + c] : at[(size_t)node * ncol + c];
                if (f < 0) break;
                path.push_back(f);
                node = right ? ea[f] : eb[f];
                right = !right;
                c = (c == al) ? be : al;
            }
            for (int32_t f : path) {
                at[(size_t)ea[f] * ncol + colour[f]] = -1;
                bt[(size_t)eb[f] * ncol + colour[f]] = -1;
            }
            for (int32_t f : path) {
                colour[f] = colour[f] == al ? be : al;
                at[(size_t)ea[f] * ncol + colour[f]] = f;
                bt[(size_t)eb[f] * ncol + colour[f]] = f;
            }
        }
        colour[e] = al;
        at[(size_t)a * ncol + al] = (int32_t)e;
        bt[(size_t)b * ncol + al] = (int32_t)e;
    }
    return colour;
}

} // namespace

bool onchip_cf_layout(const std::vector<int32_t> &rowptr, const std::vector<int32_t> &col,
                      const std::vector<int32_t> &row_class, int32_t m, int32_t n, int32_t rpt, int32_t cpt,
                      int32_t dvs, uint32_t dvp, OnchipLayout *out) {
        const int64_t E = (int64_t)col.size();
    if (m < 1 || n < 1 || E < 1 || n >= 65536 || E >= 65536 || rpt < 1 || cpt < 1) return false;
    int32_t dc = 0;
    for (int32_t i = 0; i < m; ++i) dc = std::max(dc, rowptr[i + 1] - rowptr[i]);
    std::vector<int32_t> cdeg(n, 0);
    for (int32_t j : col) ++cdeg[j];
    const int32_t dv = *std::max_element(cdeg.begin(), cdeg.end());
    if (dc > 16 || dv > 16 || dvs < dv || dvs > 16) return false;
    const int32_t need = std::max((m + rpt - 1) / rpt, (n + cpt - 1) / cpt);
    const int32_t nt = std::max<int32_t>(64, (need + 63) / 64 * 64);
    if (nt > 512) return false;
    const int32_t S = rpt * nt;        // row slots: s = r nt + t
    const int32_t G = S / 32;         // half-groups of 32 row slots
    auto group_of = [&](int32_t s) { return (s / nt) * (nt / 32) + (s % nt) / 32; };

    // ---- 1. rows into slots 0 .. m-1 and bits into slots of their own 64-slot
    // block (with a degree profile: bits in ascending degree, then moves
    // among the slots of one degree), evening out each half-group's classes
    // (bit slot modulo 32) by local search on the sum of squared (half-group,
    // class) counts
    std::vector<int32_t> slot_row(m), row_slot(m);
    std::iota(slot_row.begin(), slot_row.end(), 0);
    std::iota(row_slot.begin(), row_slot.end(), 0);
    const int32_t nblk = (n + 63) / 64;
    std::vector<int32_t> bit_slot(n), slot_bit((size_t)nblk * 64, -1);
    for (int32_t j = 0; j < n; ++j) {
        bit_slot[j] = j;
        slot_bit[j] = j;
    }
    // with a profile: [lo, hi) of the slots that hold bits of slot p's degree
    std::vector<int32_t> grp_lo, grp_hi;
    if (dvp != 0u) {
        std::stable_sort(slot_bit.begin(), slot_bit.begin() + n,
                         [&](int32_t a, int32_t b) { return cdeg[a] < cdeg[b]; });
        grp_lo.assign(n, 0);
        grp_hi.assign(n, 0);
        for (int32_t p = 0; p < n; ++p) {
            const int32_t j = slot_bit[p];
            bit_slot[j] = p;
            if ((int32_t)((dvp >> (4 * (p / nt))) & 15u) < cdeg[j]) return false; // the profile does not hold it
            grp_lo[p] = (p > 0 && cdeg[slot_bit[p - 1]] == cdeg[j]) ? grp_lo[p - 1] : p;
        }
        for (int32_t p = n - 1; p >= 0; --p)
            grp_hi[p] = (p + 1 < n && cdeg[slot_bit[p + 1]] == cdeg[slot_bit[p]]) ? grp_hi[p + 1] : p + 1;
    }
    std::vector<std::vector<int32_t>> rows_of(n);
    for (int32_t i = 0; i < m; ++i)
        for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) rows_of[col[e]].push_back(i);
    std::vector<int32_t> hist((size_t)G * 32, 0);
    for (int32_t i = 0; i < m; ++i)
        for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) ++hist[(size_t)group_of(i) * 32 + bit_slot[col[e]] % 32];
    std::mt19937_64 rng(0x5eed1234u);
    // change of the sum of squared counts for a list of (bin, +-1) changes
    auto bin_delta = [&](std::vector<std::pair<int64_t, int32_t>> &ch) {
        std::sort(ch.begin(), ch.end());
        int64_t delta = 0;
        size_t t = 0;
        while (t < ch.size()) {
            size_t u = t;
            int64_t x = 0;
            while (u < ch.size() && ch[u].first == ch[t].first) x += ch[u++].second;
            const int64_t h = hist[(size_t)ch[t].first];
            delta += 2 * x * h + x * x;
            t = u;
        }
        return delta;
    };
    std::vector<std::pair<int64_t, int32_t>> ch;
    const int64_t moves = std::min<int64_t>(3000000, 3000 * (int64_t)m);
    for (int64_t it = 0; it < moves; ++it) {
        ch.clear();
        const bool rowmove = (it & 1) == 0 || n < 2;
        int32_t s1 = 0, s2 = 0, i1 = 0, i2 = 0, j1 = -1, j2 = -1, p1 = 0, p2 = 0;
        if (rowmove) {
            if (m < 2) continue;
            s1 = (int32_t)(rng() % (uint64_t)m);
            s2 = (int32_t)(rng() % (uint64_t)m);
            const int32_t g1 = group_of(s1), g2 = group_of(s2);
            if (g1 == g2) continue;
            i1 = slot_row[s1];
            i2 = slot_row[s2];
            for (int32_t e = rowptr[i1]; e < rowptr[i1 + 1]; ++e) {
                const int32_t c = bit_slot[col[e]] % 32;
                ch.push_back({(int64_t)g1 * 32 + c, -1});
                ch.push_back({(int64_t)g2 * 32 + c, +1});
            }
            for (int32_t e = rowptr[i2]; e < rowptr[i2 + 1]; ++e) {
                const int32_t c = bit_slot[col[e]] % 32;
                ch.push_back({(int64_t)g2 * 32 + c, -1});
                ch.push_back({(int64_t)g1 * 32 + c, +1});
            }
        } else {
            // slots below n only, so that slots n .. are the empty ones
            if (dvp != 0u) {
                p1 = (int32_t)(rng() % (uint64_t)n);
                p2 = grp_lo[p1] + (int32_t)(rng() % (uint64_t)(grp_hi[p1] - grp_lo[p1]));
            } else {
                const int32_t b = (int32_t)(rng() % (uint64_t)nblk);
                const int32_t w = std::min<int32_t>(64, n - 64 * b);
                p1 = 64 * b + (int32_t)(rng() % (uint64_t)w);
                p2 = 64 * b + (int32_t)(rng() % (uint64_t)w);
            }
            if (p1 % 32 == p2 % 32) continue;
            j1 = slot_bit[p1];
            j2 = slot_bit[p2];
            for (int32_t i : rows_of[j1]) {
                ch.push_back({(int64_t)group_of(row_slot[i]) * 32 + p1 % 32, -1});
                ch.push_back({(int64_t)group_of(row_slot[i]) * 32 + p2 % 32, +1});
            }
            for (int32_t i : rows_of[j2]) {
                ch.push_back({(int64_t)group_of(row_slot[i]) * 32 + p2 % 32, -1});
                ch.push_back({(int64_t)group_of(row_slot[i]) * 32 + p1 % 32, +1});
            }
        }
        const int64_t delta = bin_delta(ch);
        if (!(delta < 0 || (delta == 0 && (rng() & 1)))) continue;
        for (auto &c : ch) hist[(size_t)c.first] += c.second;
        if (rowmove) {
            std::swap(slot_row[s1], slot_row[s2]);
            row_slot[i1] = s2;
            row_slot[i2] = s1;
        } else {
            std::swap(slot_bit[p1], slot_bit[p2]);
            bit_slot[j1] = p2;
            bit_slot[j2] = p1;
        }
    }

    // ---- 2. edge order of each row: colour the (rows x classes) multigraph of
    // each half-group with dc colours (the colour is the edge's position k)
    std::vector<int32_t> kpos(E, -1); // position of CSR edge e in its row's order
    {
        std::vector<int32_t> ea, eb, ids;
        for (int32_t g = 0; g < G; ++g) {
            ea.clear();
            eb.clear();
            ids.clear();
            std::vector<int32_t> split(32, 0), node_of_class(32 * 64, -1);
            int32_t nright = 0;
            int32_t a = 0;
            for (int32_t q = 0; q < 32; ++q) {
                const int32_t s = (g / (nt / 32)) * nt + (g % (nt / 32)) * 32 + q;
                if (s >= m) continue;
                const int32_t i = slot_row[s];
                for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
                    const int32_t c = bit_slot[col[e]] % 32;
                    const int32_t part = split[c]++ / dc; // at most dc edges per right node
                    int32_t &nd = node_of_class[c * 64 + part];
                    if (nd < 0) nd = nright++;
                    ea.push_back(a);
                    eb.push_back(nd);
                    ids.push_back(e);
                }
                ++a;
            }
            if (ids.empty()) continue;
            const std::vector<int32_t> k = bipartite_edge_colour(a, nright, ea, eb, dc);
            for (size_t t = 0; t < ids.size(); ++t) kpos[ids[t]] = k[t];
        }
    }

    // ---- 3. message positions: classes by colouring (see the file comment)
    // check instruction of an edge: (wave, r, k), lane; bit instruction: (c, wave, u), lane
    std::vector<int32_t> rank(E); // rank of the edge's row in its column (ascending)
    {
        std::vector<int32_t> cnt(n, 0);
        for (int32_t i = 0; i < m; ++i)
            for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) rank[e] = cnt[col[e]]++;
    }
    const int32_t nw = nt / 64;
    auto chk_quarter = [&](int64_t e, int32_t i) {
        const int32_t s = row_slot[i], r = s / nt, t = s % nt;
        return (((int64_t)(t / 64) * rpt + r) * 16 + kpos[e]) * 4 + (t % 64) / 16;
    };
    auto bit_half = [&](int64_t e) {
        const int32_t j = bit_slot[col[e]], c = j / nt, t = j % nt;
        return (((int64_t)c * nw + t / 64) * 16 + rank[e]) * 2 + (t % 64) / 32;
    };
    std::vector<int32_t> row_of(E);
    for (int32_t i = 0; i < m; ++i)
        for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) row_of[e] = i;
    std::vector<int32_t> x(E), hbit(E, -1);
    {
        // left: check quarters; right: halves of bit halves (<= 16 edges each)
        std::vector<int64_t> qk(E), bk(E);
        for (int64_t e = 0; e < E; ++e) {
            qk[e] = chk_quarter(e, row_of[e]);
            bk[e] = bit_half(e);
        }
        auto dense = [](const std::vector<int64_t> &key, std::vector<int32_t> &id) {
            std::vector<int64_t> u(key);
            std::sort(u.begin(), u.end());
            u.erase(std::unique(u.begin(), u.end()), u.end());
            id.resize(key.size());
            for (size_t e = 0; e < key.size(); ++e)
                id[e] = (int32_t)(std::lower_bound(u.begin(), u.end(), key[e]) - u.begin());
            return (int32_t)u.size();
        };
        std::vector<int32_t> qid, bid;
        const int32_t nq = dense(qk, qid), nb = dense(bk, bid);
        std::vector<int32_t> fill(nb, 0), sub(E);
        for (int64_t e = 0; e < E; ++e) sub[e] = 2 * bid[e] + (fill[bid[e]]++ >= 16 ? 1 : 0);
        x = bipartite_edge_colour(nq, 2 * nb, qid, sub, 16);
        // partners: same x in the same check half (other quarter) / same bit half
        std::vector<int64_t> ck(E), bk2(E);
        for (int64_t e = 0; e < E; ++e) {
            ck[e] = (qk[e] / 2) * 16 + x[e]; // half = quarter / 2
            bk2[e] = bk[e] * 16 + x[e];
        }
        std::vector<int32_t> cpart(E, -1), bpart(E, -1);
        auto pair_up = [&](const std::vector<int64_t> &key, std::vector<int32_t> &part) {
            std::vector<int32_t> ord(E);
            std::iota(ord.begin(), ord.end(), 0);
            std::sort(ord.begin(), ord.end(), [&](int32_t p, int32_t q) { return key[p] < key[q]; });
            for (int64_t t = 0; t + 1 < E; ++t)
                if (key[ord[t]] == key[ord[t + 1]]) {
                    part[ord[t]] = ord[t + 1];
                    part[ord[t + 1]] = ord[t];
                }
        };
        pair_up(ck, cpart);
        pair_up(bk2, bpart);
        // 2-colour each path / cycle, choosing the start so the classes stay even
        std::vector<int64_t> count(32, 0);
        std::vector<int32_t> comp;
        for (int64_t e0 = 0; e0 < E; ++e0) {
            if (hbit[e0] >= 0) continue;
            comp.clear();
            hbit[e0] = 0;
            comp.push_back((int32_t)e0);
            for (size_t t = 0; t < comp.size(); ++t) {
                const int32_t e = comp[t];
                for (int32_t f : {cpart[e], bpart[e]}) {
                    if (f < 0) continue;
                    if (hbit[f] < 0) {
                        hbit[f] = hbit[e] ^ 1;
                        comp.push_back(f);
                    } else if (hbit[f] == hbit[e]) {
                        return false; // cannot happen: the cycles are even
                    }
                }
            }
            int64_t c0 = 0, c1 = 0;
            for (int32_t e : comp) {
                c0 += count[x[e] + 16 * hbit[e]];
                c1 += count[x[e] + 16 * (hbit[e] ^ 1)];
            }
            const bool flip = c1 < c0;
            for (int32_t e : comp) {
                if (flip) hbit[e] ^= 1;
                ++count[x[e] + 16 * hbit[e]];
            }
        }
    }
    std::vector<int32_t> pos(E);
    std::vector<int32_t> used(32, 0);
    for (int64_t e = 0; e < E; ++e) {
        const int32_t c = x[e] + 16 * hbit[e];
        pos[e] = c + 32 * used[c]++;
    }
    const int32_t rows32 = *std::max_element(used.begin(), used.end());
    // 32 zero positions (one per class, never written but with zeros) for the
    // bit-side entries past a bit's degree and for bit slots past n, then one
    // position that rows past m read and write
    const int32_t zero = 32 * rows32;
    const int32_t dummy = zero + 32;
    const int32_t npos = dummy + 1;
    if (npos >= 65536) return false;

    // ---- tables
    out->nt = nt;
    out->rpt = rpt;
    out->cpt = cpt;
    out->dvp = dvp;
    out->dc = dc;
    out->dv = dvs;
    out->npos = npos;
    out->edge.assign((size_t)S * dc, (uint32_t)dummy << 16); // bit 0's s, the dummy position
    out->row_class.assign(S, 0);
    for (int32_t s = 0; s < m; ++s) {
        const int32_t i = slot_row[s];
        out->row_class[s] = row_class[i] < 0 ? 0 : row_class[i];
        for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e)
            out->edge[(size_t)s * dc + kpos[e]] = (uint32_t)bit_slot[col[e]] | ((uint32_t)pos[e] << 16);
    }
    const int32_t P = cpt * nt; // bit slots
    out->bitpos.assign((size_t)P * dvs, 0xffffffffu);
    for (int32_t i = 0; i < m; ++i)
        for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e)
            out->bitpos[(size_t)bit_slot[col[e]] * dvs + rank[e]] = (uint32_t)pos[e];
    // Entries without a message read a zero position in a class that no real
    // entry of their bit instruction's half uses (the real ones are distinct
    // modulo 32, so at most 31 classes are taken when one entry is missing).
    for (int32_t base = 0; base < P; base += 32)
        for (int32_t u = 0; u < dvs; ++u) {
            uint32_t taken = 0u;
            for (int32_t p = base; p < base + 32; ++p) {
                const uint32_t v = out->bitpos[(size_t)p * dvs + u];
                if (v != 0xffffffffu) taken |= 1u << (v % 32);
            }
            int32_t c = 0;
            while (c < 32 && ((taken >> c) & 1u)) ++c;
            for (int32_t p = base; p < base + 32; ++p) {
                uint32_t &v = out->bitpos[(size_t)p * dvs + u];
                if (v == 0xffffffffu) v = (uint32_t)(zero + (c < 32 ? c : 0));
            }
        }
    out->slot_bit.assign(slot_bit.begin(), slot_bit.begin() + n);
    return true;
}

} // namespace ldpc
