// Tanner graph construction from a dense parity matrix on the device.
//
// The neighbour sets of Sec. II-B: N_i (the bits of check row i, the ones of
// row i of H) and M_j (the checks of bit j, the ones of column j).  They are
// stored as CSR (row_ptr, col_idx) and as a CSC view (col_ptr, csc_edge) that
// points back into the CSR edge numbering, so one per-edge message array
// serves both the check update (row order) and the bit update (column order).
#include <algorithm>
#include <cstring>

#include "ldpc_internal.h"

namespace {

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// One wavefront per row: count the ones of the row and flag entries > 1.
__global__ __launch_bounds__(256) void k_row_count(const uint8_t *__restrict__ H, int32_t m, int32_t n,
                                                   int32_t *__restrict__ row_deg, int32_t *__restrict__ bad) {
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= m) return;
    const uint8_t *h = H + row * (int64_t)n;
    int cnt = 0, big = 0;
    for (int32_t k = lane; k < n; k += 64) {
        const uint8_t v = h[k];
        cnt += v;
        big |= v > 1;
    }
    cnt = wave_sum(cnt);
    big = wave_sum(big);
    if (lane == 0) {
        row_deg[row] = cnt;
        if (big) atomicOr(bad, 1);
    }
}

// One wavefront per row: write the bit index of every one, ascending, by a
// ballot over each 64-entry chunk and a popcount of the lower lanes.
__global__ __launch_bounds__(256) void k_row_fill(const uint8_t *__restrict__ H, int32_t m, int32_t n,
                                                  const int32_t *__restrict__ row_ptr,
                                                  int32_t *__restrict__ col_idx) {
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= m) return;
    const uint8_t *h = H + row * (int64_t)n;
    int32_t out = row_ptr[row];
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int32_t base = 0; base < n; base += 64) {
        const int32_t k = base + lane;
        const bool one = k < n && h[k] != 0;
        const uint64_t mask = __ballot(one);
        if (one) col_idx[out + __popcll(mask & below)] = k;
        out += __popcll(mask);
    }
}

__global__ void k_col_count(const int32_t *__restrict__ col_idx, int64_t E, int32_t *__restrict__ col_deg) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < E) atomicAdd(&col_deg[col_idx[e]], 1);
}

// Scatter every edge into its column's segment (slot order arbitrary) ...
__global__ void k_csc_scatter(const int32_t *__restrict__ col_idx, int64_t E, const int32_t *__restrict__ col_ptr,
                              int32_t *__restrict__ fill, int32_t *__restrict__ csc_edge) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    const int32_t j = col_idx[e];
    const int32_t slot = atomicAdd(&fill[j], 1);
    csc_edge[col_ptr[j] + slot] = (int32_t)e;
}

// ... then sort each segment: CSR numbers grow with the row index, so an
// ascending segment lists the column's checks in ascending order.
__global__ void k_csc_sort(const int32_t *__restrict__ col_ptr, int32_t n, int32_t *__restrict__ csc_edge) {
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int32_t a = col_ptr[j], b = col_ptr[j + 1];
    for (int32_t p = a + 1; p < b; ++p) {
        const int32_t v = csc_edge[p];
        int32_t q = p - 1;
        while (q >= a && csc_edge[q] > v) {
            csc_edge[q + 1] = csc_edge[q];
            --q;
        }
        csc_edge[q + 1] = v;
    }
}

__global__ void k_edge_pos(const int32_t *__restrict__ csc_edge, int64_t E, int32_t *__restrict__ edge_pos) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < E) edge_pos[csc_edge[k]] = (int32_t)k;
}

// Order of each row's edges in the on-chip table.  The on-chip decoder reads
// s[bit] and writes eta[slot] for edge k of 64 consecutive rows in one
// wavefront instruction, as 8-byte LDS accesses (two frames).  The results do
// not depend on the order of a row's edges, so it is chosen here to spread
// each instruction's accesses over the LDS banks.  For every block of 32
// consecutive rows, with h_k(b) the number of rows whose k-th edge has its
// bit (or its slot) in bank pair b (8-byte words modulo 32), a local search
// swaps edges within rows while that lowers sum_k sum_b h_k(b)^2.
std::vector<uint32_t> bank_balanced_edge_tab(const std::vector<int32_t> &rowptr, const std::vector<int32_t> &col,
                                             const std::vector<int32_t> &pos, int32_t m) {
    constexpr int kPairs = 32, kGroup = 32, kPasses = 8;
    std::vector<int32_t> order(col.size()); // CSR edge placed at each table position
    for (size_t e = 0; e < order.size(); ++e) order[e] = (int32_t)e;
    for (int32_t g0 = 0; g0 < m; g0 += kGroup) {
        const int32_t g1 = std::min<int32_t>(m, g0 + kGroup);
        int32_t dmax = 0;
        for (int32_t i = g0; i < g1; ++i) dmax = std::max(dmax, rowptr[i + 1] - rowptr[i]);
        std::vector<int32_t> hs((size_t)dmax * kPairs, 0), he((size_t)dmax * kPairs, 0);
        for (int32_t i = g0; i < g1; ++i)
            for (int32_t k = 0; k < rowptr[i + 1] - rowptr[i]; ++k) {
                const int32_t e = order[rowptr[i] + k];
                ++hs[(size_t)k * kPairs + col[e] % kPairs];
                ++he[(size_t)k * kPairs + pos[e] % kPairs];
            }
        // change of sum of squares when one unit moves from bin x to bin y at
        // step k1 and one from y to x at step k2
        auto delta = [&](std::vector<int32_t> &h, int k1, int k2, int x, int y) {
            if (x == y) return 0;
            const int32_t *a = &h[(size_t)k1 * kPairs], *b = &h[(size_t)k2 * kPairs];
            return 2 * (b[x] - a[x] + a[y] - b[y]) + 4;
        };
        for (int pass = 0; pass < kPasses; ++pass) {
            bool improved = false;
            for (int32_t i = g0; i < g1; ++i) {
                const int32_t d = rowptr[i + 1] - rowptr[i];
                for (int k1 = 0; k1 < d; ++k1)
                    for (int k2 = k1 + 1; k2 < d; ++k2) {
                        int32_t &e1 = order[rowptr[i] + k1], &e2 = order[rowptr[i] + k2];
                        const int s1 = col[e1] % kPairs, s2 = col[e2] % kPairs;
                        const int p1 = pos[e1] % kPairs, p2 = pos[e2] % kPairs;
                        if (delta(hs, k1, k2, s1, s2) + delta(he, k1, k2, p1, p2) >= 0) continue;
                        --hs[(size_t)k1 * kPairs + s1]; ++hs[(size_t)k1 * kPairs + s2];
                        --hs[(size_t)k2 * kPairs + s2]; ++hs[(size_t)k2 * kPairs + s1];
                        --he[(size_t)k1 * kPairs + p1]; ++he[(size_t)k1 * kPairs + p2];
                        --he[(size_t)k2 * kPairs + p2]; ++he[(size_t)k2 * kPairs + p1];
                        std::swap(e1, e2);
                        improved = true;
                    }
            }
            if (!improved) break;
        }
    }
    std::vector<uint32_t> tab(col.size());
    for (size_t t = 0; t < tab.size(); ++t) tab[t] = (uint32_t)col[order[t]] | ((uint32_t)pos[order[t]] << 16);
    return tab;
}

void free_graph_arrays(ldpc_graph *g) {
    if (!g) return;
    (void)hipFree(g->row_ptr);
    (void)hipFree(g->col_idx);
    (void)hipFree(g->col_ptr);
    (void)hipFree(g->csc_edge);
    (void)hipFree(g->row_class);
    (void)hipFree(g->edge_pos);
    (void)hipFree(g->edge_tab);
    (void)hipFree(g->dense_h);
    (void)hipFree(g->cf.edge);
    (void)hipFree(g->cf.bitpos);
    (void)hipFree(g->cf.slot_bit);
    (void)hipFree(g->cf.row_class);
    (void)hipFree(g->stream_order.col_idx);
    (void)hipFree(g->stream_order.csc_edge);
    (void)hipFree(g->stream_order.row_class);
    g->stream_order.col_idx = g->stream_order.csc_edge = g->stream_order.row_class = nullptr;
    g->cf.edge = g->cf.bitpos = nullptr;
    g->cf.slot_bit = g->cf.row_class = nullptr;
    g->cf.nt = g->cf.npos = 0;
    g->cf.rpt = g->cf.cpt = g->cf.dvs = 0;
    g->cf.dvp = 0;
    g->row_ptr = g->col_idx = g->col_ptr = g->csc_edge = g->row_class = g->edge_pos = nullptr;
    g->edge_tab = nullptr;
    g->dense_h = nullptr;
}

template <class T> hipError_t dalloc(T **p, size_t count) {
    return hipMalloc((void **)p, sizeof(T) * std::max<size_t>(count, 1));
}

int build(const uint8_t *H, int32_t m, int32_t n, hipStream_t s, ldpc_graph *g) {
    int32_t *row_deg = nullptr, *bad = nullptr, *col_deg = nullptr, *fill = nullptr;
    int status = LDPC_OK;
    auto fail = [&](int st) {
        status = st;
        return st;
    };
    std::vector<int32_t> h_row(m), h_col(n);
    int32_t h_bad = 0;
    int64_t E = 0;
    do {
        if (dalloc(&row_deg, m) != hipSuccess || dalloc(&bad, 1) != hipSuccess ||
            dalloc(&col_deg, n) != hipSuccess || dalloc(&fill, n) != hipSuccess) {
            fail(LDPC_ENOMEM);
            break;
        }
        if (hipMemsetAsync(bad, 0, sizeof(int32_t), s) != hipSuccess) { fail(LDPC_EHIP); break; }
        k_row_count<<<(m + 3) / 4, 256, 0, s>>>(H, m, n, row_deg, bad);
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(h_row.data(), row_deg, sizeof(int32_t) * m, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(&h_bad, bad, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            fail(LDPC_EHIP);
            break;
        }
        if (h_bad) { fail(LDPC_EBADH); break; }
        std::vector<int32_t> h_rowptr(m + 1);
        int32_t dcmax = 0;
        std::vector<uint8_t> present(n + 1, 0);
        for (int32_t i = 0; i < m; ++i) {
            h_rowptr[i] = (int32_t)E;
            E += h_row[i];
            dcmax = std::max(dcmax, h_row[i]);
            present[h_row[i]] = 1;
        }
        bool deg1 = false;
        for (int32_t i = 0; i < m; ++i) deg1 |= h_row[i] == 1;
        if (deg1 || E >= INT32_MAX) { fail(LDPC_EBADH); break; }
        h_rowptr[m] = (int32_t)E;
        g->E = E;
        g->dc_max = dcmax;
        g->dc_min = *std::min_element(h_row.begin(), h_row.end());
        std::vector<int32_t> rank(n + 1, -1);
        g->class_degrees.clear();
        for (int32_t d = 1; d <= n; ++d)
            if (present[d]) {
                rank[d] = (int32_t)g->class_degrees.size();
                g->class_degrees.push_back(d);
            }
        std::vector<int32_t> h_class(m);
        for (int32_t i = 0; i < m; ++i) h_class[i] = h_row[i] ? rank[h_row[i]] : -1;

        if (dalloc(&g->row_ptr, m + 1) != hipSuccess || dalloc(&g->col_idx, E) != hipSuccess ||
            dalloc(&g->col_ptr, n + 9) != hipSuccess || dalloc(&g->csc_edge, E + 8) != hipSuccess || // 8 entries of padding: readers load groups of 8
            hipMemsetAsync(g->csc_edge + E, 0, 8 * sizeof(int32_t), s) != hipSuccess ||
            dalloc(&g->row_class, m) != hipSuccess || dalloc(&g->edge_pos, E) != hipSuccess) {
            fail(LDPC_ENOMEM);
            break;
        }
        if (hipMemcpyAsync(g->row_ptr, h_rowptr.data(), sizeof(int32_t) * (m + 1), hipMemcpyHostToDevice, s) !=
                hipSuccess ||
            hipMemcpyAsync(g->row_class, h_class.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice, s) !=
                hipSuccess ||
            hipMemsetAsync(col_deg, 0, sizeof(int32_t) * n, s) != hipSuccess ||
            hipMemsetAsync(fill, 0, sizeof(int32_t) * n, s) != hipSuccess) {
            fail(LDPC_EHIP);
            break;
        }
        k_row_fill<<<(m + 3) / 4, 256, 0, s>>>(H, m, n, g->row_ptr, g->col_idx);
        const unsigned eblocks = (unsigned)((E + 255) / 256);
        if (E > 0) k_col_count<<<eblocks, 256, 0, s>>>(g->col_idx, E, col_deg);
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(h_col.data(), col_deg, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            fail(LDPC_EHIP);
            break;
        }
        std::vector<int32_t> h_colptr(n + 9);
        int32_t dvmax = 0;
        int64_t acc = 0;
        for (int32_t j = 0; j < n; ++j) {
            h_colptr[j] = (int32_t)acc;
            acc += h_col[j];
            dvmax = std::max(dvmax, h_col[j]);
        }
        for (int32_t j = n; j < n + 9; ++j) h_colptr[j] = (int32_t)acc; // col_ptr[n] and 8 entries of padding
        g->dv_max = dvmax;
        g->dv_min = *std::min_element(h_col.begin(), h_col.end());
        if (hipMemcpyAsync(g->col_ptr, h_colptr.data(), sizeof(int32_t) * (n + 9), hipMemcpyHostToDevice, s) !=
            hipSuccess) {
            fail(LDPC_EHIP);
            break;
        }
        if (E > 0) {
            k_csc_scatter<<<eblocks, 256, 0, s>>>(g->col_idx, E, g->col_ptr, fill, g->csc_edge);
            k_csc_sort<<<(n + 255) / 256, 256, 0, s>>>(g->col_ptr, n, g->csc_edge);
            k_edge_pos<<<eblocks, 256, 0, s>>>(g->csc_edge, E, g->edge_pos);
        }
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
            fail(LDPC_EHIP);
            break;
        }
        if (n < 65536 && E < 65536) {
            std::vector<int32_t> h_bit(E), h_pos(E);
            if (E > 0 &&
                (hipMemcpy(h_bit.data(), g->col_idx, sizeof(int32_t) * E, hipMemcpyDeviceToHost) != hipSuccess ||
                 hipMemcpy(h_pos.data(), g->edge_pos, sizeof(int32_t) * E, hipMemcpyDeviceToHost) != hipSuccess)) {
                fail(LDPC_EHIP);
                break;
            }
            const std::vector<uint32_t> tab = bank_balanced_edge_tab(h_rowptr, h_bit, h_pos, m);
            if (dalloc(&g->edge_tab, E) != hipSuccess) {
                fail(LDPC_ENOMEM);
                break;
            }
            if (E > 0 && hipMemcpy(g->edge_tab, tab.data(), sizeof(uint32_t) * E, hipMemcpyHostToDevice) != hipSuccess) {
                fail(LDPC_EHIP);
                break;
            }
            // the bank-conflict-free layout, for rows of one degree, in the
            // geometry of the layout variants that fits the graph best
            ldpc::OnchipLayout lay;
            int32_t rpt = 0, cpt = 0, dvs = 0;
            uint32_t dvp = 0;
            if (E > 0 && g->dc_min == g->dc_max && ldpc::onchip_cf_geometry(*g, h_col, &rpt, &cpt, &dvs, &dvp) &&
                ldpc::onchip_cf_layout(h_rowptr, h_bit, h_class, m, n, rpt, cpt, dvs, dvp, &lay)) {
                const size_t S = (size_t)lay.rpt * lay.nt;
                if (dalloc(&g->cf.edge, lay.edge.size()) != hipSuccess ||
                    dalloc(&g->cf.bitpos, lay.bitpos.size()) != hipSuccess ||
                    dalloc(&g->cf.slot_bit, lay.slot_bit.size()) != hipSuccess ||
                    dalloc(&g->cf.row_class, S) != hipSuccess) {
                    fail(LDPC_ENOMEM);
                    break;
                }
                if (hipMemcpy(g->cf.edge, lay.edge.data(), sizeof(uint32_t) * lay.edge.size(),
                              hipMemcpyHostToDevice) != hipSuccess ||
                    hipMemcpy(g->cf.bitpos, lay.bitpos.data(), sizeof(uint32_t) * lay.bitpos.size(),
                              hipMemcpyHostToDevice) != hipSuccess ||
                    hipMemcpy(g->cf.slot_bit, lay.slot_bit.data(), sizeof(int32_t) * lay.slot_bit.size(),
                              hipMemcpyHostToDevice) != hipSuccess ||
                    hipMemcpy(g->cf.row_class, lay.row_class.data(), sizeof(int32_t) * S, hipMemcpyHostToDevice) !=
                        hipSuccess) {
                    fail(LDPC_EHIP);
                    break;
                }
                g->cf.nt = lay.nt;
                g->cf.npos = lay.npos;
                g->cf.rpt = lay.rpt;
                g->cf.cpt = lay.cpt;
                g->cf.dvs = lay.dv;
                g->cf.dvp = lay.dvp;
            }
        }
        // Row order of the streaming path, where its check kernel reads
        // posteriors with its unrolled form (rows of 6 or 7 edges) and a tile
        // of them (256 bytes per bit) exceeds an XCD's 4 MB L2.
        if (E > 0 && g->dc_min == g->dc_max && (g->dc_max == 6 || g->dc_max == 7) && (size_t)n * 256 > ((size_t)4 << 20)) {
            std::vector<int32_t> h_colidx(E);
            if (hipMemcpy(h_colidx.data(), g->col_idx, sizeof(int32_t) * E, hipMemcpyDeviceToHost) != hipSuccess) {
                fail(LDPC_EHIP);
                break;
            }
            std::vector<int32_t> h_csc(E);
            if (hipMemcpy(h_csc.data(), g->csc_edge, sizeof(int32_t) * E, hipMemcpyDeviceToHost) != hipSuccess) {
                fail(LDPC_EHIP);
                break;
            }
            const std::vector<int32_t> ord = ldpc::stream_row_order(h_rowptr, h_colidx, m, n);
            const int32_t dc = g->dc_max;
            std::vector<int32_t> ncol(E), ncsc(E + 8, 0), nrc(m), old2new(E);
            for (int32_t p = 0; p < m; ++p) {
                const int32_t i = ord[p];
                nrc[p] = h_class[i];
                for (int32_t k = 0; k < dc; ++k) {
                    ncol[(size_t)p * dc + k] = h_colidx[(size_t)i * dc + k];
                    old2new[(size_t)i * dc + k] = p * dc + k;
                }
            }
            for (int64_t q = 0; q < E; ++q) ncsc[q] = old2new[h_csc[q]];
            if (dalloc(&g->stream_order.col_idx, E) != hipSuccess || dalloc(&g->stream_order.csc_edge, E + 8) != hipSuccess ||
                dalloc(&g->stream_order.row_class, m) != hipSuccess) {
                fail(LDPC_ENOMEM);
                break;
            }
            if (hipMemcpy(g->stream_order.col_idx, ncol.data(), sizeof(int32_t) * E, hipMemcpyHostToDevice) != hipSuccess ||
                hipMemcpy(g->stream_order.csc_edge, ncsc.data(), sizeof(int32_t) * (E + 8), hipMemcpyHostToDevice) !=
                    hipSuccess ||
                hipMemcpy(g->stream_order.row_class, nrc.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice) != hipSuccess) {
                fail(LDPC_EHIP);
                break;
            }
        }
    } while (false);
    (void)hipFree(row_deg);
    (void)hipFree(bad);
    (void)hipFree(col_deg);
    (void)hipFree(fill);
    return status;
}

} // namespace

extern "C" int ldpc_build_graph(const uint8_t *H_dev, int32_t m, int32_t n, hipStream_t stream,
                                ldpc_graph **out) {
    if (!out) return LDPC_EINVAL;
    *out = nullptr;
    if (!H_dev || m < 1 || n < 1) return LDPC_EINVAL;
    ldpc_graph *g = new (std::nothrow) ldpc_graph();
    if (!g) return LDPC_ENOMEM;
    g->m = m;
    g->n = n;
    if (hipGetDevice(&g->device) != hipSuccess ||
        hipDeviceGetAttribute(&g->num_cu, hipDeviceAttributeMultiprocessorCount, g->device) != hipSuccess ||
        hipDeviceGetAttribute(&g->lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, g->device) != hipSuccess) {
        delete g;
        return LDPC_EHIP;
    }
    int st = build(H_dev, m, n, stream, g);
    if (st == LDPC_OK && (size_t)m * (size_t)n <= ldpc::kDenseMaxBytes) {
        if (dalloc(&g->dense_h, (size_t)m * (size_t)n) != hipSuccess)
            st = LDPC_ENOMEM;
        else if (hipMemcpyAsync(g->dense_h, H_dev, (size_t)m * (size_t)n, hipMemcpyDeviceToDevice, stream) !=
                 hipSuccess)
            st = LDPC_EHIP;
    }
    if (st != LDPC_OK) {
        (void)hipStreamSynchronize(stream);
        free_graph_arrays(g);
        delete g;
        return st;
    }
    *out = g;
    return LDPC_OK;
}

extern "C" int ldpc_graph_info(const ldpc_graph *g, int32_t *m, int32_t *n, int64_t *n_edges, int32_t *dc_max,
                               int32_t *dv_max, int32_t *n_classes, int32_t *check_degrees, int32_t cap) {
    if (!g) return LDPC_EINVAL;
    if (m) *m = g->m;
    if (n) *n = g->n;
    if (n_edges) *n_edges = g->E;
    if (dc_max) *dc_max = g->dc_max;
    if (dv_max) *dv_max = g->dv_max;
    if (n_classes) *n_classes = (int32_t)g->class_degrees.size();
    if (check_degrees)
        for (int32_t k = 0; k < cap && k < (int32_t)g->class_degrees.size(); ++k) check_degrees[k] = g->class_degrees[k];
    return LDPC_OK;
}

extern "C" void ldpc_graph_destroy(ldpc_graph *g) {
    if (!g) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(g->device);
    (void)hipDeviceSynchronize();
    free_graph_arrays(g);
    (void)hipSetDevice(cur);
    delete g;
}
