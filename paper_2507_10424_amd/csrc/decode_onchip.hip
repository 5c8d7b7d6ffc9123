// On-chip Min-Sum decoder: one workgroup decodes one frame at a time with the
// whole decoding state in LDS, for codes whose state fits (n, E < 2^16 and
// tables + state within the workgroup's LDS).
//
// Workgroups are persistent: each takes frame numbers from an atomic counter
// until the batch is exhausted, so a frame that stops early frees its
// workgroup for the next frame at once (per-frame early exit costs nothing)
// and the graph tables are loaded into LDS once per workgroup.
//
// LDS (32-bit words):  row_ptr[m+1]  edge_tab[E]  col_ptr[n+1]   (graph)
//                      s[n]  r[n]  eta[E]                         (frame)
// eta is kept in CSC order (slot = position in the bit's list), so the bit
// update reads each bit's messages contiguously; the check update finds the
// slot of each of its edges in edge_tab (bit index | slot << 16).
//
// Check update of row i (one thread per row, rows strided over the
// workgroup): x_e = s_j - eta_e (eta = 0 in iteration 1), kept in registers;
// the two smallest |x| (min1 = min(min1, max(min0, |x|)), min0 = min(min0,
// |x|), on the bit patterns of non-negative floats, which order like the
// values); the XOR of the sign bits of x.  Then eta_e = magnitude of min1
// where |x_e| == min0 and of min0 elsewhere (Observation 1: on a tie min1 ==
// min0, so every edge attaining the minimum may take min1), with the sign
// bit of x_e XOR the row's sign parity (Observation 2).  The sign of a value
// is read from its sign bit: the channel LLRs are loaded as r + 0.0f, which
// turns -0 into +0, and no later s or x can then be -0, so the sign bit
// agrees with the comparison v < 0 that defines sign() (sign(0) = +1).
// The same pass XORs the sign bits of the s it reads per row: the syndrome
// of the previous iteration's hard decision, reduced over the workgroup by
// __syncthreads_or.
#include "ldpc_internal.h"

namespace ldpc {
namespace {

constexpr int kMaxThreads = 256;

size_t onchip_lds_bytes(const ldpc_graph &g) {
    // one padding word after eta keeps clamped reads of empty columns inside
    return 4ull * ((size_t)(g.m + 1) + (size_t)g.E + (size_t)(g.n + 1) + 2ull * g.n + (size_t)g.E + 1);
}

__global__ void k_zero_u32(uint32_t *p) { *p = 0u; }

// DC: row degree (RX: every row has exactly DC edges, else at most DC);
// DV: column degree (CX: every column exactly DV, else at most DV).  All
// loads of a row or column are issued before any use (branch-free masking),
// so their LDS latencies overlap.
template <int DC, bool RX, int DV, bool CX>
__global__ __launch_bounds__(kMaxThreads) void k_onchip(
    const int32_t *__restrict__ row_ptr, const uint32_t *__restrict__ edge_tab, const int32_t *__restrict__ col_ptr,
    const int32_t *__restrict__ row_class, int32_t m, int32_t n, int32_t E, const float *__restrict__ llr, int32_t B,
    int32_t L, int32_t early, const float *__restrict__ alpha, const float *__restrict__ beta, int32_t ncls,
    uint8_t *__restrict__ bits, float *__restrict__ post, int32_t *__restrict__ iters, uint8_t *__restrict__ ok,
    uint32_t *__restrict__ queue) {
    extern __shared__ uint32_t lds[];
    __shared__ int32_t frame_sh;
    uint32_t *rp = lds;
    uint32_t *tab = rp + (m + 1);
    uint32_t *cp = tab + E;
    float *s = reinterpret_cast<float *>(cp + (n + 1));
    float *r = s + n;
    float *eta = r + n; // E + 1 words
    const int tid = threadIdx.x;
    const int nt = blockDim.x;

    for (int32_t k = tid; k <= m; k += nt) rp[k] = (uint32_t)row_ptr[k];
    for (int32_t k = tid; k < E; k += nt) tab[k] = edge_tab[k];
    for (int32_t k = tid; k <= n; k += nt) cp[k] = (uint32_t)col_ptr[k];
    if (tid == 0) eta[E] = 0.0f;

    for (;;) {
        if (tid == 0) frame_sh = (int32_t)atomicAdd(queue, 1u);
        __syncthreads();
        const int32_t f = frame_sh;
        if (f >= B) break;
        const float *lf = llr + (size_t)f * n;
        for (int32_t j = tid; j < n; j += nt) {
            const float v = lf[j] + 0.0f; // -0 -> +0
            s[j] = v;
            r[j] = v;
        }
        for (int32_t k = tid; k < E; k += nt) eta[k] = 0.0f; // no message before iteration 1
        __syncthreads();

        int32_t it = L, conv = 0;
        for (int32_t t = 1;; ++t) {
            const bool msgs = t <= L; // iteration t computes messages; t = L + 1 only checks
            uint32_t unsat = 0;
            for (int32_t i = tid; i < m; i += nt) {
                const int32_t e0 = (int32_t)rp[i];
                const int32_t d = RX ? DC : (int32_t)rp[i + 1] - e0;
                if (!RX && d == 0) continue;
                uint32_t w[DC];
                float sv[DC], ev[DC];
#pragma unroll
                for (int k = 0; k < DC; ++k) w[k] = tab[e0 + (RX || k < d ? k : 0)];
#pragma unroll
                for (int k = 0; k < DC; ++k) {
                    sv[k] = s[w[k] & 0xffffu];
                    ev[k] = eta[w[k] >> 16];
                }
                uint32_t syn = 0, par = 0, mn0 = 0x7f800000u, mn1 = 0x7f800000u;
                float x[DC];
#pragma unroll
                for (int k = 0; k < DC; ++k) {
                    const bool valid = RX || k < d;
                    x[k] = sv[k] - ev[k];
                    const uint32_t xb = __float_as_uint(x[k]);
                    const uint32_t a = valid ? (xb & 0x7fffffffu) : 0x7f800000u;
                    syn ^= valid ? __float_as_uint(sv[k]) : 0u;
                    par ^= valid ? xb : 0u;
                    mn1 = min(mn1, max(mn0, a));
                    mn0 = min(mn0, a);
                }
                unsat |= syn >> 31;
                if (msgs) {
                    float m0 = __uint_as_float(mn0), m1 = __uint_as_float(mn1);
                    if (alpha != nullptr) {
                        const int32_t c = row_class[i];
                        const float al = alpha[(t - 1) * ncls + c], be = beta[(t - 1) * ncls + c];
                        const float v0 = fmaf(al, m0, -be), v1 = fmaf(al, m1, -be);
                        m0 = v0 > 0.0f ? v0 : 0.0f;
                        m1 = v1 > 0.0f ? v1 : 0.0f;
                    }
                    const uint32_t b0 = __float_as_uint(m0), b1 = __float_as_uint(m1);
                    const uint32_t sg = par & 0x80000000u;
#pragma unroll
                    for (int k = 0; k < DC; ++k) {
                        if (RX || k < d) {
                            const uint32_t xb = __float_as_uint(x[k]);
                            const uint32_t mag = ((xb & 0x7fffffffu) == mn0) ? b1 : b0;
                            eta[w[k] >> 16] = __uint_as_float(mag | ((xb ^ sg) & 0x80000000u));
                        }
                    }
                }
            }
            const int any = __syncthreads_or((int)unsat);
            if ((early && !any) || !msgs) {
                it = (early && !any) ? t - 1 : L;
                conv = !any;
                break;
            }
            for (int32_t j = tid; j < n; j += nt) {
                const uint32_t k0 = cp[j];
                const int32_t dv = CX ? DV : (int32_t)(cp[j + 1] - k0);
                float ev[DV];
#pragma unroll
                for (int k = 0; k < DV; ++k) ev[k] = eta[k0 + (CX || k < dv ? k : 0)];
                float acc = 0.0f;
#pragma unroll
                for (int k = 0; k < DV; ++k) acc = acc + ((CX || k < dv) ? ev[k] : 0.0f); // +0 adds are exact
                s[j] = acc + r[j];
            }
            __syncthreads();
        }

        float *pf = post ? post + (size_t)f * n : nullptr;
        uint8_t *bf = bits + (size_t)f * n;
        for (int32_t j = tid; j < n; j += nt) {
            const float v = s[j];
            if (pf) pf[j] = v;
            bf[j] = v < 0.0f ? 1 : 0;
        }
        if (tid == 0) {
            iters[f] = it;
            if (ok) ok[f] = (uint8_t)conv;
        }
        __syncthreads();
    }
}

using KernelFn = decltype(&k_onchip<8, false, 8, false>);

struct Variant {
    int dc;
    bool rx;
    int dv;
    bool cx;
    KernelFn fn;
};

#define V(DC, RX, DV, CX) Variant{DC, RX, DV, CX, &k_onchip<DC, RX, DV, CX>}
// Exact-degree variants for the regular codes in use, then masked ones.
const Variant kVariants[] = {
    V(6, true, 3, true),   V(6, true, 8, false),  V(9, true, 8, false),   V(12, true, 8, false),
    V(16, true, 8, false), V(8, false, 4, false), V(8, false, 8, false),  V(16, false, 8, false),
    V(16, false, 16, false), V(32, false, 8, false), V(32, false, 16, false), V(32, false, 32, false),
};
#undef V

const Variant *pick(const ldpc_graph &g) {
    for (const Variant &v : kVariants) {
        const bool rows_ok = v.rx ? (g.dc_min == v.dc && g.dc_max == v.dc) : g.dc_max <= v.dc;
        const bool cols_ok = v.cx ? (g.dv_min == v.dv && g.dv_max == v.dv) : g.dv_max <= v.dv;
        if (rows_ok && cols_ok) return &v;
    }
    return nullptr;
}

int onchip_threads(const ldpc_graph &g) {
    // about two rows per thread, whole wavefronts, at most 256 threads
    const int want = (g.m + 1) / 2;
    int t = ((want + 63) / 64) * 64;
    return t < 64 ? 64 : (t > kMaxThreads ? kMaxThreads : t);
}

} // namespace

bool onchip_fits(const ldpc_graph &g) {
    return g.edge_tab != nullptr && pick(g) != nullptr && onchip_lds_bytes(g) + 512 <= (size_t)g.lds_max;
}

size_t onchip_workspace_bytes(const ldpc_graph &g, int32_t B) {
    (void)g;
    (void)B;
    return 256; // frame counter
}

int onchip_decode(const ldpc_graph &g, const float *llr, int32_t B, int32_t L, uint32_t flags, const float *alpha,
                  const float *beta, int32_t T, uint8_t *bits, float *post, int32_t *iters, uint8_t *ok, void *ws,
                  size_t ws_bytes, hipStream_t stream) {
    (void)T;
    if (!onchip_fits(g)) return LDPC_EUNSUPPORTED;
    if (ws == nullptr || ws_bytes < onchip_workspace_bytes(g, B)) return LDPC_EWORKSPACE;
    KernelFn fn = pick(g)->fn;
    const int threads = onchip_threads(g);
    const size_t lds = onchip_lds_bytes(g);
    if (hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return LDPC_EHIP;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)fn, threads, lds) != hipSuccess)
        return LDPC_EHIP;
    per_cu = per_cu < 1 ? 1 : per_cu;
    const int64_t want = (int64_t)g.num_cu * per_cu;
    const int32_t grid = (int32_t)(want < B ? want : B);
    uint32_t *queue = (uint32_t *)ws;
    const int32_t early = (flags & LDPC_NO_EARLY_EXIT) ? 0 : 1;
    const int32_t ncls = (int32_t)g.class_degrees.size();
    k_zero_u32<<<1, 1, 0, stream>>>(queue);
    timed_launch(K_ONCHIP, stream, [&] {
        fn<<<grid, threads, lds, stream>>>(g.row_ptr, g.edge_tab, g.col_ptr, g.row_class, g.m, g.n, (int32_t)g.E, llr,
                                            B, L, early, alpha, beta, ncls, bits, post, iters, ok, queue);
    });
    return hipGetLastError() == hipSuccess ? LDPC_OK : LDPC_EHIP;
}

} // namespace ldpc
