// On-chip Min-Sum decoder: the whole decoding state of a frame lives in LDS
// and registers, for codes whose state fits (n, E < 2^16, row and column
// degrees <= 16, at most 1024 threads of <= 2 rows and <= 8 bits each, state
// within one workgroup's LDS).
//
// Workgroups are persistent.  Each holds F = 2 frame "slots" and decodes
// both in lock step, one iteration per round; a slot whose frame stops takes
// the next frame number from an atomic counter at once, so per-frame early
// exit wastes no rounds and the graph is read from global memory only once
// per workgroup.
//
// Ownership.  Thread `tid` owns check rows tid + r*nt (r < RPT) and bits
// tid + c*nt (c < CPT).  It keeps in registers, for the whole launch, the LDS
// byte addresses of its edges' s and eta entries, and per slot the messages
// it sent along its edges in the previous iteration (eta_prev) and the
// channel LLRs of its bits.  LDS holds, per bit, s of both slots (float2) and,
// per edge in CSC order, the current messages of both slots (float2), so one
// 8-byte LDS access serves both frames.
//
// Round (iteration t of each slot):
//   check pass  per own row and slot: x_e = s_j - eta_prev_e; min0/min1 with
//               integer min/max on the bit patterns of |x| (non-negative
//               floats order like their bit patterns); sign parity = XOR of
//               the sign bits of x; then eta_e = (|x_e| == min0 ? min1 : min0)
//               with sign bit(x_e) XOR parity (Observations 1 and 2; on a tie
//               min1 == min0, so every edge at the minimum may take min1).
//               The XOR of the sign bits of the s values read per row is the
//               syndrome of the previous hard decision.
//   barrier     the per-slot "some row unsatisfied" bits are OR-reduced.
//   decisions   a slot whose previous decision is a codeword (or that has run
//               L iterations) writes its outputs and is refilled.
//   bit pass    per own bit: s_j = (+0 + eta over the column in ascending
//               check order) + r_j; a refilled slot gets s_j = r_j instead.
//   barrier
// Signs are read from sign bits: LLRs are loaded as r + 0.0f, which turns -0
// into +0; after that no s or x can be -0, so the sign bit agrees with the
// comparison v < 0 that defines sign() (sign(0) = +1).
#include "ldpc_internal.h"

namespace ldpc {
namespace {

constexpr int kF = 2; // frame slots per workgroup
typedef float vf2 __attribute__((ext_vector_type(2)));

struct Shared {          // small shared words, placed after s and eta
    int32_t first[kF];   // first frame of each slot
    int32_t next[kF][2]; // prefetched next frame of each slot, by refill parity
    uint32_t red[2];     // OR of the per-slot unsatisfied bits, by round parity
};

size_t state_bytes(const ldpc_graph &g) { return align_up(sizeof(vf2) * ((size_t)g.n + (size_t)g.E + 1), 16); }

size_t onchip_lds_bytes(const ldpc_graph &g) {
    // s[n] and eta[E + 1] (one padding slot) as float2, then Shared
    return state_bytes(g) + sizeof(Shared);
}

__global__ void k_zero_u32(uint32_t *p) { *p = 0u; }

__device__ __forceinline__ vf2 lds_ld(const unsigned char *base, uint32_t off) {
    return *reinterpret_cast<const vf2 *>(base + off);
}
__device__ __forceinline__ void lds_st(unsigned char *base, uint32_t off, vf2 v) {
    *reinterpret_cast<vf2 *>(base + off) = v;
}

// DC: row degree (RX: every row exactly DC, else at most DC); DV: column
// degree (CX: every column exactly DV, else at most DV); RPT: rows per
// thread; CPT: bits per thread (at most); MAXT: workgroup size limit (1024
// threads leave 128 VGPRs per thread, 512 leave 256).
template <int DC, bool RX, int DV, bool CX, int RPT, int CPT, int MAXT>
__global__ __launch_bounds__(MAXT) void k_onchip(
    const int32_t *__restrict__ row_ptr, const uint32_t *__restrict__ edge_tab, const int32_t *__restrict__ col_ptr,
    const int32_t *__restrict__ row_class, int32_t m, int32_t n, int32_t E, uint32_t sh_off,
    const float *__restrict__ llr, int32_t B, int32_t L, int32_t early, const float *__restrict__ alpha,
    const float *__restrict__ beta, int32_t ncls, uint8_t *__restrict__ bits, float *__restrict__ post,
    int32_t *__restrict__ iters, uint8_t *__restrict__ ok, uint32_t *__restrict__ queue) {
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
    const uint32_t eta0 = (uint32_t)sizeof(vf2) * (uint32_t)n; // byte offset of eta
    Shared *sh = reinterpret_cast<Shared *>(lds + sh_off);
    const int tid = threadIdx.x;
    const int nt = blockDim.x;

    // ---- static per-thread graph data -------------------------------------
    int32_t deg[RPT], rcls[RPT];
    uint32_t sa[RPT][DC], ea[RPT][DC]; // LDS byte addresses of s_j and eta_e
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int32_t i = tid + r * nt;
        const int32_t e0 = i < m ? row_ptr[i] : 0;
        const int32_t d = i < m ? row_ptr[i + 1] - e0 : 0;
        deg[r] = d;
        rcls[r] = (i < m && alpha != nullptr) ? row_class[i] : 0;
#pragma unroll
        for (int k = 0; k < DC; ++k) {
            const bool v = k < d;
            const uint32_t w = v ? edge_tab[e0 + k] : 0u;
            sa[r][k] = (uint32_t)sizeof(vf2) * (w & 0xffffu);
            ea[r][k] = eta0 + (uint32_t)sizeof(vf2) * (v ? (w >> 16) : (uint32_t)E); // padding slot
        }
    }
    uint32_t ckd[CPT]; // first CSC slot | degree << 16 of each own bit
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const int32_t j = tid + c * nt;
        const int32_t k0 = j < n ? col_ptr[j] : E;
        ckd[c] = (uint32_t)k0 | ((uint32_t)(j < n ? col_ptr[j + 1] - k0 : 0) << 16);
    }

    // ---- slots --------------------------------------------------------------
    if (tid == 0) {
        const int32_t base = (int32_t)atomicAdd(queue, 2u * kF);
#pragma unroll
        for (int q = 0; q < kF; ++q) {
            sh->first[q] = base + q;
            sh->next[q][0] = base + kF + q;
        }
        sh->red[0] = sh->red[1] = 0u;
    }
    __syncthreads();
    int32_t fr[kF], tt[kF], gen[kF];
#pragma unroll
    for (int q = 0; q < kF; ++q) {
        fr[q] = sh->first[q];
        tt[q] = 1;
        gen[q] = 0;
    }
    vf2 eprev[RPT][DC];
    vf2 rc[CPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r)
#pragma unroll
        for (int k = 0; k < DC; ++k) eprev[r][k] = vf2{0.0f, 0.0f};
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const int32_t j = tid + c * nt;
        rc[c] = vf2{0.0f, 0.0f};
        if (j < n) {
#pragma unroll
            for (int q = 0; q < kF; ++q) rc[c][q] = fr[q] < B ? llr[(size_t)fr[q] * n + j] + 0.0f : 0.0f; // -0 -> +0
            lds_st(lds, (uint32_t)sizeof(vf2) * (uint32_t)j, rc[c]);
        }
    }
    __syncthreads();

    for (int32_t round = 0;; ++round) {
        bool live = false;
#pragma unroll
        for (int q = 0; q < kF; ++q) live |= fr[q] < B;
        if (!live) break;

        // ---- check pass -------------------------------------------------------
        uint32_t umask = 0;
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const int32_t d = RX ? DC : deg[r];
            const bool rowv = deg[r] > 0;
            vf2 sv[DC];
#pragma unroll
            for (int k = 0; k < DC; ++k) sv[k] = lds_ld(lds, sa[r][k]);
#pragma unroll
            for (int q = 0; q < kF; ++q) {
                uint32_t syn = 0, par = 0, mn0 = 0x7f800000u, mn1 = 0x7f800000u;
                float x[DC];
#pragma unroll
                for (int k = 0; k < DC; ++k) {
                    const bool valid = RX ? rowv : (k < d);
                    x[k] = sv[k][q] - eprev[r][k][q];
                    const uint32_t xb = __float_as_uint(x[k]);
                    const uint32_t a = valid ? (xb & 0x7fffffffu) : 0x7f800000u;
                    syn ^= valid ? __float_as_uint(sv[k][q]) : 0u;
                    par ^= valid ? xb : 0u;
                    mn1 = min(mn1, max(mn0, a));
                    mn0 = min(mn0, a);
                }
                umask |= (syn >> 31) << q;
                uint32_t b0 = mn0, b1 = mn1;
                if (alpha != nullptr && tt[q] <= L && rowv) {
                    const float al = alpha[(tt[q] - 1) * ncls + rcls[r]], be = beta[(tt[q] - 1) * ncls + rcls[r]];
                    const float v0 = fmaf(al, __uint_as_float(mn0), -be), v1 = fmaf(al, __uint_as_float(mn1), -be);
                    b0 = __float_as_uint(v0 > 0.0f ? v0 : 0.0f);
                    b1 = __float_as_uint(v1 > 0.0f ? v1 : 0.0f);
                }
                const uint32_t sg = par & 0x80000000u;
#pragma unroll
                for (int k = 0; k < DC; ++k) {
                    const uint32_t xb = __float_as_uint(x[k]);
                    const uint32_t mag = ((xb & 0x7fffffffu) == mn0) ? b1 : b0;
                    eprev[r][k][q] = __uint_as_float(mag | ((xb ^ sg) & 0x80000000u));
                }
            }
#pragma unroll
            for (int k = 0; k < DC; ++k)
                if (RX ? rowv : (k < d)) lds_st(lds, ea[r][k], eprev[r][k]);
        }

        // ---- per-slot syndrome over the workgroup ------------------------------
        const int p = round & 1;
        uint32_t wm = 0;
#pragma unroll
        for (int q = 0; q < kF; ++q) wm |= (__ballot((umask >> q) & 1u) != 0ull ? 1u : 0u) << q;
        if ((tid & 63) == 0 && wm) atomicOr(&sh->red[p], wm);
        __syncthreads();
        const uint32_t U = sh->red[p];
        if (tid == 0) sh->red[p ^ 1] = 0u;

        // ---- decisions, outputs, refills --------------------------------------
        uint32_t fin = 0;
#pragma unroll
        for (int q = 0; q < kF; ++q) {
            if (fr[q] >= B) continue;
            const bool clean = ((U >> q) & 1u) == 0u;
            if (!((early && clean) || tt[q] > L)) continue;
            fin |= 1u << q;
            const int32_t f = fr[q];
#pragma unroll
            for (int c = 0; c < CPT; ++c) {
                const int32_t j = tid + c * nt;
                if (j < n) {
                    const float v = lds_ld(lds, (uint32_t)sizeof(vf2) * (uint32_t)j)[q];
                    if (post) post[(size_t)f * n + j] = v;
                    bits[(size_t)f * n + j] = v < 0.0f ? 1 : 0;
                }
            }
            if (tid == 0) {
                iters[f] = (early && clean) ? tt[q] - 1 : L;
                if (ok) ok[f] = clean ? 1 : 0;
            }
            const int32_t nf = sh->next[q][gen[q] & 1];
            if (tid == 0) sh->next[q][(gen[q] + 1) & 1] = (int32_t)atomicAdd(queue, 1u);
            fr[q] = nf;
            gen[q] += 1;
#pragma unroll
            for (int r = 0; r < RPT; ++r)
#pragma unroll
                for (int k = 0; k < DC; ++k) eprev[r][k][q] = 0.0f;
        }

        // ---- bit pass -------------------------------------------------------------
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            const int32_t j = tid + c * nt;
            if (j < n) {
                const uint32_t base = eta0 + (uint32_t)sizeof(vf2) * (ckd[c] & 0xffffu);
                const int32_t dv = (int32_t)(ckd[c] >> 16);
                vf2 ev[DV];
#pragma unroll
                for (int k = 0; k < DV; ++k)
                    ev[k] = lds_ld(lds, base + (uint32_t)sizeof(vf2) * (uint32_t)(CX || k < dv ? k : 0));
                vf2 acc = vf2{0.0f, 0.0f};
#pragma unroll
                for (int k = 0; k < DV; ++k)
                    acc = acc + ((CX || k < dv) ? ev[k] : vf2{0.0f, 0.0f}); // +0 adds are exact
                vf2 sn = acc + rc[c];
#pragma unroll
                for (int q = 0; q < kF; ++q) {
                    if ((fin >> q) & 1u) {
                        const float v = fr[q] < B ? llr[(size_t)fr[q] * n + j] + 0.0f : 0.0f;
                        rc[c][q] = v;
                        sn[q] = v;
                    }
                }
                lds_st(lds, (uint32_t)sizeof(vf2) * (uint32_t)j, sn);
            }
        }
#pragma unroll
        for (int q = 0; q < kF; ++q) tt[q] = ((fin >> q) & 1u) ? 1 : tt[q] + 1;
        __syncthreads();
    }
}

using KernelFn = decltype(&k_onchip<6, true, 3, true, 2, 4, 512>);

struct Variant {
    int dc;
    bool rx;
    int dv;
    bool cx;
    int rpt;
    int cpt;
    int max_threads;
    KernelFn fn;
};

#define V(DC, RX, DV, CX, RPT, CPT, MAXT) \
    Variant{DC, RX, DV, CX, RPT, CPT, MAXT, &k_onchip<DC, RX, DV, CX, RPT, CPT, MAXT>}
// Exact-degree variants for the regular codes in use first, then masked ones.
const Variant kVariants[] = {
    V(6, true, 3, true, 2, 4, 512),    V(6, true, 8, false, 2, 4, 512),   V(9, true, 8, false, 1, 4, 1024),
    V(12, true, 8, false, 1, 4, 512),  V(16, true, 8, false, 1, 8, 512),  V(8, false, 8, false, 2, 4, 512),
    V(16, false, 16, false, 1, 8, 512),
};
#undef V

// Threads: whole wavefronts, enough for RPT rows and CPT bits per thread.
int threads_for(const ldpc_graph &g, const Variant &v) {
    const int a = (g.m + v.rpt - 1) / v.rpt, b = (g.n + v.cpt - 1) / v.cpt;
    const int want = a > b ? a : b;
    const int t = ((want + 63) / 64) * 64;
    return t < 64 ? 64 : t;
}

const Variant *pick(const ldpc_graph &g) {
    for (const Variant &v : kVariants) {
        const bool rows_ok = v.rx ? (g.dc_min == v.dc && g.dc_max == v.dc) : g.dc_max <= v.dc;
        const bool cols_ok = v.cx ? (g.dv_min == v.dv && g.dv_max == v.dv) : g.dv_max <= v.dv;
        if (rows_ok && cols_ok && threads_for(g, v) <= v.max_threads) return &v;
    }
    return nullptr;
}

} // namespace

bool onchip_fits(const ldpc_graph &g) {
    return g.edge_tab != nullptr && pick(g) != nullptr && onchip_lds_bytes(g) + 1024 <= (size_t)g.lds_max;
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
    const Variant &var = *pick(g);
    KernelFn fn = var.fn;
    const int threads = threads_for(g, var);
    const size_t lds = onchip_lds_bytes(g);
    if (hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return LDPC_EHIP;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)fn, threads, lds) != hipSuccess)
        return LDPC_EHIP;
    per_cu = per_cu < 1 ? 1 : per_cu;
    const int64_t slot_groups = ((int64_t)B + 2 * kF - 1) / (2 * kF);
    const int64_t want = (int64_t)g.num_cu * per_cu;
    const int32_t grid = (int32_t)(want < slot_groups ? want : slot_groups);
    uint32_t *queue = (uint32_t *)ws;
    const int32_t early = (flags & LDPC_NO_EARLY_EXIT) ? 0 : 1;
    const int32_t ncls = (int32_t)g.class_degrees.size();
    const uint32_t sh_off = (uint32_t)state_bytes(g);
    k_zero_u32<<<1, 1, 0, stream>>>(queue);
    timed_launch(K_ONCHIP, stream, [&] {
        fn<<<grid, threads, lds, stream>>>(g.row_ptr, g.edge_tab, g.col_ptr, g.row_class, g.m, g.n, (int32_t)g.E,
                                            sh_off, llr, B, L, early, alpha, beta, ncls, bits, post, iters, ok, queue);
    });
    return hipGetLastError() == hipSuccess ? LDPC_OK : LDPC_EHIP;
}

} // namespace ldpc
