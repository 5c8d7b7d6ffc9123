// On-chip Min-Sum decoder, device side (shared by the kernel sources of
// each register budget and the host side in decode_onchip.hip).
//
// The whole decoding state of a frame lives in LDS
// and registers, for codes whose state fits (n, E < 2^16, row and column
// degrees <= 16, at most 512 threads of <= 2 rows and <= 8 bits each, state
// within one workgroup's LDS).
//
// Workgroups are persistent.  Each holds F frame "slots" (F = 2 or 4, a
// choice of the kernel variant) and decodes them in lock step, one iteration
// per round; a slot whose frame stops takes the next frame number from
// atomic counters at once (several, so that no single address serialises
// the workgroups), so per-frame early exit wastes no rounds and the graph is
// read from global memory only once per workgroup.
//
// Ownership.  Thread `tid` owns check rows tid + r*nt (r < RPT) and bits
// tid + c*nt (c < CPT).  It keeps in registers, for the whole launch, the LDS
// byte addresses of its edges' s and eta entries, and per slot the messages
// it sent along its edges in the previous iteration (eta_prev) and the
// channel LLRs of its bits.  LDS holds, per bit, s of all slots (F floats)
// and, per edge in CSC order, the current messages of all slots (F floats),
// so one 8- or 16-byte LDS access serves all F frames.
//
// Round (iteration t of each slot):
//   check pass  per own row and slot: x_e = s_j - eta_prev_e; min0/min1 of
//               |x| by a tournament of three-input min / median instructions
//               (|x| is a free source modifier); sign parity = XOR of the sign
//               bits of x; then eta_e = (|x_e| == min0 ? min1 : min0) with
//               sign bit(x_e) XOR parity (Observations 1 and 2; on a tie
//               min1 == min0, so every edge at the minimum may take min1),
//               formed for plain Min-Sum as K - clamp(x_e, -min1, min1) on
//               the bit patterns (edge_message in minsum_row.h), for learned
//               weights by a compare and a select of the two weighted
//               magnitudes.  The XOR of the sign bits of the s values read
//               per row is the syndrome of the previous hard decision.
//   barrier     the per-slot "some row unsatisfied" bits are OR-reduced.
//   decisions   a slot whose previous decision is a codeword (or that has run
//               L iterations) writes its outputs and is refilled.
//   bit pass    per own bit: s_j = (eta over the column in ascending check
//               order) + r_j; a refilled slot gets s_j = r_j instead.
//   barrier
// Signs are read from sign bits: LLRs are loaded as r + 0.0f, which turns -0
// into +0; after that no s or x can be -0, so the sign bit agrees with the
// comparison v < 0 that defines sign() (sign(0) = +1).  For the same reason
// the column sum may start from its first message instead of from +0: the
// two partial sums can differ only in the sign of a zero, and adding an r
// that is not -0 gives the same s either way.
#pragma once

#include <algorithm>

#include "ldpc_internal.h"
#include "minsum_row.h"

namespace ldpc {
namespace onchip {

constexpr int kMaxF = 4; // frame slots per workgroup: 2 or 4 (a kernel variant's choice)
template <int F> struct Vec;
template <> struct Vec<1> {
    typedef float type __attribute__((ext_vector_type(1)));
};
template <> struct Vec<2> {
    typedef float type __attribute__((ext_vector_type(2)));
};
template <> struct Vec<4> {
    typedef float type __attribute__((ext_vector_type(4)));
};

struct Shared {          // small shared words, placed after s and eta
    int32_t first[kMaxF];   // first frame of each slot
    int32_t next[kMaxF][2]; // prefetched next frame of each slot, by refill parity
    uint32_t red[2];     // OR of the per-slot unsatisfied bits, by round parity
    int32_t hc;          // thread 0: the frame counter this workgroup draws from
    uint32_t dead;       // thread 0: counters found exhausted
};

// Frame counters.  One counter handing out every frame number would be a
// single address that every refill of every workgroup increments atomically;
// when frames stop after a few iterations, those atomics (one per frame, all
// serialised at one address) bound the decoder.  So each job has kQueues
// counters, each in a 128-byte line of its own: counter c hands out frames
// c, c + kQueues, c + 2 kQueues, ...  A workgroup draws from one counter and
// moves to another live one when it finds its counter exhausted, so all
// frames are taken before any workgroup runs out.
constexpr int kQueues = 16;
constexpr int kQueueStride = 32; // 32-bit words between counters
// the counters, then one word (in a line of its own) with a bit for every
// counter some workgroup has found exhausted
constexpr int kQueueWords = (kQueues + 1) * kQueueStride;

// Frame number of the k-th value taken from counter c of nq.
__device__ __forceinline__ int64_t frame_of(uint32_t k, int32_t c, int32_t nq) { return (int64_t)k * nq + c; }

// Counters a batch of B frames uses: one per 1,024 frames, at most kQueues
// (a small batch needs no spreading, and every counter a workgroup finds
// exhausted costs it one atomic round trip at the end).
inline int32_t queues_for(int32_t B) {
    const int32_t q = B / 1024;
    return q < 1 ? 1 : (q > kQueues ? kQueues : q);
}

// The next live counter after c, or c when none is left.
__device__ __forceinline__ int32_t next_live(int32_t c, uint32_t dead, int32_t nq) {
    for (int d = 1; d < nq; ++d) {
        const int32_t x = (c + d) % nq;
        if (!((dead >> x) & 1u)) return x;
    }
    return c;
}

// Records that counter c is exhausted and learns which others are, in one
// atomic on the shared exhausted-counter word.
__device__ __forceinline__ uint32_t mark_dead(uint32_t *queue, int32_t c, uint32_t dead) {
    return dead | (1u << c) | atomicOr(queue + kQueues * kQueueStride, 1u << c);
}

// One thread: a frame number below B from the live counters (blocking), or B
// when all are exhausted.  `hc` is the counter to try first (live unless all
// are dead); each failed attempt marks at least one more counter dead, so
// the loop ends after at most nq attempts.
__device__ __forceinline__ int32_t take_frame(uint32_t *queue, int32_t B, int32_t nq, int32_t &hc, uint32_t &dead) {
    const uint32_t all = (1u << nq) - 1u;
    while ((dead & all) != all) {
        if ((dead >> hc) & 1u) hc = next_live(hc, dead, nq); // some counter is live
        const int64_t f = frame_of(atomicAdd(queue + hc * kQueueStride, 1u), hc, nq);
        if (f < B) return (int32_t)f;
        dead = mark_dead(queue, hc, dead);
    }
    return B;
}

// s[n] and eta[E + 1] (one padding slot), F floats per entry, then Shared
inline size_t state_bytes(const ldpc_graph &g, int F) {
    return align_up(sizeof(float) * (size_t)F * ((size_t)g.n + (size_t)g.E + 1), 16);
}


// The bank-conflict-free layout (two frame slots, 8-byte entries): s[n], then
// the messages from a 256-byte boundary (so that a position's bank class is
// the position modulo 32), cf.npos entries.
inline uint32_t cf_eta_offset(const ldpc_graph &g) { return (uint32_t)align_up(8 * (size_t)g.n, 256); }
inline size_t cf_state_bytes(const ldpc_graph &g) { return align_up(cf_eta_offset(g) + 8 * (size_t)g.cf.npos, 16); }

template <class V> __device__ __forceinline__ V lds_ld(const unsigned char *base, uint32_t off) {
    return *reinterpret_cast<const V *>(base + off);
}
template <class V> __device__ __forceinline__ void lds_st(unsigned char *base, uint32_t off, V v) {
    *reinterpret_cast<V *>(base + off) = v;
}
template <class V> __device__ __forceinline__ V vzero() {
    V z;
#pragma unroll
    for (int q = 0; q < (int)(sizeof(V) / sizeof(float)); ++q) z[q] = 0.0f;
    return z;
}

// Messages an own bit slot c reads in the bit pass: DV, or with a column
// degree profile DVP (bits placed in ascending degree, 4 bits per slot
// index) the largest degree among the bits of slot index c.
template <uint32_t DVP, int DV> __host__ __device__ constexpr int slot_cap(int c) {
    return DVP == 0u ? DV : (int)((DVP >> (4 * c)) & 15u);
}
template <uint32_t DVP, int DV, int CPT> __host__ __device__ constexpr int cap_sum() {
    int t = 0;
    for (int c = 0; c < CPT; ++c) t += slot_cap<DVP, DV>(c);
    return t;
}

// One decoding job: a graph, its frames and outputs.
struct Job {
    const int32_t *row_ptr;
    const uint32_t *edge_tab;
    const int32_t *col_ptr;
    const int32_t *row_class;
    int32_t m, n, E;
    uint32_t sh_off; // LDS byte offset of Shared for this graph
    const float *llr;
    int32_t B;
    uint8_t *bits;
    float *post;
    int32_t *iters;
    uint8_t *ok;
    const float *alpha, *beta; // learned weights (T x ncls) or null
    int32_t ncls;
    int32_t variant;  // index into kVariants
    uint32_t *queue;  // kQueues frame counters (kQueueStride words apart), zero before the launch
    int32_t nq;       // counters in use (queues_for(B))
    // bank-conflict-free layout (CF variants): tables of the graph, the LDS
    // byte offset of the messages and their number of positions
    const uint32_t *cf_edge;
    const uint32_t *cf_bitpos;
    const int32_t *cf_slot_bit;
    const int32_t *cf_row_class;
    uint32_t cf_eta_off;
    int32_t cf_npos;
};

// Decodes all frames of one job with the workgroup (see the file comment).
// DC: row degree (RX: every row exactly DC, else at most DC); DV: column
// degree (CX: every column exactly DV, else at most DV); RPT: rows per
// thread; CPT: bits per thread (at most); F: frame slots.  Every thread of
// the workgroup calls it; it returns once all frames of the job handed to
// this workgroup are done.
// NMS: the learned check update (J.alpha, J.beta non-null); plain Min-Sum
// instantiations carry no trace of it.
// CF: the bank-conflict-free layout of the graph (layout.hip): rows and bits
// in the thread slots its tables give, and every edge's message at an LDS
// position of its own; needs rows of degree DC, a layout built for this
// geometry (RPT, CPT) and a bit-side stride of DV (columns of lower degree
// read zero messages past their degree, so the bit pass is the exact-degree
// one; with a column degree profile DVP the bits are sorted by degree and own
// bit slot c reads slot_cap(c) messages).  CF & 3 = 1: the check pass reads
// each edge's previous message back from its position (no registers for
// them); CF & 3 = 2: it keeps them in registers, as without the layout (a
// third fewer LDS reads).  CF & 4: columns
// padded to DV (else every column has degree DV, and the zero positions are
// never read by a bit below n).
template <int DC, bool RX, int DV, bool CX, int RPT, int CPT, int F, bool NMS, int CF, uint32_t DVP = 0u>
__device__ __forceinline__ void run_onchip(const Job &J, int32_t L, int32_t early, unsigned char *lds) {
    constexpr bool kLay = (CF & 3) != 0;     // the layout's tables
    constexpr bool kPrevLds = (CF & 3) == 1; // previous messages read from LDS
    constexpr bool kPad = (CF & 4) != 0;     // columns padded with zero messages
    static_assert(!kLay || (RX && CX && F == 2), "layout: rows of one degree, padded columns, 8-byte entries");
    typedef typename Vec<F>::type V;
    constexpr uint32_t kEnt = sizeof(V); // bytes of one LDS entry (F floats)
    // read all s (messages) of the check (bit) pass up front when that takes
    // at most 32 registers (s: only with exact column degrees; the masked
    // variants, and the layout with padded columns, need those registers to
    // stay within four waves per SIMD)
    constexpr bool kPrefetchS = RPT > 1 && RPT * DC * F <= 32 && CX && !kPad;
    constexpr bool kPrefetchEta = CPT > 1 && cap_sum<DVP, DV, CPT>() * F <= 32;
    // keep the channel LLRs of every slot's next frame in registers, read
    // ahead, when that takes at most 8 registers and the column degree is
    // exact (the masked-column variants are the ones near the 128-register
    // budget of four waves per SIMD, which the 8 would push into spills);
    // the learned update only with exact row degrees, where its weights sit
    // in scalar registers and leave room for the 8, and not in the
    // conflict-free layout, whose bit-side message addresses take them
    constexpr bool kAheadLLR = CPT * F <= 8 && CX && (!NMS || (RX && !kLay));
    const int32_t *__restrict__ row_ptr = J.row_ptr;
    const uint32_t *__restrict__ edge_tab = J.edge_tab;
    const int32_t *__restrict__ col_ptr = J.col_ptr;
    const int32_t *__restrict__ row_class = J.row_class;
    const int32_t m = J.m, n = J.n, E = J.E;
    const uint32_t sh_off = J.sh_off;
    const float *__restrict__ llr = J.llr;
    const int32_t B = J.B;
    uint8_t *__restrict__ bits = J.bits;
    float *__restrict__ post = J.post;
    int32_t *__restrict__ iters = J.iters;
    uint8_t *__restrict__ ok = J.ok;
    const float *__restrict__ alpha = J.alpha;
    const float *__restrict__ beta = J.beta;
    const int32_t ncls = J.ncls;
    uint32_t *__restrict__ queue = J.queue;
    const int32_t nq = J.nq;
    const uint32_t eta0 = kLay ? J.cf_eta_off : kEnt * (uint32_t)n; // byte offset of eta
    Shared *sh = reinterpret_cast<Shared *>(lds + sh_off);
    const int tid = threadIdx.x;
    const int nt = blockDim.x;

    // ---- static per-thread graph data -------------------------------------
    int32_t deg[RPT], rcls[RPT];
    uint32_t sa[RPT][DC], ea[RPT][DC]; // LDS byte addresses of s_j and eta_e
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int32_t i = tid + r * nt;
        if constexpr (kLay) {
            // every slot has a table entry (slots past m: bit 0, the spare position)
            deg[r] = DC;
            rcls[r] = NMS ? J.cf_row_class[i] : 0;
#pragma unroll
            for (int k = 0; k < DC; ++k) {
                const uint32_t w = J.cf_edge[(size_t)i * DC + k];
                sa[r][k] = kEnt * (w & 0xffffu);
                ea[r][k] = eta0 + kEnt * (w >> 16);
            }
            continue;
        }
        const int32_t e0 = i < m ? row_ptr[i] : 0;
        const int32_t d = i < m ? row_ptr[i + 1] - e0 : 0;
        deg[r] = d;
        rcls[r] = (NMS && i < m) ? row_class[i] : 0;
#pragma unroll
        for (int k = 0; k < DC; ++k) {
            const bool v = k < d;
            const uint32_t w = v ? edge_tab[e0 + k] : 0u;
            sa[r][k] = kEnt * (w & 0xffffu);
            ea[r][k] = eta0 + kEnt * (v ? (w >> 16) : (uint32_t)E); // padding slot
        }
    }
    uint32_t ckd[CPT]; // first CSC slot | degree << 16 of each own bit
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const int32_t j = tid + c * nt;
        const int32_t k0 = j < n ? col_ptr[j] : E;
        ckd[c] = (uint32_t)k0 | ((uint32_t)(j < n ? col_ptr[j + 1] - k0 : 0) << 16);
    }
    // Own bit slots p = tid + c nt (LDS s at kEnt p): the bit index they hold
    // (frame I/O) and, in the layout, their messages' LDS addresses.
    int32_t gj[CPT];
    uint32_t ba[kLay ? CPT : 1][kLay ? DV : 1];
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const int32_t p = tid + c * nt;
        gj[c] = kLay ? (p < n ? J.cf_slot_bit[p] : 0) : p;
        if constexpr (kLay) {
#pragma unroll
            for (int u = 0; u < DV; ++u)
                if (u < slot_cap<DVP, DV>(c))
                    ba[c][u] = eta0 + kEnt * (kPad || p < n ? J.cf_bitpos[(size_t)p * DV + u] : (uint32_t)(J.cf_npos - 1));
        }
    }

    // ---- slots --------------------------------------------------------------
    if (tid == 0) {
        // 2 F consecutive values of the home counter with one atomic; any
        // that fall past B come from the other counters
        int32_t hc = (int32_t)(blockIdx.x % (uint32_t)nq);
        uint32_t dead = 0u;
        const uint32_t k0 = atomicAdd(queue + hc * kQueueStride, 2u * F);
        const int32_t home = hc;
        int32_t fs[2 * F];
#pragma unroll
        for (int i = 0; i < 2 * F; ++i) {
            const int64_t f = frame_of(k0 + (uint32_t)i, home, nq);
            if (f < B) {
                fs[i] = (int32_t)f;
            } else {
                if (!((dead >> home) & 1u)) {
                    dead = mark_dead(queue, home, dead);
                    hc = next_live(home, dead, nq);
                }
                fs[i] = take_frame(queue, B, nq, hc, dead);
            }
        }
#pragma unroll
        for (int q = 0; q < F; ++q) {
            sh->first[q] = fs[q];
            sh->next[q][0] = fs[F + q];
        }
        sh->hc = hc;
        sh->dead = dead;
        sh->red[0] = sh->red[1] = 0u;
    }
    __syncthreads();
    int32_t fr[F], tt[F], gen[F], ph[F]; // ph = (tt - 1) mod the test period
#pragma unroll
    for (int q = 0; q < F; ++q) {
        fr[q] = __builtin_amdgcn_readfirstlane(sh->first[q]); // uniform: kept in scalar registers
        tt[q] = 1;
        gen[q] = 0;
        ph[q] = 0;
    }
    V eprev[RPT][DC];
    V rc[CPT];
    // Channel LLRs of each slot's next frame (its frame number is known one
    // refill ahead), read while the slot still decodes its current frame, so
    // that a refill does not wait for global memory.
    V rnx[CPT];
    uint32_t pend = 0; // slots whose next frame's LLRs are still to be read
    if constexpr (kAheadLLR) {
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            const int32_t j = tid + c * nt;
            rnx[c] = vzero<V>();
#pragma unroll
            for (int q = 0; q < F; ++q) {
                const int32_t nx = __builtin_amdgcn_readfirstlane(sh->next[q][0]);
                rnx[c][q] = llr[(size_t)(nx < B ? nx : 0) * n + (j < n ? gj[c] : 0)];
            }
        }
    }
#pragma unroll
    for (int r = 0; r < RPT; ++r)
#pragma unroll
        for (int k = 0; k < DC; ++k) eprev[r][k] = vzero<V>();
    if constexpr (kPrevLds) { // every message starts at 0 (first iteration of every slot)
        for (int32_t e = tid; e < J.cf_npos; e += nt) lds_st<V>(lds, eta0 + kEnt * (uint32_t)e, vzero<V>());
    } else if constexpr (kPad) { // the 32 zero positions (before the last one) stay 0
        if (tid < 32) lds_st<V>(lds, eta0 + kEnt * (uint32_t)(J.cf_npos - 33 + tid), vzero<V>());
    }
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const int32_t j = tid + c * nt;
        rc[c] = vzero<V>();
        if (j < n) {
#pragma unroll
            for (int q = 0; q < F; ++q)
                rc[c][q] = fr[q] < B ? llr[(size_t)fr[q] * n + gj[c]] + 0.0f : 0.0f; // -0 -> +0
            lds_st<V>(lds, kEnt * (uint32_t)j, rc[c]);
        }
    }
    __syncthreads();

    for (int32_t round = 0;; ++round) {
        // The slot state is the same in every lane; saying so keeps it in
        // scalar registers and makes the branches on it scalar.
#pragma unroll
        for (int q = 0; q < F; ++q) {
            fr[q] = __builtin_amdgcn_readfirstlane(fr[q]);
            tt[q] = __builtin_amdgcn_readfirstlane(tt[q]);
            gen[q] = __builtin_amdgcn_readfirstlane(gen[q]);
            ph[q] = __builtin_amdgcn_readfirstlane(ph[q]);
        }
        bool live = false;
#pragma unroll
        for (int q = 0; q < F; ++q) live |= fr[q] < B;
        if (!live) break;

        // ---- check pass -------------------------------------------------------
        // When the registers allow, the s values of all own rows are read
        // before the first row's messages are written (the compiler cannot
        // move a read of s above an LDS write it cannot tell apart from it),
        // so the reads of later rows overlap the work of earlier ones.
        // In the layout (CF), each edge's previous message is read from its
        // LDS position as well, in the same batch.
        V svp[RPT][DC], pvp[kPrevLds ? RPT : 1][kPrevLds ? DC : 1];
        if constexpr (kPrefetchS) {
#pragma unroll
            for (int r = 0; r < RPT; ++r)
#pragma unroll
                for (int k = 0; k < DC; ++k) {
                    svp[r][k] = lds_ld<V>(lds, sa[r][k]);
                    if constexpr (kPrevLds) pvp[r][k] = lds_ld<V>(lds, ea[r][k]);
                }
        }
        // per slot, the OR of the syndrome words of the own rows: its sign bit
        // says that one of them is unsatisfied
        uint32_t usyn[F];
#pragma unroll
        for (int q = 0; q < F; ++q) usyn[q] = 0u;
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const int32_t d = RX ? DC : deg[r];
            const bool rowv = RX ? (tid + r * nt < m) : deg[r] > 0; // RX: recomputed, saves a register
            V sv[DC], pv_[DC], msg[DC];
#pragma unroll
            for (int k = 0; k < DC; ++k) {
                sv[k] = kPrefetchS ? svp[r][k] : lds_ld<V>(lds, sa[r][k]);
                if constexpr (kPrevLds) pv_[k] = kPrefetchS ? pvp[r][k] : lds_ld<V>(lds, ea[r][k]);
                else pv_[k] = eprev[r][k];
            }
#pragma unroll
            for (int q = 0; q < F; ++q) {
                // RX: every edge of a real row is valid; rows past m compute
                // garbage that only reaches the padding slot and is masked
                // out of the syndrome.  Otherwise edges k >= d are masked.
                uint32_t xb[DC];
                float a[DC];
#pragma unroll
                for (int k = 0; k < DC; ++k) {
                    const bool valid = RX || k < d;
                    const float x = sv[k][q] - pv_[k][q];
                    xb[k] = __float_as_uint(x);
                    a[k] = valid ? fabsf(x) : __builtin_inff();
                }
                float mn0, mn1;
                min_pair<DC>(a, mn0, mn1);
                uint32_t pv[DC], sb[DC];
#pragma unroll
                for (int k = 0; k < DC; ++k) {
                    const bool valid = RX || k < d;
                    pv[k] = valid ? xb[k] : 0u;
                    sb[k] = valid ? __float_as_uint(sv[k][q]) : 0u;
                }
                uint32_t par = xor_all<DC>(pv), syn = xor_all<DC>(sb);
                // RX: a row past m reads bit 0's s on all DC edges, so with DC
                // even its syndrome is 0 without a mask
                if (RX && (DC % 2) == 1 && !rowv) syn = 0u;
                usyn[q] |= syn;
                if constexpr (NMS) {
                    uint32_t b0 = __float_as_uint(mn0), b1 = __float_as_uint(mn1);
                    if (tt[q] <= L && rowv) {
                        float al, be;
                        if constexpr (RX) {
                            // every row has degree DC, so one class: the
                            // weights are the workgroup's, read through the
                            // scalar cache (constant address space) instead of
                            // a vector load each lane waits on.  A scalar load
                            // ignores the lane mask, so its index is clamped
                            // into the table (1 <= tt <= L <= T inside this
                            // branch; the clamp keeps it there whatever code
                            // the compiler emits around the branch).
                            int32_t tw = tt[q] > L ? L : tt[q];
                            tw = tw < 1 ? 1 : tw; // L = 0: no iteration reads it
                            const int32_t wi = __builtin_amdgcn_readfirstlane((tw - 1) * ncls);
                            al = *(const __attribute__((address_space(4))) float *)(alpha + wi);
                            be = *(const __attribute__((address_space(4))) float *)(beta + wi);
                        } else {
                            al = alpha[(tt[q] - 1) * ncls + rcls[r]];
                            be = beta[(tt[q] - 1) * ncls + rcls[r]];
                        }
                        const float v0 = fmaf(al, mn0, -be), v1 = fmaf(al, mn1, -be);
                        b0 = __float_as_uint(v0 > 0.0f ? v0 : 0.0f);
                        b1 = __float_as_uint(v1 > 0.0f ? v1 : 0.0f);
                    }
                    // the row's sign parity folded into both magnitudes; each
                    // edge then XORs in its own sign bit.  The empty asm keeps
                    // the compiler from moving the parity XOR back onto every edge.
                    const uint32_t sg = par & 0x80000000u;
                    uint32_t b0s = b0 ^ sg, b1s = b1 ^ sg;
                    asm("" : "+v"(b0s), "+v"(b1s));
#pragma unroll
                    for (int k = 0; k < DC; ++k)
                        msg[k][q] = __uint_as_float(((a[k] == mn0) ? b1s : b0s) ^ (xb[k] & 0x80000000u));
                } else {
                    // two instructions per edge (edge_message); a zero message's
                    // sign changes no s (r is never -0, and s = sum + r)
                    const uint32_t K = row_word(mn0, mn1, par);
#pragma unroll
                    for (int k = 0; k < DC; ++k) msg[k][q] = edge_message(__uint_as_float(xb[k]), mn1, K);
                }
            }
#pragma unroll
            for (int k = 0; k < DC; ++k) {
                if constexpr (!kPrevLds) eprev[r][k] = msg[k];
                if (RX || k < d) lds_st<V>(lds, ea[r][k], msg[k]); // rows past m write the padding slot
            }
        }

        // ---- per-slot syndrome over the workgroup ------------------------------
        const int p = round & 1;
        uint32_t wm = 0;
#pragma unroll
        for (int q = 0; q < F; ++q) wm |= (__ballot((int32_t)usyn[q] < 0) != 0ull ? 1u : 0u) << q;
        if ((tid & 63) == 0 && wm) atomicOr(&sh->red[p], wm);
        __syncthreads();
        const uint32_t U = __builtin_amdgcn_readfirstlane(sh->red[p]);
        if (tid == 0) sh->red[p ^ 1] = 0u;
        if constexpr (kAheadLLR) {
            // the next frames of the slots refilled last round (stored by
            // thread 0 in last round's decision step)
            pend = __builtin_amdgcn_readfirstlane(pend);
            if (pend) {
#pragma unroll
                for (int q = 0; q < F; ++q) {
                    if (!((pend >> q) & 1u)) continue;
                    const int32_t nx = __builtin_amdgcn_readfirstlane(sh->next[q][gen[q] & 1]);
                    // Unconditional loads from a valid address (frame 0 and bit 0
                    // stand in past B and n; a dead slot's or an absent bit's
                    // values are never output), and no arithmetic on the value
                    // here: anything that reads it would make the wavefront wait
                    // for the load now instead of at the slot's next refill.
#pragma unroll
                    for (int c = 0; c < CPT; ++c) {
                        const int32_t j = tid + c * nt;
                        rnx[c][q] = llr[(size_t)(nx < B ? nx : 0) * n + (j < n ? gj[c] : 0)];
                    }
                }
                pend = 0;
            }
        }

        // ---- decisions, outputs, refills --------------------------------------
        uint32_t fin = 0;
#pragma unroll
        for (int q = 0; q < F; ++q) {
            if (fr[q] >= B) continue;
            // a codeword test is due when the decision's iteration tt - 1 is
            // a multiple of the period (early = 0: never)
            const bool clean = ((U >> q) & 1u) == 0u && ph[q] == 0 && early != 0;
            if (!(clean || tt[q] > L)) continue;
            fin |= 1u << q;
            const int32_t f = fr[q];
#pragma unroll
            for (int c = 0; c < CPT; ++c) {
                const int32_t j = tid + c * nt;
                if (j < n) {
                    const float v = lds_ld<V>(lds, kEnt * (uint32_t)j)[q];
                    if (post) post[(size_t)f * n + gj[c]] = v;
                    bits[(size_t)f * n + gj[c]] = v < 0.0f ? 1 : 0;
                }
            }
            if (tid == 0) {
                iters[f] = clean ? tt[q] - 1 : L;
                if (ok) ok[f] = ((U >> q) & 1u) == 0u ? 1 : 0;
            }
            const int32_t nf = __builtin_amdgcn_readfirstlane(sh->next[q][gen[q] & 1]);
            if (tid == 0) { // the slot's frame after next
                int32_t hc = sh->hc;
                uint32_t dead = sh->dead;
                sh->next[q][(gen[q] + 1) & 1] = take_frame(queue, B, nq, hc, dead);
                sh->hc = hc;
                sh->dead = dead;
            }
            fr[q] = nf;
            gen[q] += 1;
            if constexpr (!kPrevLds) { // (else the bit pass zeroes the slot's messages in LDS)
#pragma unroll
                for (int r = 0; r < RPT; ++r)
#pragma unroll
                    for (int k = 0; k < DC; ++k) eprev[r][k][q] = 0.0f;
            }
        }

        fin = __builtin_amdgcn_readfirstlane(fin);
        pend = fin;
        // next round's iteration numbers (the bit pass below does not use
        // them; updated here, they stay out of its divergent branches)
#pragma unroll
        for (int q = 0; q < F; ++q) {
            const bool refilled = (fin >> q) & 1u;
            tt[q] = refilled ? 1 : tt[q] + 1;
            ph[q] = (refilled || ph[q] + 1 == early) ? 0 : ph[q] + 1;
        }

        // ---- bit pass -------------------------------------------------------------
        // As in the check pass: when the registers allow, the messages of all
        // own bits are read before the first s is written; otherwise those of
        // the next own bit are read before this bit's s is written (the
        // compiler cannot move a read of a message above an LDS write it
        // cannot tell apart from it), so each bit's reads overlap the previous
        // bit's sum.  Every own slot reads valid addresses (the layout's
        // tables cover all slots; otherwise bits past n read bit 0's or the
        // padding slot); only bits below n write s.  CF: each message at its
        // own position (ba), in ascending check order.
        if constexpr (kPrefetchEta) {
            V evp[CPT][DV];
#pragma unroll
            for (int c = 0; c < CPT; ++c) {
                const int32_t j = tid + c * nt;
                const uint32_t base =
                    eta0 + kEnt * (CX ? (uint32_t)(DV * (j < n ? j : 0)) : (ckd[c] & 0xffffu));
                const int32_t dv = CX ? DV : (int32_t)(ckd[c] >> 16);
#pragma unroll
                for (int k = 0; k < DV; ++k)
                    if (k < slot_cap<DVP, DV>(c))
                        evp[c][k] = kLay ? lds_ld<V>(lds, ba[kLay ? c : 0][kLay ? k : 0])
                                       : lds_ld<V>(lds, base + kEnt * (uint32_t)(CX || k < dv ? k : 0));
            }
#pragma unroll
            for (int c = 0; c < CPT; ++c) {
                const int32_t j = tid + c * nt;
                if (j < n) {
                    const int32_t dv = CX ? DV : (int32_t)(ckd[c] >> 16);
                    V acc = (CX || 0 < dv) ? evp[c][0] : vzero<V>();
#pragma unroll
                    for (int k = 1; k < DV; ++k)
                        if (k < slot_cap<DVP, DV>(c))
                            acc = acc + ((CX || k < dv) ? evp[c][k] : vzero<V>()); // +0 adds change no s
                    lds_st<V>(lds, kEnt * (uint32_t)j, acc + rc[c]);
                }
            }
        } else {
            auto bit_msgs = [&](int c, V(&ev)[DV]) {
                const int32_t j = tid + c * nt;
                const uint32_t base =
                    eta0 + kEnt * (CX ? (uint32_t)(DV * (j < n ? j : 0)) : (ckd[c] & 0xffffu));
                const int32_t dv = CX ? DV : (int32_t)(ckd[c] >> 16);
#pragma unroll
                for (int k = 0; k < DV; ++k)
                    if (k < slot_cap<DVP, DV>(c))
                        ev[k] = kLay ? lds_ld<V>(lds, ba[kLay ? c : 0][kLay ? k : 0])
                                     : lds_ld<V>(lds, base + kEnt * (uint32_t)(CX || k < dv ? k : 0));
            };
            V evn[DV];
            bit_msgs(0, evn);
#pragma unroll
            for (int c = 0; c < CPT; ++c) {
                const int32_t j = tid + c * nt;
                V ev[DV];
#pragma unroll
                for (int k = 0; k < DV; ++k) ev[k] = evn[k];
                if (c + 1 < CPT) bit_msgs(c + 1, evn);
                if (j < n) {
                    const int32_t dv = CX ? DV : (int32_t)(ckd[c] >> 16);
                    V acc = (CX || 0 < dv) ? ev[0] : vzero<V>();
#pragma unroll
                    for (int k = 1; k < DV; ++k)
                        if (k < slot_cap<DVP, DV>(c))
                            acc = acc + ((CX || k < dv) ? ev[k] : vzero<V>()); // +0 adds change no s
                    lds_st<V>(lds, kEnt * (uint32_t)j, acc + rc[c]);
                }
            }
        }
        // Slots refilled this round start their new frame from s = r: their
        // entries are overwritten (the same thread wrote them just above).  A
        // refill happens in few rounds, so this is a branch on the uniform
        // refill mask rather than a select on every bit of every round.
        if (fin) {
#pragma unroll
            for (int c = 0; c < CPT; ++c) {
                const int32_t j = tid + c * nt;
                if (j < n) {
#pragma unroll
                    for (int q = 0; q < F; ++q) {
                        if ((fin >> q) & 1u) {
                            const float v = kAheadLLR ? rnx[c][q] + 0.0f // -0 -> +0
                                                      : (fr[q] < B ? llr[(size_t)fr[q] * n + gj[c]] + 0.0f : 0.0f);
                            rc[c][q] = v;
                            lds_st<float>(lds, kEnt * (uint32_t)j + 4u * (uint32_t)q, v);
                            if constexpr (kPrevLds) { // the new frame's first iteration reads 0 messages
#pragma unroll
                                for (int u = 0; u < DV; ++u)
                                    if (u < slot_cap<DVP, DV>(c))
                                        lds_st<float>(lds, ba[kLay ? c : 0][kLay ? u : 0] + 4u * (uint32_t)q, 0.0f);
                            }
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
}

constexpr int kMaxThreads = 512;

struct Variant {
    int dc;
    bool rx;
    int dv;
    bool cx;
    int rpt;
    int cpt;
    int f;  // frame slots per workgroup
    int cf; // the graph's bank-conflict-free layout: 0 no, 1 previous messages in LDS, 2 in registers,
            // + 4 columns of degree below dv padded
    uint32_t dvp; // layout with bits sorted by degree: messages read per own bit slot c (4 bits each), 0 dv
};

// Exact-degree variants for the regular codes in use first, then masked ones,
// then four-slot variants of the (3,6) shape (float4 LDS entries: half the
// LDS instructions and per-frame loop work per frame, twice the LDS per
// workgroup), then bit degree masked at 6 (fewer registers and LDS loads
// than 8 for codes whose bits have at most 6 checks).  The order is the
// dispatch order of pick below.
constexpr Variant kVariants[] = {
    {6, true, 3, true, 2, 4, 2},   {6, true, 8, false, 2, 4, 2},  {9, true, 8, false, 2, 8, 2},
    {12, true, 8, false, 1, 4, 2}, {16, true, 8, false, 1, 8, 2}, {8, false, 8, false, 2, 4, 2},
    {16, false, 16, false, 1, 8, 2}, {6, true, 3, true, 1, 4, 2}, {6, true, 3, true, 2, 4, 4},
    {6, true, 3, true, 1, 4, 4},     {6, true, 6, false, 2, 4, 2},  {9, true, 6, false, 2, 8, 2},
    {12, true, 6, false, 1, 4, 2},   {16, true, 6, false, 1, 8, 2}, {6, true, 3, true, 2, 4, 2, 1},
    {6, true, 3, true, 2, 4, 2, 2},
    // one frame slot (half the per-slot registers and LDS of the two-slot
    // variant of the same shape) for the shapes whose two-slot kernels need
    // more than 128 VGPRs, and bit degree masked at 4 (codes of rate 5/6)
    {9, true, 6, false, 2, 8, 1},    {16, true, 6, false, 1, 8, 1}, {12, true, 6, false, 1, 4, 1},
    {6, true, 6, false, 2, 4, 1},    {16, true, 4, false, 1, 8, 2}, {16, true, 4, false, 1, 8, 1},
    // the bank-conflict-free layout for rows of one degree and columns of
    // degree at most DV (padded), in a geometry per row degree: rate 1/2 (two
    // geometries), 2/3, 3/4 and 5/6 shapes; previous messages in LDS, then in
    // registers
    {6, true, 6, true, 2, 4, 2, 5},  {6, true, 6, true, 2, 4, 2, 6},  {6, true, 6, true, 1, 2, 2, 5},
    {6, true, 6, true, 1, 2, 2, 6},  {9, true, 6, true, 2, 6, 2, 5},  {9, true, 6, true, 2, 6, 2, 6},
    {12, true, 6, true, 1, 4, 2, 5}, {12, true, 6, true, 1, 4, 2, 6}, {16, true, 4, true, 1, 6, 2, 5},
    {16, true, 4, true, 1, 6, 2, 6},
    // the same shapes with bits placed in ascending column degree: each bit
    // slot index reads only as many messages as its bits' largest degree
    // (profiles of codes whose bits have degrees 2, 3 and 6 or 4 in the
    // proportions 3:2:1)
    {6, true, 6, true, 2, 4, 2, 5, 0x6332u},      {6, true, 6, true, 2, 4, 2, 6, 0x6332u},
    {6, true, 6, true, 1, 2, 2, 5, 0x63u},        {6, true, 6, true, 1, 2, 2, 6, 0x63u},
    {9, true, 6, true, 2, 6, 2, 5, 0x633222u},    {9, true, 6, true, 2, 6, 2, 6, 0x633222u},
    {12, true, 6, true, 1, 4, 2, 5, 0x6332u},     {12, true, 6, true, 1, 4, 2, 6, 0x6332u},
    {16, true, 4, true, 1, 6, 2, 5, 0x433222u},   {16, true, 4, true, 1, 6, 2, 6, 0x433222u},
};
constexpr int kNumVariants = (int)(sizeof(kVariants) / sizeof(kVariants[0]));

template <int V, bool NMS>
__device__ __forceinline__ void run_v(const Job &J, int32_t L, int32_t early, unsigned char *lds) {
    constexpr Variant v = kVariants[V];
    run_onchip<v.dc, v.rx, v.dv, v.cx, v.rpt, v.cpt, v.f, NMS, v.cf, v.dvp>(J, L, early, lds);
}


// Jobs of one launch: every workgroup works through them in order, each
// until that job's frame counter is exhausted (no grid-wide barrier: a
// workgroup moves on while others finish their last frames, so the last
// frames of one job overlap the first ones of the next).
constexpr int kMaxJobs = 16;
struct JobTable {
    int32_t njobs;
    Job job[kMaxJobs];
};

// One variant instantiated, one or more jobs that all use it.  W > 0 asks
// the compiler for at least W waves per SIMD (fewer registers per thread,
// more resident waves to hide LDS latency); W = 0 leaves the register budget
// to it.
template <int V, int W, bool NMS>
__global__ __launch_bounds__(kMaxThreads) __attribute__((amdgpu_waves_per_eu(W > 0 ? W : 1))) void k_onchip(
    const JobTable jt, int32_t L, int32_t early) {
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
    for (int32_t c = 0; c < jt.njobs; ++c) {
        run_v<V, NMS>(jt.job[c], L, early, lds);
        __syncthreads();
    }
}

using KernelFn = void (*)(const JobTable, int32_t, int32_t);
// [learned][register budget][variant]
#define LDPC_ONCHIP_ROW(W, N)                                                                                      \
    {&k_onchip<0, W, N>, &k_onchip<1, W, N>, &k_onchip<2, W, N>, &k_onchip<3, W, N>, &k_onchip<4, W, N>,         \
     &k_onchip<5, W, N>, &k_onchip<6, W, N>, &k_onchip<7, W, N>, &k_onchip<8, W, N>, &k_onchip<9, W, N>,         \
     &k_onchip<10, W, N>, &k_onchip<11, W, N>, &k_onchip<12, W, N>, &k_onchip<13, W, N>, &k_onchip<14, W, N>,        \
     &k_onchip<15, W, N>, &k_onchip<16, W, N>, &k_onchip<17, W, N>, &k_onchip<18, W, N>, &k_onchip<19, W, N>,         \
     &k_onchip<20, W, N>, &k_onchip<21, W, N>, &k_onchip<22, W, N>, &k_onchip<23, W, N>, &k_onchip<24, W, N>,         \
     &k_onchip<25, W, N>, &k_onchip<26, W, N>, &k_onchip<27, W, N>, &k_onchip<28, W, N>, &k_onchip<29, W, N>,         \
     &k_onchip<30, W, N>, &k_onchip<31, W, N>, &k_onchip<32, W, N>, &k_onchip<33, W, N>, &k_onchip<34, W, N>,         \
     &k_onchip<35, W, N>, &k_onchip<36, W, N>, &k_onchip<37, W, N>, &k_onchip<38, W, N>, &k_onchip<39, W, N>,         \
     &k_onchip<40, W, N>, &k_onchip<41, W, N>}
// The kernels of each register budget (waves per SIMD 0, 4, 3), one source
// file each: [learned][variant].
extern const KernelFn kKernelsW0[2][kNumVariants];
extern const KernelFn kKernelsW4[2][kNumVariants];
extern const KernelFn kKernelsW3[2][kNumVariants];

} // namespace onchip
} // namespace ldpc
