// On-chip Min-Sum decoder: the whole decoding state of a frame lives in LDS
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
#include <algorithm>

#include "ldpc_internal.h"
#include "minsum_row.h"

namespace ldpc {
namespace {

constexpr int kMaxF = 4; // frame slots per workgroup: 2 or 4 (a kernel variant's choice)
template <int F> struct Vec;
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
__device__ int32_t take_frame(uint32_t *queue, int32_t B, int32_t nq, int32_t &hc, uint32_t &dead) {
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
size_t state_bytes(const ldpc_graph &g, int F) {
    return align_up(sizeof(float) * (size_t)F * ((size_t)g.n + (size_t)g.E + 1), 16);
}

size_t lds_bytes_for(const ldpc_graph &g, int F) { return state_bytes(g, F) + sizeof(Shared); }

// The bank-conflict-free layout (two frame slots, 8-byte entries): s[n], then
// the messages from a 256-byte boundary (so that a position's bank class is
// the position modulo 32), cf.npos entries.
uint32_t cf_eta_offset(const ldpc_graph &g) { return (uint32_t)align_up(8 * (size_t)g.n, 256); }
size_t cf_state_bytes(const ldpc_graph &g) { return align_up(cf_eta_offset(g) + 8 * (size_t)g.cf.npos, 16); }

__global__ void k_zero_u32(uint32_t *p) { *p = 0u; }

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
// position of its own; needs exact degrees and its geometry (two rows, four
// bits per thread).  CF = 1: the check pass reads each edge's previous
// message back from its position (no registers for them); CF = 2: it keeps
// them in registers, as without the layout (a third fewer LDS reads).
template <int DC, bool RX, int DV, bool CX, int RPT, int CPT, int F, bool NMS, int CF>
__device__ __forceinline__ void run_onchip(const Job &J, int32_t L, int32_t early, unsigned char *lds) {
    constexpr bool kLay = CF != 0;     // the layout's tables
    constexpr bool kPrevLds = CF == 1; // previous messages read from LDS
    static_assert(!kLay || (RX && CX && RPT == 2 && CPT == 4 && F == 2), "layout geometry");
    typedef typename Vec<F>::type V;
    constexpr uint32_t kEnt = sizeof(V); // bytes of one LDS entry (F floats)
    // read all s (messages) of the check (bit) pass up front when that takes
    // at most 32 registers (s: only with exact column degrees; the masked
    // variants need those registers to stay within four waves per SIMD)
    constexpr bool kPrefetchS = RPT > 1 && RPT * DC * F <= 32 && CX;
    constexpr bool kPrefetchEta = CPT > 1 && CPT * DV * F <= 32;
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
                ba[c][u] = eta0 + kEnt * (p < n ? J.cf_bitpos[(size_t)p * DV + u] : (uint32_t)(J.cf_npos - 1));
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
        // own bits are read before the first s is written.  Bits past n read
        // a valid slot (bit 0's, or the padding slot) and write nothing.
        // CF: each message at its own position (ba), in ascending check order.
        V evp[CPT][DV];
        if constexpr (kPrefetchEta) {
#pragma unroll
            for (int c = 0; c < CPT; ++c) {
                const int32_t j = tid + c * nt;
                const uint32_t base =
                    eta0 + kEnt * (CX ? (uint32_t)(DV * (j < n ? j : 0)) : (ckd[c] & 0xffffu));
                const int32_t dv = CX ? DV : (int32_t)(ckd[c] >> 16);
#pragma unroll
                for (int k = 0; k < DV; ++k)
                    evp[c][k] = kLay ? lds_ld<V>(lds, ba[kLay ? c : 0][kLay ? k : 0])
                                   : lds_ld<V>(lds, base + kEnt * (uint32_t)(CX || k < dv ? k : 0));
            }
        }
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            const int32_t j = tid + c * nt;
            if (j < n) {
                // CX: every bit has DV slots, so bit j's first slot is DV j
                const uint32_t base =
                    eta0 + kEnt * (CX ? (uint32_t)(DV * j) : (ckd[c] & 0xffffu));
                const int32_t dv = CX ? DV : (int32_t)(ckd[c] >> 16);
                V ev[DV];
#pragma unroll
                for (int k = 0; k < DV; ++k)
                    ev[k] = kPrefetchEta ? evp[c][k]
                            : kLay       ? lds_ld<V>(lds, ba[kLay ? c : 0][kLay ? k : 0])
                                         : lds_ld<V>(lds, base + kEnt * (uint32_t)(CX || k < dv ? k : 0));
                V acc = (CX || 0 < dv) ? ev[0] : vzero<V>();
#pragma unroll
                for (int k = 1; k < DV; ++k)
                    acc = acc + ((CX || k < dv) ? ev[k] : vzero<V>()); // +0 adds change no s
                lds_st<V>(lds, kEnt * (uint32_t)j, acc + rc[c]);
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
    int cf; // the graph's bank-conflict-free layout: 0 no, 1 previous messages in LDS, 2 in registers
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
};
constexpr int kNumVariants = (int)(sizeof(kVariants) / sizeof(kVariants[0]));

template <int V, bool NMS>
__device__ __forceinline__ void run_v(const Job &J, int32_t L, int32_t early, unsigned char *lds) {
    constexpr Variant v = kVariants[V];
    run_onchip<v.dc, v.rx, v.dv, v.cx, v.rpt, v.cpt, v.f, NMS, v.cf>(J, L, early, lds);
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
// The widest masked variant is left out of the multi-code kernel: the
// register demand of a kernel is that of its largest variant, and that one
// alone would push every variant of the launch into spills.  Jobs that need
// it get a launch of their own.  So is the bank-conflict-free layout: its
// tables are built for the graph's own thread count, and the shared launch
// runs the largest thread count of its jobs.
constexpr int kWideVariant = 6;
constexpr bool shared_launch_ok(int v) { return v != kWideVariant && kVariants[v].cf == 0; }
static_assert(kNumVariants == 16, "k_onchip_multi dispatches variants 0-5 and 7-13");

__global__ __launch_bounds__(kMaxThreads) void k_onchip_multi(const JobTable jt, int32_t L, int32_t early) {
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
    for (int32_t c = 0; c < jt.njobs; ++c) {
        switch (jt.job[c].variant) {
        case 0: run_v<0, false>(jt.job[c], L, early, lds); break;
        case 1: run_v<1, false>(jt.job[c], L, early, lds); break;
        case 2: run_v<2, false>(jt.job[c], L, early, lds); break;
        case 3: run_v<3, false>(jt.job[c], L, early, lds); break;
        case 4: run_v<4, false>(jt.job[c], L, early, lds); break;
        case 5: run_v<5, false>(jt.job[c], L, early, lds); break;
        case 7: run_v<7, false>(jt.job[c], L, early, lds); break;
        case 8: run_v<8, false>(jt.job[c], L, early, lds); break;
        case 9: run_v<9, false>(jt.job[c], L, early, lds); break;
        case 10: run_v<10, false>(jt.job[c], L, early, lds); break;
        case 11: run_v<11, false>(jt.job[c], L, early, lds); break;
        case 12: run_v<12, false>(jt.job[c], L, early, lds); break;
        case 13: run_v<13, false>(jt.job[c], L, early, lds); break;
        default: break; // the host places no variant here that fails shared_launch_ok
        }
        __syncthreads();
    }
}

using KernelFn = void (*)(const JobTable, int32_t, int32_t);
// [learned][register budget][variant]
#define LDPC_ONCHIP_ROW(W, N)                                                                                      \
    {&k_onchip<0, W, N>, &k_onchip<1, W, N>, &k_onchip<2, W, N>, &k_onchip<3, W, N>, &k_onchip<4, W, N>,         \
     &k_onchip<5, W, N>, &k_onchip<6, W, N>, &k_onchip<7, W, N>, &k_onchip<8, W, N>, &k_onchip<9, W, N>,         \
     &k_onchip<10, W, N>, &k_onchip<11, W, N>, &k_onchip<12, W, N>, &k_onchip<13, W, N>, &k_onchip<14, W, N>,        \
     &k_onchip<15, W, N>}
const KernelFn kKernels[2][2][kNumVariants] = {{LDPC_ONCHIP_ROW(0, false), LDPC_ONCHIP_ROW(4, false)},
                                               {LDPC_ONCHIP_ROW(0, true), LDPC_ONCHIP_ROW(4, true)}};
#undef LDPC_ONCHIP_ROW

// Threads: whole wavefronts, enough for RPT rows and CPT bits per thread.
int threads_for(const ldpc_graph &g, const Variant &v) {
    const int a = (g.m + v.rpt - 1) / v.rpt, b = (g.n + v.cpt - 1) / v.cpt;
    const int want = a > b ? a : b;
    const int t = ((want + 63) / 64) * 64;
    return t < 64 ? 64 : t;
}

bool variant_ok(const ldpc_graph &g, int k) {
    if (k < 0 || k >= kNumVariants) return false;
    const Variant &v = kVariants[k];
    const bool rows_ok = v.rx ? (g.dc_min == v.dc && g.dc_max == v.dc) : g.dc_max <= v.dc;
    const bool cols_ok = v.cx ? (g.dv_min == v.dv && g.dv_max == v.dv) : g.dv_max <= v.dv;
    // the layout's tables are for exact degrees and their own thread count
    const bool cf_ok = v.cf == 0 || (g.cf.edge != nullptr && g.dc_min == v.dc && g.dv_min == v.dv &&
                                 threads_for(g, v) == g.cf.nt);
    const size_t state = v.cf != 0 ? cf_state_bytes(g) : state_bytes(g, v.f);
    return rows_ok && cols_ok && cf_ok && threads_for(g, v) <= kMaxThreads && g.edge_tab != nullptr &&
           state + sizeof(Shared) + 1024 <= (size_t)g.lds_max;
}

size_t state_of(const ldpc_graph &g, int variant) {
    return kVariants[variant].cf != 0 ? cf_state_bytes(g) : state_bytes(g, kVariants[variant].f);
}
size_t lds_of(const ldpc_graph &g, int variant) { return state_of(g, variant) + sizeof(Shared); }

// Default preference when nothing is tuned: the bank-conflict-free layout,
// then exact degrees, a column mask of 6 before one of 8, two frame slots
// before four.
constexpr int kPickOrder[] = {15, 14, 0, 7, 10, 1, 11, 2, 12, 3, 13, 4, 5, 6, 8, 9};
static_assert(sizeof(kPickOrder) / sizeof(kPickOrder[0]) == kNumVariants, "every variant has a place");

// The tuned variant if one is set and valid, else the first that fits.
int pick(const ldpc_graph &g) {
    if (g.tuning.set && variant_ok(g, g.tuning.variant)) return g.tuning.variant;
    for (int k : kPickOrder)
        if (variant_ok(g, k)) return k;
    return -1;
}

Job make_job(const ldpc_graph &g, int variant, const float *llr, int32_t B, uint8_t *bits, float *post,
             int32_t *iters, uint8_t *ok, const float *alpha, const float *beta, uint32_t *queue) {
    Job J;
    J.row_ptr = g.row_ptr;
    J.edge_tab = g.edge_tab;
    J.col_ptr = g.col_ptr;
    J.row_class = g.row_class;
    J.m = g.m;
    J.n = g.n;
    J.E = (int32_t)g.E;
    J.sh_off = (uint32_t)state_of(g, variant);
    J.cf_edge = g.cf.edge;
    J.cf_bitpos = g.cf.bitpos;
    J.cf_slot_bit = g.cf.slot_bit;
    J.cf_row_class = g.cf.row_class;
    J.cf_eta_off = cf_eta_offset(g);
    J.cf_npos = g.cf.npos;
    J.llr = llr;
    J.B = B;
    J.bits = bits;
    J.post = post;
    J.iters = iters;
    J.ok = ok;
    J.alpha = alpha;
    J.beta = beta;
    J.ncls = (int32_t)g.class_degrees.size();
    J.variant = variant;
    J.queue = queue;
    J.nq = queues_for(B);
    return J;
}

__global__ void k_zero_words(uint32_t *p, int32_t count) {
    const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < count) p[k] = 0u;
}

// Grid of a persistent launch: every CU filled to its occupancy, but no more
// workgroups than there are groups of 2 F frames.
int launch_grid(const void *fn, int threads, size_t lds, int num_cu, int64_t frames, int cap_per_cu, int *grid,
                int F = 2) {
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) return LDPC_EHIP;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, lds) != hipSuccess) return LDPC_EHIP;
    if (cap_per_cu > 0 && per_cu > cap_per_cu) per_cu = cap_per_cu;
    per_cu = per_cu < 1 ? 1 : per_cu;
    const int64_t groups = (frames + 2 * F - 1) / (2 * F);
    const int64_t want = (int64_t)num_cu * per_cu;
    *grid = (int)(want < groups ? want : groups);
    if (*grid < 1) *grid = 1;
    return LDPC_OK;
}

} // namespace

bool onchip_fits(const ldpc_graph &g) { return g.edge_tab != nullptr && pick(g) >= 0; }

bool onchip_variant_fits(const ldpc_graph &g, int variant) { return variant_ok(g, variant); }

int onchip_num_variants() { return kNumVariants; }

bool onchip_kernel_spill_free(int variant, int waves_per_simd) {
    if (variant < 0 || variant >= kNumVariants) return false;
    hipFuncAttributes a{};
    if (hipFuncGetAttributes(&a, (const void *)kKernels[0][waves_per_simd == 4 ? 1 : 0][variant]) != hipSuccess)
        return false;
    return a.localSizeBytes == 0;
}

size_t onchip_workspace_bytes(const ldpc_graph &g, int32_t B) {
    (void)g;
    (void)B;
    return 4ull * kQueueWords; // frame counters
}

int onchip_decode(const ldpc_graph &g, const float *llr, int32_t B, int32_t L, uint32_t flags, const float *alpha,
                  const float *beta, int32_t T, uint8_t *bits, float *post, int32_t *iters, uint8_t *ok, void *ws,
                  size_t ws_bytes, hipStream_t stream) {
    (void)T;
    if (!onchip_fits(g)) return LDPC_EUNSUPPORTED;
    if (ws == nullptr || ws_bytes < onchip_workspace_bytes(g, B)) return LDPC_EWORKSPACE;
    const int v = pick(g);
    const KernelFn fn = kKernels[alpha != nullptr ? 1 : 0][(g.tuning.set && g.tuning.waves_per_simd == 4) ? 1 : 0][v];
    const int threads = threads_for(g, kVariants[v]);
    const size_t lds = lds_of(g, v);
    int grid = 0;
    int st = launch_grid((const void *)fn, threads, lds, g.num_cu, B, g.tuning.set ? g.tuning.wg_per_cu : 0, &grid,
                         kVariants[v].f);
    if (st) return st;
    uint32_t *queue = (uint32_t *)ws;
    const int32_t early = test_period(flags);
    JobTable jt{};
    jt.njobs = 1;
    jt.job[0] = make_job(g, v, llr, B, bits, post, iters, ok, alpha, beta, queue);
    k_zero_words<<<(kQueueWords + 255) / 256, 256, 0, stream>>>(queue, kQueueWords);
    timed_launch(K_ONCHIP, fn, grid, threads, lds, stream, jt, L, early);
    return hipGetLastError() == hipSuccess ? LDPC_OK : LDPC_EHIP;
}

size_t onchip_multi_workspace_bytes(int32_t njobs) {
    return align_up(4ull * kQueueWords * (size_t)(njobs > 0 ? njobs : 1), 256);
}

int onchip_decode_multi(const ldpc_job *jobs, int32_t njobs, int32_t L, uint32_t flags, void *ws, size_t ws_bytes,
                        hipStream_t stream) {
    if (njobs > kMaxJobs) return LDPC_EUNSUPPORTED;
    if (ws == nullptr || ws_bytes < onchip_multi_workspace_bytes(njobs)) return LDPC_EWORKSPACE;
    // largest jobs first, so the last frames of the shared launch come from small jobs
    std::vector<int32_t> order(njobs);
    for (int32_t k = 0; k < njobs; ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        return (int64_t)jobs[a].B * jobs[a].g->E > (int64_t)jobs[b].B * jobs[b].g->E;
    });
    // A job whose batch alone fills every CU at least once gets a launch of
    // its own kernel (its own LDS size, workgroup size, register budget and
    // tuned workgroups per CU); so does a job that only the widest variant
    // fits.  The other jobs share one persistent launch, whose workgroup size
    // and LDS are the maxima over them.
    constexpr int64_t kOwnLaunchRounds = 1;
    JobTable jt{};
    int threads = 64;
    size_t lds = 0;
    int64_t frames = 0;
    int num_cu = 0;
    uint32_t *queues = (uint32_t *)ws;
    struct Own {
        Job J;
        KernelFn fn;
        int threads;
        size_t lds;
        int num_cu;
        int wg_per_cu; // tuned cap, 0 for none
    };
    std::vector<Own> own;
    int32_t nj = 0;
    for (int32_t k = 0; k < njobs; ++k) {
        const ldpc_job &jb = jobs[order[k]];
        const ldpc_graph &g = *jb.g;
        if (!onchip_fits(g)) return LDPC_EUNSUPPORTED;
        if (jb.B == 0) continue;
        const int v_own = pick(g);
        int v = v_own;
        if (!shared_launch_ok(v)) // another variant that fits keeps the job eligible for the shared launch
            for (int c : kPickOrder)
                if (shared_launch_ok(c) && variant_ok(g, c)) {
                    v = c;
                    break;
                }
        const KernelFn fn = kKernels[0][(g.tuning.set && g.tuning.waves_per_simd == 4) ? 1 : 0][v_own];
        const int t_own = threads_for(g, kVariants[v_own]);
        const size_t l_own = lds_of(g, v_own);
        bool alone = !shared_launch_ok(v);
        if (!alone) {
            int per_cu = 0;
            if (hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)l_own) !=
                    hipSuccess ||
                hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)fn, t_own, l_own) != hipSuccess)
                return LDPC_EHIP;
            const int64_t in_flight = (int64_t)(per_cu < 1 ? 1 : per_cu) * g.num_cu * kVariants[v_own].f;
            alone = (int64_t)jb.B >= kOwnLaunchRounds * in_flight;
        }
        if (alone) {
            own.push_back(Own{make_job(g, v_own, jb.llr_dev, jb.B, jb.bits_dev, jb.post_dev, jb.iters_dev, jb.ok_dev,
                                       nullptr, nullptr, queues + (size_t)k * kQueueWords),
                              fn, t_own, l_own, g.num_cu, g.tuning.set ? g.tuning.wg_per_cu : 0});
            continue;
        }
        const int t = threads_for(g, kVariants[v]);
        threads = t > threads ? t : threads;
        lds = lds_of(g, v) > lds ? lds_of(g, v) : lds;
        frames += jb.B;
        num_cu = g.num_cu;
        jt.job[nj++] = make_job(g, v, jb.llr_dev, jb.B, jb.bits_dev, jb.post_dev, jb.iters_dev, jb.ok_dev, nullptr,
                                nullptr, queues + (size_t)k * kQueueWords);
    }
    jt.njobs = nj;
    const int32_t early = test_period(flags);
    if (frames == 0 && own.empty()) return LDPC_OK;
    k_zero_words<<<(njobs * kQueueWords + 255) / 256, 256, 0, stream>>>(queues, njobs * kQueueWords);
    // Jobs with a launch of their own that use the same kernel, workgroup size,
    // LDS size and workgroup cap (the same graph, or graphs of one shape) go
    // into one launch of it, in order (largest first), so that each job's last
    // frames overlap the next job's first ones.
    std::vector<bool> placed(own.size(), false);
    for (size_t a = 0; a < own.size(); ++a) {
        if (placed[a]) continue;
        JobTable ot{};
        int t = 0;
        size_t l = 0;
        int64_t fr = 0;
        for (size_t b = a; b < own.size(); ++b) {
            if (placed[b] || own[b].fn != own[a].fn || own[b].wg_per_cu != own[a].wg_per_cu ||
                own[b].threads != own[a].threads || own[b].lds != own[a].lds)
                continue;
            placed[b] = true;
            ot.job[ot.njobs++] = own[b].J;
            t = own[b].threads > t ? own[b].threads : t;
            l = own[b].lds > l ? own[b].lds : l;
            fr += own[b].J.B;
        }
        int grid = 0;
        const int st = launch_grid((const void *)own[a].fn, t, l, own[a].num_cu, fr, own[a].wg_per_cu, &grid,
                                   kVariants[own[a].J.variant].f);
        if (st) return st;
        timed_launch(K_ONCHIP, own[a].fn, grid, t, l, stream, ot, L, early);
    }
    if (frames > 0) {
        int grid = 0;
        const int st = launch_grid((const void *)k_onchip_multi, threads, lds, num_cu, frames, 0, &grid);
        if (st) return st;
        timed_launch(K_ONCHIP, k_onchip_multi, grid, threads, lds, stream, jt, L, early);
    }
    return hipGetLastError() == hipSuccess ? LDPC_OK : LDPC_EHIP;
}

} // namespace ldpc
