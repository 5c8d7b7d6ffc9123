// HBM-streaming Min-Sum decoder: any code size, state in device memory.
//
// Layout ("frames in lanes"): frames are grouped in tiles of 64, one
// wavefront per tile, lane = frame.  Every per-bit and per-edge quantity is
// stored tile-major with the 64 frames innermost:
//     r[tile][j][64], s[tile][j][64]  (channel LLR, posterior)   4 B each
//     eta[tile][e][64]                (check-to-bit message)      4 B each
// so each wavefront load or store of one edge or bit is 256 contiguous bytes,
// whatever the structure of H.  The edge and bit indices are the same for
// every lane, so they come in through scalar loads.
//
// One iteration is two launches (a kernel boundary is the grid-wide barrier
// between the check and the bit phase):
//   check kernel  per (row, frame): x_e = s_j - eta_e over the row (eta = 0 in
//                 iteration 1, s = r), the row's two smallest |x|, the first
//                 position of the smallest, the parity of the negative x,
//                 then eta_e = (+-)(e == argmin ? min1 : min0) with the sign
//                 from the parity without e's own sign (Observations 1, 2 of
//                 Sec. III).  The XOR of the row's hard decisions of the s it
//                 reads is the syndrome of the previous iteration.
//   bit kernel    per (bit, frame): s_j = (+0 + eta_e over the column in
//                 ascending check order) + r_j (eq. lambda_j), unless the
//                 previous syndrome was zero: then the frame is finished and
//                 keeps the s of that iteration.
// The first check launch computes the syndrome of the channel decision, so a
// frame whose channel decision is a codeword stops with 0 iterations (the
// pre-loop test of the paper's kernel listing).
//
// Batches whose state exceeds the last-level (Infinity) cache are decoded in
// chunks of whole tiles, all iterations of one chunk before the next, so that
// every launch after a chunk's first finds its state in that cache.  Within a
// chunk, the frames still decoding are packed into fewer tiles from time to
// time (frame compaction, below), since a tile runs until its last frame
// stops.
#include <type_traits>

#include "ldpc_internal.h"
#include "minsum_row.h"

namespace ldpc {
namespace {

constexpr int kWaves = 4;       // wavefronts per workgroup of the transpose kernels
constexpr int kRowsPerWave = 2; // rows per wavefront of the unrolled check kernel
constexpr int kColsPerWave = 4; // bit columns per wavefront of the bit kernel

// Per-slot arrays of the state (slot = tile * 64 + lane), in two sets: frame
// compaction (below) copies the frames still decoding from one set into the
// other, packed into the first tiles.
struct Set {
    float *r, *s, *eta;
    uint32_t *done;     // slot's frame has stopped, or the slot is empty
    uint32_t *unsat[2]; // syndrome nonzero, indexed by iteration parity
    int32_t *conv;      // iteration at which the frame stopped, -1 if not
    int32_t *fid;       // the frame in the slot, -1 for none
};
// Per chunk: which set holds its frames, and the last compaction plan.
struct Ctrl {
    uint32_t cur;   // set holding the chunk's frames at the last plan
    uint32_t go;    // the last plan compacts: from its copy on, the frames are in set cur ^ 1
    int32_t active; // frames still decoding at the last plan
    uint32_t pad;
};
// What every streaming kernel of a chunk receives: both sets, offset to the
// chunk's first tile, and its control words.  Kernels read them once.
struct Bufs {
    Set set[2];
    Ctrl *ctrl;
};
// A set's syndrome flags of parity p.  (A select, not an index: indexing
// the kernel argument's array with a run-time value makes the compiler copy
// the struct through LDS and turn its pointers into per-lane values.)
__device__ __forceinline__ uint32_t *unsat_of(const Set &S, int32_t p) { return (p & 1) ? S.unsat[1] : S.unsat[0]; }
// The set holding the chunk's frames outside a compaction (after the copy of
// the last plan that went ahead).
__device__ __forceinline__ Set cur_set(const Bufs &b) {
    const uint32_t c = __builtin_amdgcn_readfirstlane(b.ctrl->cur ^ b.ctrl->go);
    const Set s0 = b.set[0], s1 = b.set[1];
    return c ? s1 : s0;
}
// The set the last plan counted (the source of its copy).
__device__ __forceinline__ Set plan_set(const Bufs &b) {
    const uint32_t c = __builtin_amdgcn_readfirstlane(b.ctrl->cur);
    const Set s0 = b.set[0], s1 = b.set[1];
    return c ? s1 : s0;
}

struct StreamWs {
    Set set[2];
    Ctrl *ctrl;
    int32_t *base; // compaction: first destination slot of every tile of a chunk
};

size_t tiles_of(int32_t B) { return (size_t)((B + kTile - 1) / kTile); }

StreamWs carve(const ldpc_graph &g, int32_t B, void *base, size_t *total) {
    const size_t nt = tiles_of(B);
    const size_t fr = nt * kTile;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    size_t o_r[2], o_s[2], o_e[2], o_d[2], o_u0[2], o_u1[2], o_c[2], o_f[2];
    for (int k = 0; k < 2; ++k) {
        o_r[k] = take(nt * (size_t)g.n * kTile * 4);
        o_s[k] = take(nt * (size_t)g.n * kTile * 4);
        o_e[k] = take(nt * (size_t)g.E * kTile * 4);
        o_d[k] = take(fr * 4);
        o_u0[k] = take(fr * 4);
        o_u1[k] = take(fr * 4);
        o_c[k] = take(fr * 4);
        o_f[k] = take(fr * 4);
    }
    const size_t o_ctrl = take(sizeof(Ctrl));
    const size_t o_base = take(nt * 4);
    if (total) *total = off;
    StreamWs w{};
    char *b = (char *)base;
    if (b) {
        for (int k = 0; k < 2; ++k) {
            w.set[k].r = (float *)(b + o_r[k]);
            w.set[k].s = (float *)(b + o_s[k]);
            w.set[k].eta = (float *)(b + o_e[k]);
            w.set[k].done = (uint32_t *)(b + o_d[k]);
            w.set[k].unsat[0] = (uint32_t *)(b + o_u0[k]);
            w.set[k].unsat[1] = (uint32_t *)(b + o_u1[k]);
            w.set[k].conv = (int32_t *)(b + o_c[k]);
            w.set[k].fid = (int32_t *)(b + o_f[k]);
        }
        w.ctrl = (Ctrl *)(b + o_ctrl);
        w.base = (int32_t *)(b + o_base);
    }
    return w;
}

// The chunk of tiles c0 .. of both sets.
Bufs chunk_bufs(const StreamWs &w, const ldpc_graph &g, int32_t c0) {
    const size_t fo = (size_t)c0 * kTile;
    Bufs b{};
    for (int k = 0; k < 2; ++k) {
        const Set &x = w.set[k];
        b.set[k] = Set{x.r + fo * g.n, x.s + fo * g.n, x.eta + fo * (size_t)g.E, x.done + fo,
                       {x.unsat[0] + fo, x.unsat[1] + fo}, x.conv + fo, x.fid + fo};
    }
    b.ctrl = w.ctrl;
    return b;
}

// Message (eta) accesses, optionally non-temporal: one iteration's messages
// stream through the caches once, and marked so they leave the L2 to the
// posterior gathers of the check kernel.
template <bool NT> __device__ __forceinline__ float ld_msg(const float *p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <bool NT> __device__ __forceinline__ void st_msg(float *p, float v) {
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

__global__ void k_flags_init(int32_t B, int32_t frames, uint32_t *done, uint32_t *u0, uint32_t *u1, int32_t *conv) {
    const int32_t f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= frames) return;
    done[f] = f >= B;
    u0[f] = 0;
    u1[f] = 0;
    conv[f] = -1;
}

// Set 0 of the streaming decoder: frame f in slot f, nothing stopped.
__global__ void k_slots_init(int32_t B, int32_t frames, Set S) {
    const int32_t f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= frames) return;
    S.done[f] = f >= B;
    S.unsat[0][f] = 0;
    S.unsat[1][f] = 0;
    S.conv[f] = -1;
    S.fid[f] = f < B ? f : -1;
}

// A chunk starts in set 0 with no compaction planned.
__global__ void k_ctrl_reset(Ctrl *ctrl) {
    ctrl->cur = 0u;
    ctrl->go = 0u;
    ctrl->active = 0;
}

// llr[B][n] -> r[tile][j][64] through a 64 x 64 LDS tile.
__global__ __launch_bounds__(256) void k_to_tiles(const float *__restrict__ llr, int32_t B, int32_t n,
                                                  float *__restrict__ r) {
    __shared__ float t[kTile][kTile + 1];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int32_t nchunks = (n + 63) / 64;
    const int32_t tile = blockIdx.x / nchunks, j0 = (blockIdx.x % nchunks) * 64;
#pragma unroll 4
    for (int k = w; k < kTile; k += kWaves) {
        const int64_t f = (int64_t)tile * kTile + k;
        const int32_t j = j0 + lane;
        t[k][lane] = (f < B && j < n) ? llr[f * n + j] + 0.0f : 0.0f; // -0 -> +0: no s or x is ever -0
    }
    __syncthreads();
    float *rt = r + (size_t)tile * n * kTile;
#pragma unroll 4
    for (int k = w; k < kTile; k += kWaves) {
        const int32_t j = j0 + k;
        if (j < n) rt[(size_t)j * kTile + lane] = t[lane][k];
    }
}

// One wavefront = one check row x one frame tile.  `t` is the iteration
// being computed (1-based).
template <bool NT>
__global__ __launch_bounds__(512) void k_check(const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col_idx,
                                               const int32_t *__restrict__ row_class, int32_t m, int32_t n, int64_t E,
                                               int32_t row_blocks, const Bufs bufs, int32_t t,
                                               const float *__restrict__ alpha, const float *__restrict__ beta,
                                               int32_t n_classes) {
    const Set S = cur_set(bufs);
    const float *__restrict__ r = S.r;
    const float *__restrict__ s = S.s;
    float *__restrict__ eta = S.eta;
    const uint32_t *__restrict__ done = S.done;
    uint32_t *__restrict__ unsat = unsat_of(S, t);
    const uint32_t bid = xcd_swizzle(blockIdx.x, gridDim.x);
    const int32_t tile = bid / row_blocks;
    const int32_t w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int32_t row = (bid % row_blocks) * (int32_t)(blockDim.x >> 6) + w;
    const int lane = threadIdx.x & 63;
    const int32_t f = tile * kTile + lane;
    const bool act = !done[f];
    if (row >= m || !__any(act)) return;

    const float *sv = (t == 1 ? r : s) + (size_t)tile * n * kTile + lane;
    float *et = eta + (size_t)tile * E * kTile + lane;
    const int32_t e0 = row_ptr[row], e1 = row_ptr[row + 1];

    float min0 = __builtin_inff(), min1 = __builtin_inff();
    int32_t am = -1;
    uint32_t negs = 0, par = 0, syn = 0;
    for (int32_t e = e0; e < e1; ++e) {
        const float sj = sv[(size_t)col_idx[e] * kTile];
        syn ^= sj < 0.0f;
        const float x = (t == 1) ? sj : sj - ld_msg<NT>(&et[(size_t)e * kTile]);
        const float a = fabsf(x);
        const uint32_t ng = x < 0.0f;
        par ^= ng;
        const int32_t k = e - e0;
        if (k < 32) negs |= ng << k;
        if (a < min0) {
            min1 = min0;
            min0 = a;
            am = k;
        } else if (a < min1) {
            min1 = a;
        }
    }
    if (alpha != nullptr && e1 > e0) {
        const int32_t c = row_class[row];
        const float al = alpha[(t - 1) * n_classes + c], be = beta[(t - 1) * n_classes + c];
        const float v0 = fmaf(al, min0, -be), v1 = fmaf(al, min1, -be);
        min0 = v0 > 0.0f ? v0 : 0.0f;
        min1 = v1 > 0.0f ? v1 : 0.0f;
    }
    for (int32_t e = e0; e < e1; ++e) {
        const int32_t k = e - e0;
        uint32_t ng;
        if (k < 32) {
            ng = (negs >> k) & 1u;
        } else { // rows longer than 32: recompute the sign of x (inputs unchanged so far)
            const float sj = sv[(size_t)col_idx[e] * kTile];
            const float x = (t == 1) ? sj : sj - ld_msg<NT>(&et[(size_t)e * kTile]);
            ng = x < 0.0f;
        }
        const float mag = (k == am) ? min1 : min0;
        if (act) st_msg<NT>(&et[(size_t)e * kTile], (par ^ ng) ? -mag : mag);
    }
    if (act && syn) unsat[f] = 1u;
}

// The same check update for graphs whose rows all have DC edges, RPW rows
// per wavefront: the loops are unrolled and every load of the wavefront's
// rows is issued before any use, so it keeps 2 DC RPW requests in flight,
// and there are RPW times fewer wavefronts to launch.  The row's two
// smallest magnitudes come from the min3 / med3 tournament, its sign parity
// and syndrome from XORs of sign bits (r is loaded as r + 0, so no s or x is
// -0 and a sign bit is the sign), and plain Min-Sum messages (PLAIN) take
// two instructions per edge (edge_message); learned weights apply to the two
// magnitudes before the per-edge selection.
template <int DC, int RPW, bool NT, bool PLAIN>
__global__ __launch_bounds__(512) void k_check_dc(const int32_t *__restrict__ col_idx,
                                                  const int32_t *__restrict__ row_class, int32_t m, int32_t n,
                                                  int64_t E, int32_t row_blocks, const Bufs bufs, int32_t t,
                                                  const float *__restrict__ alpha, const float *__restrict__ beta,
                                                  int32_t n_classes) {
    const Set S = cur_set(bufs);
    const float *__restrict__ r = S.r;
    const float *__restrict__ s = S.s;
    float *__restrict__ eta = S.eta;
    const uint32_t *__restrict__ done = S.done;
    uint32_t *__restrict__ unsat = unsat_of(S, t);
    const uint32_t bid = xcd_swizzle(blockIdx.x, gridDim.x);
    const int32_t tile = bid / row_blocks;
    const int32_t w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int32_t row0 = ((bid % row_blocks) * (int32_t)(blockDim.x >> 6) + w) * RPW;
    const int lane = threadIdx.x & 63;
    if (row0 >= m) return;
    const int32_t f = tile * kTile + lane;
    const uint32_t dn = done[f];
    // The rows' column indices (scalar loads) are requested before the frame
    // flags are tested, so that their latencies overlap; the empty asm, which
    // takes a value that depends on every index, keeps the compiler from
    // moving the index loads behind the test.
    // the wavefront's rows (a row past m repeats row0, and computes nothing)
    int32_t rw[RPW];
#pragma unroll
    for (int q = 0; q < RPW; ++q) rw[q] = row0 + q < m ? row0 + q : row0;
    int32_t ci[RPW][DC];
    int32_t all = 0;
#pragma unroll
    for (int q = 0; q < RPW; ++q) {
        // rows of equal degree: CSR offsets are row * DC
        const int64_t e0 = (int64_t)rw[q] * DC;
#pragma unroll
        for (int k = 0; k < DC; ++k) ci[q][k] = col_idx[e0 + k];
    }
#pragma unroll
    for (int q = 0; q < RPW; ++q)
#pragma unroll
        for (int k = 0; k < DC; ++k) all ^= ci[q][k];
    asm volatile("" ::"s"(all));
    const bool act = dn == 0u;
    if (!__any(act)) return;

    const float *sv = (t == 1 ? r : s) + (size_t)tile * n * kTile + lane;
    float *et = eta + (size_t)tile * E * kTile + lane;
    float sj[RPW][DC], ev[RPW][DC];
#pragma unroll
    for (int q = 0; q < RPW; ++q) {
        const int64_t e0 = (int64_t)rw[q] * DC;
#pragma unroll
        for (int k = 0; k < DC; ++k) sj[q][k] = sv[(size_t)ci[q][k] * kTile];
#pragma unroll
        for (int k = 0; k < DC; ++k) ev[q][k] = (t == 1) ? 0.0f : ld_msg<NT>(&et[(size_t)(e0 + k) * kTile]);
    }
    uint32_t syn = 0;
#pragma unroll
    for (int q = 0; q < RPW; ++q) {
        if (row0 + q >= m) break;
        const int32_t row = rw[q];
        float x[DC], a[DC];
        uint32_t xb[DC], sb[DC];
#pragma unroll
        for (int k = 0; k < DC; ++k) {
            x[k] = (t == 1) ? sj[q][k] : sj[q][k] - ev[q][k];
            a[k] = fabsf(x[k]);
            xb[k] = __float_as_uint(x[k]);
            sb[k] = __float_as_uint(sj[q][k]);
        }
        syn |= xor_all<DC>(sb); // sign bit: parity of the row's hard decisions
        const uint32_t par = xor_all<DC>(xb);
        float min0, min1;
        min_pair<DC>(a, min0, min1);
        if (act) {
            const int64_t e0 = (int64_t)row * DC;
            if constexpr (PLAIN) {
                const uint32_t K = row_word(min0, min1, par);
#pragma unroll
                for (int k = 0; k < DC; ++k) st_msg<NT>(&et[(size_t)(e0 + k) * kTile], edge_message(x[k], min1, K));
            } else {
                const int32_t c = row_class[row];
                const float al = alpha[(t - 1) * n_classes + c], be = beta[(t - 1) * n_classes + c];
                const float v0 = fmaf(al, min0, -be), v1 = fmaf(al, min1, -be);
                const uint32_t b0 = __float_as_uint(v0 > 0.0f ? v0 : 0.0f) ^ (par & 0x80000000u);
                const uint32_t b1 = __float_as_uint(v1 > 0.0f ? v1 : 0.0f) ^ (par & 0x80000000u);
                // the edges at the minimum take the second magnitude (on a tie
                // the two are equal)
#pragma unroll
                for (int k = 0; k < DC; ++k)
                    st_msg<NT>(&et[(size_t)(e0 + k) * kTile],
                               __uint_as_float(((a[k] == min0) ? b1 : b0) ^ (xb[k] & 0x80000000u)));
            }
        }
    }
    if (act && (syn >> 31)) unsat[f] = 1u; // some row of this wavefront is unsatisfied
}

// CPW bit columns x one frame tile per wavefront.  The first 8 messages of
// every column are loaded (8 indices per column with one scalar load, then 8
// message loads) before any add, so a wavefront keeps up to 9 CPW requests in
// flight; longer columns continue in groups of 8.  The adds of a column run
// in ascending check order from +0, then r is added.
template <int CPW, bool NT>
__global__ __launch_bounds__(512) void k_bit(const int32_t *__restrict__ col_ptr, const int32_t *__restrict__ csc_edge,
                                             int32_t n, int64_t E, int32_t col_blocks, const Bufs bufs, int32_t t,
                                             int32_t test_now) {
    const Set S = cur_set(bufs);
    const float *__restrict__ r = S.r;
    float *__restrict__ s = S.s;
    const float *__restrict__ eta = S.eta;
    uint32_t *__restrict__ done = S.done;
    const uint32_t *__restrict__ unsat_cur = unsat_of(S, t);
    uint32_t *__restrict__ unsat_next = unsat_of(S, t + 1);
    int32_t *__restrict__ conv = S.conv;
    const uint32_t bid = xcd_swizzle(blockIdx.x, gridDim.x);
    const int32_t tile = bid / col_blocks;
    const int32_t w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int32_t cb = bid % col_blocks;
    static_assert(CPW <= 8, "col_ptr has 8 entries of padding");
    const int32_t col0 = (cb * (int32_t)(blockDim.x >> 6) + w) * CPW;
    const int lane = threadIdx.x & 63;
    if (col0 >= n) return;
    const int32_t f = tile * kTile + lane;
    const uint32_t dn = done[f], uc = unsat_cur[f];
    // Column pointers and the first 8 CSC entries of each column (scalar
    // loads) are requested before the frame flags are tested, so that their
    // latencies overlap; the empty asm, which takes a value that depends on
    // every index and the test flag, keeps the compiler from moving those
    // loads behind the test.
    // col_ptr at col0 .. col0 + CPW (in bounds: 8 entries of padding equal to
    // E, so that columns past n get k0 = k1 = E, no messages)
    int32_t kp[CPW + 1], k0[CPW], k1[CPW], idx0[CPW][8];
#pragma unroll
    for (int c = 0; c <= CPW; ++c) kp[c] = col_ptr[col0 + c];
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
        k0[c] = kp[c];
        k1[c] = kp[c + 1];
    }
#pragma unroll
    for (int c = 0; c < CPW; ++c)
#pragma unroll
        for (int u = 0; u < 8; ++u) idx0[c][u] = csc_edge[k0[c] + u]; // in bounds: 8 entries of padding
    int32_t all = 0;
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
        all ^= k1[c];
#pragma unroll
        for (int u = 0; u < 8; ++u) all ^= idx0[c][u];
    }
    asm volatile("" ::"s"(all), "v"(uc));
    bool act = dn == 0u;
    if (!__any(act)) return;
    const bool stop = act && test_now && uc == 0u;
    if (col0 == 0) { // the wavefront of column 0 keeps the per-frame flags
        if (stop) {
            done[f] = 1u;
            conv[f] = t - 1;
        } else if (act) {
            unsat_next[f] = 0u;
        }
    }
    act = act && !stop;
    if (!__any(act)) return;
    const float *et = eta + (size_t)tile * E * kTile + lane;
    float rv[CPW], acc[CPW], ev[CPW][8];
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
        const int32_t col = col0 + c < n ? col0 + c : col0;
        rv[c] = r[((size_t)tile * n + col) * kTile + lane];
    }
    // Only a column's own messages are loaded: the bounds are uniform across
    // the wavefront, so each load sits behind a scalar branch (a column of
    // 2 or 3 checks issues 2 or 3 loads, not 8).
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            ev[c][u] = 0.0f;
            if (k0[c] + u < k1[c]) ev[c][u] = ld_msg<NT>(&et[(size_t)idx0[c][u] * kTile]);
        }
    }
    // The adds below are under the same conditions as the loads; the compiler
    // would merge them into the load branches, where the first add waits for
    // its load before the other loads are issued.  Passing every loaded value
    // through an empty asm once all loads are issued keeps the adds after it.
#pragma unroll
    for (int c = 0; c < CPW; ++c)
        asm volatile("" : "+v"(ev[c][0]), "+v"(ev[c][1]), "+v"(ev[c][2]), "+v"(ev[c][3]), "+v"(ev[c][4]),
                     "+v"(ev[c][5]), "+v"(ev[c][6]), "+v"(ev[c][7]));
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
        acc[c] = 0.0f;
#pragma unroll
        for (int u = 0; u < 8; ++u) acc[c] = (k0[c] + u < k1[c]) ? acc[c] + ev[c][u] : acc[c]; // a select
        for (int32_t k = k0[c] + 8; k < k1[c]; k += 8) { // columns with more than 8 checks
            int32_t idx[8];
            float e2[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) idx[u] = csc_edge[k + u];
#pragma unroll
            for (int u = 0; u < 8; ++u) e2[u] = ld_msg<NT>(&et[(size_t)(k + u < k1[c] ? idx[u] : idx[0]) * kTile]);
#pragma unroll
            for (int u = 0; u < 8; ++u) acc[c] = (k + u < k1[c]) ? acc[c] + e2[u] : acc[c];
        }
    }
    if (act) {
#pragma unroll
        for (int c = 0; c < CPW; ++c)
            if (col0 + c < n) s[((size_t)tile * n + col0 + c) * kTile + lane] = acc[c] + rv[c];
    }
}

// Syndrome of the current decision only (after the last iteration).
__global__ __launch_bounds__(512) void k_syndrome(const int32_t *__restrict__ row_ptr,
                                                  const int32_t *__restrict__ col_idx, int32_t m, int32_t n,
                                                  int32_t row_blocks, const Bufs bufs, int32_t use_r, int32_t upar) {
    const Set S = cur_set(bufs);
    const uint32_t bid = xcd_swizzle(blockIdx.x, gridDim.x);
    const int32_t tile = bid / row_blocks;
    const int32_t w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int32_t row = (bid % row_blocks) * (int32_t)(blockDim.x >> 6) + w;
    const int lane = threadIdx.x & 63;
    const int32_t f = tile * kTile + lane;
    const bool act = !S.done[f];
    if (row >= m || !__any(act)) return;
    const float *sv = (use_r ? S.r : S.s) + (size_t)tile * n * kTile + lane;
    uint32_t syn = 0;
    for (int32_t e = row_ptr[row]; e < row_ptr[row + 1]; ++e) syn ^= sv[(size_t)col_idx[e] * kTile] < 0.0f;
    if (act && syn) unsat_of(S, upar)[f] = 1u;
}

// Outputs of the frames in a chunk's slots: iterations and convergence flag
// per frame (after the last iteration), and (below) posteriors and decisions.
__global__ void k_out_flags(const Bufs bufs, int32_t slots, int32_t L, int32_t upar, int32_t *__restrict__ iters,
                            uint8_t *__restrict__ ok) {
    const Set S = cur_set(bufs);
    const int32_t f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= slots) return;
    const int32_t id = S.fid[f];
    if (id < 0) return;
    const int32_t c = S.conv[f];
    iters[id] = c >= 0 ? c : L;
    if (ok) ok[id] = (c >= 0 || unsat_of(S, upar)[f] == 0u) ? 1 : 0;
}

// s (or r for frames that stopped at iteration 0) -> post[B][n], bits[B][n]
// through a 64 x 64 LDS tile.  STOPPED: at a compaction that goes ahead,
// only the frames that have stopped (they are not copied on), and their
// iterations and convergence flags too; else, after the last iteration,
// every frame still in a slot.
template <bool STOPPED>
__global__ __launch_bounds__(256) void k_out_tiles(const Bufs bufs, int32_t n, int32_t L, int32_t items,
                                                   float *__restrict__ post, uint8_t *__restrict__ bits,
                                                   int32_t *__restrict__ iters, uint8_t *__restrict__ ok) {
    if (STOPPED && !bufs.ctrl->go) return;
    const Set S = STOPPED ? plan_set(bufs) : cur_set(bufs);
    __shared__ float t[kTile][kTile + 1];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int32_t nchunks = (n + 63) / 64;
    for (int32_t item = blockIdx.x; item < items; item += gridDim.x) { // (tile, 64 bits)
        const int32_t tile = item / nchunks, j0 = (item % nchunks) * 64;
        const int32_t f_lane = tile * kTile + lane;
        const int32_t id_lane = S.fid[f_lane];
        const bool emit = id_lane >= 0 && (!STOPPED || S.done[f_lane]);
        if (!__syncthreads_or(emit)) continue;
        if (STOPPED && j0 == 0 && w == 0 && emit) { // a stopped frame: it stopped by the codeword test
            iters[id_lane] = S.conv[f_lane];
            if (ok) ok[id_lane] = 1;
        }
        const bool use_r = L == 0 || S.conv[f_lane] == 0;
        const float *src = (use_r ? S.r : S.s) + (size_t)tile * n * kTile;
#pragma unroll 4
        for (int k = w; k < kTile; k += kWaves) {
            const int32_t j = j0 + k;
            t[lane][k] = (j < n) ? src[(size_t)j * kTile + lane] : 0.0f;
        }
        __syncthreads();
#pragma unroll 4
        for (int k = w; k < kTile; k += kWaves) {
            const int32_t fk = tile * kTile + k;
            const int64_t id = S.fid[fk];
            const int32_t j = j0 + lane;
            if (id >= 0 && (!STOPPED || S.done[fk]) && j < n) {
                const float v = t[k][lane];
                if (post) post[id * n + j] = v;
                bits[id * n + j] = v < 0.0f ? 1 : 0;
            }
        }
        __syncthreads(); // t is rewritten by the next item
    }
}

// Dense decoder outputs (frame f in slot f): iterations and convergence flag.
__global__ void k_finalize(int32_t B, int32_t L, const int32_t *__restrict__ conv,
                           const uint32_t *__restrict__ unsat_final, int32_t *__restrict__ iters,
                           uint8_t *__restrict__ ok) {
    const int32_t f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= B) return;
    const int32_t c = conv[f];
    iters[f] = c >= 0 ? c : L;
    if (ok) ok[f] = (c >= 0 || unsat_final[f] == 0u) ? 1 : 0;
}

// Dense decoder: s (or r for frames that stopped at iteration 0) -> post[B][n], bits[B][n].
__global__ __launch_bounds__(256) void k_from_tiles(const float *__restrict__ r, const float *__restrict__ s,
                                                    const int32_t *__restrict__ conv, int32_t B, int32_t n,
                                                    int32_t L, float *__restrict__ post, uint8_t *__restrict__ bits) {
    __shared__ float t[kTile][kTile + 1];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int32_t nchunks = (n + 63) / 64;
    const int32_t tile = blockIdx.x / nchunks, j0 = (blockIdx.x % nchunks) * 64;
    const int32_t f_lane = tile * kTile + lane;
    const bool use_r = L == 0 || (f_lane < B && conv[f_lane] == 0);
    const float *src = (use_r ? r : s) + (size_t)tile * n * kTile;
#pragma unroll 4
    for (int k = w; k < kTile; k += kWaves) {
        const int32_t j = j0 + k;
        t[lane][k] = (j < n) ? src[(size_t)j * kTile + lane] : 0.0f;
    }
    __syncthreads();
#pragma unroll 4
    for (int k = w; k < kTile; k += kWaves) {
        const int64_t f = (int64_t)tile * kTile + k;
        const int32_t j = j0 + lane;
        if (f < B && j < n) {
            const float v = t[k][lane];
            if (post) post[f * n + j] = v;
            bits[f * n + j] = v < 0.0f ? 1 : 0;
        }
    }
}

// ---- frame compaction ------------------------------------------------------
// A 64-frame tile runs until its last frame stops.  Every so often (a fixed
// schedule of iterations) one workgroup counts the frames still decoding in
// the chunk; if packing them into fewer tiles saves enough tile-iterations
// over the iterations left, the frames that have stopped are output, the others
// are copied into the other set, packed (a tile's frames keep their order
// and go to consecutive slots, so every store of a row is at most two
// 256-byte pieces; the packed tiles are spread over the chunk so that every
// XCD keeps some), the rest of that set's slots are marked empty, and the
// chunk continues in that set (the kernels take the set from the control
// words: the set of the last plan, the other one if it went ahead).  Each
// frame's own
// arithmetic is unchanged: it sees the same launches in the same order.
constexpr int kPlanThreads = 1024;
constexpr int kMoveRows = 128; // rows of r, s and eta per wavefront of the copy

__global__ __launch_bounds__(kPlanThreads) void k_compact_plan(const Bufs bufs, int32_t ct, int32_t remaining,
                                                               int32_t *__restrict__ base) {
    __shared__ int32_t part[kPlanThreads], tiles_on[kPlanThreads];
    // the frames are where the previous plan left them (copied if it went ahead)
    const uint32_t c = __builtin_amdgcn_readfirstlane(bufs.ctrl->cur ^ bufs.ctrl->go);
    const Set S = c ? bufs.set[1] : bufs.set[0];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, nw = kPlanThreads / 64;
    for (int32_t tile = w; tile < ct; tile += nw) {
        const uint64_t on = __ballot(S.done[tile * kTile + lane] == 0u);
        if (lane == 0) base[tile] = __popcll(on);
    }
    __syncthreads();
    // exclusive scan of the per-tile counts: a contiguous segment per thread
    const int32_t per = (ct + kPlanThreads - 1) / kPlanThreads;
    const int32_t a0 = tid * per, a1 = a0 + per < ct ? a0 + per : ct;
    int32_t sum = 0, on = 0;
    for (int32_t k = a0; k < a1; ++k) {
        sum += base[k];
        on += base[k] > 0;
    }
    part[tid] = sum;
    tiles_on[tid] = on;
    __syncthreads();
    for (int d = 1; d < kPlanThreads; d <<= 1) { // inclusive Hillis-Steele scan of part, sum of tiles_on
        const int32_t x = tid >= d ? part[tid - d] : 0;
        const int32_t y = tid >= d ? tiles_on[tid - d] : 0;
        __syncthreads();
        part[tid] += x;
        tiles_on[tid] += y;
        __syncthreads();
    }
    int32_t run = part[tid] - sum; // exclusive prefix of this segment
    for (int32_t k = a0; k < a1; ++k) {
        const int32_t c = base[k];
        base[k] = run;
        run += c;
    }
    if (tid == 0) {
        const int32_t active = part[kPlanThreads - 1], t_on = tiles_on[kPlanThreads - 1];
        const int32_t packed = (active + kTile - 1) / kTile;
        bufs.ctrl->cur = c;
        bufs.ctrl->active = active;
        // the copy reads the running tiles and writes the packed ones, about
        // 0.4 of an iteration's bytes per tile for rate-1/2 codes: go when
        // the tiles saved over the iterations left repay that twice
        bufs.ctrl->go = (t_on - packed >= 1 && (int64_t)(t_on - packed) * remaining >= (int64_t)(t_on + packed))
                            ? 1u
                            : 0u;
    }
}

// Packed tile k goes to tile spread(k): consecutive packed tiles land in
// different eighths of the chunk, so that the launches' XCD-contiguous block
// ranges (xcd_swizzle) keep every XCD busy after a compaction.  A bijection
// of 0 .. ct-1 (the identity past the largest multiple of 8).
__device__ __forceinline__ int32_t spread(int32_t k, int32_t ct) {
    const int32_t stride = ct / 8;
    return k < 8 * stride ? (k % 8) * stride + k / 8 : k;
}
__device__ __forceinline__ int32_t unspread(int32_t p, int32_t ct) {
    const int32_t stride = ct / 8;
    return p < 8 * stride ? (p % stride) * 8 + p / stride : p;
}

// Items 0 .. ct * blocks_per_tile - 1 copy the frames still decoding (one
// source tile per blocks_per_tile items); the items after them mark the
// destination slots past the packed frames empty.  A grid of at most a few
// thousand workgroups walks the items, so a plan that does not go ahead
// costs only that grid's launch.
__global__ __launch_bounds__(256) void k_compact_move(const Bufs bufs, const int32_t *__restrict__ base, int32_t n,
                                                      int64_t E, int32_t ct, int32_t blocks_per_tile, int32_t items) {
    if (!bufs.ctrl->go) return;
    const uint32_t c = __builtin_amdgcn_readfirstlane(bufs.ctrl->cur);
    const Set src = c ? bufs.set[1] : bufs.set[0];
    const Set dst = c ? bufs.set[0] : bufs.set[1];
    const int32_t w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int32_t active = bufs.ctrl->active;
    for (int32_t item = blockIdx.x; item < items; item += gridDim.x) {
        if (item >= ct * blocks_per_tile) {
            const int32_t p = (item - ct * blocks_per_tile) * (int32_t)blockDim.x + threadIdx.x;
            if (p < ct * kTile && unspread(p / kTile, ct) * kTile + p % kTile >= active) {
                dst.done[p] = 1u;
                dst.unsat[0][p] = 0u;
                dst.unsat[1][p] = 0u;
                dst.conv[p] = -1;
                dst.fid[p] = -1;
            }
            continue;
        }
        const int32_t tile = item / blocks_per_tile, wb = item % blocks_per_tile;
        const int32_t f = tile * kTile + lane;
        const bool act = src.done[f] == 0u;
        const uint64_t on = __ballot(act);
        if (on == 0ull) continue;
        const int32_t k = base[tile] + __popcll(on & ((1ull << lane) - 1ull)); // packed index
        const int32_t dt = spread(k / kTile, ct), dl = k % kTile;
        const int32_t ds = dt * kTile + dl; // destination slot
        if (wb == 0 && w == 0 && act) {
            dst.done[ds] = 0u;
            dst.unsat[0][ds] = src.unsat[0][f];
            dst.unsat[1][ds] = src.unsat[1][f];
            dst.conv[ds] = src.conv[f];
            dst.fid[ds] = src.fid[f];
        }
        // rows q of [r: n][s: n][eta: E] of this wavefront
        const int64_t R = 2 * (int64_t)n + E;
        const int64_t q0 = ((int64_t)wb * (blockDim.x >> 6) + w) * kMoveRows;
        const int64_t q1 = q0 + kMoveRows < R ? q0 + kMoveRows : R;
        auto copy = [&](const float *a, float *d, int64_t rows_per_tile, int64_t lo, int64_t hi) {
            const float *ap = a + (size_t)tile * rows_per_tile * kTile + lane;
            float *dp = d + (size_t)dt * rows_per_tile * kTile + dl;
#pragma unroll 8
            for (int64_t q = lo; q < hi; ++q) {
                const float v = ap[(size_t)q * kTile];
                if (act) dp[(size_t)q * kTile] = v;
            }
        };
        if (q0 < n) copy(src.r, dst.r, n, q0, q1 < n ? q1 : n);
        if (q1 > n && q0 < 2 * (int64_t)n)
            copy(src.s, dst.s, n, (q0 > n ? q0 : n) - n, (q1 < 2 * (int64_t)n ? q1 : 2 * (int64_t)n) - n);
        if (q1 > 2 * (int64_t)n)
            copy(src.eta, dst.eta, E, (q0 > 2 * (int64_t)n ? q0 : 2 * (int64_t)n) - 2 * n, q1 - 2 * n);
    }
}

// Iterations after which a compaction is planned (roughly geometric: frames
// stop early at high Eb/N0 and late at low).
constexpr int32_t kCompactAt[] = {4, 6, 8, 11, 15, 20, 26, 32, 37, 42, 46};
constexpr int32_t kCompactGrid = 2048; // workgroups of the output and copy kernels of a plan
constexpr int32_t kCompactMinTiles = 16; // chunks of fewer tiles are not compacted

} // namespace

// Chunk budget of the size rule: a chunk's r, s and messages (4 (2n + E)
// bytes per frame) take at most this much of the 256 MiB Infinity Cache.
constexpr double kChunkBytes = 200.0 * 1024 * 1024;

int32_t stream_chunk_tiles(const ldpc_graph &g, int32_t B, int32_t chunk) {
    const int32_t nt = (int32_t)tiles_of(B);
    if (chunk == 0) return nt;
    if (chunk > 0) return chunk < nt ? chunk : nt;
    const double per_tile = (double)kTile * 4.0 * (2.0 * g.n + (double)g.E);
    const double k = kChunkBytes / per_tile;
    const int32_t c = k < 1.0 ? 1 : (k > nt ? nt : (int32_t)k);
    return c;
}

size_t stream_workspace_bytes(const ldpc_graph &g, int32_t B) {
    size_t total = 0;
    carve(g, B, nullptr, &total);
    return total;
}

int stream_decode(const ldpc_graph &g, const float *llr, int32_t B, int32_t L, uint32_t flags, const float *alpha,
                  const float *beta, int32_t T, uint8_t *bits, float *post, int32_t *iters, uint8_t *ok, void *ws,
                  size_t ws_bytes, hipStream_t stream) {
    (void)T;
    size_t need = 0;
    StreamWs w = carve(g, B, ws, &need);
    if (ws == nullptr || ws_bytes < need) return LDPC_EWORKSPACE;
    const int32_t nt = (int32_t)tiles_of(B);
    const int32_t frames = nt * kTile;
    const int32_t period = test_period(flags); // 0: no early exit
    // wavefronts per workgroup of the check / bit kernels (tuning record, else 4)
    const int32_t waves = (g.tuning.set && g.tuning.stream_waves > 0) ? g.tuning.stream_waves : 4;
    const int32_t row_blocks = (g.m + waves - 1) / waves;                     // one row per wavefront
    const int32_t row_blocks_dc = (g.m + waves * kRowsPerWave - 1) / (waves * kRowsPerWave);
    const int32_t col_blocks = (g.n + waves * kColsPerWave - 1) / (waves * kColsPerWave);
    const int32_t nchunks = (g.n + 63) / 64;
    const int32_t ncls = (int32_t)g.class_degrees.size();
    // unrolled check kernel when every row has 6 or 7 edges
    const int32_t regular = (g.dc_min == g.dc_max && (g.dc_max == 6 || g.dc_max == 7)) ? g.dc_max : 0;

    // Chunks: all L iterations of `chunk` tiles before the next tiles, so that
    // a chunk that fits the Infinity Cache is read from there, not from HBM,
    // by every launch after its first.  Each frame sees the same launches in
    // the same order as without chunks; only frames of different chunks are
    // interleaved differently.
    const bool tuned = g.tuning.set && g.tuning.path == 2;
    const int32_t chunk = stream_chunk_tiles(g, B, tuned ? g.tuning.stream_chunk : -1);
    // Non-temporal message accesses: the tuning record's choice, else when one
    // iteration's messages of a chunk (4 E bytes per frame) exceed 2 GiB and
    // so cannot stay in the caches between the two kernels anyway.
    const bool nt_msgs = (tuned && g.tuning.stream_nt >= 0)
                             ? g.tuning.stream_nt == 1
                             : (double)chunk * kTile * 4.0 * (double)g.E > 2.0 * 1024 * 1024 * 1024;

    k_slots_init<<<(frames + 255) / 256, 256, 0, stream>>>(B, frames, w.set[0]);
    k_to_tiles<<<nt * nchunks, 256, 0, stream>>>(llr, B, g.n, w.set[0].r);
    // frame compaction needs early exit and chunks large enough to shrink
    const bool compact = period > 0 && chunk >= kCompactMinTiles;
    const int32_t move_blocks = (int32_t)((2 * (int64_t)g.n + g.E + 4 * kMoveRows - 1) / (4 * kMoveRows));
    auto iterate = [&](auto nt_tag) {
        constexpr bool NT = decltype(nt_tag)::value;
        for (int32_t c0 = 0; c0 < nt; c0 += chunk) {
            // the chunk's tiles c0 .. c0 + ct - 1: every array offset to its first tile
            const int32_t ct = chunk < nt - c0 ? chunk : nt - c0;
            const Bufs b = chunk_bufs(w, g, c0);
            k_ctrl_reset<<<1, 1, 0, stream>>>(w.ctrl);
            size_t next_plan = 0;
            for (int32_t t = 1; t <= L; ++t) {
                if (regular == 6 || regular == 7) {
                    auto *fn = regular == 6 ? (alpha ? k_check_dc<6, kRowsPerWave, NT, false>
                                                     : k_check_dc<6, kRowsPerWave, NT, true>)
                                            : (alpha ? k_check_dc<7, kRowsPerWave, NT, false>
                                                     : k_check_dc<7, kRowsPerWave, NT, true>);
                    // the graph's rows in the streaming order where it has one
                    const int32_t *cidx = g.stream_order.col_idx ? g.stream_order.col_idx : g.col_idx;
                    const int32_t *rcls = g.stream_order.row_class ? g.stream_order.row_class : g.row_class;
                    timed_launch(K_CHECK, fn, ct * row_blocks_dc, 64 * waves, 0, stream, cidx, rcls, g.m, g.n, g.E,
                                 row_blocks_dc, b, t, alpha, beta, ncls);
                } else
                    timed_launch(K_CHECK, k_check<NT>, ct * row_blocks, 64 * waves, 0, stream, g.row_ptr, g.col_idx,
                                 g.row_class, g.m, g.n, g.E, row_blocks, b, t, alpha, beta, ncls);
                // is the decision of iteration t - 1 tested?
                const int32_t test_now = (period > 0 && (t - 1) % period == 0) ? 1 : 0;
                timed_launch(K_BIT, k_bit<kColsPerWave, NT>, ct * col_blocks, 64 * waves, 0, stream, g.col_ptr,
                             (regular && g.stream_order.csc_edge) ? g.stream_order.csc_edge : g.csc_edge, g.n, g.E,
                             col_blocks, b, t, test_now);
                while (next_plan < sizeof(kCompactAt) / sizeof(kCompactAt[0]) && kCompactAt[next_plan] < t) ++next_plan;
                if (compact && t < L && next_plan < sizeof(kCompactAt) / sizeof(kCompactAt[0]) &&
                    kCompactAt[next_plan] == t) {
                    const int32_t out_items = ct * nchunks;
                    const int32_t move_items = ct * move_blocks + (ct * kTile + 255) / 256;
                    k_compact_plan<<<1, kPlanThreads, 0, stream>>>(b, ct, L - t, w.base);
                    k_out_tiles<true><<<out_items < kCompactGrid ? out_items : kCompactGrid, 256, 0, stream>>>(
                        b, g.n, L, out_items, post, bits, iters, ok);
                    k_compact_move<<<move_items < kCompactGrid ? move_items : kCompactGrid, 256, 0, stream>>>(
                        b, w.base, g.n, g.E, ct, move_blocks, move_items);
                }
            }
            // the chunk's last decisions, then its outputs
            const int32_t upar = (L + 1) & 1;
            k_syndrome<<<ct * row_blocks, 64 * waves, 0, stream>>>(g.row_ptr, g.col_idx, g.m, g.n, row_blocks, b,
                                                                   L == 0 ? 1 : 0, upar);
            k_out_flags<<<(ct * kTile + 255) / 256, 256, 0, stream>>>(b, ct * kTile, L, upar, iters, ok);
            k_out_tiles<false><<<ct * nchunks, 256, 0, stream>>>(b, g.n, L, ct * nchunks, post, bits, iters, ok);
        }
    };
    if (nt_msgs)
        iterate(std::true_type{});
    else
        iterate(std::false_type{});
    return hipGetLastError() == hipSuccess ? LDPC_OK : LDPC_EHIP;
}

} // namespace ldpc

// ---------------------------------------------------------------------------
// Dense map-reduce decoder (Algorithm 2, Sec. III), kept as an ablation of the
// sparse design.  Same frames-in-lanes tiles, but lambda and eta are full
// m x n matrices per frame: eta[tile][i][j][64], zero wherever H(i,j) = 0.
// Per iteration and frame it moves 12 m n bytes of messages (read + write in
// the row reductions, read in the column sums) instead of 12 E.
//   row kernel     per (row i, frame): lambda(i,j) = s(j) H(i,j) - eta(i,j)
//                  (s = r and eta = 0 in iteration 1) for every j; min0, its
//                  first position, min1 and the sign parity over the j with
//                  H(i,j) = 1; the syndrome of the previous decision; then
//                  eta(i,j) = H(i,j) sign(lambda(i,j)) (total sign) (the other
//                  bits' minimum) for every j (eq. etaCalculation, with the
//                  argmin entry taking min1 as Observation 1 says).
//   column kernel  per (bit j, frame): s(j) = (sum over all i ascending of
//                  eta(i,j), from +0) + r(j) (eq. sCalculation).
// The zero entries add only +-0 to the column sums, so the outputs equal the
// sparse decoders' up to the sign of a zero posterior.
// ---------------------------------------------------------------------------
namespace ldpc {
namespace {

__global__ __launch_bounds__(512) void k_dense_row(const uint8_t *__restrict__ H, int32_t m, int32_t n,
                                                   int32_t row_blocks, const float *__restrict__ r,
                                                   const float *__restrict__ s, float *__restrict__ eta,
                                                   const uint32_t *__restrict__ done, uint32_t *__restrict__ unsat,
                                                   int32_t t) {
    const uint32_t bid = xcd_swizzle(blockIdx.x, gridDim.x);
    const int32_t tile = bid / row_blocks;
    const int32_t w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int32_t row = (bid % row_blocks) * (int32_t)(blockDim.x >> 6) + w;
    const int lane = threadIdx.x & 63;
    const int32_t f = tile * kTile + lane;
    const bool act = !done[f];
    if (row >= m || !__any(act)) return;
    const float *sv = (t == 1 ? r : s) + (size_t)tile * n * kTile + lane;
    float *et = eta + ((size_t)tile * m + row) * (size_t)n * kTile + lane;
    const uint8_t *h = H + (size_t)row * n;
    float min0 = __builtin_inff(), min1 = __builtin_inff();
    int32_t am = -1;
    uint32_t par = 0, syn = 0;
    for (int32_t j = 0; j < n; ++j) {
        const bool hj = h[j] != 0;
        const float sj = sv[(size_t)j * kTile];
        const float lam = sj * (hj ? 1.0f : 0.0f) - (t == 1 ? 0.0f : et[(size_t)j * kTile]);
        if (hj) {
            syn ^= sj < 0.0f;
            par ^= lam < 0.0f;
            const float a = fabsf(lam);
            if (a < min0) {
                min1 = min0;
                min0 = a;
                am = j;
            } else if (a < min1) {
                min1 = a;
            }
        }
    }
    if (act) {
        for (int32_t j = 0; j < n; ++j) {
            const bool hj = h[j] != 0;
            float v = 0.0f;
            if (hj) {
                const float sj = sv[(size_t)j * kTile];
                const float lam = sj - (t == 1 ? 0.0f : et[(size_t)j * kTile]);
                const float mag = (j == am) ? min1 : min0;
                v = (par ^ (lam < 0.0f ? 1u : 0u)) ? -mag : mag;
            }
            et[(size_t)j * kTile] = v;
        }
        if (syn) unsat[f] = 1u;
    }
}

__global__ __launch_bounds__(512) void k_dense_col(int32_t m, int32_t n, int32_t col_blocks,
                                                   const float *__restrict__ r, float *__restrict__ s,
                                                   const float *__restrict__ eta, uint32_t *__restrict__ done,
                                                   const uint32_t *__restrict__ unsat_cur,
                                                   uint32_t *__restrict__ unsat_next, int32_t *__restrict__ conv,
                                                   int32_t t, int32_t test_now) {
    const uint32_t bid = xcd_swizzle(blockIdx.x, gridDim.x);
    const int32_t tile = bid / col_blocks;
    const int32_t w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int32_t cb = bid % col_blocks;
    const int32_t col = cb * (int32_t)(blockDim.x >> 6) + w;
    const int lane = threadIdx.x & 63;
    const int32_t f = tile * kTile + lane;
    bool act = !done[f];
    if (col >= n || !__any(act)) return;
    const bool stop = act && test_now && unsat_cur[f] == 0u;
    if (cb == 0 && w == 0) { // the wavefront of column 0 keeps the per-frame flags
        if (stop) {
            done[f] = 1u;
            conv[f] = t - 1;
        } else if (act) {
            unsat_next[f] = 0u;
        }
    }
    act = act && !stop;
    if (!__any(act)) return;
    const float *et = eta + (size_t)tile * m * (size_t)n * kTile + (size_t)col * kTile + lane;
    float acc = 0.0f;
    for (int32_t i = 0; i < m; ++i) acc = acc + et[(size_t)i * n * kTile];
    const size_t o = ((size_t)tile * n + col) * kTile + lane;
    if (act) s[o] = acc + r[o];
}

// Syndrome of the final decision, over the dense rows.
__global__ __launch_bounds__(512) void k_dense_syndrome(const uint8_t *__restrict__ H, int32_t m, int32_t n,
                                                        int32_t row_blocks, const float *__restrict__ sv_all,
                                                        const uint32_t *__restrict__ done,
                                                        uint32_t *__restrict__ unsat) {
    const uint32_t bid = xcd_swizzle(blockIdx.x, gridDim.x);
    const int32_t tile = bid / row_blocks;
    const int32_t w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int32_t row = (bid % row_blocks) * (int32_t)(blockDim.x >> 6) + w;
    const int lane = threadIdx.x & 63;
    const int32_t f = tile * kTile + lane;
    const bool act = !done[f];
    if (row >= m || !__any(act)) return;
    const float *sv = sv_all + (size_t)tile * n * kTile + lane;
    const uint8_t *h = H + (size_t)row * n;
    uint32_t syn = 0;
    for (int32_t j = 0; j < n; ++j)
        if (h[j]) syn ^= sv[(size_t)j * kTile] < 0.0f;
    if (act && syn) unsat[f] = 1u;
}

struct DenseWs {
    float *r, *s, *eta;
    uint32_t *done, *unsat[2];
    int32_t *conv;
};

DenseWs carve_dense(const ldpc_graph &g, int32_t B, void *base, size_t *total) {
    const size_t nt = tiles_of(B);
    const size_t fr = nt * kTile;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    const size_t o_r = take(nt * (size_t)g.n * kTile * 4);
    const size_t o_s = take(nt * (size_t)g.n * kTile * 4);
    const size_t o_e = take(nt * (size_t)g.m * (size_t)g.n * kTile * 4);
    const size_t o_d = take(fr * 4);
    const size_t o_u0 = take(fr * 4);
    const size_t o_u1 = take(fr * 4);
    const size_t o_c = take(fr * 4);
    if (total) *total = off;
    DenseWs w{};
    char *b = (char *)base;
    if (b) {
        w.r = (float *)(b + o_r);
        w.s = (float *)(b + o_s);
        w.eta = (float *)(b + o_e);
        w.done = (uint32_t *)(b + o_d);
        w.unsat[0] = (uint32_t *)(b + o_u0);
        w.unsat[1] = (uint32_t *)(b + o_u1);
        w.conv = (int32_t *)(b + o_c);
    }
    return w;
}

} // namespace

size_t dense_workspace_bytes(const ldpc_graph &g, int32_t B) {
    size_t total = 0;
    carve_dense(g, B, nullptr, &total);
    return total;
}

int dense_decode(const ldpc_graph &g, const float *llr, int32_t B, int32_t L, uint32_t flags, uint8_t *bits,
                 float *post, int32_t *iters, uint8_t *ok, void *ws, size_t ws_bytes, hipStream_t stream) {
    if (g.dense_h == nullptr) return LDPC_EUNSUPPORTED;
    size_t need = 0;
    DenseWs w = carve_dense(g, B, ws, &need);
    if (ws == nullptr || ws_bytes < need) return LDPC_EWORKSPACE;
    const int32_t nt = (int32_t)tiles_of(B);
    const int32_t frames = nt * kTile;
    const int32_t period = test_period(flags);
    const int32_t waves = 4;
    const int32_t row_blocks = (g.m + waves - 1) / waves;
    const int32_t col_blocks = (g.n + waves - 1) / waves;
    const int32_t nchunks = (g.n + 63) / 64;
    k_flags_init<<<(frames + 255) / 256, 256, 0, stream>>>(B, frames, w.done, w.unsat[0], w.unsat[1], w.conv);
    k_to_tiles<<<nt * nchunks, 256, 0, stream>>>(llr, B, g.n, w.r);
    for (int32_t t = 1; t <= L; ++t) {
        timed_launch(K_DENSE_ROW, k_dense_row, nt * row_blocks, 64 * waves, 0, stream, g.dense_h, g.m, g.n, row_blocks,
                     w.r, w.s, w.eta, w.done, w.unsat[t & 1], t);
        const int32_t test_now = (period > 0 && (t - 1) % period == 0) ? 1 : 0;
        timed_launch(K_DENSE_COL, k_dense_col, nt * col_blocks, 64 * waves, 0, stream, g.m, g.n, col_blocks, w.r, w.s,
                     w.eta, w.done, w.unsat[t & 1], w.unsat[(t + 1) & 1], w.conv, t, test_now);
    }
    uint32_t *unsat_final = w.unsat[(L + 1) & 1];
    k_dense_syndrome<<<nt * row_blocks, 64 * waves, 0, stream>>>(g.dense_h, g.m, g.n, row_blocks,
                                                                 L == 0 ? w.r : w.s, w.done, unsat_final);
    k_finalize<<<(B + 255) / 256, 256, 0, stream>>>(B, L, w.conv, unsat_final, iters, ok);
    k_from_tiles<<<nt * nchunks, 256, 0, stream>>>(w.r, w.s, w.conv, B, g.n, L, post, bits);
    return hipGetLastError() == hipSuccess ? LDPC_OK : LDPC_EHIP;
}

} // namespace ldpc
