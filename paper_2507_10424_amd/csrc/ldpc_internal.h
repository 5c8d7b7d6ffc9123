// Internal declarations of libldpc (not part of the C-ABI).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <tuple>
#include <vector>

#include "ldpc.h"

// Device-side Tanner graph.  Edges are numbered row by row (CSR order), bits
// ascending inside a row; the CSC side lists, for every bit, the CSR numbers
// of its edges in ascending check index.
struct ldpc_graph {
    int device = 0;
    int num_cu = 0;   // compute units of the device
    int lds_max = 0;  // LDS bytes a workgroup may allocate
    int32_t m = 0, n = 0;
    int64_t E = 0;
    int32_t dc_max = 0, dv_max = 0;
    int32_t dc_min = 0, dv_min = 0; // smallest row / column degree (0 included)
    std::vector<int32_t> class_degrees; // distinct nonzero row degrees, ascending
    int32_t *row_ptr = nullptr;   // m + 1
    int32_t *col_idx = nullptr;   // E: bit of each edge
    int32_t *col_ptr = nullptr;   // n + 1 (+ 8 padding entries equal to E)
    int32_t *csc_edge = nullptr;  // E (+ 8 padding entries): CSR edge number of the k-th CSC entry
    int32_t *row_class = nullptr; // m: degree class of the row (-1 for degree 0)
    int32_t *edge_pos = nullptr;  // E: CSC slot of each CSR edge (inverse of csc_edge)
    // On-chip path tables (built when n and E are below 2^16): per CSR edge
    // the bit index in the low 16 bits and the CSC slot in the high 16 bits.
    uint32_t *edge_tab = nullptr; // E, or null
    // Bank-conflict-free on-chip layout (OnchipLayout), built for graphs with
    // one row degree that a layout variant fits; null otherwise.
    struct {
        uint32_t *edge = nullptr;     // [row slot][k]: bit slot | message position << 16
        uint32_t *bitpos = nullptr;   // [bit slot][u]: message position
        int32_t *slot_bit = nullptr;  // [bit slot]: bit index
        int32_t *row_class = nullptr; // [row slot]: degree class
        int32_t nt = 0, npos = 0;     // threads of its geometry, message positions
        int32_t rpt = 0, cpt = 0, dvs = 0; // rows and bits per thread, bit-side stride
        uint32_t dvp = 0;                  // column degree profile, 0 none
    } cf;
    // Streaming path, for graphs of one row degree (6 or 7) whose tile of
    // posteriors exceeds an L2: the rows renumbered in a cache-friendly order
    // (stream_row_order), so that the check kernel's launch order follows it
    // and the messages of consecutive rows stay consecutive in memory.  Row p
    // of the new numbering is row order[p]; its edges are p DC .. p DC + DC - 1
    // (bits ascending), csc_edge lists every column's edges in ascending
    // original row (the column-sum order) by their new numbers.  Null when
    // the graph keeps its own order.
    struct {
        int32_t *col_idx = nullptr;   // E
        int32_t *csc_edge = nullptr;  // E + 8 (8 entries of padding, 0)
        int32_t *row_class = nullptr; // m
    } stream_order;
    // Device copy of the dense m x n H (0/1 bytes) for the dense map-reduce
    // decoder, kept when m * n <= kDenseMaxBytes; null otherwise.
    uint8_t *dense_h = nullptr;
    // Launch choices picked by ldpc_autotune or set by ldpc_graph_set_tuning.
    struct {
        bool set = false;
        int path = 0;         // 1 on-chip, 2 streaming
        int variant = -1;     // on-chip kernel variant
        int wg_per_cu = 0;    // on-chip workgroups per CU (0: occupancy limit)
        int waves_per_simd = 0; // on-chip register budget: 0 compiler's, 4 / 3 at least 4 / 3 waves per SIMD
        int stream_waves = 4; // wavefronts per workgroup of the streaming kernels
        int stream_nt = -1;   // non-temporal message accesses: 1 yes, 0 no, -1 by size
        int stream_chunk = -1; // tiles per chunk of the streaming path: 0 all, -1 by size
    } tuning;
};

#define LDPC_HIP_TRY(expr)                                   \
    do {                                                     \
        if ((expr) != hipSuccess) return LDPC_EHIP;          \
    } while (0)

namespace ldpc {

constexpr int kTile = 64; // frames per tile of the streaming layout (one wavefront)

// Streaming (HBM-resident) decoder: workspace bytes and launch sequence.
size_t stream_workspace_bytes(const ldpc_graph &g, int32_t B);
int stream_decode(const ldpc_graph &g, const float *llr, int32_t B, int32_t L, uint32_t flags,
                  const float *alpha, const float *beta, int32_t T, uint8_t *bits, float *post,
                  int32_t *iters, uint8_t *ok, void *ws, size_t ws_bytes, hipStream_t stream);
// Tiles of 64 frames per chunk of the streaming decoder for a batch of B
// frames: chunk 0 = all tiles, k > 0 = at most k, -1 = by size.
int32_t stream_chunk_tiles(const ldpc_graph &g, int32_t B, int32_t chunk);

// On-chip (LDS-resident) decoder: whether the graph fits, workspace, launch.
bool onchip_fits(const ldpc_graph &g);
bool onchip_variant_fits(const ldpc_graph &g, int variant);
int onchip_num_variants();
// Whether the kernel of (variant, register budget) needs no scratch (no spills).
bool onchip_kernel_spill_free(int variant, int waves_per_simd);
// Scratch bytes per thread of that kernel (register spills), -1 if unknown.
int64_t onchip_kernel_spill_bytes(int variant, int waves_per_simd);
// Vector registers per thread of that kernel (-1 if unknown).
int onchip_kernel_vgprs(int variant, int waves_per_simd);
size_t onchip_workspace_bytes(const ldpc_graph &g, int32_t B);
int onchip_decode(const ldpc_graph &g, const float *llr, int32_t B, int32_t L, uint32_t flags,
                  const float *alpha, const float *beta, int32_t T, uint8_t *bits, float *post,
                  int32_t *iters, uint8_t *ok, void *ws, size_t ws_bytes, hipStream_t stream);

// Bank-conflict-free on-chip layout (layout.hip) for a geometry of rpt rows
// and cpt bits per thread: check row slot s = r nt + t and bit slot p = c nt + t
// hold the row and bit given by the tables (a bit stays in its 64-slot block,
// slots n and up are empty).  The bit-side table has a stride of dv >= the
// largest column degree; entries past a bit's degree name zero positions.
struct OnchipLayout {
    int32_t nt = 0;         // threads
    int32_t rpt = 0, cpt = 0; // rows / bits per thread
    uint32_t dvp = 0;         // column degree profile (4 bits per bit slot index), 0 none
    int32_t dc = 0, dv = 0; // largest row degree, bit-side stride
    int32_t npos = 0;       // message positions (the last one for rows past m)
    std::vector<uint32_t> edge;      // [row slot][k]: bit slot | message position << 16
    std::vector<uint32_t> bitpos;    // [bit slot < cpt nt][u]: message position of the bit's u-th check (ascending)
    std::vector<int32_t> slot_bit;   // [bit slot < n]: the bit it holds
    std::vector<int32_t> row_class;  // [slot]: degree class of the row (0 past m)
};
bool onchip_cf_layout(const std::vector<int32_t> &rowptr, const std::vector<int32_t> &col,
                      const std::vector<int32_t> &row_class, int32_t m, int32_t n, int32_t rpt, int32_t cpt,
                      int32_t dvs, uint32_t dvp, OnchipLayout *out);
// The layout geometry the on-chip variants offer for a graph (rows of one
// degree): rows and bits per thread, bit-side stride and column degree
// profile; false if none fits.
bool onchip_cf_geometry(const ldpc_graph &g, const std::vector<int32_t> &col_deg, int32_t *rpt, int32_t *cpt,
                        int32_t *dvs, uint32_t *dvp);

// Order of the rows for the streaming check kernel (roworder.hip): a
// permutation of 0 .. m-1 that keeps rows sharing bits close together.
std::vector<int32_t> stream_row_order(const std::vector<int32_t> &rowptr, const std::vector<int32_t> &col, int32_t m,
                                      int32_t n);

// Several graphs in one on-chip launch.
size_t onchip_multi_workspace_bytes(int32_t njobs);
int onchip_decode_multi(const ldpc_job *jobs, int32_t njobs, int32_t L, uint32_t flags, void *ws, size_t ws_bytes,
                        hipStream_t stream);

// Dense map-reduce decoder (Algorithm 2 on m x n matrices): workspace, launch.
constexpr size_t kDenseMaxBytes = size_t(1) << 26;
size_t dense_workspace_bytes(const ldpc_graph &g, int32_t B);
int dense_decode(const ldpc_graph &g, const float *llr, int32_t B, int32_t L, uint32_t flags, uint8_t *bits,
                 float *post, int32_t *iters, uint8_t *ok, void *ws, size_t ws_bytes, hipStream_t stream);

// Kernel ids of the optional per-kernel timing (ldpc_timing_read).
enum KernelId { K_CHECK = 0, K_BIT = 1, K_ONCHIP = 2, K_DENSE_ROW = 3, K_DENSE_COL = 4, K_COUNT = 5 };
bool timing_on();
void timing_record(int kid, hipEvent_t a, hipEvent_t b);

// Launch `kernel` on `s`.  When timing is enabled the launch goes through
// hipExtLaunchKernel with two HIP events that take the start and end
// timestamps of that dispatch itself (no event packets between kernels).
template <class... P, class... A>
inline void timed_launch(int kid, void (*kernel)(P...), dim3 grid, dim3 block, uint32_t lds, hipStream_t s,
                         A... a) {
    static_assert(sizeof...(P) == sizeof...(A), "argument count");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timing_on() && hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
        std::tuple<P...> args{P(a)...};
        void *ptrs[sizeof...(P)];
        std::apply([&](auto &...x) {
            size_t i = 0;
            ((ptrs[i++] = (void *)&x), ...);
        }, args);
        (void)hipExtLaunchKernel((const void *)kernel, grid, block, ptrs, lds, s, e0, e1, 0);
        timing_record(kid, e0, e1);
        return;
    }
    if (e0) (void)hipEventDestroy(e0);
    kernel<<<grid, block, lds, s>>>(a...);
}

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Flag bits the decode entry points accept.
constexpr uint32_t kKnownFlags = LDPC_NO_EARLY_EXIT | LDPC_FORCE_STREAM | LDPC_FORCE_ONCHIP | LDPC_CHECK_PERIOD(0xff);

// Codeword-test period of a decode: 0 = never (no early exit), else k >= 1.
inline int32_t test_period(uint32_t flags) {
    if (flags & LDPC_NO_EARLY_EXIT) return 0;
    const int32_t k = (int32_t)((flags >> LDPC_CHECK_PERIOD_SHIFT) & 0xffu);
    return k < 1 ? 1 : k;
}

// Linear workgroup id -> logical id such that consecutive logical ids stay on
// one XCD.  Workgroups are dealt to the 8 XCDs round-robin, so XCD x runs the
// ids x, x+8, x+16, ...; mapping them to a contiguous logical range keeps the
// blocks that share data (one frame tile) inside one XCD's L2.
__device__ __forceinline__ uint32_t xcd_swizzle(uint32_t bid, uint32_t nblocks) {
    constexpr uint32_t kXcd = 8;
    const uint32_t per = nblocks / kXcd; // blocks per XCD in the full part
    const uint32_t full = per * kXcd;
    if (bid >= full) return bid;         // ragged tail keeps its id
    return (bid % kXcd) * per + bid / kXcd;
}

} // namespace ldpc
