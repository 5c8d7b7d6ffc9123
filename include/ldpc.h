/*
 * libldpc: batched Min-Sum LDPC decoding on AMD Instinct MI355X (gfx950).
 *
 * Method: "A mapping of the Min-Sum decoder to reduction operations, and its
 * implementation using CUDA kernels" (Sella & Heinis).  The parity matrix H is
 * a run-time argument; only its dimensions are fixed when a graph is built.
 *
 * Conventions shared by every entry point
 *   - Pointers named *_dev are device memory on the current HIP device; the
 *     caller allocates and owns them.  The library owns only the arrays inside
 *     an ldpc_graph (allocated by ldpc_build_graph, freed by
 *     ldpc_graph_destroy).
 *   - Matrices are dense and row-major: H is m x n, per-frame arrays are
 *     B x n with frame b's n values contiguous.
 *   - LLR polarity: a positive LLR favours bit 0.  Hard decision: bit = 1 iff
 *     the posterior is < 0 (so a posterior of +-0 decides 0).
 *   - Decoding calls are asynchronous on `stream`, allocate nothing, never
 *     synchronise the host and do not read anything back; they can be
 *     captured into a HIP graph.  Argument errors are reported before
 *     anything is launched; launch failures are reported as LDPC_EHIP.
 *   - Every entry point returns an LDPC_* status (0 = success) unless noted.
 *
 * The decoding interface proper is ldpc_build_graph, ldpc_graph_info,
 * ldpc_graph_destroy, ldpc_decode_workspace_bytes, ldpc_minsum_decode and
 * ldpc_status_string with the statuses LDPC_OK .. LDPC_EWORKSPACE.  Beyond
 * it, as extensions: the `flags` argument of ldpc_decode_workspace_bytes (the
 * workspace depends on the kernel path, which flags can force), the `cap`
 * argument of ldpc_graph_info (the length of the caller's check_degrees
 * array, so the call never writes past it), the status LDPC_EUNSUPPORTED (a
 * forced kernel path that the graph does not fit), the path flags, and every
 * entry point declared after ldpc_minsum_decode.
 */
#ifndef LDPC_H
#define LDPC_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ldpc_graph ldpc_graph; /* opaque; immutable once built, except its tuning record */

enum ldpc_status {
    LDPC_OK = 0,
    LDPC_EINVAL = -1,      /* bad argument: null pointer, negative size, ... */
    LDPC_EBADH = -2,       /* H holds a value other than 0/1, or a row of degree 1 */
    LDPC_ENOMEM = -3,      /* device or host allocation failed (graph build only) */
    LDPC_EHIP = -4,        /* a HIP call or kernel launch failed */
    LDPC_EWORKSPACE = -5,  /* workspace null or smaller than required */
    LDPC_EUNSUPPORTED = -6 /* the graph exceeds a limit of the requested kernel path */
};

/* Decode flags (bitwise OR). */
enum ldpc_flags {
    /* Run exactly max_iter iterations for every frame (no syndrome exit). */
    LDPC_NO_EARLY_EXIT = 1u << 0,
    /* Force the HBM-streaming kernels (state in device memory, one launch per
     * half-iteration) even where the graph fits the on-chip path. */
    LDPC_FORCE_STREAM = 1u << 1,
    /* Force the on-chip kernel (one workgroup per frame group, state in LDS);
     * LDPC_EUNSUPPORTED if the graph does not fit. */
    LDPC_FORCE_ONCHIP = 1u << 2
};

/* Codeword-test period (the paper's termination variant, Sec. IV: its GPU
 * decoder tests for a codeword after every 6th iteration).  With early exit a
 * frame is tested before the first iteration and after every k-th one, and
 * stops at the first test it passes.  k sits in bits 8..15 of the flags;
 * 0 and 1 both test after every iteration.  Other flag bits must be 0. */
#define LDPC_CHECK_PERIOD_SHIFT 8
#define LDPC_CHECK_PERIOD(k) ((((uint32_t)(k)) & 0xffu) << LDPC_CHECK_PERIOD_SHIFT)

/*
 * Build the Tanner graph of H (Sec. II-B: the neighbour sets N_i of each check
 * row and M_j of each bit column) on the device.
 *   H_dev   m x n uint8 row-major, entries 0 or 1.  Read only; may be freed
 *           after the call returns.
 *   m, n    numbers of checks and bits, m >= 1, n >= 1, number of ones < 2^31.
 *   stream  stream for the build kernels; the call synchronises it before it
 *           returns (it reads degree counts back), so it must not be captured.
 *   out     receives the graph.  On failure *out is set to NULL.
 * Edges are numbered row by row with ascending bit index inside a row; each
 * bit's checks are kept in ascending check index, which fixes the order of
 * the bit-node sum.  Check rows are grouped by degree into classes (rank of
 * the degree among the distinct nonzero row degrees, ascending), used by the
 * learned decoder's per-degree weights.
 * Errors: LDPC_EINVAL (null pointer, m or n < 1), LDPC_EBADH (entry not 0/1,
 * or a row with exactly one 1, whose Min-Sum message is undefined; also more
 * than 2^31 - 1 ones), LDPC_ENOMEM, LDPC_EHIP.
 */
int ldpc_build_graph(const uint8_t *H_dev, int32_t m, int32_t n, hipStream_t stream,
                     ldpc_graph **out);

/*
 * Graph facts.  Any output pointer may be NULL.  check_degrees (host memory,
 * `cap` entries) receives the distinct nonzero row degrees in ascending order;
 * n_classes receives their count.
 */
int ldpc_graph_info(const ldpc_graph *g, int32_t *m, int32_t *n, int64_t *n_edges,
                    int32_t *dc_max, int32_t *dv_max, int32_t *n_classes,
                    int32_t *check_degrees, int32_t cap);

/* Free a graph (NULL is allowed).  Synchronises the device first. */
void ldpc_graph_destroy(ldpc_graph *g);

/*
 * Bytes of device workspace that ldpc_minsum_decode / ldpc_nms_decode need
 * for B frames with the given flags (the kernel path depends on both).
 * Returns 0 for g == NULL or B <= 0.
 */
size_t ldpc_decode_workspace_bytes(const ldpc_graph *g, int32_t B, uint32_t flags);

/*
 * Min-Sum decoding of B frames (Algorithm 1, with the pre-loop codeword test
 * of the paper's kernel listing, Sec. IV).
 *   llr_dev   B x n float32 channel LLRs, finite.  A frame holding an
 *             infinite or NaN LLR gets unspecified outputs (bits still 0/1,
 *             iterations still within 0..L); the other frames' outputs and
 *             the status are unaffected, and no access leaves the buffers.
 *   B         frames, B >= 0 (B == 0 is a no-op).
 *   max_iter  L >= 0 iterations at most.
 *   flags     LDPC_* decode flags.
 *   bits_dev  B x n uint8 out: hard decisions 0/1.
 *   post_dev  B x n float32 out, may be NULL: posterior LLRs s_j.
 *   iters_dev B int32 out: 0 if the channel decision is a codeword, else the
 *             first iteration t after which the syndrome is zero, else L.
 *             With LDPC_NO_EARLY_EXIT always L.  With a check period k > 1
 *             only multiples of k are tested (t = 0, k, 2k, ...).
 *   ok_dev    B uint8 out, may be NULL: 1 iff the final decision is a codeword.
 *   ws_dev, ws_bytes  workspace of at least ldpc_decode_workspace_bytes(g, B,
 *             flags) bytes, 256-byte aligned; its contents need not be set.
 * Each iteration: every check sends each of its bits the product of the signs
 * of the other bits' extrinsic values times the smallest of their magnitudes
 * (eq. eta_update, computed through Observations 1 and 2); every bit sums its
 * channel LLR and its incoming messages (eq. lambda_j, in ascending check
 * order starting from +0, the channel LLR added last); the posteriors are
 * sliced (eq. slice) and a frame stops once H b = 0.  A stopped frame's
 * outputs are those of the iteration at which it stopped.  All arithmetic is
 * IEEE binary32 with round-to-nearest-even and no contraction.
 * Errors: LDPC_EINVAL (null g / llr / bits / iters with B > 0, B < 0,
 * max_iter < 0, an unknown flag bit), LDPC_EWORKSPACE, LDPC_EUNSUPPORTED,
 * LDPC_EHIP.
 */
int ldpc_minsum_decode(const ldpc_graph *g, const float *llr_dev, int32_t B, int32_t max_iter,
                       uint32_t flags, uint8_t *bits_dev, float *post_dev, int32_t *iters_dev,
                       uint8_t *ok_dev, void *ws_dev, size_t ws_bytes, hipStream_t stream);

/*
 * Largest workspace ldpc_minsum_decode_noalloc can serve from the library's
 * own device memory: 16 MiB per GPU.  The on-chip path needs about 2 KiB for
 * any batch; the streaming path needs 8 (2 n + E) + 40 bytes per frame (two
 * copies of its state, for frame compaction), rounded up to tiles of 64
 * frames.
 */
#define LDPC_NOALLOC_SCRATCH_BYTES ((size_t)16 << 20)

/*
 * ldpc_minsum_decode without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops that
 * must not call hipMalloc, harnesses that forbid it).  The kernels use a
 * fixed scratch array that the library holds on every GPU it runs on (its
 * address is looked up once per device, at the first call on that device);
 * the call itself allocates nothing.  Inputs, outputs, flags, results and the
 * other errors are those of ldpc_minsum_decode.  The graph must live on the
 * current device (else LDPC_EINVAL).  A decode whose workspace
 * (ldpc_decode_workspace_bytes(g, B, flags)) exceeds
 * LDPC_NOALLOC_SCRATCH_BYTES returns LDPC_EWORKSPACE and launches nothing.
 * Every call on one GPU shares that GPU's scratch array, and each call
 * re-initialises what it needs from it: calls that may overlap on one GPU
 * (other streams, other host threads) race and must be serialised by the
 * caller, e.g. by issuing them on one stream.
 */
int ldpc_minsum_decode_noalloc(const ldpc_graph *g, const float *llr_dev, int32_t B, int32_t max_iter,
                               uint32_t flags, uint8_t *bits_dev, float *post_dev, int32_t *iters_dev,
                               uint8_t *ok_dev, hipStream_t stream);

/*
 * The paper's dense map-reduce form of the same decoder (Algorithm 2, Sec. III),
 * as an ablation of the sparse design: per frame, lambda and eta are full
 * m x n matrices (zero where H(i,j) = 0), each row reduction runs over all n
 * columns and each column sum over all m rows, on HBM-resident frames-in-lanes
 * tiles (12 m n message bytes per frame and iteration instead of 12 E).
 * Arguments, outputs and errors are those of ldpc_minsum_decode; the outputs
 * equal it except that a zero posterior may have the other sign.  Accepted
 * flags: LDPC_NO_EARLY_EXIT and a check period.  Needs the graph's copy of the
 * dense H, which ldpc_build_graph keeps when m * n <= 2^26; otherwise
 * LDPC_EUNSUPPORTED.  ldpc_dense_workspace_bytes returns 0 in that case.
 */
size_t ldpc_dense_workspace_bytes(const ldpc_graph *g, int32_t B);
int ldpc_minsum_decode_dense(const ldpc_graph *g, const float *llr_dev, int32_t B, int32_t max_iter,
                             uint32_t flags, uint8_t *bits_dev, float *post_dev, int32_t *iters_dev,
                             uint8_t *ok_dev, void *ws_dev, size_t ws_bytes, hipStream_t stream);

/*
 * One job of a multi-code decode: a graph with its B frames and outputs,
 * laid out as for ldpc_minsum_decode (post_dev and ok_dev may be NULL).
 */
typedef struct ldpc_job {
    const ldpc_graph *g;
    const float *llr_dev;
    int32_t B;
    uint8_t *bits_dev;
    float *post_dev;
    int32_t *iters_dev;
    uint8_t *ok_dev;
} ldpc_job;

enum { LDPC_MAX_JOBS = 16 };

/* Workspace bytes of ldpc_minsum_decode_multi for njobs jobs. */
size_t ldpc_multi_workspace_bytes(int32_t njobs);

/*
 * Min-Sum decoding of the frames of several codes (up to LDPC_MAX_JOBS
 * graphs, each with its own batch) in one call, with the semantics of
 * ldpc_minsum_decode for every frame (per-frame early exit; LDPC_NO_EARLY_EXIT
 * and the check period are honoured, the path flags are ignored).  Every graph
 * must fit the on-chip kernel and live on the current device.  Jobs whose
 * batch alone fills the GPU run as launches of their own kernels (with the
 * graph's tuning record), one launch for all such jobs of the same kernel and
 * launch shape (the same graph, or graphs of one shape); the others share one
 * persistent launch.  In each launch workgroups take frames from per-job
 * counters, largest job (frames x edges) first, and move to the next job
 * without waiting for the others.  Several launches run side by side: the
 * first on `stream`, the others on side streams that the library creates
 * once per device (default priority) and forks from `stream` and joins back
 * into it in this call, so that the call is ordered on `stream` like one
 * kernel.  Calls on one device take a lock while they enqueue.  The first
 * call on a device that needs them creates the side streams: make it before
 * capturing such a call into a HIP graph (a capture records the fork and the
 * join as graph dependencies).
 * Errors: LDPC_EINVAL (null or empty job list, null pointers in a job with
 * B > 0, B < 0, max_iter < 0), LDPC_EUNSUPPORTED (a graph does not fit, or
 * more than LDPC_MAX_JOBS jobs), LDPC_EWORKSPACE, LDPC_EHIP.
 */
int ldpc_minsum_decode_multi(const ldpc_job *jobs, int32_t njobs, int32_t max_iter, uint32_t flags, void *ws_dev,
                             size_t ws_bytes, hipStream_t stream);

/*
 * Normalised / offset Min-Sum with learned weights (an extension; the paper
 * decodes with plain Min-Sum).  Identical to ldpc_minsum_decode except that in
 * iteration t (1-based) the message magnitude mu of a check row whose degree
 * class is c (see ldpc_build_graph) becomes
 *     max(fma(alpha[t-1][c], mu, -beta[t-1][c]), 0)
 * before the sign is applied.  alpha = 1, beta = 0 everywhere reproduces
 * ldpc_minsum_decode bit for bit.
 *   alpha_dev, beta_dev  T x n_classes float32 device arrays, row-major,
 *                        owned by the caller; they must not change until the
 *                        call's kernels have finished (they may be read through
 *                        the scalar cache).
 *   T                    number of weight rows; requires max_iter <= T.
 * Errors: as ldpc_minsum_decode, and LDPC_EINVAL for null weights, T < 1 or
 * max_iter > T.
 */
int ldpc_nms_decode(const ldpc_graph *g, const float *llr_dev, int32_t B, int32_t max_iter, uint32_t flags,
                    const float *alpha_dev, const float *beta_dev, int32_t T, uint8_t *bits_dev,
                    float *post_dev, int32_t *iters_dev, uint8_t *ok_dev, void *ws_dev, size_t ws_bytes,
                    hipStream_t stream);

/*
 * Training of the learned decoder of ldpc_nms_decode (an extension; not in
 * the paper).  The objective unrolls exactly T iterations (no syndrome exit)
 * and is the mean over frames and bits of
 *     sum_{t=1..T} softplus((2 c_j - 1) s_j^(t)),
 * the binary cross-entropy of every iteration's posterior against the
 * transmitted bits c (P(bit = 1) = sigmoid(-s)).
 *
 * ldpc_nms_train_workspace_bytes: workspace for B frames, T iterations and a
 * checkpoint of the decoder state every `ckpt_every` iterations (the
 * forward's checkpoints stay there for the backward).
 *
 * ldpc_nms_train_forward: runs the T iterations with the weights (alpha_dev,
 * beta_dev: T x n_classes float32, device), writes the mean loss to
 * loss_dev[0] and, if post_dev is non-null, the iteration-T posteriors
 * (B x n).  target_dev: B x n bits of the transmitted codewords, or NULL for
 * the all-zero codeword.  The posteriors equal those of ldpc_nms_decode with
 * LDPC_NO_EARLY_EXIT and max_iter = T, bit for bit.
 *
 * ldpc_nms_train_backward: gradient of grad_loss * loss with respect to alpha
 * and beta (written to galpha_dev, gbeta_dev, T x n_classes) and, if
 * gllr_dev is non-null, to the channel LLRs (B x n).  It reads the
 * checkpoints of the last forward call on the same workspace and inputs and
 * recomputes each segment of ckpt_every iterations.  The derivative of a
 * check message's magnitude goes to the edge attaining the minimum over the
 * row's other edges (lowest position on a tie), the sign product is held
 * constant and the clip max(v, 0) passes the gradient where v > 0.  Sums over
 * frames are taken in a fixed order (deterministic).
 *
 * The per-frame state lives in LDS when it fits one workgroup; otherwise it
 * lives in the workspace (4 n + 2 E + ckpt_every (n + E) floats per frame).
 * Errors: LDPC_EINVAL (null pointers, B, T or ckpt_every < 1),
 * LDPC_EWORKSPACE, LDPC_EUNSUPPORTED (more than 8 degree classes),
 * LDPC_EHIP.
 */
size_t ldpc_nms_train_workspace_bytes(const ldpc_graph *g, int32_t B, int32_t T, int32_t ckpt_every);
int ldpc_nms_train_forward(const ldpc_graph *g, const float *llr_dev, const uint8_t *target_dev, int32_t B,
                           int32_t T, const float *alpha_dev, const float *beta_dev, int32_t ckpt_every,
                           float *loss_dev, float *post_dev, void *ws_dev, size_t ws_bytes, hipStream_t stream);
int ldpc_nms_train_backward(const ldpc_graph *g, const float *llr_dev, const uint8_t *target_dev, int32_t B,
                            int32_t T, const float *alpha_dev, const float *beta_dev, int32_t ckpt_every,
                            float grad_loss, float *galpha_dev, float *gbeta_dev, float *gllr_dev, void *ws_dev,
                            size_t ws_bytes, hipStream_t stream);

/*
 * Synthetic channel frames on the device: LLRs of BPSK over AWGN (bit c ->
 * 1 - 2c, y = x + sigma z, LLR = 2 y / sigma^2, sigma^2 = 1 / (2 rate
 * 10^(EbN0/10))) for the codewords cw_dev (B x n bits, NULL = all-zero), with
 * Eb/N0 in dB drawn per frame uniformly from [ebn0_lo_db, ebn0_hi_db]
 * (equal bounds: fixed) and written to ebn0_dev (B floats) if non-null.  The
 * normals come from the counter-based Philox4x32-10 generator (Salmon et al.,
 * SC 2011) keyed by `seed` and the Box-Muller transform, so a seed fixes the
 * frames.  Errors: LDPC_EINVAL, LDPC_EHIP.
 */
int ldpc_awgn_llr(const uint8_t *cw_dev, int32_t B, int32_t n, float rate, float ebn0_lo_db, float ebn0_hi_db,
                  uint64_t seed, float *llr_dev, float *ebn0_dev, hipStream_t stream);

/*
 * One Adam step (Kingma & Ba) on `count` float32 parameters in place, with
 * first/second moment buffers m1_dev, m2_dev (zero before step 1) and the
 * 1-based step number for the bias correction.  Errors: LDPC_EINVAL, LDPC_EHIP.
 */
int ldpc_adam_step(float *param_dev, const float *grad_dev, float *m1_dev, float *m2_dev, int32_t count, float lr,
                   float beta1, float beta2, float eps, int32_t step, hipStream_t stream);

/*
 * Launch choices of a graph ("tuning record").  Without one, decoding takes
 * the on-chip path whenever the graph fits (the preferred fitting kernel
 * variant: exact degrees, then the tightest degree masks, two frame slots;
 * as many workgroups as fit on each CU) and otherwise the streaming path with
 * 4 wavefronts per workgroup.
 *   path          1 on-chip, 2 streaming (0 in ldpc_graph_get_tuning: none set)
 *   variant       on-chip kernel variant (degree templates, rows and bits
 *                 per thread, frame slots), -1 for the preferred one
 *   wg_per_cu     on-chip workgroups per CU, 0 for the occupancy limit
 *   stream_waves  wavefronts per workgroup of the streaming kernels (1..8)
 *   waves_per_simd  on-chip register budget: 0 the compiler's, 4 (3) at least
 *                 four (three) resident waves per SIMD (fewer registers per
 *                 thread)
 *   ms            ldpc_autotune: mean time of one decode of the tuning batch
 *   stream_nt     streaming path: 1 marks the message loads and stores
 *                 non-temporal (they stream through the caches and leave them
 *                 to the posterior gathers), 0 not, -1 by size (non-temporal
 *                 when one iteration's messages of a chunk exceed 2 GiB)
 *   stream_chunk  streaming path: tiles of 64 frames decoded together, all
 *                 iterations of one chunk before the next, so that a chunk's
 *                 state can stay in the last-level (Infinity) cache between
 *                 the launches; 0 all tiles at once, k > 0 k tiles, -1 by size
 *                 (as many tiles as fit 200 MiB of posteriors, channel LLRs
 *                 and messages, at least one)
 * LDPC_FORCE_STREAM / LDPC_FORCE_ONCHIP still override the path.
 */
typedef struct ldpc_tuning {
    int32_t path;
    int32_t variant;
    int32_t wg_per_cu;
    int32_t stream_waves;
    int32_t waves_per_simd;
    float ms;
    int32_t stream_nt;
    int32_t stream_chunk;
} ldpc_tuning;

/* Set (t != NULL) or clear (t == NULL) the tuning record.  Not thread-safe
 * against concurrent decodes of the same graph.  Errors: LDPC_EINVAL,
 * LDPC_EUNSUPPORTED (the variant does not fit the graph). */
int ldpc_graph_set_tuning(ldpc_graph *g, const ldpc_tuning *t);
int ldpc_graph_get_tuning(const ldpc_graph *g, ldpc_tuning *t);

/*
 * Autotuner: generates B all-zero frames at ebn0_db on the device, times one
 * warm-up and three decodes (at most max_iter iterations, early exit) for
 * every launch choice that applies to the graph (each fitting on-chip
 * variant under three register budgets, the compiler's and at least 4 or 3
 * waves per SIMD, a tighter one only where the compiler's kernel takes more
 * than 128 or 168 registers, 0..4 workgroups per CU, leaving out kernels
 * that spill under the compiler's budget unless nothing else fits and those
 * that spill more than 320 bytes under a tighter one; the streaming path
 * with 1, 2, 4, 8 wavefronts per workgroup, with and without non-temporal
 * message accesses, whole batch and chunks by size where those differ), times the four fastest again (three interleaved rounds
 * of four decodes), and stores the fastest of those in the graph's tuning
 * record (also returned in *best if non-null).  It synchronises `stream` and
 * creates two HIP events; do not capture it.  The workspace needs
 * ldpc_autotune_workspace_bytes(g, B) bytes.
 * Errors: LDPC_EINVAL, LDPC_EWORKSPACE, LDPC_EHIP.
 */
size_t ldpc_autotune_workspace_bytes(const ldpc_graph *g, int32_t B);
int ldpc_autotune(ldpc_graph *g, int32_t B, int32_t max_iter, float ebn0_db, void *ws_dev, size_t ws_bytes,
                  hipStream_t stream, ldpc_tuning *best);

/*
 * Per-kernel timing for benchmarks (decoding does not need it).
 * ldpc_timing_enable(1) clears the record and starts bracketing every launch
 * of the timed kernels with two HIP events on its launch stream (this adds
 * event records to the stream and is not meant for graph capture);
 * ldpc_timing_enable(0) clears and stops.  ldpc_timing_read waits for the
 * recorded events and returns the summed elapsed milliseconds and the number
 * of launches of one kernel since the last enable:
 *   kernel 0  streaming check-node kernel
 *   kernel 1  streaming bit-node kernel
 *   kernel 2  on-chip whole-decode kernel
 *   kernel 3  dense row-reduction kernel
 *   kernel 4  dense column-sum kernel
 * Errors: LDPC_EINVAL (unknown kernel), LDPC_EHIP.
 */
int ldpc_timing_enable(int on);
int ldpc_timing_read(int32_t kernel, double *total_ms, int64_t *launches);

/* Text for a status code (static storage). */
const char *ldpc_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* LDPC_H */
