// Training of the learned (normalised / offset) Min-Sum decoder on the GPU.
//
// The learned decoder replaces the message magnitude mu of eq. eta_update in
// iteration t by max(fma(alpha[t-1][c], mu, -beta[t-1][c]), 0), c the degree
// class of the check row.  Training unrolls exactly T iterations (no
// syndrome exit) and minimises
//     loss = 1/(B n) sum_frames sum_{t=1..T} sum_j softplus((2 c_j - 1) s_j^(t))
// (binary cross-entropy of every iteration's posterior against the
// transmitted bits; P(bit = 1) = sigmoid(-s)).
//
// Forward: one workgroup per frame, state in LDS (or, for codes whose state
// does not fit, in a per-frame region of the workspace), the same binary32
// arithmetic as the decoder (so the posteriors equal those of
// ldpc_nms_decode with LDPC_NO_EARLY_EXIT bit for bit).  Every K iterations
// the state (s, eta) is written to a checkpoint in the workspace.
// Backward: one workgroup per frame; for each segment of K iterations, last
// first, the state is reloaded from its checkpoint and the segment is
// recomputed, keeping x = s - eta of every iteration of the segment in LDS;
// then the reverse sweep runs through the segment:
//   ds^(t)_j   = scale (2c_j-1) sigmoid((2c_j-1) s_j^(t)) + sum_{e in M_j} dx^(t+1)_e
//   deta^(t)_e = ds^(t)_j - dx^(t+1)_e
//   with v_e = fma(alpha, mu_e, -beta) > 0:  dv = deta sign_e
//     dalpha += dv mu_e,  dbeta -= dv,  dx^(t)_a(e) += dv alpha sign(x_a(e))
// where a(e) is the edge attaining the minimum over the row's other edges
// (lowest position on a tie) and the sign product is held constant.
// Per-frame partial sums are reduced over frames in a fixed order, so the
// gradients are deterministic.
#include "ldpc_internal.h"

namespace ldpc {
namespace {

constexpr int kThreads = 256;
constexpr int kMaxClasses = 8;

__device__ __forceinline__ float softplusf(float z) { return fmaxf(z, 0.0f) + log1pf(expf(-fabsf(z))); }
__device__ __forceinline__ float sigmoidf(float z) {
    const float e = expf(-fabsf(z));
    return z >= 0.0f ? 1.0f / (1.0f + e) : e / (1.0f + e);
}
__device__ __forceinline__ float sgnf(float v) { return v < 0.0f ? -1.0f : 1.0f; }

// Fixed-order block sum of one float per thread (wave shuffles, then the
// wave partials in order); result valid in thread 0.
__device__ float block_sum(float v, float *red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) red[w] = v;
    __syncthreads();
    float t = 0.0f;
    if (threadIdx.x == 0)
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += red[k];
    __syncthreads();
    return t;
}

struct Row {
    float min0, min1; // two smallest |x| (min1 over the edges other than loc0)
    int32_t loc0, loc1;
    uint32_t par;     // parity of the negative x
};

// Scan of a row's x (from LDS, CSR order): minima with first positions, sign
// parity.  Edges with equal |x| keep the first position.
__device__ __forceinline__ Row scan_row(const float *x, int32_t d) {
    Row R{__builtin_inff(), __builtin_inff(), -1, -1, 0u};
    for (int32_t k = 0; k < d; ++k) {
        const float a = fabsf(x[k]);
        R.par ^= x[k] < 0.0f ? 1u : 0u;
        if (a < R.min0) {
            R.min1 = R.min0;
            R.loc1 = R.loc0;
            R.min0 = a;
            R.loc0 = k;
        } else if (a < R.min1) {
            R.min1 = a;
            R.loc1 = k;
        }
    }
    return R;
}

// One check-node pass of iteration t (1-based) on CSR-ordered LDS arrays:
// x = s - eta (kept in xout if non-null), then eta in place.
__device__ void check_pass(const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col_idx,
                           const int32_t *__restrict__ row_class, int32_t m, const float *s, float *eta, float *xout,
                           const float *__restrict__ alpha, const float *__restrict__ beta, int32_t ncls, int32_t t) {
    for (int32_t i = threadIdx.x; i < m; i += blockDim.x) {
        const int32_t e0 = row_ptr[i], d = row_ptr[i + 1] - e0;
        if (d == 0) continue;
        float *x = xout + e0; // x of this row, CSR positions
        for (int32_t k = 0; k < d; ++k) x[k] = s[col_idx[e0 + k]] - eta[e0 + k];
        const Row R = scan_row(x, d);
        const int32_t c = row_class[i];
        const float al = alpha[(t - 1) * ncls + c], be = beta[(t - 1) * ncls + c];
        const float v0 = fmaf(al, R.min0, -be), v1 = fmaf(al, R.min1, -be);
        const float m0 = v0 > 0.0f ? v0 : 0.0f, m1 = v1 > 0.0f ? v1 : 0.0f;
        for (int32_t k = 0; k < d; ++k) {
            const float mag = (k == R.loc0) ? m1 : m0;
            const bool neg = (R.par ^ (x[k] < 0.0f ? 1u : 0u)) != 0u;
            eta[e0 + k] = neg ? -mag : mag;
        }
    }
}

// Bit-node pass: s_j = (+0 + eta over M_j ascending) + r_j.
__device__ void bit_pass(const int32_t *__restrict__ col_ptr, const int32_t *__restrict__ csc_edge, int32_t n,
                         const float *r, const float *eta, float *s) {
    for (int32_t j = threadIdx.x; j < n; j += blockDim.x) {
        float acc = 0.0f;
        for (int32_t k = col_ptr[j]; k < col_ptr[j + 1]; ++k) acc = acc + eta[csc_edge[k]];
        s[j] = acc + r[j];
    }
}

// ONCHIP: the per-frame state lives in LDS; otherwise in a per-frame region
// of `scratch` (global memory), for codes whose state does not fit.
template <bool ONCHIP>
__global__ __launch_bounds__(kThreads) void k_nms_fwd(
    const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col_idx, const int32_t *__restrict__ col_ptr,
    const int32_t *__restrict__ csc_edge, const int32_t *__restrict__ row_class, int32_t m, int32_t n, int32_t E,
    int32_t ncls, const float *__restrict__ llr, const uint8_t *__restrict__ target, int32_t T, int32_t K,
    const float *__restrict__ alpha, const float *__restrict__ beta, float *__restrict__ ckpt,
    float *__restrict__ loss_part, float *__restrict__ post, float *__restrict__ scratch) {
    extern __shared__ float sm[];
    __shared__ float red[16];
    const int32_t f = blockIdx.x;
    float *base = ONCHIP ? sm : scratch + (size_t)f * (2ull * n + 2ull * E);
    float *s = base, *r = s + n, *eta = r + n, *x = eta + E;
    const int32_t nck = (T + K - 1) / K;
    for (int32_t j = threadIdx.x; j < n; j += blockDim.x) {
        const float v = llr[(size_t)f * n + j];
        s[j] = v;
        r[j] = v;
    }
    for (int32_t e = threadIdx.x; e < E; e += blockDim.x) eta[e] = 0.0f;
    __syncthreads();
    float lacc = 0.0f;
    for (int32_t t = 1; t <= T; ++t) {
        if ((t - 1) % K == 0) {
            float *ck = ckpt + ((size_t)f * nck + (t - 1) / K) * (size_t)(n + E);
            for (int32_t j = threadIdx.x; j < n; j += blockDim.x) ck[j] = s[j];
            for (int32_t e = threadIdx.x; e < E; e += blockDim.x) ck[n + e] = eta[e];
            __syncthreads();
        }
        check_pass(row_ptr, col_idx, row_class, m, s, eta, x, alpha, beta, ncls, t);
        __syncthreads();
        bit_pass(col_ptr, csc_edge, n, r, eta, s);
        for (int32_t j = threadIdx.x; j < n; j += blockDim.x) {
            const float y = (target && target[(size_t)f * n + j]) ? 1.0f : -1.0f;
            lacc += softplusf(y * s[j]);
        }
        __syncthreads();
    }
    if (post)
        for (int32_t j = threadIdx.x; j < n; j += blockDim.x) post[(size_t)f * n + j] = s[j];
    const float tot = block_sum(lacc, red);
    if (threadIdx.x == 0) loss_part[f] = tot;
}

template <bool ONCHIP>
__global__ __launch_bounds__(kThreads) void k_nms_bwd(
    const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col_idx, const int32_t *__restrict__ col_ptr,
    const int32_t *__restrict__ csc_edge, const int32_t *__restrict__ row_class, int32_t m, int32_t n, int32_t E,
    int32_t ncls, const float *__restrict__ llr, const uint8_t *__restrict__ target, int32_t T, int32_t K,
    const float *__restrict__ alpha, const float *__restrict__ beta, const float *__restrict__ ckpt, float scale,
    float *__restrict__ gpart /* [B][2][T][ncls] */, float *__restrict__ gllr, float *__restrict__ scratch) {
    extern __shared__ float sm[];
    __shared__ float red[16];
    const int32_t f = blockIdx.x;
    // state: s, r, gs, gr (n each); eta, gxn (E each); xbuf (K*E), sbuf (K*n)
    float *base = ONCHIP ? sm : scratch + (size_t)f * (4ull * n + 2ull * E + (size_t)K * E + (size_t)K * n);
    float *s = base, *r = s + n, *gs = r + n, *gr = gs + n, *eta = gr + n, *gxn = eta + E, *xbuf = gxn + E,
          *sbuf = xbuf + (size_t)K * E;
    const int32_t nck = (T + K - 1) / K;
    float *gp = gpart + (size_t)f * 2 * T * ncls;
    for (int32_t j = threadIdx.x; j < n; j += blockDim.x) {
        r[j] = llr[(size_t)f * n + j];
        gr[j] = 0.0f;
    }
    for (int32_t e = threadIdx.x; e < E; e += blockDim.x) gxn[e] = 0.0f;
    for (int32_t seg = nck - 1; seg >= 0; --seg) {
        const int32_t t0 = seg * K, t1 = (t0 + K < T) ? t0 + K : T;
        const float *ck = ckpt + ((size_t)f * nck + seg) * (size_t)(n + E);
        for (int32_t j = threadIdx.x; j < n; j += blockDim.x) s[j] = ck[j];
        for (int32_t e = threadIdx.x; e < E; e += blockDim.x) eta[e] = ck[n + e];
        __syncthreads();
        for (int32_t t = t0 + 1; t <= t1; ++t) { // recompute the segment
            float *xt = xbuf + (size_t)(t - t0 - 1) * E;
            check_pass(row_ptr, col_idx, row_class, m, s, eta, xt, alpha, beta, ncls, t);
            __syncthreads();
            bit_pass(col_ptr, csc_edge, n, r, eta, s);
            float *st = sbuf + (size_t)(t - t0 - 1) * n;
            for (int32_t j = threadIdx.x; j < n; j += blockDim.x) st[j] = s[j];
            __syncthreads();
        }
        for (int32_t t = t1; t > t0; --t) { // reverse sweep
            const float *xt = xbuf + (size_t)(t - t0 - 1) * E;
            const float *st = sbuf + (size_t)(t - t0 - 1) * n;
            for (int32_t j = threadIdx.x; j < n; j += blockDim.x) {
                const float y = (target && target[(size_t)f * n + j]) ? 1.0f : -1.0f;
                float g = scale * y * sigmoidf(y * st[j]);
                for (int32_t k = col_ptr[j]; k < col_ptr[j + 1]; ++k) g += gxn[csc_edge[k]];
                gs[j] = g;
                gr[j] += g;
            }
            __syncthreads();
            float ga[kMaxClasses], gb[kMaxClasses];
#pragma unroll
            for (int c = 0; c < kMaxClasses; ++c) ga[c] = gb[c] = 0.0f;
            for (int32_t i = threadIdx.x; i < m; i += blockDim.x) {
                const int32_t e0 = row_ptr[i], d = row_ptr[i + 1] - e0;
                if (d == 0) continue;
                const float *x = xt + e0;
                const Row R = scan_row(x, d);
                const int32_t c = row_class[i];
                const float al = alpha[(t - 1) * ncls + c], be = beta[(t - 1) * ncls + c];
                float gx0 = 0.0f, gx1 = 0.0f; // the only edges that receive: loc0 and loc1
                float dga = 0.0f, dgb = 0.0f;
                for (int32_t k = 0; k < d; ++k) {
                    const bool at0 = k == R.loc0;
                    const float mu = at0 ? R.min1 : R.min0;
                    const float v = fmaf(al, mu, -be);
                    if (!(v > 0.0f)) continue;
                    const float sg = ((R.par ^ (x[k] < 0.0f ? 1u : 0u)) != 0u) ? -1.0f : 1.0f;
                    const float geta = gs[col_idx[e0 + k]] - gxn[e0 + k];
                    const float gv = geta * sg;
                    dga += gv * mu;
                    dgb -= gv;
                    if (at0) gx1 += gv * al; // routed to the minimum over the others: loc1
                    else gx0 += gv * al;     // routed to loc0
                }
#pragma unroll
                for (int cc = 0; cc < kMaxClasses; ++cc)
                    if (cc == c) {
                        ga[cc] += dga;
                        gb[cc] += dgb;
                    }
                // x^(t) = s^(t-1) - eta^(t-1): this row's dx^(t), written in place
                for (int32_t k = 0; k < d; ++k) {
                    float g = 0.0f;
                    if (k == R.loc0) g = gx0 * sgnf(x[k]);
                    else if (k == R.loc1) g = gx1 * sgnf(x[k]);
                    gxn[e0 + k] = g;
                }
            }
            __syncthreads();
#pragma unroll
            for (int c = 0; c < kMaxClasses; ++c) {
                if (c >= ncls) break; // uniform
                const float a = block_sum(ga[c], red);
                const float b = block_sum(gb[c], red);
                if (threadIdx.x == 0) {
                    gp[(size_t)(t - 1) * ncls + c] = a;
                    gp[(size_t)T * ncls + (size_t)(t - 1) * ncls + c] = b;
                }
            }
        }
        __syncthreads();
    }
    if (gllr) { // x^(1) = r: the last dx goes to the channel LLRs too
        for (int32_t j = threadIdx.x; j < n; j += blockDim.x) {
            float g = gr[j];
            for (int32_t k = col_ptr[j]; k < col_ptr[j + 1]; ++k) g += gxn[csc_edge[k]];
            gllr[(size_t)f * n + j] = g;
        }
    }
}

// Sum over frames: out[k] = mult * sum_f part[f * stride + offset + k], one
// workgroup per output k.  Thread i adds frames i, i + 256, ... in order, then
// the block reduction adds the threads' partials in a fixed tree; the order
// depends only on B, so the result is the same on every run.
__global__ __launch_bounds__(kThreads) void k_sum_frames(const float *__restrict__ part, int32_t B, int32_t stride,
                                                          int32_t offset, float mult, float *__restrict__ out) {
    __shared__ float red[16];
    const int32_t k = blockIdx.x;
    float acc = 0.0f;
    for (int32_t f = threadIdx.x; f < B; f += kThreads) acc += part[(size_t)f * stride + offset + k];
    const float tot = block_sum(acc, red);
    if (threadIdx.x == 0) out[k] = tot * mult;
}

// ---- synthetic frames --------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
// as 1, 2, 3", SC 2011): 10 rounds of two 32x32 -> 64-bit products on a
// 128-bit counter with a 64-bit key bumped by the Weyl constants.
struct U4 {
    uint32_t x, y, z, w;
};
__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
    constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        const uint32_t lo0 = M0 * c.x, hi0 = __umulhi(M0, c.x);
        const uint32_t lo1 = M1 * c.z, hi1 = __umulhi(M1, c.z);
        c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
        k0 += W0;
        k1 += W1;
    }
    return c;
}
// uniform in (0, 1]
__device__ __forceinline__ float u01(uint32_t v) { return ((float)(v >> 8) + 1.0f) * (1.0f / 16777216.0f); }

// LLRs of BPSK over AWGN for codewords (bits, or all-zero when null), with
// Eb/N0 per frame uniform in [lo_db, hi_db] (lo == hi: fixed), Box-Muller
// normals from the Philox stream keyed by `seed`; LLR = 2 y / sigma^2.
__global__ void k_awgn(const uint8_t *__restrict__ cw, int32_t B, int32_t n, float rate, float lo_db, float hi_db,
                       uint32_t seed_lo, uint32_t seed_hi, float *__restrict__ llr, float *__restrict__ ebn0_out) {
    const int32_t j0 = (blockIdx.x * blockDim.x + threadIdx.x) * 4;
    for (int32_t f = blockIdx.y; f < B; f += gridDim.y) {
        const U4 u = philox4x32_10(U4{0xFFFFFFFFu, (uint32_t)f, 0u, 0u}, seed_lo, seed_hi);
        const float eb = lo_db + (hi_db - lo_db) * (u01(u.x) - 1.0f / 16777216.0f);
        const float sigma2 = 1.0f / (2.0f * rate * exp10f(0.1f * eb));
        const float sigma = sqrtf(sigma2);
        if (ebn0_out && blockIdx.x == 0 && threadIdx.x == 0) ebn0_out[f] = eb;
        if (j0 >= n) continue;
        const U4 v = philox4x32_10(U4{(uint32_t)j0, (uint32_t)f, 1u, 0u}, seed_lo, seed_hi);
        const float r1 = sqrtf(-2.0f * logf(u01(v.x))), r2 = sqrtf(-2.0f * logf(u01(v.z)));
        const float a1 = 6.2831853071795864f * u01(v.y), a2 = 6.2831853071795864f * u01(v.w);
        const float z[4] = {r1 * cosf(a1), r1 * sinf(a1), r2 * cosf(a2), r2 * sinf(a2)};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int32_t j = j0 + k;
            if (j < n) {
                const float x = (cw && cw[(size_t)f * n + j]) ? -1.0f : 1.0f;
                llr[(size_t)f * n + j] = 2.0f * (x + sigma * z[k]) / sigma2;
            }
        }
    }
}

// Adam (Kingma & Ba) on a flat parameter array; step is 1-based.
__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m1,
                       float *__restrict__ m2, int32_t count, float lr, float b1, float b2, float eps, int32_t step) {
    const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    const float gk = g[k];
    const float a = b1 * m1[k] + (1.0f - b1) * gk;
    const float b = b2 * m2[k] + (1.0f - b2) * gk * gk;
    m1[k] = a;
    m2[k] = b;
    const float ah = a / (1.0f - powf(b1, (float)step)), bh = b / (1.0f - powf(b2, (float)step));
    p[k] -= lr * ah / (sqrtf(bh) + eps);
}

struct TrainWs {
    float *ckpt, *loss_part, *gpart, *scratch;
};

size_t fwd_lds(const ldpc_graph &g) { return 4ull * (2ull * g.n + 2ull * g.E); }
size_t bwd_lds(const ldpc_graph &g, int32_t K) {
    return 4ull * (4ull * g.n + 2ull * g.E + (size_t)K * g.E + (size_t)K * g.n);
}
// the backward needs the larger state; both kernels use LDS or both global
bool train_onchip(const ldpc_graph &g, int32_t K) { return bwd_lds(g, K) + 1024 <= (size_t)g.lds_max; }

TrainWs carve_train(const ldpc_graph &g, int32_t B, int32_t T, int32_t K, void *base, size_t *total) {
    const int32_t nck = (T + K - 1) / K;
    const int32_t ncls = (int32_t)g.class_degrees.size();
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    const size_t o_ck = take((size_t)B * nck * ((size_t)g.n + (size_t)g.E) * 4);
    const size_t o_lp = take((size_t)B * 4);
    const size_t o_gp = take((size_t)B * 2 * T * ncls * 4);
    const size_t o_sc = take(train_onchip(g, K) ? 0 : (size_t)B * bwd_lds(g, K));
    if (total) *total = off;
    TrainWs w{};
    if (base) {
        char *b = (char *)base;
        w.ckpt = (float *)(b + o_ck);
        w.loss_part = (float *)(b + o_lp);
        w.gpart = (float *)(b + o_gp);
        w.scratch = (float *)(b + o_sc);
    }
    return w;
}

int train_check(const ldpc_graph *g, const float *llr, int32_t B, int32_t T, int32_t K, const float *alpha,
                const float *beta) {
    if (!g || !llr || !alpha || !beta || B < 1 || T < 1 || K < 1) return LDPC_EINVAL;
    if ((int)g->class_degrees.size() > kMaxClasses) return LDPC_EUNSUPPORTED;
    return LDPC_OK;
}

} // namespace
} // namespace ldpc

using namespace ldpc;

extern "C" size_t ldpc_nms_train_workspace_bytes(const ldpc_graph *g, int32_t B, int32_t T, int32_t ckpt_every) {
    if (!g || B < 1 || T < 1 || ckpt_every < 1) return 0;
    size_t total = 0;
    carve_train(*g, B, T, ckpt_every, nullptr, &total);
    return total;
}

extern "C" int ldpc_nms_train_forward(const ldpc_graph *g, const float *llr_dev, const uint8_t *target_dev, int32_t B,
                                      int32_t T, const float *alpha_dev, const float *beta_dev, int32_t ckpt_every,
                                      float *loss_dev, float *post_dev, void *ws_dev, size_t ws_bytes,
                                      hipStream_t stream) {
    int st = train_check(g, llr_dev, B, T, ckpt_every, alpha_dev, beta_dev);
    if (st) return st;
    if (!loss_dev) return LDPC_EINVAL;
    size_t need = 0;
    TrainWs w = carve_train(*g, B, T, ckpt_every, ws_dev, &need);
    if (!ws_dev || ws_bytes < need) return LDPC_EWORKSPACE;
    const bool on = train_onchip(*g, ckpt_every);
    const size_t lds = on ? fwd_lds(*g) : 0;
    auto fn = on ? &k_nms_fwd<true> : &k_nms_fwd<false>;
    if (on && hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
                  hipSuccess)
        return LDPC_EHIP;
    fn<<<B, kThreads, lds, stream>>>(g->row_ptr, g->col_idx, g->col_ptr, g->csc_edge, g->row_class, g->m, g->n,
                                     (int32_t)g->E, (int32_t)g->class_degrees.size(), llr_dev, target_dev, T,
                                     ckpt_every, alpha_dev, beta_dev, w.ckpt, w.loss_part, post_dev, w.scratch);
    k_sum_frames<<<1, kThreads, 0, stream>>>(w.loss_part, B, 1, 0, 1.0f / ((float)B * (float)g->n), loss_dev);
    return hipGetLastError() == hipSuccess ? LDPC_OK : LDPC_EHIP;
}

extern "C" int ldpc_nms_train_backward(const ldpc_graph *g, const float *llr_dev, const uint8_t *target_dev, int32_t B,
                                       int32_t T, const float *alpha_dev, const float *beta_dev, int32_t ckpt_every,
                                       float grad_loss, float *galpha_dev, float *gbeta_dev, float *gllr_dev,
                                       void *ws_dev, size_t ws_bytes, hipStream_t stream) {
    int st = train_check(g, llr_dev, B, T, ckpt_every, alpha_dev, beta_dev);
    if (st) return st;
    if (!galpha_dev || !gbeta_dev) return LDPC_EINVAL;
    size_t need = 0;
    TrainWs w = carve_train(*g, B, T, ckpt_every, ws_dev, &need);
    if (!ws_dev || ws_bytes < need) return LDPC_EWORKSPACE;
    const bool on = train_onchip(*g, ckpt_every);
    const size_t lds = on ? bwd_lds(*g, ckpt_every) : 0;
    auto fn = on ? &k_nms_bwd<true> : &k_nms_bwd<false>;
    if (on && hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
                  hipSuccess)
        return LDPC_EHIP;
    const int32_t ncls = (int32_t)g->class_degrees.size();
    const float scale = grad_loss / ((float)B * (float)g->n);
    fn<<<B, kThreads, lds, stream>>>(g->row_ptr, g->col_idx, g->col_ptr, g->csc_edge, g->row_class, g->m, g->n,
                                     (int32_t)g->E, ncls, llr_dev, target_dev, T, ckpt_every, alpha_dev, beta_dev,
                                     w.ckpt, scale, w.gpart, gllr_dev, w.scratch);
    const int32_t width = T * ncls;
    k_sum_frames<<<width, kThreads, 0, stream>>>(w.gpart, B, 2 * width, 0, 1.0f, galpha_dev);
    k_sum_frames<<<width, kThreads, 0, stream>>>(w.gpart, B, 2 * width, width, 1.0f, gbeta_dev);
    return hipGetLastError() == hipSuccess ? LDPC_OK : LDPC_EHIP;
}

extern "C" int ldpc_awgn_llr(const uint8_t *cw_dev, int32_t B, int32_t n, float rate, float ebn0_lo_db,
                             float ebn0_hi_db, uint64_t seed, float *llr_dev, float *ebn0_dev, hipStream_t stream) {
    if (B < 0 || n < 1 || !(rate > 0.0f) || !(ebn0_hi_db >= ebn0_lo_db) || (B > 0 && !llr_dev)) return LDPC_EINVAL;
    if (B == 0) return LDPC_OK;
    const dim3 grid((unsigned)((n + 4 * 256 - 1) / (4 * 256)), (unsigned)(B < 65535 ? B : 65535));
    k_awgn<<<grid, 256, 0, stream>>>(cw_dev, B, n, rate, ebn0_lo_db, ebn0_hi_db, (uint32_t)seed,
                                     (uint32_t)(seed >> 32), llr_dev, ebn0_dev);
    return hipGetLastError() == hipSuccess ? LDPC_OK : LDPC_EHIP;
}

extern "C" int ldpc_adam_step(float *param_dev, const float *grad_dev, float *m1_dev, float *m2_dev, int32_t count,
                              float lr, float beta1, float beta2, float eps, int32_t step, hipStream_t stream) {
    if (!param_dev || !grad_dev || !m1_dev || !m2_dev || count < 0 || step < 1) return LDPC_EINVAL;
    if (count == 0) return LDPC_OK;
    k_adam<<<(count + 255) / 256, 256, 0, stream>>>(param_dev, grad_dev, m1_dev, m2_dev, count, lr, beta1, beta2, eps,
                                                    step);
    return hipGetLastError() == hipSuccess ? LDPC_OK : LDPC_EHIP;
}
