// On-chip Min-Sum decoder, host side: variant choice, launch geometry, the
// single-graph and multi-graph launches.  The kernels are in onchip_kernel.h
// (one instantiation per source file and register budget).
#include <algorithm>
#include <mutex>
#include <new>

#include "onchip_kernel.h"

namespace ldpc {
namespace {
using namespace onchip;

// The widest masked variant is left out of the multi-code kernel: the
// register demand of a kernel is that of its largest variant, and that one
// alone would push every variant of the launch into spills.  Jobs that need
// it get a launch of their own.  So is the bank-conflict-free layout: its
// tables are built for the graph's own thread count, and the shared launch
// runs the largest thread count of its jobs.
constexpr int kWideVariant = 6;
constexpr bool shared_launch_ok(int v) { return v != kWideVariant && kVariants[v].cf == 0 && v < 16; }
static_assert(kNumVariants == 42, "k_onchip_multi dispatches variants 0-5 and 7-13");

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

// [register budget][learned][variant]; register budgets: the compiler's, at
// least 4 and at least 3 waves per SIMD
const KernelFn (*const kKernels[3])[kNumVariants] = {kKernelsW0, kKernelsW4, kKernelsW3};
// Index of a register budget (waves per SIMD: 0, 4 or 3) in kKernels.
inline int budget_index(int waves_per_simd) { return waves_per_simd == 4 ? 1 : waves_per_simd == 3 ? 2 : 0; }
inline int tuned_budget(const ldpc_graph &g) { return g.tuning.set ? budget_index(g.tuning.waves_per_simd) : 0; }

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
    // (a padded layout variant, cf & 4, takes columns of any degree up to its dv)
    const bool cols_ok = (v.cx && !(v.cf & 4)) ? (g.dv_min == v.dv && g.dv_max == v.dv) : g.dv_max <= v.dv;
    // the layout's tables are for their own geometry, stride and thread count
    const bool cf_ok = v.cf == 0 || (g.cf.edge != nullptr && g.cf.rpt == v.rpt && g.cf.cpt == v.cpt &&
                                     g.cf.dvs == v.dv && g.cf.dvp == v.dvp && threads_for(g, v) == g.cf.nt);
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
constexpr int kPickOrder[] = {15, 14, 33, 32, 35, 34, 37, 36, 39, 38, 41, 40, 22, 23, 24, 25, 26, 27, 28, 29, 30,
                              31, 0,  7,  10, 1,  11, 2,  12, 3,  13, 4,  5,  6,  8,  9,  16, 17, 18, 19, 20, 21};
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

// Side streams of the multi-code decoder, one set per device, created on
// first use (default priority, non-blocking) and kept until the process
// ends; `mu` serialises the calls that fork onto them.
constexpr int kSideStreams = 3;
struct SideStreams {
    hipStream_t s[kSideStreams];
    hipEvent_t fork, join[kSideStreams];
    std::mutex mu;
};
SideStreams *side_streams() {
    constexpr int kMaxDevices = 64;
    static SideStreams *sets[kMaxDevices] = {};
    static bool failed[kMaxDevices] = {};
    static std::mutex make;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(make);
    if (!sets[dev] && !failed[dev]) {
        failed[dev] = true; // until the set is complete
        SideStreams *x = new (std::nothrow) SideStreams();
        if (!x) return nullptr;
        bool ok = hipEventCreateWithFlags(&x->fork, hipEventDisableTiming) == hipSuccess;
        for (int k = 0; k < kSideStreams && ok; ++k)
            ok = hipStreamCreateWithFlags(&x->s[k], hipStreamNonBlocking) == hipSuccess &&
                 hipEventCreateWithFlags(&x->join[k], hipEventDisableTiming) == hipSuccess;
        if (!ok) return nullptr; // (a partial set is left to the process end; every call runs on `stream`)
        sets[dev] = x;
        failed[dev] = false;
    }
    return sets[dev];
}

} // namespace

bool onchip_cf_geometry(const ldpc_graph &g, const std::vector<int32_t> &col_deg, int32_t *rpt, int32_t *cpt,
                        int32_t *dvs, uint32_t *dvp) {
    // Among the layout variants for the graph's row degree whose stride (or
    // degree profile) holds its columns: the least lane work issued per round
    // (threads round up to whole wavefronts; a check edge weighs about four
    // bit-side adds, and a bit slot index reads its profile entry's messages),
    // then the exact stride, then more threads (more wavefronts to hide LDS
    // latency when LDS limits the workgroups per CU).
    std::vector<int32_t> sorted(col_deg);
    std::sort(sorted.begin(), sorted.end());
    int best = -1;
    int64_t best_cost = 0;
    for (int k = 0; k < kNumVariants; ++k) {
        const Variant &v = kVariants[k];
        if (v.cf == 0 || g.dc_min != g.dc_max || g.dc_max != v.dc || g.dv_max > v.dv) continue;
        if (!(v.cf & 4) && (g.dv_min != v.dv || g.dv_max != v.dv)) continue; // exact columns only
        const int t = threads_for(g, v);
        if (t > kMaxThreads) continue;
        int64_t reads = (int64_t)v.cpt * v.dv;
        if (v.dvp != 0u) { // bits in ascending degree: slot index c holds sorted[c t .. c t + t)
            bool holds = true;
            for (size_t p = 0; p < sorted.size() && holds; ++p)
                holds = (int32_t)((v.dvp >> (4 * (p / t))) & 15u) >= sorted[p];
            if (!holds) continue;
            reads = 0;
            for (int c = 0; c < v.cpt; ++c) reads += (v.dvp >> (4 * c)) & 15u;
        }
        const int64_t cost = (int64_t)t * (4 * v.rpt * v.dc + reads);
        const Variant *b = best >= 0 ? &kVariants[best] : nullptr;
        if (best < 0 || cost < best_cost ||
            (cost == best_cost && (v.dv < b->dv || (v.dv == b->dv && t > threads_for(g, *b))))) {
            best = k;
            best_cost = cost;
        }
    }
    if (best < 0) return false;
    *rpt = kVariants[best].rpt;
    *cpt = kVariants[best].cpt;
    *dvs = kVariants[best].dv;
    *dvp = kVariants[best].dvp;
    return true;
}

bool onchip_fits(const ldpc_graph &g) { return g.edge_tab != nullptr && pick(g) >= 0; }

bool onchip_variant_fits(const ldpc_graph &g, int variant) { return variant_ok(g, variant); }

int onchip_num_variants() { return kNumVariants; }

bool onchip_kernel_spill_free(int variant, int waves_per_simd) { return onchip_kernel_spill_bytes(variant, waves_per_simd) == 0; }

int64_t onchip_kernel_spill_bytes(int variant, int waves_per_simd) {
    if (variant < 0 || variant >= kNumVariants) return -1;
    hipFuncAttributes a{};
    if (hipFuncGetAttributes(&a, (const void *)kKernels[budget_index(waves_per_simd)][0][variant]) != hipSuccess)
        return -1;
    return (int64_t)a.localSizeBytes;
}

int onchip_kernel_vgprs(int variant, int waves_per_simd) {
    if (variant < 0 || variant >= kNumVariants) return -1;
    hipFuncAttributes a{};
    if (hipFuncGetAttributes(&a, (const void *)kKernels[budget_index(waves_per_simd)][0][variant]) != hipSuccess)
        return -1;
    return a.numRegs;
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
    const KernelFn fn = kKernels[tuned_budget(g)][alpha != nullptr ? 1 : 0][v];
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
        const KernelFn fn = kKernels[tuned_budget(g)][0][v_own];
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
    struct Launch {
        KernelFn fn;
        int grid, threads;
        size_t lds;
        JobTable jt;
    };
    std::vector<Launch> launches;
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
        launches.push_back(Launch{own[a].fn, grid, t, l, ot});
    }
    if (frames > 0) {
        int grid = 0;
        const int st = launch_grid((const void *)k_onchip_multi, threads, lds, num_cu, frames, 0, &grid);
        if (st) return st;
        launches.push_back(Launch{k_onchip_multi, grid, threads, lds, jt});
    }
    // Several launches run side by side: all but the first go round-robin to
    // the library's side streams of the device, which wait for everything
    // enqueued on `stream` so far and which `stream` waits for at the end.
    // Each launch's last frames (and the shared launch of small jobs) then
    // overlap the others instead of leaving CUs idle.
    SideStreams *side = launches.size() > 1 ? side_streams() : nullptr;
    std::unique_lock<std::mutex> hold;
    if (side) {
        hold = std::unique_lock<std::mutex>(side->mu);
        LDPC_HIP_TRY(hipEventRecord(side->fork, stream));
        for (int k = 0; k < kSideStreams; ++k) LDPC_HIP_TRY(hipStreamWaitEvent(side->s[k], side->fork, 0));
    }
    for (size_t k = 0; k < launches.size(); ++k) {
        const Launch &x = launches[k];
        const hipStream_t on = (side && k % (kSideStreams + 1) != 0) ? side->s[k % (kSideStreams + 1) - 1] : stream;
        timed_launch(K_ONCHIP, x.fn, x.grid, x.threads, x.lds, on, x.jt, L, early);
    }
    if (side) {
        for (int k = 0; k < kSideStreams; ++k) {
            LDPC_HIP_TRY(hipEventRecord(side->join[k], side->s[k]));
            LDPC_HIP_TRY(hipStreamWaitEvent(stream, side->join[k], 0));
        }
    }
    return hipGetLastError() == hipSuccess ? LDPC_OK : LDPC_EHIP;
}

} // namespace ldpc
