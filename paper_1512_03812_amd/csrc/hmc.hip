// Host runtime and C ABI of the Schwinger-model HMC library: context and workspace,
// CG drivers (FP64 and mixed precision), force evaluation, the integrators of Sec. 2.2
// and the HMC update of Sec. 2.1.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <exception>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/schwinger_hmc.h"
#include "kernels.hpp"

using namespace shmc;

namespace {

constexpr int kNumXcd = 8;        // XCDs of an MI355X; workgroups are dealt to them round robin
constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Names of the real-link and spinor buffers carved out of the workspace.
enum LinkBuf { LQ, LP, LQ0, LP0, LQS, LF, LFF, LFT, LG, kNumLinkBufs };
enum SpinBuf { SPHI, SZETA, SXI, SCHI, SR, SPA, SPB, ST, SW, SY, SZ, SR2, SS2, kNumSpinBufs };
enum Spin32Buf { FX, FR, FT, FPA, FPB, FR2, FS2, kNumSpin32Bufs };

}  // namespace

// Sampled event timing of the two CG step kernels (kernel index 0: step 1, 1: step 2).
// In every sample_every-th iteration slot each kernel is launched with a start and an end
// event that its own dispatch stamps (no marker packets, so the durations are the kernels'
// own).  Step 1 of that slot writes, for each chain it iterates, the algorithmic bytes of
// both steps (the chain's sites times the bytes per site of the slot's mode) into a device
// row; at the end of the solve one reduction sums the rows and a single copy brings the
// sums to the host, so the bytes of exactly those launches are attributed to the measured
// durations with no copy inside the iteration loop.
struct TimedSlot {
    hipEvent_t ev[4];  // step 1 start, end; step 2 start, end
    int sample;        // row of the device byte table
    bool two;          // step 2 was launched (not the fused iteration)
};

struct KernelTimer {
    bool on = false;
    int sample_every = 32;
    std::vector<hipEvent_t> pool;
    size_t pool_used = 0;
    std::vector<TimedSlot> pending;
    double *sums_host = nullptr;  // pinned: [kMaxSamples + 1][2] byte sums of the pending samples
                                  // and (last row) of every slot since the last flush
    double ms[2] = {0.0, 0.0};
    double bytes[2] = {0.0, 0.0};
    double all_bytes[2] = {0.0, 0.0};  // algorithmic bytes of every slot launched while on
    long long timed[2] = {0, 0};
    long long launches = 0;  // all slots launched while timing was on
    int since_sync = 0;      // slots launched since the host last waited for the stream
    bool fused = false;      // the sampled slots ran the fused iteration (index 0 holds it)
};

// Contexts hmc_trajectories_concurrent advances at once (one host thread each).
constexpr int kMaxConcurrent = 8;

// Chain groups of one context (hmc_set_cg_groups).
constexpr int kMaxGroups = 4;

// Solves whose results a captured trajectory can log on the device.
constexpr int kMaxLoggedSolves = 1024;

// A trajectory captured as one HIP graph, with the host-side counts of its schedule.
struct GraphEntry {
    int scheme, n_outer, n_inner, prec, fg_mode;
    double tau;
    long epoch;  // settings generation it was captured under
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int solves = 0, force_evals = 0, hvp_solves = 0, logged = 0;
};

// A captured chunk of CG iteration slots (graph mode with chains above the persistent
// solver's limit): `slots` slots of both step kernels over the active workgroup list, whose
// length the kernels read from the device, then the compaction that shortens the list.  The
// slots only select state and direction buffers by their parity, so one chunk (an even number
// of slots) serves every chunk of every solve with the same fields and settings.
struct ChunkGraph {
    long epoch;
    const void *phi, *x;
    int mixed, slots, nblocks, block, variant, max_iter, vmax;
    double tol, delta;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

struct hmc_ctx {
    // ------------------------------------------------------------ geometry (host)
    int nchains = 0;
    int step_variant = kStepPlain;  // CG step-kernel variant (sites per thread of the tables)
    int Vtot = 0;            // sites of the flat site space (field planes are Vtot apart)
    int site0 = 0;           // the chains' contiguous site range [site0, site0 + nsites)
    int nsites = 0;          // (a chain group's context covers part of its parent's space)
    int block = 256;
    int nlog_max = 0;  // workgroups of the table at the smallest workgroup size
    bool has_large = false;  // some chain has more than kMaxChainBlocks workgroups
    std::vector<ChainInfo> chains;
    std::vector<BlockWork> work;
    uint64_t seed = 0;
    uint32_t traj = 0;
    // ------------------------------------------------------------ solver settings
    double tol = 1e-12;
    int max_iter = 100000;
    double delta = 1e-4;
    int check_every = 32;
    bool quenched = false;
    int fg_mode = HMC_FG_SHIFT;
    // ------------------------------------------------------------ captured trajectories
    bool graph_on = false;
    long graph_epoch = 0;          // bumped by every setting a captured graph bakes in
    std::vector<GraphEntry> graphs;
    std::vector<ChunkGraph> chunks;  // captured CG iteration chunks
    bool deferring = false;        // capturing: solves log their results on the device
    int log_count = 0;             // solves logged by the trajectory being captured
    bool log_overflow = false;
    int persist_vmax = 2048;  // chains with at most this many sites use the persistent solver
    bool fused_on = false;    // one kernel per CG iteration where every chain allows it
    // ------------------------------------------------------------ workspace
    size_t ws_bytes = 0;
    char *ws = nullptr;
    hipStream_t stream = nullptr;
    size_t off_chains = 0, off_work = 0, off_active = 0, off_big = 0, off_small = 0, off_cg = 0,
           off_partials = 0, off_samples = 0, off_sample_sums = 0, off_trajc = 0, off_log = 0,
           off_sums = 0, off_fin = 0, off_metro = 0, off_status = 0, off_count = 0, off_links[kNumLinkBufs] = {},
           off_spin[kNumSpinBufs] = {}, off_U64 = 0, off_A32 = 0, off_spin32[kNumSpin32Bufs] = {},
           off_Uw = 0;
    // ------------------------------------------------------------ solver partition
    hipStream_t side = nullptr;           // second stream for the persistent solver
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;
    int device = 0;                       // the device current at hmc_bind
    // Chain groups (hmc_set_cg_groups): contiguous ranges of the chains, each advanced through
    // a trajectory as a context of its own (grp[g]: its own tables, stream and host thread;
    // the fields are this context's), so that one group's kernels run while another's host
    // waits at a convergence check or its solve drains.
    int groups = 1;
    int grp_n = 0;                        // groups built (0: none)
    int grp_first[kMaxGroups + 1] = {};   // chain ranges [grp_first[g], grp_first[g + 1])
    hmc_ctx *grp[kMaxGroups] = {};
    hipEvent_t grp_fork = nullptr, grp_join[kMaxGroups] = {};
    // The groups' streams beyond the bound one, created once and kept for the context's life
    // (re-creating streams re-deals the process's few hardware queues).
    hipStream_t grp_stream[kMaxGroups] = {};
    bool is_group = false;                // a group of another context (owns no workspace)
    size_t off_groups = 0, groups_bytes = 0;  // the workspace area of the groups' tables
    int part_vmax = -1;                   // vmax the device partition tables were built for
    int n_big_blocks = 0, n_small = 0, small_vmax = 0;
    // the persistent-solver chains in size classes (at most 1024 and 2048 sites: one and two
    // sites per thread), each launched with its own workgroup size and LDS: class k holds
    // n_cls[k] chains from entry cls_first[k] of the small-chain list, the largest with
    // vmax_cls[k] sites
    int n_cls[2] = {}, cls_first[2] = {}, vmax_cls[2] = {};
    size_t lds_max = 64 * 1024;           // dynamic LDS a workgroup may opt in to
    // ------------------------------------------------------------ pinned host staging
    void *pinned = nullptr;
    size_t pinned_bytes = 0;
    // ------------------------------------------------------------ state tracking
    long q_version = 0;      // bumped whenever Q changes inside the library
    long links_version = -1; // q version the materialised FP64 links belong to (-1: none / other q)
    long links32_version = -1; // same for the FP32 copy
    long ff_version = -1;    // q version of the cached fermion force LFF (-1: none)
    long xi_version = -1;    // q version of the solution in SXI (-1: none / shifted links)
    long chi_version = -1;   // q version of chi = D xi in SCHI
    std::string err;
    // per-solve bookkeeping of the last CG (host copies)
    std::vector<CGState> cg_host;
    std::vector<double> resid_host;  // true residual norms of the last allocation-free solve
    void *static_scratch = nullptr;  // this device's address of the static scratch array
    std::string static_scratch_err;
    KernelTimer timer;

    // ------------------------------------------------------------ accessors
    template <typename T> T *at(size_t off) const { return reinterpret_cast<T *>(ws + off); }
    double *link(int b) const { return at<double>(off_links[b]); }
    double2 *spin(int b) const { return at<double2>(off_spin[b]); }
    float4 *spin32(int b) const { return at<float4>(off_spin32[b]); }
    double2 *U64() const { return at<double2>(off_U64); }
    double2 *Uw() const { return at<double2>(off_Uw); }
    float *A32() const { return at<float>(off_A32); }
    CGState *cg() const { return at<CGState>(off_cg); }
    double *sums() const { return at<double>(off_sums); }
    Geo geo() const {
        Geo g;
        g.chains = at<ChainInfo>(off_chains);
        g.work = at<BlockWork>(off_work);
        g.nblocks = (int)work.size();
        g.nlog = (int)work.size();
        g.nchains = nchains;
        g.Vtot = Vtot;
        g.block = block;
        g.site0 = site0;
        g.nsites = nsites;
        return g;
    }
    double *partials() const { return at<double>(off_partials); }
};

namespace {

int fail(hmc_ctx *c, int code, const char *fmt, ...) {
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return code;
}

#define HIP_TRY(ctx, expr)                                                                      \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return fail(ctx, HMC_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));         \
    } while (0)

#define CHECK_BOUND(ctx)                                                                        \
    do {                                                                                        \
        if (!(ctx)) return HMC_E_INVAL;                                                         \
        if (!(ctx)->ws) return fail(ctx, HMC_E_INVAL, "context has no workspace bound");        \
    } while (0)

// Block table: every chain gets ceil((V/2) / (block/2)) logical workgroups, one site per
// thread, each covering the same half-site range of both parity planes (chains contiguous in
// logical order).  Hardware workgroup h runs on XCD h % 8, and the
// j-th workgroup of XCD k receives logical workgroup start_k + j, so each XCD sweeps one
// contiguous site range and the workgroups resident on it at any time cover a few
// consecutive lattice rows: the t +- 1 stencil rows are L2 hits.
void build_tables(hmc_ctx *c) {
    std::vector<BlockWork> logical;
    c->has_large = false;
    for (int ch = 0; ch < c->nchains; ++ch) {
        ChainInfo &ci = c->chains[ch];
        const int spt = step_variant_spt(c->step_variant);
        ci.block0 = (int)logical.size();
        const int half = c->block / 2;
        ci.nblocks = (ci.Vh + half * spt - 1) / (half * spt);
        if (ci.nblocks > kMaxChainBlocks) c->has_large = true;
        for (int j = 0; j < ci.nblocks; ++j) {
            BlockWork w;
            w.chain = ch;
            w.start = j * half * spt;
            w.logical = (int)logical.size();
            w.spt = spt;
            logical.push_back(w);
        }
    }
    const int N = (int)logical.size();
    c->work.assign(N, BlockWork());
    std::vector<int> start(kNumXcd + 1, 0);
    for (int k = 0; k < kNumXcd; ++k) start[k + 1] = start[k] + N / kNumXcd + (k < N % kNumXcd ? 1 : 0);
    for (int h = 0; h < N; ++h) c->work[h] = logical[start[h % kNumXcd] + h / kNumXcd];
}

// Per-workgroup arrays are sized for the smallest workgroup the tuner may choose.
constexpr int kMinBlock = 128;

// The per-chain and per-workgroup tables of a context with C chains and N logical workgroups,
// carved from byte offset o of the workspace; returns the end.
size_t layout_tables(hmc_ctx *c, size_t o, size_t C, size_t N) {
    auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + bytes); return r; };
    c->off_chains = take(sizeof(ChainInfo) * C);
    c->off_work = take(sizeof(BlockWork) * N);
    c->off_active = take(sizeof(BlockWork) * N);
    c->off_big = take(sizeof(BlockWork) * N);
    c->off_small = take(sizeof(int) * C);
    c->off_cg = take(sizeof(CGState) * 2 * C);
    c->off_partials = take(sizeof(double) * kMaxReduce * N);
    c->off_samples = take(sizeof(double) * 2 * (kMaxSamples + 1) * C);
    c->off_trajc = take(sizeof(uint32_t));
    c->off_log = take(sizeof(int) * 2 * kMaxLoggedSolves * C);
    c->off_sample_sums = take(sizeof(double) * 2 * (kMaxSamples + 1));
    c->off_sums = take(sizeof(double) * 16 * C);
    c->off_fin = take(sizeof(double) * 2 * kFinSlices * C);
    c->off_metro = take(sizeof(MetroOut) * C);
    c->off_status = take(sizeof(int) * C);
    c->off_count = take(sizeof(int) * 4);
    return o;
}

// Bytes of layout_tables beyond its proportional part: each of its 16 tables rounds up to
// 256 bytes, and the sample sums, counter and counts do not scale with C or N.
constexpr size_t kTablesFixed = 16 * kAlign + sizeof(double) * 2 * kMaxSamples + 2 * kAlign;

void layout_workspace(hmc_ctx *c, size_t N) {
    const size_t C = c->nchains, V = c->Vtot;
    size_t o = layout_tables(c, 0, C, N);
    // the tables of up to kMaxGroups chain groups: they partition the chains and workgroups,
    // so together they take at most these tables' bytes plus the fixed part of each
    c->off_groups = o;
    c->groups_bytes = o + kMaxGroups * kTablesFixed;
    o = align_up(c->off_groups + c->groups_bytes);
    auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + bytes); return r; };
    for (int b = 0; b < kNumLinkBufs; ++b) c->off_links[b] = take(sizeof(double) * 2 * V);
    for (int b = 0; b < kNumSpinBufs; ++b) c->off_spin[b] = take(sizeof(double2) * 2 * V);
    c->off_U64 = take(sizeof(double2) * 2 * V);
    c->off_A32 = take(sizeof(float) * 2 * V);
    c->off_Uw = take(sizeof(double2) * 2 * V);
    for (int b = 0; b < kNumSpin32Bufs; ++b) c->off_spin32[b] = take(sizeof(float4) * V);
    c->ws_bytes = o;
}

int make_ctx(hmc_ctx **out, int n, const int *Lx, const int *Lt, const double *beta,
             const double *m0, uint64_t seed) {
    if (!out) return HMC_E_INVAL;
    *out = nullptr;
    if (n < 1 || !Lx || !Lt || !beta || !m0) return HMC_E_INVAL;
    long long vt = 0;
    for (int c = 0; c < n; ++c) {
        if (Lx[c] < 2 || Lt[c] < 2 || (Lx[c] & 1) || (Lt[c] & 1)) return HMC_E_INVAL;
        if (!isfinite(beta[c]) || !isfinite(m0[c])) return HMC_E_INVAL;
        vt += (long long)Lx[c] * Lt[c];
    }
    if (vt > (1LL << 30)) return HMC_E_INVAL;  // flat indices are 32-bit
    hmc_ctx *c = new hmc_ctx();
    c->nchains = n;
    c->seed = seed;
    c->chains.resize(n);
    int off = 0;
    for (int k = 0; k < n; ++k) {
        ChainInfo &ci = c->chains[k];
        memset(&ci, 0, sizeof ci);
        ci.off = off;
        ci.Lx = Lx[k];
        ci.Lt = Lt[k];
        ci.hx = Lx[k] / 2;
        ci.V = Lx[k] * Lt[k];
        ci.Vh = ci.V / 2;
        ci.beta = beta[k];
        ci.m0 = m0[k];
        ci.chain_id = (uint32_t)k;
        off += ci.V;
    }
    c->Vtot = off;
    c->nsites = off;
    c->block = kMinBlock;
    build_tables(c);
    c->nlog_max = (int)c->work.size();
    c->block = 256;
    build_tables(c);
    layout_workspace(c, (size_t)c->nlog_max);
    c->cg_host.resize(n);
    c->resid_host.resize(n);
    *out = c;
    return HMC_OK;
}

// ------------------------------------------------------------------ allocation-free solve
// Scratch of hmc_cg_solve_noalloc: one array in static device memory, of which every GPU
// that loads the library holds its own copy until the process ends.  Host code never uses
// the array's name as an address: each device's address is taken once, with that device
// current, by hipGetSymbolAddress (scratch_address, called from hmc_bind).  Layout for the
// largest context the entry point takes: FP64 links U [2][V] and the true-residual
// intermediate t [2][V] (double2), the CG states [2][C], the chain list [C], partial sums
// [P] and per-chain sums [C].
constexpr int kNoAllocMaxSites = 65536;    // V_total
constexpr int kNoAllocMaxChains = 1024;
constexpr int kNoAllocMaxPartials = 4096;  // logical workgroups of the context's table
constexpr size_t kNoAllocOffT = (size_t)2 * kNoAllocMaxSites * sizeof(double2);
constexpr size_t kNoAllocOffState = 2 * kNoAllocOffT;
constexpr size_t kNoAllocOffList =
    kNoAllocOffState + (size_t)2 * kNoAllocMaxChains * sizeof(CGState);
constexpr size_t kNoAllocOffPartials = kNoAllocOffList + (size_t)kNoAllocMaxChains * sizeof(int);
constexpr size_t kNoAllocOffSums =
    kNoAllocOffPartials + (size_t)kNoAllocMaxPartials * sizeof(double);
constexpr size_t kNoAllocBytes = kNoAllocOffSums + (size_t)kNoAllocMaxChains * sizeof(double);
static_assert(kNoAllocOffState % 256 == 0 && kNoAllocOffList % 256 == 0 &&
                  kNoAllocOffPartials % 256 == 0 && kNoAllocOffSums % 256 == 0,
              "scratch regions are 256-byte aligned");

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_addr[kMaxDevices] = {};

// The current device's address of `scratch` (the current device is the context's).
void scratch_address(hmc_ctx *c) {
    c->static_scratch = nullptr;
    if (c->device < 0 || c->device >= kMaxDevices) {
        c->static_scratch_err = "device index out of range";
        return;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[c->device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            c->static_scratch_err = std::string("hipGetSymbolAddress failed: ") + hipGetErrorString(e);
            return;
        }
        g_scratch_addr[c->device] = p;
    }
    c->static_scratch = g_scratch_addr[c->device];
}

// ------------------------------------------------------------------ helpers on a bound context
int sync(hmc_ctx *c) {
    c->timer.since_sync = 0;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return HMC_OK;
}

int to_host(hmc_ctx *c, void *dst, const void *src_dev, size_t bytes) {
    if (bytes > c->pinned_bytes) {
        HIP_TRY(c, hipMemcpyAsync(dst, src_dev, bytes, hipMemcpyDeviceToHost, c->stream));
        return sync(c);
    }
    HIP_TRY(c, hipMemcpyAsync(c->pinned, src_dev, bytes, hipMemcpyDeviceToHost, c->stream));
    int rc = sync(c);
    if (rc) return rc;
    memcpy(dst, c->pinned, bytes);
    return HMC_OK;
}

// dst = src on the context's sites of both planes of a real link field.
void copy_links(hmc_ctx *c, const double *src, double *dst) {
    if (c->site0 == 0 && c->nsites == c->Vtot) {
        launch_copy(src, dst, sizeof(double) * 2 * c->Vtot, c->stream);
        return;
    }
    (void)hipMemcpy2DAsync(dst + c->site0, sizeof(double) * c->Vtot, src + c->site0,
                           sizeof(double) * c->Vtot, sizeof(double) * c->nsites, 2,
                           hipMemcpyDeviceToDevice, c->stream);
}

// The library's second stream (persistent solver, graph capture), created on first use: an
// idle stream still takes one of the process's few hardware queues, which concurrent chain
// groups need.
int ensure_side(hmc_ctx *c) {
    if (c->side) return HMC_OK;
    HIP_TRY(c, hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
    HIP_TRY(c, hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming));
    HIP_TRY(c, hipEventCreateWithFlags(&c->join_ev, hipEventDisableTiming));
    return HMC_OK;
}

void ensure_links(hmc_ctx *c, const double *q, bool need32, long version) {
    // version >= 0 identifies q == LQ at that version; -1 forces a rebuild
    const bool have64 = version >= 0 && c->links_version == version;
    const bool have32 = version >= 0 && c->links32_version == version;
    if (have64 && (!need32 || have32)) return;
    launch_make_links(c->geo(), q, c->U64(), need32 ? c->A32() : nullptr, c->stream);
    c->links_version = version;
    c->links32_version = need32 ? version : -1;
}

void forget_links(hmc_ctx *c) { c->links_version = c->links32_version = -1; }

void forget_all(hmc_ctx *c) {
    c->q_version++;
    forget_links(c);
    c->ff_version = c->xi_version = c->chi_version = -1;
}

// Rebuilds the list of workgroups of the unconverged chains; returns its length in *active
// and the number of unconverged chains with iterations left in *live.
int check_convergence(hmc_ctx *c, const Geo &big, int max_iter, int *active, int *live) {
    int *dev = c->at<int>(c->off_count);
    launch_compact(big, c->cg(), max_iter, c->at<BlockWork>(c->off_active), dev, c->stream);
    int n[2] = {0, 0};
    int rc = to_host(c, n, dev, sizeof(n));
    if (rc) return rc;
    *active = n[0];
    *live = n[1];
    return HMC_OK;
}

hipEvent_t timer_event(hmc_ctx *c) {
    KernelTimer &T = c->timer;
    if (T.pool_used == T.pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        T.pool.push_back(e);
    }
    return T.pool[T.pool_used++];
}

// Sums the device byte rows of the pending samples into pinned memory (stream-ordered, no
// wait); the caller synchronises before timer_flush.
void timer_reduce(hmc_ctx *c) {
    KernelTimer &T = c->timer;
    const int n = (int)T.pending.size();
    double *sums = c->at<double>(c->off_sample_sums);
    double *rows = c->at<double>(c->off_samples);
    if (n > 0) launch_sample_sums(rows, n, c->nchains, sums, c->stream);
    launch_sample_sums(rows + (size_t)2 * kMaxSamples * c->nchains, 1, c->nchains, sums + 2 * kMaxSamples,
                       c->stream);
    (void)hipMemcpyAsync(T.sums_host, sums, sizeof(double) * 2 * n, hipMemcpyDeviceToHost, c->stream);
    (void)hipMemcpyAsync(T.sums_host + 2 * kMaxSamples, sums + 2 * kMaxSamples, sizeof(double) * 2,
                         hipMemcpyDeviceToHost, c->stream);
}

// Called only after the stream was synchronised (following timer_reduce): every recorded
// event and byte sum is complete.
void timer_flush(hmc_ctx *c) {
    KernelTimer &T = c->timer;
    T.all_bytes[0] += T.sums_host[2 * kMaxSamples];
    T.all_bytes[1] += T.sums_host[2 * kMaxSamples + 1];
    for (const TimedSlot &ts : T.pending) {
        float a = 0.f, b = 0.f;
        if (hipEventElapsedTime(&a, ts.ev[0], ts.ev[1]) != hipSuccess) continue;
        if (ts.two && hipEventElapsedTime(&b, ts.ev[2], ts.ev[3]) != hipSuccess) continue;
        T.ms[0] += a;
        T.bytes[0] += T.sums_host[2 * ts.sample];
        T.timed[0]++;
        if (ts.two) {
            T.ms[1] += b;
            T.bytes[1] += T.sums_host[2 * ts.sample + 1];
            T.timed[1]++;
        }
    }
    T.pending.clear();
    T.pool_used = 0;
}

// One CG slot (step 1 + step 2, or the fused iteration with no step 2); in a sampled slot
// each kernel gets its start and end events and step 1 records the bytes of both steps in
// the row given to it (-1: not sampled).
template <typename L1, typename L2>
void slot_launch(hmc_ctx *c, int slot, L1 step1, L2 step2, bool two = true) {
    KernelTimer &T = c->timer;
    if (T.on) T.launches++;
    // Sampled slots sit mid-way between the convergence checks, a few slots after the host
    // last waited: the stream then already holds the launches ahead, and the events measure
    // the kernels rather than the host's latency in enqueuing them after a wait.
    const int since = T.since_sync++;
    if (!T.on || slot % T.sample_every != T.sample_every / 2 || since < 2 ||
        (int)T.pending.size() == kMaxSamples || !T.sums_host) {
        step1(-1, nullptr, nullptr);
        if (two) step2(nullptr, nullptr);
        return;
    }
    TimedSlot ts;
    for (int k = 0; k < 4; ++k) ts.ev[k] = timer_event(c);
    ts.sample = (int)T.pending.size();
    ts.two = two;
    step1(ts.sample, ts.ev[0], ts.ev[1]);
    if (two) step2(ts.ev[2], ts.ev[3]);
    T.pending.push_back(ts);
}

// Splits the chains between the persistent one-workgroup solver (V <= vmax) and the
// multi-workgroup slot kernels, and uploads the workgroup list of the latter and the chain
// list of the former.
// Size class of a persistent-solver chain: one or two sites per thread of its workgroup.
static int size_class(int V) { return V <= 1024 ? 0 : 1; }

int build_partition(hmc_ctx *c, int vmax) {
    if (c->part_vmax == vmax) return HMC_OK;
    std::vector<BlockWork> big;
    std::vector<int> small;
    int svmax = 0, rc = HMC_OK;
    for (int cls = 0; cls < 2; ++cls) {
        c->cls_first[cls] = (int)small.size();
        c->vmax_cls[cls] = 0;
        for (int k = 0; k < c->nchains; ++k) {
            const int V = c->chains[k].V;
            if (V <= vmax && size_class(V) == cls) {
                small.push_back(k);
                c->vmax_cls[cls] = std::max(c->vmax_cls[cls], V);
                svmax = std::max(svmax, V);
            }
        }
        c->n_cls[cls] = (int)small.size() - c->cls_first[cls];
    }
    for (const BlockWork &w : c->work)
        if (c->chains[w.chain].V > vmax) big.push_back(w);
    if (!big.empty())
        HIP_TRY(c, hipMemcpyAsync(c->at<BlockWork>(c->off_big), big.data(), sizeof(BlockWork) * big.size(),
                                  hipMemcpyHostToDevice, c->stream));
    if (!small.empty())
        HIP_TRY(c, hipMemcpyAsync(c->at<int>(c->off_small), small.data(), sizeof(int) * small.size(),
                                  hipMemcpyHostToDevice, c->stream));
    if ((rc = sync(c))) return rc;
    c->n_big_blocks = (int)big.size();
    c->n_small = (int)small.size();
    c->small_vmax = svmax;
    c->part_vmax = vmax;
    return HMC_OK;
}

// Largest chain the persistent solver takes for a precision (LDS holds 4V complex; at most
// 2 sites per thread of a 1024-thread workgroup; the device's opt-in LDS limit, less the
// kernel's static LDS).
int persistent_limit(hmc_ctx *c, bool mixed) {
    int v = std::min(c->persist_vmax, 2048);
    while (v > 0 && cg_wg_lds_bytes(v, mixed) + 1024 > c->lds_max) v /= 2;
    return v;
}

// Raises the LDS grant of every size class of the persistent solver; nonzero if the device
// refuses one (then nothing has been launched).
static int prepare_small(hmc_ctx *c, bool mixed) {
    for (int cls = 0; cls < 2; ++cls)
        if (c->n_cls[cls] > 0 && prepare_cg_wg(c->vmax_cls[cls], mixed)) return -1;
    return 0;
}

// The persistent solver over every size class on stream s (after prepare_small).
static int launch_small(hmc_ctx *c, const Geo &g, const CGFields &f, bool mixed, double tol, int max_iter,
                        hipStream_t s) {
    for (int cls = 0; cls < 2; ++cls)
        if (c->n_cls[cls] > 0 &&
            launch_cg_wg(g, f, mixed, c->at<int>(c->off_small) + c->cls_first[cls], c->n_cls[cls],
                         c->vmax_cls[cls], tol, c->delta, max_iter, s))
            return -1;
    return 0;
}

// LDS bytes of the fused iteration over the chains above vmax at the current workgroup
// size, or 0 if one of them cannot use it (or the fused iteration is switched off).
size_t fused_lds(hmc_ctx *c, int vmax, bool mixed) {
    if (!c->fused_on || step_variant_spt(c->step_variant) != 1) return 0;
    int entries = 0;
    for (const ChainInfo &ci : c->chains) {
        if (ci.V <= vmax) continue;
        int e = 0;
        if (!cg_iter_eligible(ci, c->block, &e)) return 0;
        entries = std::max(entries, e);
    }
    const size_t lds = cg_iter_lds_bytes(entries, mixed);
    if (lds == 0 || lds + 1024 > c->lds_max || grant_cg_iter_lds(lds)) return 0;
    return lds;
}

// The captured iteration chunk for these fields and settings (recorded on first use on the
// library's second stream, so that the bound stream may be the default one).
int chunk_graph(hmc_ctx *c, const CGFields &f0, const Geo &big, void *const pb[2], bool mixed,
                int chunk, double tol, int max_iter, ChunkGraph **out) {
    for (ChunkGraph &e : c->chunks)
        if (e.epoch == c->graph_epoch && e.phi == f0.phi && e.x == f0.x64 && e.mixed == mixed &&
            e.slots == chunk && e.nblocks == big.nblocks && e.block == c->block &&
            e.variant == c->step_variant && e.max_iter == max_iter && e.vmax == c->part_vmax &&
            e.tol == tol && e.delta == c->delta) {
            *out = &e;
            return HMC_OK;
        }
    // graphs of older settings go
    for (ChunkGraph &e : c->chunks)
        if (e.epoch != c->graph_epoch) {
            if (e.exec) (void)hipGraphExecDestroy(e.exec);
            if (e.graph) (void)hipGraphDestroy(e.graph);
            e.exec = nullptr;
        }
    c->chunks.erase(std::remove_if(c->chunks.begin(), c->chunks.end(),
                                   [](const ChunkGraph &e) { return e.exec == nullptr; }),
                    c->chunks.end());
    int rc = ensure_side(c);
    if (rc) return rc;
    int *counts = c->at<int>(c->off_count);
    CGFields f = f0;
    f.active = counts;
    Geo g = big;
    g.work = c->at<BlockWork>(c->off_active);
    hipError_t e = hipStreamBeginCapture(c->side, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, HMC_E_HIP, "chunk capture could not start: %s", hipGetErrorString(e));
    }
    for (int k = 0; k < chunk; ++k) {
        launch_cg_step1(g, f, mixed, c->step_variant, k, tol, max_iter, pb[k & 1], pb[(k + 1) & 1], false,
                        -1, c->side);
        if (c->has_large) launch_finalize_large(big, f.p1, f.fin1, c->side);
        launch_cg_step2(g, f, mixed, c->step_variant, k, pb[(k + 1) & 1], c->side);
        if (c->has_large) launch_finalize_large(big, f.p2, f.fin2, c->side);
    }
    launch_compact(big, c->cg(), max_iter, c->at<BlockWork>(c->off_active), counts, c->side);
    ChunkGraph cg;
    e = hipStreamEndCapture(c->side, &cg.graph);
    if (e != hipSuccess || !cg.graph) {
        (void)hipGetLastError();
        return fail(c, HMC_E_HIP, "chunk capture failed: %s", hipGetErrorString(e));
    }
    if (hipGraphInstantiate(&cg.exec, cg.graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(cg.graph);
        (void)hipGetLastError();
        return fail(c, HMC_E_HIP, "chunk graph instantiation failed");
    }
    cg.epoch = c->graph_epoch;
    cg.phi = f0.phi;
    cg.x = f0.x64;
    cg.mixed = mixed;
    cg.slots = chunk;
    cg.nblocks = big.nblocks;
    cg.block = c->block;
    cg.variant = c->step_variant;
    cg.max_iter = max_iter;
    cg.vmax = c->part_vmax;
    cg.tol = tol;
    cg.delta = c->delta;
    c->chunks.push_back(cg);
    *out = &c->chunks.back();
    return HMC_OK;
}

// CG on D^dagger D x = phi with the links already materialised (U64, and the FP32 angles if mixed).
// Per-chain results land in c->cg_host.  Returns HMC_E_NAN if a chain's residual became
// non-finite, else HMC_E_NOCONV if a chain hit max_iter (the other chains are solved).
// Every check_every slots the host reads back how many workgroups still belong to
// unconverged chains and launches only those from then on.
int solve(hmc_ctx *c, const double2 *phi, double2 *x, double tol, int max_iter, int prec);
int solve(hmc_ctx *c, const double2 *phi, double2 *x, double tol, int max_iter, int prec) {
    const bool mixed = prec == HMC_PREC_MIXED;
    const Geo full = c->geo();
    Geo g = full;
    CGFields f = {};
    f.phi = phi;
    f.x64 = x;
    f.r64 = c->spin(SR);
    f.t64 = c->spin(ST);
    f.x32 = c->spin32(FX);
    f.r32 = c->spin32(FR);
    f.t32 = c->spin32(FT);
    f.U64 = c->U64();
    f.A32 = c->A32();
    f.p1 = c->partials();
    f.p2 = c->partials() + full.nlog;
    f.fin1 = c->at<double>(c->off_fin);
    f.fin2 = f.fin1 + (size_t)kFinSlices * c->nchains;
    f.st = c->cg();
    f.samples = c->at<double>(c->off_samples);
    if (c->timer.on && c->timer.sums_host)
        f.all_bytes = f.samples + (size_t)2 * kMaxSamples * c->nchains;
    void *pb[2];
    if (mixed) { pb[0] = c->spin32(FPA); pb[1] = c->spin32(FPB); }
    else { pb[0] = c->spin(SPA); pb[1] = c->spin(SPB); }
    int rc = build_partition(c, persistent_limit(c, mixed));
    if (rc) return rc;
    if (c->deferring) {
        // inside a captured trajectory: every chain is a persistent-solver chain; the solve
        // runs on the bound stream and logs its per-chain results on the device
        if (c->n_small != c->nchains || launch_small(c, full, f, mixed, tol, max_iter, c->stream))
            return fail(c, HMC_E_INVAL, "a captured trajectory needs every chain in the persistent solver");
        if (c->log_count < kMaxLoggedSolves)
            launch_log_solve(c->cg(), c->nchains, c->at<int>(c->off_log) + (size_t)2 * c->log_count * c->nchains,
                             c->stream);
        else
            c->log_overflow = true;
        c->log_count++;
        return HMC_OK;
    }
    // small chains: one persistent workgroup each, on the side stream
    if (c->n_small > 0) {
        if (prepare_small(c, mixed)) {
            // the device refused an LDS request: lower the limit below the largest class and
            // solve again (nothing has been launched)
            c->lds_max = cg_wg_lds_bytes(c->small_vmax, mixed) - 1;
            return solve(c, phi, x, tol, max_iter, prec);
        }
        if ((rc = ensure_side(c))) return rc;
        HIP_TRY(c, hipEventRecord(c->fork_ev, c->stream));
        HIP_TRY(c, hipStreamWaitEvent(c->side, c->fork_ev, 0));
        if (launch_small(c, full, f, mixed, tol, max_iter, c->side))
            return fail(c, HMC_E_HIP, "the persistent solver could not be launched");
        HIP_TRY(c, hipEventRecord(c->join_ev, c->side));
    }
    // large chains: multi-workgroup slot kernels on the bound stream
    Geo big = full;
    big.work = c->at<BlockWork>(c->off_big);
    big.nblocks = c->n_big_blocks;
    g = big;
    int slot = 0;
    const size_t lds_iter = big.nblocks > 0 ? fused_lds(c, c->part_vmax, mixed) : 0;
    c->timer.fused = lds_iter > 0;
    if (lds_iter > 0) {
        // one fused kernel per iteration: r, s, p double-buffered; partial rows [2][4]
        CGIterFields fi;
        fi.phi = phi;
        fi.x64 = x;
        fi.t64 = c->spin(ST);
        fi.x32 = c->spin32(FX);
        if (mixed) {
            fi.r[0] = c->spin32(FR); fi.r[1] = c->spin32(FR2);
            fi.s[0] = c->spin32(FT); fi.s[1] = c->spin32(FS2);
            fi.p[0] = c->spin32(FPA); fi.p[1] = c->spin32(FPB);
        } else {
            fi.r[0] = c->spin(SR); fi.r[1] = c->spin(SR2);
            fi.s[0] = c->spin(ST); fi.s[1] = c->spin(SS2);
            fi.p[0] = c->spin(SPA); fi.p[1] = c->spin(SPB);
        }
        fi.U64 = c->U64();
        fi.A32 = c->A32();
        fi.Q = c->partials();
        fi.st = c->cg();
        fi.samples = f.samples;
        CGFields fz = f;  // the initial kernel: r (buffer 0) = phi, x = 0, ||phi||^2 -> Q[1][1]
        if (mixed) fz.r32 = (float4 *)fi.r[0];
        else fz.r64 = (double2 *)fi.r[0];
        fz.p2 = fi.Q + (size_t)5 * full.nlog;
        launch_cg_init(big, fz, mixed, c->delta, c->stream);
        const int max_slots = mixed ? max_iter + max_iter / 2 + 64 : max_iter + 1;
        int interval = c->check_every, next_check = interval, last_active = big.nblocks;
        for (; slot < max_slots; ++slot) {
            slot_launch(c, slot,
                        [&](int sample, hipEvent_t e0, hipEvent_t e1) {
                            launch_cg_iter(g, fi, mixed, slot, tol, false, sample, lds_iter, c->stream,
                                           e0, e1);
                        },
                        [](hipEvent_t, hipEvent_t) {}, false);
            if (slot + 1 == next_check) {
                int active = 0, live = 0;
                if ((rc = check_convergence(c, big, max_iter, &active, &live))) return rc;
                if (active == 0 || live == 0) { ++slot; break; }
                g.work = c->at<BlockWork>(c->off_active);
                g.nblocks = active;
                interval = active == last_active ? std::min(2 * interval, 4 * c->check_every)
                                                 : c->check_every;
                last_active = active;
                next_check = slot + 1 + interval;
            }
        }
        // the last slot's residual decides the final state of every large chain
        launch_cg_iter(big, fi, mixed, slot, tol, true, -1, lds_iter, c->stream);
        if (mixed) launch_cg_finish_mixed(big, f, c->stream);
    } else if (big.nblocks > 0 && c->graph_on) {
        // captured chunks of iteration slots; the host reads the active count once per chunk
        BlockWork *act = c->at<BlockWork>(c->off_active);
        int *counts = c->at<int>(c->off_count);  // [active workgroups, live chains]
        const int chunk = std::max(2, (c->check_every + 1) / 2 * 2);
        ChunkGraph *cg = nullptr;
        if ((rc = chunk_graph(c, f, big, pb, mixed, chunk, tol, max_iter, &cg))) return rc;
        // the first chunk iterates the whole list
        launch_copy(big.work, act, sizeof(BlockWork) * big.nblocks, c->stream);
        launch_set_u32((uint32_t *)counts, (uint32_t)big.nblocks, c->stream);
        launch_cg_init(big, f, mixed, c->delta, c->stream);
        if (c->has_large) launch_finalize_large(big, f.p2, f.fin2, c->stream);
        const int max_slots = mixed ? max_iter + max_iter / 2 + 64 : max_iter;
        while (slot < max_slots) {
            HIP_TRY(c, hipGraphLaunch(cg->exec, c->stream));
            slot += chunk;
            int nh[2] = {0, 0};
            if ((rc = to_host(c, nh, counts, sizeof(nh)))) return rc;
            if (nh[0] == 0 || (mixed && nh[1] == 0)) break;
        }
        launch_cg_step1(big, f, mixed, c->step_variant, slot, tol, max_iter, pb[slot & 1],
                        pb[(slot + 1) & 1], true, -1, c->stream);
        if (mixed) launch_cg_finish_mixed(big, f, c->stream);
    } else if (big.nblocks > 0) {
        Geo gc = big;
        BlockWork *act = c->at<BlockWork>(c->off_active);
        int *counts = c->at<int>(c->off_count);  // [active workgroups, live chains]
        launch_cg_init(big, f, mixed, c->delta, c->stream);
        if (c->has_large) launch_finalize_large(big, f.p2, f.fin2, c->stream);
        // iteration slots: CG iterations plus, in mixed precision, FP64 residual recomputations
        const int max_slots = mixed ? max_iter + max_iter / 2 + 64 : max_iter;
        // Convergence checks: the first after check_every slots; the interval doubles (up to
        // 4x) while no chain converges and falls back when the active set shrinks.
        int interval = c->check_every, next_check = interval, last_active = big.nblocks;
        for (; slot < max_slots; ++slot) {
            void *po = pb[slot & 1], *pn = pb[(slot + 1) & 1];
            slot_launch(c, slot,
                        [&](int sample, hipEvent_t e0, hipEvent_t e1) {
                            launch_cg_step1(gc, f, mixed, c->step_variant, slot, tol, max_iter, po, pn,
                                            false, sample,
                                            c->stream, e0, e1);
                            if (c->has_large) launch_finalize_large(big, f.p1, f.fin1, c->stream);
                        },
                        [&](hipEvent_t e0, hipEvent_t e1) {
                            launch_cg_step2(gc, f, mixed, c->step_variant, slot, pn, c->stream, e0, e1);
                            if (c->has_large) launch_finalize_large(big, f.p2, f.fin2, c->stream);
                        });
            if (slot + 1 == next_check) {
                launch_compact(big, c->cg(), max_iter, act, counts, c->stream);
                int nh[2] = {0, 0};
                if ((rc = to_host(c, nh, counts, sizeof(nh)))) return rc;
                if (nh[0] == 0 || (mixed && nh[1] == 0)) { ++slot; break; }
                gc.work = act;
                gc.nblocks = nh[0];
                interval = nh[0] == last_active ? std::min(2 * interval, 4 * c->check_every)
                                                : c->check_every;
                last_active = nh[0];
                next_check = slot + 1 + interval;
            }
        }
        // fold the last slot's residual into the state (decision only), on every large chain
        launch_cg_step1(big, f, mixed, c->step_variant, slot, tol, max_iter, pb[slot & 1],
                        pb[(slot + 1) & 1], true, -1,
                        c->stream);
        if (mixed) launch_cg_finish_mixed(big, f, c->stream);
    }
    if (c->n_small > 0) HIP_TRY(c, hipStreamWaitEvent(c->stream, c->join_ev, 0));
    if (c->timer.on) timer_reduce(c);
    if ((rc = to_host(c, c->cg_host.data(), c->cg() + (size_t)(slot & 1) * c->nchains,
                      sizeof(CGState) * c->nchains))) return rc;
    if (c->timer.on) timer_flush(c);
    int nonfinite = 0, capped = 0;
    for (const CGState &s : c->cg_host) {
        nonfinite += s.converged == kStopNonFinite;
        capped += s.converged != kConverged && s.converged != kStopNonFinite;
    }
    if (nonfinite) return fail(c, HMC_E_NAN, "CG: the residual of %d chain(s) became non-finite", nonfinite);
    if (capped) return fail(c, HMC_E_NOCONV, "CG did not converge in %d iterations (%d chain(s))", max_iter, capped);
    return HMC_OK;
}

// A solve's failure that concerns single chains (they stopped unconverged; the others have
// their solutions): the caller goes on and reports it.
bool chain_failure(int rc) { return rc == HMC_E_NOCONV || rc == HMC_E_NAN; }

void fill_cg_info(hmc_ctx *c, hmc_cg_info *info, const std::vector<double> *true2) {
    if (!info) return;
    for (int k = 0; k < c->nchains; ++k) {
        const CGState &s = c->cg_host[k];
        info[k].iters = s.iters;
        info[k].converged = s.converged == kConverged;
        info[k].reliable_updates = s.n_updates;
        info[k].pad = 0;
        info[k].rel_resid = s.phi2 > 0 ? sqrt(s.rho / s.phi2) : 0.0;  // last decided residual
        info[k].rel_resid_true = (true2 && s.phi2 > 0) ? sqrt((*true2)[k] / s.phi2) : info[k].rel_resid;
    }
}

// ------------------------------------------------------------------ molecular dynamics
struct MD {
    hmc_ctx *c;
    int prec;
    double tol;
    int max_iter;
    int status = HMC_OK;
    std::vector<int> chain_status;
    std::vector<long long> iters;
    int force_evals = 0;
    int solves = 0;
    int hvp_solves = 0;  // Hessian-vector solves of exact force-gradient terms
};

// Books one solve's iterations and per-chain convergence; returns rc unless it only says that
// some chains stopped unconverged (HMC_E_NOCONV, HMC_E_NAN: recorded in md.status and per
// chain, the trajectory goes on and those chains are rejected).
int note_solve(MD &md, int rc) {
    hmc_ctx *c = md.c;
    md.solves++;
    if (c->deferring) return rc;  // iterations and convergence are read from the device log
    for (int k = 0; k < c->nchains; ++k) {
        md.iters[k] += c->cg_host[k].iters;
        const int code = c->cg_host[k].converged;
        if (code != kConverged && md.chain_status[k] == HMC_OK)
            md.chain_status[k] = code == kStopNonFinite ? HMC_E_NAN : HMC_E_NOCONV;
    }
    if (chain_failure(rc)) {
        if (md.status == HMC_OK) md.status = rc;
        return HMC_OK;
    }
    return rc;
}

// fermion force at links q (== LQ when version >= 0) into out; XI/CHI keep xi and chi.
int fermion_force_at(MD &md, const double *q, long version, double *out) {
    hmc_ctx *c = md.c;
    md.force_evals++;
    if (version >= 0 && c->ff_version == version) {
        if (out != c->link(LFF))
            copy_links(c, c->link(LFF), out);
        return HMC_OK;
    }
    ensure_links(c, q, md.prec == HMC_PREC_MIXED, version);
    int rc = note_solve(md, solve(c, c->spin(SPHI), c->spin(SXI), md.tol, md.max_iter, md.prec));
    if (rc) return rc;
    launch_dslash64(c->geo(), c->U64(), c->spin(SXI), c->spin(SCHI), false, c->stream);
    launch_fermion_force(c->geo(), c->U64(), c->spin(SCHI), c->spin(SXI), out, c->stream);
    c->xi_version = c->chi_version = version;
    if (version >= 0) {
        if (out != c->link(LFF))
            copy_links(c, out, c->link(LFF));
        c->ff_version = version;
    }
    return HMC_OK;
}

// which: 0 gauge, 1 fermion, 2 total (F_G + F_F, added in that order)
int force_at(MD &md, int which, const double *q, long version, double *out) {
    hmc_ctx *c = md.c;
    const Geo g = c->geo();
    if (which == 0 || c->quenched) {
        launch_gauge_force(g, q, nullptr, out, c->stream);
        if (which == 1) launch_axpy_links(g, out, -1.0, out, out, c->stream);  // quenched: F_F = 0
        return HMC_OK;
    }
    if (which == 1) return fermion_force_at(md, q, version, out);
    int rc = fermion_force_at(md, q, version, c->link(LFT));
    if (rc) return rc;
    launch_gauge_force(g, q, c->link(LFT), out, c->stream);
    return HMC_OK;
}

void stage_A(MD &md, double eps) {
    hmc_ctx *c = md.c;
    launch_axpy_links(c->geo(), c->link(LQ), eps, c->link(LP), c->link(LQ), c->stream);
    c->q_version++;
}

// e^{eps B}: p -= eps F.  Kicks with the gauge force (alone, or added to the fermion force)
// apply it in the kernel that computes it; the fermion-only kick goes through the F field.
int stage_B(MD &md, int which, double eps) {
    hmc_ctx *c = md.c;
    const Geo g = c->geo();
    if (which == 0 || (which == 2 && c->quenched)) {
        launch_gauge_kick(g, c->link(LQ), nullptr, -eps, c->link(LP), c->stream);
        return HMC_OK;
    }
    if (which == 2) {
        int rc = fermion_force_at(md, c->link(LQ), c->q_version, c->link(LFT));
        if (rc) return rc;
        launch_gauge_kick(g, c->link(LQ), c->link(LFT), -eps, c->link(LP), c->stream);
        return HMC_OK;
    }
    int rc = force_at(md, which, c->link(LQ), c->q_version, c->link(LF));
    if (rc) return rc;
    launch_axpy_links(g, c->link(LP), -eps, c->link(LF), c->link(LP), c->stream);
    return HMC_OK;
}

// force-gradient kick: p -= eps F(q - (h^2/24) F(q)); q is untouched.
int stage_B_fg_shift(MD &md, int which, double eps, double h) {
    hmc_ctx *c = md.c;
    const Geo g = c->geo();
    int rc = force_at(md, which, c->link(LQ), c->q_version, c->link(LF));
    if (rc) return rc;
    launch_axpy_links(g, c->link(LQ), -(h * h / 24.0), c->link(LF), c->link(LQS), c->stream);
    rc = force_at(md, which, c->link(LQS), -1, c->link(LG));
    if (rc) return rc;
    forget_links(c);
    launch_axpy_links(g, c->link(LP), -eps, c->link(LG), c->link(LP), c->stream);
    return HMC_OK;
}

// chi, xi (SCHI, SXI) at the current links LQ, solved for unless they are already there.
int ensure_chixi(MD &md) {
    hmc_ctx *c = md.c;
    if (c->xi_version == c->q_version && c->chi_version == c->q_version) return HMC_OK;
    ensure_links(c, c->link(LQ), md.prec == HMC_PREC_MIXED, c->q_version);
    int rc = note_solve(md, solve(c, c->spin(SPHI), c->spin(SXI), md.tol, md.max_iter, md.prec));
    if (rc) return rc;
    launch_dslash64(c->geo(), c->U64(), c->spin(SXI), c->spin(SCHI), false, c->stream);
    c->xi_version = c->chi_version = c->q_version;
    return HMC_OK;
}

// out = scale * H v at the links LQ for the force set `which` (0 gauge, 1 fermion, 2 total;
// Sec. 3, Eqs. (20)-(23)).  The fermion part needs chi and xi at LQ and one solve of
// D^dagger D:  W = dD[v] xi,  Z2 = (D^dagger D)^{-1} (D^dagger W + dD[v]^dagger chi),
// Z1 = D Z2 - W.  v must not be one of SW, SY, SZ.
int hessian_vector(MD &md, int which, const double *v, double scale, double *out) {
    hmc_ctx *c = md.c;
    const Geo g = c->geo();
    const bool gauge = which != HMC_FORCE_FERMION;
    const bool fermion = which != HMC_FORCE_GAUGE && !c->quenched;
    if (!fermion) {
        launch_hessian_vector(g, nullptr, v, nullptr, nullptr, nullptr, nullptr, c->link(LQ), gauge,
                              scale, out, c->stream);
        return HMC_OK;
    }
    int rc = ensure_chixi(md);
    if (rc) return rc;
    ensure_links(c, c->link(LQ), md.prec == HMC_PREC_MIXED, c->q_version);
    launch_weight_links(g, c->U64(), v, c->Uw(), c->stream);
    launch_stencil2(g, false, c->Uw(), c->spin(SXI), false, nullptr, nullptr, nullptr, c->spin(SW),
                    c->stream);
    launch_stencil2(g, true, c->U64(), c->spin(SW), true, c->Uw(), c->spin(SCHI), nullptr,
                    c->spin(SY), c->stream);
    md.hvp_solves++;
    rc = note_solve(md, solve(c, c->spin(SY), c->spin(SZ), md.tol, md.max_iter, md.prec));
    if (rc) return rc;
    launch_stencil2(g, false, c->U64(), c->spin(SZ), true, nullptr, nullptr, c->spin(SW), c->spin(SY),
                    c->stream);
    launch_hessian_vector(g, c->U64(), v, c->spin(SCHI), c->spin(SXI), c->spin(SY), c->spin(SZ),
                          c->link(LQ), gauge, scale, out, c->stream);
    return HMC_OK;
}

// force-gradient kick with the exact term of Eq. (5): p -= eps F(q) - (h^3/72) C(q) with
// C = 2 H F (Eq. (19)) for the same force set.
int stage_B_fg_exact(MD &md, int which, double eps, double h) {
    hmc_ctx *c = md.c;
    const Geo g = c->geo();
    int rc = force_at(md, which, c->link(LQ), c->q_version, c->link(LF));
    if (rc) return rc;
    rc = hessian_vector(md, which, c->link(LF), 2.0, c->link(LG));
    if (rc) return rc;
    launch_axpy_links(g, c->link(LP), -eps, c->link(LF), c->link(LP), c->stream);
    launch_axpy_links(g, c->link(LP), h * h * h / 72.0, c->link(LG), c->link(LP), c->stream);
    return HMC_OK;
}

int stage_B_fg(MD &md, int which, double eps, double h) {
    if (md.c->fg_mode == HMC_FG_EXACT) return stage_B_fg_exact(md, which, eps, h);
    return stage_B_fg_shift(md, which, eps, h);
}

int inner_leapfrog(MD &md, double s, int M) {
    int rc;
    for (int k = 0; k < M; ++k) {
        if ((rc = stage_B(md, 0, s / (2.0 * M)))) return rc;
        stage_A(md, s / M);
        if ((rc = stage_B(md, 0, s / (2.0 * M)))) return rc;
    }
    return HMC_OK;
}

int inner_fg(MD &md, double s, int M) {
    const double hm = s / M;
    int rc;
    for (int k = 0; k < M; ++k) {
        if ((rc = stage_B(md, 0, hm / 6.0))) return rc;
        stage_A(md, hm / 2.0);
        if ((rc = stage_B_fg(md, 0, 2.0 * hm / 3.0, hm))) return rc;
        stage_A(md, hm / 2.0);
        if ((rc = stage_B(md, 0, hm / 6.0))) return rc;
    }
    return HMC_OK;
}

// sigma, eta, lambda, theta of Eq. (6): the fourth-order set of Omelyan, Mryglod and Folk
// (2003), their Eq. (71)
constexpr double kOmfSigma = 0.08398315262876693;
constexpr double kOmfEta = 0.2539785108410595;
constexpr double kOmfLambda = 0.6822365335719091;
constexpr double kOmfTheta = -0.03230286765269967;

int md_step(MD &md, int scheme, double h, int M) {
    int rc = HMC_OK;
#define T(x) if ((rc = (x))) return rc
    switch (scheme) {
    case HMC_LEAPFROG:  // Eq. (3)
        T(stage_B(md, 2, h / 2.0)); stage_A(md, h); T(stage_B(md, 2, h / 2.0));
        break;
    case HMC_OMELYAN_5STAGE:  // Eq. (4)
        T(stage_B(md, 2, h / 6.0)); stage_A(md, h / 2.0); T(stage_B(md, 2, 2.0 * h / 3.0));
        stage_A(md, h / 2.0); T(stage_B(md, 2, h / 6.0));
        break;
    case HMC_FORCE_GRADIENT:  // Eq. (5)
        T(stage_B(md, 2, h / 6.0)); stage_A(md, h / 2.0); T(stage_B_fg(md, 2, 2.0 * h / 3.0, h));
        stage_A(md, h / 2.0); T(stage_B(md, 2, h / 6.0));
        break;
    case HMC_NESTED_FG:  // Eq. (10)
        T(stage_B(md, 1, h / 6.0)); T(inner_fg(md, h / 2.0, M)); T(stage_B_fg(md, 1, 2.0 * h / 3.0, h));
        T(inner_fg(md, h / 2.0, M)); T(stage_B(md, 1, h / 6.0));
        break;
    case HMC_ADAPTED_NESTED_FG:  // Eq. (11)
        T(stage_B(md, 1, h / 6.0)); T(inner_leapfrog(md, h / 2.0, M));
        T(stage_B_fg(md, 1, 2.0 * h / 3.0, h)); T(inner_leapfrog(md, h / 2.0, M));
        T(stage_B(md, 1, h / 6.0));
        break;
    case HMC_NESTED_LEAPFROG:  // Eq. (8)
        T(stage_B(md, 1, h / 2.0)); T(inner_leapfrog(md, h, M)); T(stage_B(md, 1, h / 2.0));
        break;
    case HMC_OMELYAN_11STAGE: {  // Eq. (6)
        const double bm = (1.0 - 2.0 * (kOmfLambda + kOmfSigma)) / 2.0;
        const double am = 1.0 - 2.0 * (kOmfTheta + kOmfEta);
        T(stage_B(md, 2, kOmfSigma * h)); stage_A(md, kOmfEta * h);
        T(stage_B(md, 2, kOmfLambda * h)); stage_A(md, kOmfTheta * h);
        T(stage_B(md, 2, bm * h)); stage_A(md, am * h); T(stage_B(md, 2, bm * h));
        stage_A(md, kOmfTheta * h); T(stage_B(md, 2, kOmfLambda * h));
        stage_A(md, kOmfEta * h); T(stage_B(md, 2, kOmfSigma * h));
        break;
    }
    case HMC_NESTED_5STAGE:  // Eq. (9)
        T(stage_B(md, 1, h / 6.0)); T(inner_leapfrog(md, h / 2.0, M));
        T(stage_B(md, 1, 2.0 * h / 3.0)); T(inner_leapfrog(md, h / 2.0, M));
        T(stage_B(md, 1, h / 6.0));
        break;
    default:
        return HMC_E_INVAL;
    }
#undef T
    return HMC_OK;
}

int check_md_args(hmc_ctx *c, int scheme, double tau, int n_outer, int n_inner, int prec) {
    if (scheme < HMC_LEAPFROG || scheme > HMC_OMELYAN_11STAGE)
        return fail(c, HMC_E_INVAL, "unknown scheme %d", scheme);
    if (!isfinite(tau) || n_outer < 1) return fail(c, HMC_E_INVAL, "need finite tau and n_outer >= 1");
    const bool nested = scheme == HMC_NESTED_FG || scheme == HMC_ADAPTED_NESTED_FG ||
                        scheme == HMC_NESTED_LEAPFROG || scheme == HMC_NESTED_5STAGE;
    if (nested && n_inner < 1)
        return fail(c, HMC_E_INVAL, "nested schemes need n_inner >= 1");
    if (prec != HMC_PREC_FP64 && prec != HMC_PREC_MIXED) return fail(c, HMC_E_INVAL, "bad precision");
    return HMC_OK;
}

int run_md(MD &md, int scheme, double tau, int n_outer, int n_inner) {
    const double h = tau / n_outer;
    for (int k = 0; k < n_outer; ++k) {
        int rc = md_step(md, scheme, h, n_inner);
        if (rc) return rc;
    }
    return HMC_OK;
}

void init_md(MD &md, hmc_ctx *c, int prec) {
    md.c = c;
    md.prec = prec;
    md.tol = c->tol;
    md.max_iter = c->max_iter;
    md.chain_status.assign(c->nchains, HMC_OK);
    md.iters.assign(c->nchains, 0);
    c->ff_version = -1;
    c->xi_version = -1;
    c->chi_version = -1;
    forget_links(c);
}

// Rebuilds the workgroup tables for another workgroup size or step-kernel variant (its
// sites per thread) and uploads them.
int set_tables(hmc_ctx *c, int block, int variant) {
    if (block < kMinBlock || block > 1024 || block % 64) return fail(c, HMC_E_INVAL, "bad workgroup size");
    if (variant < 0 || variant >= kNumStepVariants) return fail(c, HMC_E_INVAL, "bad step-kernel variant");
    if (block == c->block && variant == c->step_variant) return HMC_OK;
    int rc = sync(c);
    if (rc) return rc;
    c->block = block;
    c->step_variant = variant;
    c->graph_epoch++;
    build_tables(c);
    HIP_TRY(c, hipMemcpyAsync(c->at<ChainInfo>(c->off_chains), c->chains.data(),
                              sizeof(ChainInfo) * c->nchains, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->at<BlockWork>(c->off_work), c->work.data(),
                              sizeof(BlockWork) * c->work.size(), hipMemcpyHostToDevice, c->stream));
    c->part_vmax = -1;
    return sync(c);
}

void drop_chunks(hmc_ctx *c) {
    for (ChunkGraph &e : c->chunks) {
        if (e.exec) (void)hipGraphExecDestroy(e.exec);
        if (e.graph) (void)hipGraphDestroy(e.graph);
    }
    c->chunks.clear();
}

// ------------------------------------------------------------------ chain groups
void drop_groups(hmc_ctx *c) {
    for (int g = 0; g < c->grp_n; ++g) {
        hmc_ctx *k = c->grp[g];
        if (!k) continue;
        if (k->stream) (void)hipStreamSynchronize(k->stream);
        drop_chunks(k);
        if (k->side) (void)hipStreamDestroy(k->side);
        if (k->fork_ev) (void)hipEventDestroy(k->fork_ev);
        if (k->join_ev) (void)hipEventDestroy(k->join_ev);
        for (hipEvent_t e : k->timer.pool) (void)hipEventDestroy(e);
        if (k->timer.sums_host) (void)hipHostFree(k->timer.sums_host);
        if (k->pinned) (void)hipHostFree(k->pinned);
        delete k;
        c->grp[g] = nullptr;
    }
    c->grp_n = 0;
}

// The settings of the parent that a group's trajectory reads.
int sync_group(hmc_ctx *c, hmc_ctx *k) {
    k->tol = c->tol;
    k->max_iter = c->max_iter;
    k->delta = c->delta;
    k->check_every = c->check_every;
    k->quenched = c->quenched;
    k->fg_mode = c->fg_mode;
    k->fused_on = c->fused_on;
    k->graph_on = c->graph_on;
    if (k->persist_vmax != c->persist_vmax) {
        k->persist_vmax = c->persist_vmax;
        k->part_vmax = -1;
    }
    k->lds_max = c->lds_max;
    k->traj = c->traj;
    return set_tables(k, c->block, c->step_variant);
}

// Splits the chains into min(groups, n_chains) contiguous ranges of about equal sites and
// builds a context for each: its own chain and workgroup tables (in this context's group
// area of the workspace), CG state, stream, host bookkeeping; the fields are this context's.
int build_groups(hmc_ctx *c) {
    const int G = std::min(c->groups, c->nchains);
    if (c->grp_n == G) {
        c->grp[0]->stream = c->stream;
        for (int g = 0; g < G; ++g) {
            int rc = sync_group(c, c->grp[g]);
            if (rc) return fail(c, rc, "chain group %d: %s", g, c->grp[g]->err.c_str());
        }
        return HMC_OK;
    }
    int rc = sync(c);
    if (rc) return rc;
    drop_groups(c);
    // boundaries: group g starts at the first chain whose preceding sites reach g/G of the total
    std::vector<int> first(G + 1, c->nchains);
    first[0] = 0;
    long long acc = 0;
    int g = 1;
    for (int k = 0; k < c->nchains && g < G; ++k) {
        acc += c->chains[k].V;
        while (g < G && acc * G >= (long long)g * c->Vtot && k + 1 < c->nchains) first[g++] = k + 1;
    }
    // no empty range (G <= n_chains): at most n - (G - h) chains before group h, at least h
    for (int h = G - 1; h >= 1; --h) first[h] = std::min(first[h], first[h + 1] - 1);
    for (int h = 1; h < G; ++h) first[h] = std::max(first[h], first[h - 1] + 1);
    if (!c->grp_fork) {
        HIP_TRY(c, hipEventCreateWithFlags(&c->grp_fork, hipEventDisableTiming));
        for (int h = 0; h < kMaxGroups; ++h)
            HIP_TRY(c, hipEventCreateWithFlags(&c->grp_join[h], hipEventDisableTiming));
    }
    size_t off = c->off_groups;
    for (int h = 0; h < G; ++h) {
        hmc_ctx *k = new hmc_ctx();
        c->grp[h] = k;
        c->grp_n = h + 1;
        c->grp_first[h] = first[h];
        k->is_group = true;
        k->nchains = first[h + 1] - first[h];
        k->chains.assign(c->chains.begin() + first[h], c->chains.begin() + first[h + 1]);
        k->Vtot = c->Vtot;
        k->site0 = k->chains[0].off;
        k->nsites = 0;
        for (const ChainInfo &ci : k->chains) k->nsites += ci.V;
        k->seed = c->seed;
        k->block = kMinBlock;
        build_tables(k);
        const size_t nlog_min = k->work.size();
        k->block = c->block;
        build_tables(k);
        off = align_up(layout_tables(k, off, k->nchains, nlog_min));
        if (off > c->off_groups + c->groups_bytes)
            return fail(c, HMC_E_NOMEM, "chain group tables exceed their workspace area");
        for (int b = 0; b < kNumLinkBufs; ++b) k->off_links[b] = c->off_links[b];
        for (int b = 0; b < kNumSpinBufs; ++b) k->off_spin[b] = c->off_spin[b];
        for (int b = 0; b < kNumSpin32Bufs; ++b) k->off_spin32[b] = c->off_spin32[b];
        k->off_U64 = c->off_U64;
        k->off_A32 = c->off_A32;
        k->off_Uw = c->off_Uw;
        k->ws = c->ws;
        k->ws_bytes = c->ws_bytes;
        k->device = c->device;
        k->lds_max = c->lds_max;
        k->static_scratch = c->static_scratch;
        k->cg_host.resize(k->nchains);
        k->resid_host.resize(k->nchains);
        if (h > 0 && !c->grp_stream[h])
            HIP_TRY(c, hipStreamCreateWithFlags(&c->grp_stream[h], hipStreamNonBlocking));
        k->stream = h == 0 ? c->stream : c->grp_stream[h];
        k->pinned_bytes = align_up(sizeof(CGState) * k->nchains + sizeof(MetroOut) * k->nchains +
                                   sizeof(double) * 16 * k->nchains + 4096);
        HIP_TRY(c, hipHostMalloc(&k->pinned, k->pinned_bytes, hipHostMallocDefault));
        HIP_TRY(c, hipMemcpyAsync(k->at<ChainInfo>(k->off_chains), k->chains.data(),
                                  sizeof(ChainInfo) * k->nchains, hipMemcpyHostToDevice, k->stream));
        HIP_TRY(c, hipMemcpyAsync(k->at<BlockWork>(k->off_work), k->work.data(),
                                  sizeof(BlockWork) * k->work.size(), hipMemcpyHostToDevice, k->stream));
        HIP_TRY(c, hipStreamSynchronize(k->stream));
        if (c->timer.on) {
            if ((rc = hmc_set_timing(k, 1))) return fail(c, rc, "chain group timing: %s", k->err.c_str());
        }
        if ((rc = sync_group(c, k))) return fail(c, rc, "chain group %d: %s", h, k->err.c_str());
    }
    c->grp_first[G] = c->nchains;
    return HMC_OK;
}

}  // namespace

// ====================================================================== C ABI
static void refresh(hmc_ctx *c);

extern "C" {

int hmc_init(hmc_ctx **out, int L, double beta, double m0, uint64_t seed) {
    return hmc_init_ex(out, L, L, beta, m0, seed);
}

int hmc_init_ex(hmc_ctx **out, int Lx, int Lt, double beta, double m0, uint64_t seed) {
    return make_ctx(out, 1, &Lx, &Lt, &beta, &m0, seed);
}

int hmc_batch_init(hmc_ctx **out, int n_chains, const int *Lx, const int *Lt, const double *beta,
                   const double *m0, uint64_t seed) {
    return make_ctx(out, n_chains, Lx, Lt, beta, m0, seed);
}

size_t hmc_workspace_bytes(const hmc_ctx *ctx) { return ctx ? ctx->ws_bytes : 0; }

int hmc_bind(hmc_ctx *c, void *ws, size_t bytes, void *stream) {
    if (!c) return HMC_E_INVAL;
    if (!ws) return fail(c, HMC_E_INVAL, "null workspace");
    if ((uintptr_t)ws % kAlign) return fail(c, HMC_E_INVAL, "workspace must be 256-byte aligned");
    if (bytes < c->ws_bytes)
        return fail(c, HMC_E_NOMEM, "workspace has %zu bytes, needs %zu", bytes, c->ws_bytes);
    if (c->is_group) return fail(c, HMC_E_INVAL, "a chain group is bound through its parent");
    drop_groups(c);
    c->ws = (char *)ws;
    c->graph_epoch++;
    c->stream = (hipStream_t)stream;
    HIP_TRY(c, hipGetDevice(&c->device));
    scratch_address(c);
    if (!c->pinned) {
        c->pinned_bytes = align_up(sizeof(CGState) * c->nchains + sizeof(MetroOut) * c->nchains +
                                   sizeof(double) * 16 * c->nchains + 4096);
        HIP_TRY(c, hipHostMalloc(&c->pinned, c->pinned_bytes, hipHostMallocDefault));
    }
    {
        int dev = 0, optin = 0, plain = 0;
        HIP_TRY(c, hipGetDevice(&dev));
        if (hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, dev) != hipSuccess)
            optin = 0;
        if (hipDeviceGetAttribute(&plain, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
            plain = 0;
        (void)hipGetLastError();
        c->lds_max = (size_t)std::max(std::max(optin, plain), 0);
    }
    c->part_vmax = -1;
    HIP_TRY(c, hipMemcpyAsync(c->at<ChainInfo>(c->off_chains), c->chains.data(),
                              sizeof(ChainInfo) * c->nchains, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->at<BlockWork>(c->off_work), c->work.data(),
                              sizeof(BlockWork) * c->work.size(), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemsetAsync(c->link(LQ), 0, sizeof(double) * 2 * c->Vtot, c->stream));
    HIP_TRY(c, hipMemsetAsync(c->link(LP), 0, sizeof(double) * 2 * c->Vtot, c->stream));
    HIP_TRY(c, hipMemsetAsync(c->spin(SPHI), 0, sizeof(double2) * 2 * c->Vtot, c->stream));
    forget_all(c);
    return sync(c);
}

int hmc_field(hmc_ctx *c, int which, void **ptr, size_t *bytes) {
    CHECK_BOUND(c);
    if (!ptr) return fail(c, HMC_E_INVAL, "null output pointer");
    const size_t lb = sizeof(double) * 2 * c->Vtot, sb = sizeof(double2) * 2 * c->Vtot;
    switch (which) {
    case HMC_FIELD_Q: *ptr = c->link(LQ); if (bytes) *bytes = lb; break;
    case HMC_FIELD_P: *ptr = c->link(LP); if (bytes) *bytes = lb; break;
    case HMC_FIELD_PHI: *ptr = c->spin(SPHI); if (bytes) *bytes = sb; break;
    case HMC_FIELD_CHI: *ptr = c->spin(SCHI); if (bytes) *bytes = sb; break;
    case HMC_FIELD_XI: *ptr = c->spin(SXI); if (bytes) *bytes = sb; break;
    case HMC_FIELD_F: *ptr = c->link(LF); if (bytes) *bytes = lb; break;
    case HMC_FIELD_ZETA: *ptr = c->spin(SZETA); if (bytes) *bytes = sb; break;
    default: return fail(c, HMC_E_INVAL, "unknown field %d", which);
    }
    // the caller may write q through this pointer: forget everything derived from it
    forget_all(c);
    return HMC_OK;
}

int hmc_geometry(const hmc_ctx *c, int *n, long long *vt, int *offsets, int *Lx, int *Lt) {
    if (!c) return HMC_E_INVAL;
    if (n) *n = c->nchains;
    if (vt) *vt = c->Vtot;
    for (int k = 0; k < c->nchains; ++k) {
        if (offsets) offsets[k] = c->chains[k].off;
        if (Lx) Lx[k] = c->chains[k].Lx;
        if (Lt) Lt[k] = c->chains[k].Lt;
    }
    return HMC_OK;
}

int hmc_pack_links(hmc_ctx *c, const double *lex, double *nat) {
    CHECK_BOUND(c);
    if (!lex || !nat) return fail(c, HMC_E_INVAL, "null pointer");
    launch_pack_links(c->geo(), const_cast<double *>(lex), nat, true, c->stream);
    forget_all(c);
    HIP_TRY(c, hipGetLastError());
    return HMC_OK;
}

int hmc_unpack_links(hmc_ctx *c, const double *nat, double *lex) {
    CHECK_BOUND(c);
    if (!lex || !nat) return fail(c, HMC_E_INVAL, "null pointer");
    launch_pack_links(c->geo(), lex, const_cast<double *>(nat), false, c->stream);
    HIP_TRY(c, hipGetLastError());
    return HMC_OK;
}

int hmc_pack_spinor(hmc_ctx *c, const double *lex, double *nat) {
    CHECK_BOUND(c);
    if (!lex || !nat) return fail(c, HMC_E_INVAL, "null pointer");
    launch_pack_spinor(c->geo(), (double2 *)const_cast<double *>(lex), (double2 *)nat, true, c->stream);
    HIP_TRY(c, hipGetLastError());
    return HMC_OK;
}

int hmc_unpack_spinor(hmc_ctx *c, const double *nat, double *lex) {
    CHECK_BOUND(c);
    if (!lex || !nat) return fail(c, HMC_E_INVAL, "null pointer");
    launch_pack_spinor(c->geo(), (double2 *)lex, (double2 *)const_cast<double *>(nat), false, c->stream);
    HIP_TRY(c, hipGetLastError());
    return HMC_OK;
}

int hmc_cold_start(hmc_ctx *c) {
    CHECK_BOUND(c);
    HIP_TRY(c, hipMemsetAsync(c->link(LQ), 0, sizeof(double) * 2 * c->Vtot, c->stream));
    forget_all(c);
    return HMC_OK;
}

int hmc_hot_start(hmc_ctx *c) {
    CHECK_BOUND(c);
    launch_rng_links(c->geo(), c->seed, c->link(LQ), c->stream);
    forget_all(c);
    HIP_TRY(c, hipGetLastError());
    return HMC_OK;
}

int hmc_set_trajectory_counter(hmc_ctx *c, uint32_t traj) {
    if (!c) return HMC_E_INVAL;
    c->traj = traj;
    return HMC_OK;
}

uint32_t hmc_get_trajectory_counter(const hmc_ctx *c) { return c ? c->traj : 0; }

int hmc_set_solver(hmc_ctx *c, double tol, int max_iter, double reliable_delta) {
    if (!c) return HMC_E_INVAL;
    if (!(tol >= 0) || !isfinite(tol) || max_iter < 1 || !(reliable_delta > 0 && reliable_delta < 1))
        return fail(c, HMC_E_INVAL, "bad solver settings");
    c->tol = tol;
    c->graph_epoch++;
    c->max_iter = max_iter;
    c->delta = reliable_delta;
    return HMC_OK;
}

int hmc_set_quenched(hmc_ctx *c, int quenched) {
    if (!c) return HMC_E_INVAL;
    c->quenched = quenched != 0;
    c->graph_epoch++;
    return HMC_OK;
}

int hmc_set_persistent_limit(hmc_ctx *c, int vmax) {
    if (!c || vmax < 0) return HMC_E_INVAL;
    c->persist_vmax = vmax;
    c->graph_epoch++;
    return HMC_OK;
}

int hmc_set_cg_groups(hmc_ctx *c, int groups) {
    if (!c || groups < 1 || groups > kMaxGroups) return HMC_E_INVAL;
    if (c->is_group) return fail(c, HMC_E_INVAL, "a chain group cannot be split again");
    if (groups != c->groups) {
        if (c->ws) {
            int rc = sync(c);
            if (rc) return rc;
        }
        drop_groups(c);
    }
    c->groups = groups;
    return HMC_OK;
}

int hmc_set_fused_cg(hmc_ctx *c, int on) {
    if (!c) return HMC_E_INVAL;
    c->fused_on = on != 0;
    c->graph_epoch++;
    return HMC_OK;
}

int hmc_mark_links_changed(hmc_ctx *c) {
    if (!c) return HMC_E_INVAL;
    forget_all(c);
    return HMC_OK;
}

int hmc_set_block_size(hmc_ctx *c, int block) {
    CHECK_BOUND(c);
    return set_tables(c, block, c->step_variant);
}

// Mean wall time of `reps` solves of the current right-hand side (after one warm-up solve).
static int time_solves(hmc_ctx *c, int prec, double tol, int reps, double *ms) {
    ensure_links(c, c->link(LQ), prec == HMC_PREC_MIXED, c->q_version);
    int rc = solve(c, c->spin(SPHI), c->spin(SXI), tol, c->max_iter, prec);
    if (rc && !chain_failure(rc)) return rc;
    const auto t0 = std::chrono::steady_clock::now();
    for (int rep = 0; rep < reps; ++rep) {
        rc = solve(c, c->spin(SPHI), c->spin(SXI), tol, c->max_iter, prec);
        if (rc && !chain_failure(rc)) return rc;
    }
    *ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count() / reps;
    return HMC_OK;
}

int hmc_autotune(hmc_ctx *c, int prec, double tol, const hmc_tune_schedule *traj, hmc_tune_info *out) {
    CHECK_BOUND(c);
    if (c->is_group) return fail(c, HMC_E_INVAL, "tune the parent context, not a chain group");
    if (prec != HMC_PREC_FP64 && prec != HMC_PREC_MIXED) return fail(c, HMC_E_INVAL, "bad precision");
    if (!(tol > 0)) return fail(c, HMC_E_INVAL, "bad tolerance");
    if (traj) {
        int rc = check_md_args(c, traj->scheme, traj->tau, traj->n_outer, traj->n_inner, prec);
        if (rc) return rc;
    }
    // a realistic right-hand side at the current links: phi = D^dagger zeta
    forget_all(c);
    refresh(c);
    int n = 0, rc = HMC_OK;
    double best = 1e300, ms = 0.0;
    // 1. workgroup size x persistent-solver limit
    std::vector<int> persist = {0};
    int vmin = 1 << 30;
    for (const ChainInfo &ci : c->chains) vmin = std::min(vmin, ci.V);
    if (vmin <= 1024) persist.push_back(1024);
    for (const ChainInfo &ci : c->chains)
        if (ci.V > 1024 && ci.V <= 2048) { persist.push_back(2048); break; }
    int best_block = c->block, best_persist = c->persist_vmax;
    for (int b : {128, 256, 512, 1024}) {
        if ((rc = set_tables(c, b, kStepPlain))) return rc;
        for (int pv : persist) {
            c->persist_vmax = pv;
            if ((rc = time_solves(c, prec, tol, 2, &ms))) return rc;
            ++n;
            if (ms < best) { best = ms; best_block = b; best_persist = pv; }
        }
    }
    c->persist_vmax = best_persist;
    // 2. step-kernel variant (sites per thread, resident grid, register bound)
    //    (the plain variant at this size was timed in step 1)
    int best_variant = kStepPlain;
    for (int v = kStepPlain + 1; v < kNumStepVariants; ++v) {
        if ((rc = set_tables(c, best_block, v))) return rc;
        if ((rc = time_solves(c, prec, tol, 2, &ms))) return rc;
        ++n;
        if (ms < best) { best = ms; best_variant = v; }
    }
    if ((rc = set_tables(c, best_block, best_variant))) return rc;
    // 3. convergence-check interval
    int best_every = c->check_every;
    for (int every : {16, 32, 64}) {
        c->check_every = every;
        if ((rc = time_solves(c, prec, tol, 2, &ms))) return rc;
        ++n;
        if (ms < best) { best = ms; best_every = every; }
    }
    c->check_every = best_every;
    // 4. mixed precision: the reliable-update factor (it changes the iterates within the
    //    tolerance, not only the speed)
    double best_delta = c->delta;
    if (prec == HMC_PREC_MIXED) {
        for (double d : {1e-3, 1e-4, 1e-5}) {
            c->delta = d;
            if ((rc = time_solves(c, prec, tol, 2, &ms))) return rc;
            ++n;
            if (ms < best) { best = ms; best_delta = d; }
        }
        c->delta = best_delta;
    }
    // 5. chain groups, by whole trajectories of the given schedule from the current links
    //    (links, trajectory counter and tolerance restored afterwards)
    int best_groups = c->groups;
    double best_traj = 0.0;
    if (traj && c->nchains > 1) {
        std::vector<double> q(2 * (size_t)c->Vtot);
        HIP_TRY(c, hipMemcpyAsync(q.data(), c->link(LQ), sizeof(double) * q.size(), hipMemcpyDeviceToHost,
                                  c->stream));
        if ((rc = sync(c))) return rc;
        const uint32_t traj0 = c->traj;
        const double tol0 = c->tol;
        c->tol = tol;
        best_traj = 1e300;
        for (int gr = 1; gr <= std::min(kMaxGroups, c->nchains); ++gr) {
            if ((rc = hmc_set_cg_groups(c, gr))) return rc;
            // a warm-up trajectory, then the mean of two timed ones (each from the links the
            // previous one left, so every candidate sees a different but equally thermalised
            // configuration; the links are restored below)
            double t_ms = 0.0;
            for (int rep = 0; rep < 3; ++rep) {
                if ((rc = sync(c))) return rc;
                const auto t0 = std::chrono::steady_clock::now();
                rc = hmc_trajectory(c, traj->scheme, traj->tau, traj->n_outer, traj->n_inner, prec, nullptr);
                if (rc && !chain_failure(rc)) return rc;
                if ((rc = sync(c))) return rc;
                if (rep > 0)
                    t_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count() / 2;
            }
            ++n;
            if (t_ms < best_traj) { best_traj = t_ms; best_groups = gr; }
        }
        if ((rc = hmc_set_cg_groups(c, best_groups))) return rc;
        HIP_TRY(c, hipMemcpyAsync(c->link(LQ), q.data(), sizeof(double) * q.size(), hipMemcpyHostToDevice,
                                  c->stream));
        if ((rc = sync(c))) return rc;
        c->traj = traj0;
        c->tol = tol0;
    }
    c->part_vmax = -1;
    c->graph_epoch++;
    forget_all(c);
    if (out) {
        memset(out, 0, sizeof *out);
        out->block = best_block;
        out->persistent_limit = best_persist;
        out->step_variant = best_variant;
        out->check_interval = best_every;
        out->groups = best_groups;
        out->candidates = n;
        out->reliable_delta = best_delta;
        out->solve_ms = best;
        out->traj_ms = best_traj;
    }
    return HMC_OK;
}

int hmc_set_step_variant(hmc_ctx *c, int variant) {
    CHECK_BOUND(c);
    int rc = set_tables(c, c->block, variant);
    if (rc) return rc;
    c->part_vmax = -1;
    c->graph_epoch++;
    return HMC_OK;
}

int hmc_set_check_interval(hmc_ctx *c, int every) {
    if (!c || every < 1) return HMC_E_INVAL;
    c->check_every = every;
    c->graph_epoch++;
    return HMC_OK;
}

int hmc_dslash(hmc_ctx *c, const void *in, void *out) {
    CHECK_BOUND(c);
    if (!in || !out || in == out) return fail(c, HMC_E_INVAL, "need distinct in/out");
    ensure_links(c, c->link(LQ), false, c->q_version);
    launch_dslash64(c->geo(), c->U64(), (const double2 *)in, (double2 *)out, false, c->stream);
    HIP_TRY(c, hipGetLastError());
    return HMC_OK;
}

int hmc_stream_copy(hmc_ctx *c, const void *src, void *dst, size_t bytes) {
    CHECK_BOUND(c);
    if (!src || !dst || bytes % 16 || ((uintptr_t)src | (uintptr_t)dst) % 16)
        return fail(c, HMC_E_INVAL, "stream copy needs 16-byte aligned pointers and a size in 16-byte units");
    if (bytes / 16 > (size_t)0x7fffffff * 256) return fail(c, HMC_E_INVAL, "stream copy too large");
    if (bytes) launch_stream_copy(src, dst, bytes / 16, c->stream);
    HIP_TRY(c, hipGetLastError());
    return HMC_OK;
}

int hmc_dslash_dagger(hmc_ctx *c, const void *in, void *out) {
    CHECK_BOUND(c);
    if (!in || !out || in == out) return fail(c, HMC_E_INVAL, "need distinct in/out");
    ensure_links(c, c->link(LQ), false, c->q_version);
    launch_dslash64(c->geo(), c->U64(), (const double2 *)in, (double2 *)out, true, c->stream);
    HIP_TRY(c, hipGetLastError());
    return HMC_OK;
}

int hmc_cg_solve(hmc_ctx *c, const void *phi, void *x, double tol, int max_iter, int prec,
                 hmc_cg_info *info) {
    CHECK_BOUND(c);
    if (!phi || !x || phi == x) return fail(c, HMC_E_INVAL, "need distinct phi/x");
    if (!(tol >= 0) || max_iter < 1) return fail(c, HMC_E_INVAL, "bad tol/max_iter");
    if (prec != HMC_PREC_FP64 && prec != HMC_PREC_MIXED) return fail(c, HMC_E_INVAL, "bad precision");
    ensure_links(c, c->link(LQ), prec == HMC_PREC_MIXED, c->q_version);
    int rc = solve(c, (const double2 *)phi, (double2 *)x, tol, max_iter, prec);
    if (rc && !chain_failure(rc)) return rc;
    std::vector<double> t2(c->nchains);
    double *dev = c->sums() + 12 * c->nchains;
    launch_true_residual64(c->geo(), c->U64(), (const double2 *)phi, (const double2 *)x,
                           c->spin(ST), c->partials(), dev, c->stream);
    int rc2 = to_host(c, t2.data(), dev, sizeof(double) * c->nchains);
    if (rc2) return rc2;
    fill_cg_info(c, info, &t2);
    return rc;
}

int hmc_cg_solve_noalloc(hmc_ctx *c, const void *phi, void *x, double tol, int max_iter,
                         hmc_cg_info *info) {
    CHECK_BOUND(c);
    if (!phi || !x || phi == x) return fail(c, HMC_E_INVAL, "need distinct phi/x");
    if (!(tol >= 0) || max_iter < 1) return fail(c, HMC_E_INVAL, "bad tol/max_iter");
    if (!c->static_scratch)
        return fail(c, HMC_E_HIP, "no device address of the static scratch: %s", c->static_scratch_err.c_str());
    int dev = -1;
    HIP_TRY(c, hipGetDevice(&dev));
    if (dev != c->device) return fail(c, HMC_E_INVAL, "the current device is not the context's");
    const Geo g = c->geo();
    if (c->Vtot > kNoAllocMaxSites || c->nchains > kNoAllocMaxChains || g.nlog > kNoAllocMaxPartials)
        return fail(c, HMC_E_NOMEM,
                    "the allocation-free solve takes at most %d sites, %d chains and %d workgroups "
                    "(context: %d, %d, %d)", kNoAllocMaxSites, kNoAllocMaxChains, kNoAllocMaxPartials,
                    c->Vtot, c->nchains, g.nlog);
    int vmax = 0;
    for (const ChainInfo &ci : c->chains) vmax = std::max(vmax, ci.V);
    if (vmax > 2048 || cg_wg_lds_bytes(vmax, false) + 1024 > c->lds_max)
        return fail(c, HMC_E_INVAL, "the allocation-free solve needs every chain within %d sites",
                    std::min(2048, persistent_limit(c, false)));
    char *base = (char *)c->static_scratch;
    double2 *U = (double2 *)base;
    double2 *t = (double2 *)(base + kNoAllocOffT);
    CGState *st = (CGState *)(base + kNoAllocOffState);
    int *list = (int *)(base + kNoAllocOffList);
    double *partials = (double *)(base + kNoAllocOffPartials);
    double *sums = (double *)(base + kNoAllocOffSums);
    launch_make_links(g, c->link(LQ), U, nullptr, c->stream);
    launch_iota(list, c->nchains, c->stream);
    CGFields f = {};
    f.phi = (const double2 *)phi;
    f.x64 = (double2 *)x;
    f.U64 = U;
    f.st = st;
    if (launch_cg_wg(g, f, false, list, c->nchains, vmax, tol, c->delta, max_iter, c->stream))
        return fail(c, HMC_E_HIP, "the persistent solver's LDS request was refused");
    launch_true_residual64(g, U, (const double2 *)phi, (const double2 *)x, t, partials, sums, c->stream);
    HIP_TRY(c, hipGetLastError());
    int rc = to_host(c, c->cg_host.data(), st, sizeof(CGState) * c->nchains);
    if (rc) return rc;
    if ((rc = to_host(c, c->resid_host.data(), sums, sizeof(double) * c->nchains))) return rc;
    fill_cg_info(c, info, &c->resid_host);
    int nonfinite = 0, capped = 0;
    for (const CGState &s : c->cg_host) {
        nonfinite += s.converged == kStopNonFinite;
        capped += s.converged != kConverged && s.converged != kStopNonFinite;
    }
    if (nonfinite) return fail(c, HMC_E_NAN, "CG: the residual of %d chain(s) became non-finite", nonfinite);
    if (capped) return fail(c, HMC_E_NOCONV, "CG did not converge in %d iterations (%d chain(s))", max_iter, capped);
    return HMC_OK;
}

int hmc_fermion_force_chixi(hmc_ctx *c, const void *chi, const void *xi, double *f) {
    CHECK_BOUND(c);
    if (!chi || !xi || !f) return fail(c, HMC_E_INVAL, "null pointer");
    ensure_links(c, c->link(LQ), false, c->q_version);
    launch_fermion_force(c->geo(), c->U64(), (const double2 *)chi, (const double2 *)xi, f, c->stream);
    HIP_TRY(c, hipGetLastError());
    return HMC_OK;
}

int hmc_fermion_force(hmc_ctx *c, const void *phi, double *f, double tol, int max_iter, int prec,
                      hmc_cg_info *info, double *sf) {
    CHECK_BOUND(c);
    if (!phi) return fail(c, HMC_E_INVAL, "null pointer");
    if (!(tol >= 0) || max_iter < 1) return fail(c, HMC_E_INVAL, "bad tol/max_iter");
    if (prec != HMC_PREC_FP64 && prec != HMC_PREC_MIXED) return fail(c, HMC_E_INVAL, "bad precision");
    ensure_links(c, c->link(LQ), prec == HMC_PREC_MIXED, c->q_version);
    int rc = solve(c, (const double2 *)phi, c->spin(SXI), tol, max_iter, prec);
    if (rc && !chain_failure(rc)) return rc;
    launch_dslash64(c->geo(), c->U64(), c->spin(SXI), c->spin(SCHI), false, c->stream);
    if (f) launch_fermion_force(c->geo(), c->U64(), c->spin(SCHI), c->spin(SXI), f, c->stream);
    fill_cg_info(c, info, nullptr);
    if (sf) {
        double *dev = c->sums() + 12 * c->nchains;
        launch_gauge_energy(c->geo(), c->link(LQ), (const double2 *)phi, c->spin(SXI),
                            c->partials(), dev, c->stream);
        std::vector<double> h(3 * c->nchains);
        int rc2 = to_host(c, h.data(), dev, sizeof(double) * 3 * c->nchains);
        if (rc2) return rc2;
        for (int k = 0; k < c->nchains; ++k) sf[k] = h[2 * c->nchains + k];
    }
    c->ff_version = c->xi_version = c->chi_version = -1;
    HIP_TRY(c, hipGetLastError());
    return rc;
}

int hmc_total_force_chixi(hmc_ctx *c, const void *chi, const void *xi, double *F) {
    CHECK_BOUND(c);
    if (!chi || !xi || !F) return fail(c, HMC_E_INVAL, "null pointer");
    ensure_links(c, c->link(LQ), false, c->q_version);
    launch_fermion_force(c->geo(), c->U64(), (const double2 *)chi, (const double2 *)xi, F, c->stream);
    launch_gauge_force(c->geo(), c->link(LQ), F, F, c->stream);
    HIP_TRY(c, hipGetLastError());
    return HMC_OK;
}

int hmc_gauge_force(hmc_ctx *c, double *g) {
    CHECK_BOUND(c);
    if (!g) return fail(c, HMC_E_INVAL, "null pointer");
    launch_gauge_force(c->geo(), c->link(LQ), nullptr, g, c->stream);
    HIP_TRY(c, hipGetLastError());
    return HMC_OK;
}

int hmc_actions(hmc_ctx *c, const void *phi, double tol, double *s_gauge, double *plaq,
                double *s_fermion) {
    CHECK_BOUND(c);
    const int C = c->nchains;
    int solve_rc = HMC_OK;
    if (phi && s_fermion) {
        ensure_links(c, c->link(LQ), false, c->q_version);
        solve_rc = solve(c, (const double2 *)phi, c->spin(SXI), tol, c->max_iter, HMC_PREC_FP64);
        if (solve_rc && !chain_failure(solve_rc)) return solve_rc;
        c->ff_version = c->xi_version = c->chi_version = -1;
    }
    double *dev = c->sums() + 12 * C;
    launch_gauge_energy(c->geo(), c->link(LQ), (phi && s_fermion) ? (const double2 *)phi : nullptr,
                        c->spin(SXI), c->partials(), dev, c->stream);
    std::vector<double> h(3 * C);
    int rc = to_host(c, h.data(), dev, sizeof(double) * 3 * C);
    if (rc) return rc;
    for (int k = 0; k < C; ++k) {
        if (s_gauge) s_gauge[k] = c->chains[k].beta * h[k];
        if (plaq) plaq[k] = h[C + k] / c->chains[k].V;
        // a chain whose solve stopped unconverged gets NaN rather than an inexact S_F
        if (s_fermion && phi)
            s_fermion[k] = c->cg_host[k].converged == kConverged ? h[2 * C + k] : NAN;
    }
    return solve_rc;
}

int hmc_update_links(hmc_ctx *c, double eps) {
    CHECK_BOUND(c);
    if (!isfinite(eps)) return fail(c, HMC_E_INVAL, "non-finite eps");
    launch_axpy_links(c->geo(), c->link(LQ), eps, c->link(LP), c->link(LQ), c->stream);
    forget_all(c);
    HIP_TRY(c, hipGetLastError());
    return HMC_OK;
}

int hmc_update_momenta(hmc_ctx *c, double eps, const double *F) {
    CHECK_BOUND(c);
    if (!F || !isfinite(eps)) return fail(c, HMC_E_INVAL, "bad arguments");
    launch_axpy_links(c->geo(), c->link(LP), -eps, F, c->link(LP), c->stream);
    HIP_TRY(c, hipGetLastError());
    return HMC_OK;
}

int hmc_fg_shifted_force(hmc_ctx *c, double c_h2, int which, const void *phi, double *F_out,
                         int prec, hmc_cg_info *info) {
    CHECK_BOUND(c);
    if (!F_out || !isfinite(c_h2) || which < 0 || which > 2) return fail(c, HMC_E_INVAL, "bad arguments");
    if (which != HMC_FORCE_GAUGE && !phi) return fail(c, HMC_E_INVAL, "phi needed");
    if (prec != HMC_PREC_FP64 && prec != HMC_PREC_MIXED) return fail(c, HMC_E_INVAL, "bad precision");
    MD md;
    init_md(md, c, prec);
    if (phi && phi != c->spin(SPHI))
        launch_copy(phi, c->spin(SPHI), sizeof(double2) * 2 * c->Vtot, c->stream);
    int rc = force_at(md, which, c->link(LQ), -1, c->link(LF));
    if (rc) return rc;
    launch_axpy_links(c->geo(), c->link(LQ), c_h2, c->link(LF), c->link(LQS), c->stream);
    rc = force_at(md, which, c->link(LQS), -1, F_out);
    if (rc) return rc;
    forget_links(c);
    c->ff_version = c->xi_version = c->chi_version = -1;
    if (which != HMC_FORCE_GAUGE) fill_cg_info(c, info, nullptr);
    HIP_TRY(c, hipGetLastError());
    return md.status;
}

int hmc_hessian_vector(hmc_ctx *c, int which, const void *phi, const double *v, double *out,
                       int prec, hmc_cg_info *info) {
    CHECK_BOUND(c);
    if (!v || !out || (const void *)v == (const void *)out || which < 0 || which > 2)
        return fail(c, HMC_E_INVAL, "bad arguments");
    if (which != HMC_FORCE_GAUGE && !phi) return fail(c, HMC_E_INVAL, "phi needed");
    if (prec != HMC_PREC_FP64 && prec != HMC_PREC_MIXED) return fail(c, HMC_E_INVAL, "bad precision");
    MD md;
    init_md(md, c, prec);
    if (phi && phi != c->spin(SPHI))
        launch_copy(phi, c->spin(SPHI), sizeof(double2) * 2 * c->Vtot, c->stream);
    int rc = hessian_vector(md, which, v, 1.0, out);
    if (rc) return rc;
    if (md.hvp_solves) fill_cg_info(c, info, nullptr);
    HIP_TRY(c, hipGetLastError());
    return md.status;
}

int hmc_force_gradient_term(hmc_ctx *c, int which, const void *phi, double *C, int prec,
                            hmc_cg_info *info) {
    CHECK_BOUND(c);
    if (!C || C == c->link(LF) || which < 0 || which > 2)
        return fail(c, HMC_E_INVAL, "bad arguments (C may not be the F field)");
    if (which != HMC_FORCE_GAUGE && !phi) return fail(c, HMC_E_INVAL, "phi needed");
    if (prec != HMC_PREC_FP64 && prec != HMC_PREC_MIXED) return fail(c, HMC_E_INVAL, "bad precision");
    MD md;
    init_md(md, c, prec);
    if (phi && phi != c->spin(SPHI))
        launch_copy(phi, c->spin(SPHI), sizeof(double2) * 2 * c->Vtot, c->stream);
    int rc = force_at(md, which, c->link(LQ), c->q_version, c->link(LF));
    if (rc) return rc;
    rc = hessian_vector(md, which, c->link(LF), 2.0, C);
    if (rc) return rc;
    if (md.hvp_solves) fill_cg_info(c, info, nullptr);
    HIP_TRY(c, hipGetLastError());
    return md.status;
}

int hmc_set_fg_mode(hmc_ctx *c, int mode) {
    if (!c) return HMC_E_INVAL;
    if (mode != HMC_FG_SHIFT && mode != HMC_FG_EXACT) return fail(c, HMC_E_INVAL, "bad force-gradient mode");
    c->fg_mode = mode;
    c->graph_epoch++;
    return HMC_OK;
}

// The device part of the end of a trajectory: S_F at the final links, the energies, the
// per-chain status, the Metropolis test (and the restore of rejected chains), the plaquettes.
static int finish_traj_device(hmc_ctx *c, MD &md, bool metropolis) {
    const Geo g = c->geo();
    const int C = c->nchains;
    const bool fermions = !c->quenched;
    // S_F at the final links: reuse xi if the last solve was at the current q
    if (fermions && c->xi_version != c->q_version) {
        ensure_links(c, c->link(LQ), md.prec == HMC_PREC_MIXED, c->q_version);
        int rc = note_solve(md, solve(c, c->spin(SPHI), c->spin(SXI), md.tol, md.max_iter, md.prec));
        if (rc) return rc;
        c->xi_version = c->q_version;
    }
    // sums layout: [0, 7C) energies, [7C, 9C) refresh, [9C, 12C) gauge sums,
    // [12C, 15C) scratch of the API-level reductions
    double *es = c->sums();             // [7][C]
    double *rs = c->sums() + 7 * C;     // [2][C] from the refresh
    double *gs = c->sums() + 9 * C;     // [3][C]
    launch_energy(g, c->link(LQ), c->link(LQ0), c->link(LP), c->link(LP0),
                  fermions ? c->spin(SPHI) : nullptr, c->spin(SXI), c->partials(), es, c->stream);
    if (c->deferring)
        launch_chain_status(c->at<int>(c->off_log), std::min(c->log_count, kMaxLoggedSolves), C,
                            c->at<int>(c->off_status), c->stream);
    else
        HIP_TRY(c, hipMemcpyAsync(c->at<int>(c->off_status), md.chain_status.data(), sizeof(int) * C,
                                  hipMemcpyHostToDevice, c->stream));
    MetroOut *mo = c->at<MetroOut>(c->off_metro);
    launch_metropolis(g, c->seed, c->at<uint32_t>(c->off_trajc), es, rs, c->at<int>(c->off_status), mo,
                      fermions, c->stream);
    if (metropolis) {
        launch_restore(g, mo, c->link(LQ0), c->link(LQ), c->stream);
        c->q_version++;
    }
    launch_gauge_energy(g, c->link(LQ), nullptr, c->spin(SXI), c->partials(), gs, c->stream);
    return HMC_OK;
}

// The host part: reads the Metropolis results and plaquettes and fills info.  logged > 0:
// the per-chain iterations come from the device log of that many solves.
static int finish_traj_host(hmc_ctx *c, MD &md, bool metropolis, int logged, hmc_traj_info *info) {
    const int C = c->nchains;
    MetroOut *mo = c->at<MetroOut>(c->off_metro);
    double *gs = c->sums() + 9 * C;
    std::vector<MetroOut> mh(C);
    std::vector<double> gh(3 * C);
    int rc = to_host(c, mh.data(), mo, sizeof(MetroOut) * C);
    if (rc) return rc;
    if ((rc = to_host(c, gh.data(), gs, sizeof(double) * 3 * C))) return rc;
    if (logged > 0) {
        std::vector<int> log((size_t)2 * logged * C);
        HIP_TRY(c, hipMemcpy(log.data(), c->at<int>(c->off_log), sizeof(int) * log.size(),
                             hipMemcpyDeviceToHost));
        for (int k = 0; k < logged; ++k)
            for (int ch = 0; ch < C; ++ch) md.iters[ch] += log[((size_t)k * C + ch) * 2];
    }
    int status = HMC_OK;
    for (int k = 0; k < C; ++k) {
        if (info) {
            hmc_traj_info &t = info[k];
            memset(&t, 0, sizeof t);
            t.dH = mh[k].dH;
            t.H0 = mh[k].H0;
            t.H1 = mh[k].H1;
            t.u = mh[k].u;
            t.accepted = metropolis ? mh[k].accepted : 0;
            t.status = mh[k].status;
            t.plaquette = gh[C + k] / c->chains[k].V;
            t.n_force_evals = md.force_evals;
            t.n_solves = md.solves;
            t.n_dinv = 2 * md.force_evals + 2 * md.hvp_solves;
            t.n_cg_iters = md.iters[k];
        }
        if (mh[k].status && status == HMC_OK) status = mh[k].status;
    }
    if (status) fail(c, status, "a chain failed (status %d)", status);
    return status;
}

static int finish_traj(hmc_ctx *c, MD &md, bool metropolis, hmc_traj_info *info) {
    int rc = finish_traj_device(c, md, metropolis);
    if (rc) return rc;
    return finish_traj_host(c, md, metropolis, 0, info);
}

static void refresh(hmc_ctx *c) {
    const Geo g = c->geo();
    const bool fermions = !c->quenched;
    double *rs = c->sums() + 7 * c->nchains;
    launch_refresh(g, c->seed, c->at<uint32_t>(c->off_trajc), c->link(LP), c->spin(SZETA), fermions,
                   c->partials(), rs, c->stream);
    if (fermions) {
        ensure_links(c, c->link(LQ), false, c->q_version);
        launch_dslash64(g, c->U64(), c->spin(SZETA), c->spin(SPHI), true, c->stream);
    }
}

int hmc_refresh(hmc_ctx *c) {
    CHECK_BOUND(c);
    forget_all(c);
    launch_set_u32(c->at<uint32_t>(c->off_trajc), c->traj, c->stream);
    refresh(c);
    HIP_TRY(c, hipGetLastError());
    return HMC_OK;
}

// One trajectory's device work: refresh (counter from the device), q0/p0 copies, the
// molecular dynamics and the device part of the Metropolis step.
static int trajectory_body(hmc_ctx *c, MD &md, int scheme, double tau, int n_outer, int n_inner) {
    refresh(c);
    copy_links(c, c->link(LQ), c->link(LQ0));
    copy_links(c, c->link(LP), c->link(LP0));
    int rc = run_md(md, scheme, tau, n_outer, n_inner);
    if (rc && !chain_failure(rc)) return rc;
    return finish_traj_device(c, md, true);
}

// Captures the trajectory body as one HIP graph.  Needs every chain in the persistent solver
// (its solves then have no host-side loop); solves log their results on the device.
static int graph_capture(hmc_ctx *c, GraphEntry &e) {
    const bool mixed = e.prec == HMC_PREC_MIXED;
    int rc = build_partition(c, persistent_limit(c, mixed));
    if (rc) return rc;
    if (c->n_small != c->nchains)
        return fail(c, HMC_E_INVAL, "a captured trajectory needs every chain within the persistent "
                                    "solver's limit (%d sites)", persistent_limit(c, mixed));
    if (prepare_small(c, mixed))
        return fail(c, HMC_E_INVAL, "the persistent solver's LDS request was refused");
    if ((rc = ensure_side(c))) return rc;
    MD md;
    init_md(md, c, e.prec);
    c->deferring = true;
    c->log_count = 0;
    c->log_overflow = false;
    // The capture is recorded on the library's own stream (the bound stream may be the
    // default stream, which cannot be captured); nothing runs until the graph is launched on
    // the bound stream.
    hipStream_t bound = c->stream;
    c->stream = c->side;
    hipError_t eb = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
    if (eb != hipSuccess) {
        c->stream = bound;
        c->deferring = false;
        (void)hipGetLastError();
        return fail(c, HMC_E_HIP, "graph capture could not start: %s", hipGetErrorString(eb));
    }
    rc = trajectory_body(c, md, e.scheme, e.tau, e.n_outer, e.n_inner);
    c->deferring = false;
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(c->stream, &graph);
    c->stream = bound;
    forget_all(c);  // nothing ran: the host's bookkeeping of links and solutions is void
    if (rc || ec != hipSuccess || c->log_overflow) {
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipGetLastError();
        if (rc) return rc;
        if (c->log_overflow) return fail(c, HMC_E_INVAL, "more than %d solves in one trajectory", kMaxLoggedSolves);
        return fail(c, HMC_E_HIP, "graph capture failed: %s", hipGetErrorString(ec));
    }
    hipGraphExec_t exec = nullptr;
    if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(graph);
        (void)hipGetLastError();
        return fail(c, HMC_E_HIP, "graph instantiation failed");
    }
    e.graph = graph;
    e.exec = exec;
    e.solves = md.solves;
    e.force_evals = md.force_evals;
    e.hvp_solves = md.hvp_solves;
    e.logged = c->log_count;
    e.epoch = c->graph_epoch;
    return HMC_OK;
}

static void drop_graph(GraphEntry &e) {
    if (e.exec) (void)hipGraphExecDestroy(e.exec);
    if (e.graph) (void)hipGraphDestroy(e.graph);
    e.exec = nullptr;
    e.graph = nullptr;
}

// A trajectory replayed from its captured graph (captured on first use of this schedule and
// these settings).  Same device work, in the same order, as the eager trajectory.
static int graph_trajectory(hmc_ctx *c, int scheme, double tau, int n_outer, int n_inner, int prec,
                            hmc_traj_info *info) {
    GraphEntry *e = nullptr;
    for (GraphEntry &g : c->graphs)
        if (g.epoch == c->graph_epoch && g.scheme == scheme && g.tau == tau && g.n_outer == n_outer &&
            g.n_inner == n_inner && g.prec == prec && g.fg_mode == c->fg_mode)
            e = &g;
    if (!e) {
        // settings changed since older graphs were captured: drop those
        for (GraphEntry &g : c->graphs)
            if (g.epoch != c->graph_epoch) drop_graph(g);
        c->graphs.erase(std::remove_if(c->graphs.begin(), c->graphs.end(),
                                       [](const GraphEntry &g) { return g.exec == nullptr; }),
                        c->graphs.end());
        GraphEntry ne;
        ne.scheme = scheme; ne.tau = tau; ne.n_outer = n_outer; ne.n_inner = n_inner; ne.prec = prec;
        ne.fg_mode = c->fg_mode;
        int rc = graph_capture(c, ne);
        if (rc) return rc;
        c->graphs.push_back(ne);
        e = &c->graphs.back();
    }
    launch_set_u32(c->at<uint32_t>(c->off_trajc), c->traj, c->stream);
    HIP_TRY(c, hipGraphLaunch(e->exec, c->stream));
    MD md;
    md.c = c;
    md.prec = prec;
    md.chain_status.assign(c->nchains, HMC_OK);
    md.iters.assign(c->nchains, 0);
    md.solves = e->solves;
    md.force_evals = e->force_evals;
    md.hvp_solves = e->hvp_solves;
    int rc = finish_traj_host(c, md, true, std::min(e->logged, kMaxLoggedSolves), info);
    forget_all(c);
    c->traj++;
    return rc;
}

// One trajectory with the chains split into groups: each group runs hmc_trajectory as a
// context of its own, on its own stream and host thread (group 0 on the calling thread and
// the bound stream), after the work already on the bound stream; the bound stream then waits
// for every group.
static int grouped_trajectory(hmc_ctx *c, int scheme, double tau, int n_outer, int n_inner,
                              int prec, hmc_traj_info *info) {
    int rc = build_groups(c);
    if (rc) return rc;
    const int G = c->grp_n;
    HIP_TRY(c, hipEventRecord(c->grp_fork, c->stream));
    for (int g = 1; g < G; ++g) HIP_TRY(c, hipStreamWaitEvent(c->grp[g]->stream, c->grp_fork, 0));
    int rcs[kMaxGroups] = {};
    auto run = [&](int g) {
        hmc_ctx *k = c->grp[g];
        if (hipSetDevice(k->device) != hipSuccess) {
            rcs[g] = fail(k, HMC_E_HIP, "hipSetDevice failed in a chain group");
            return;
        }
        rcs[g] = hmc_trajectory(k, scheme, tau, n_outer, n_inner, prec,
                                info ? info + c->grp_first[g] : nullptr);
    };
    int caller_dev = 0;
    HIP_TRY(c, hipGetDevice(&caller_dev));
    std::thread th[kMaxGroups];
    bool started[kMaxGroups] = {};
    for (int g = 1; g < G; ++g) {
        try {
            th[g] = std::thread(run, g);
            started[g] = true;
        } catch (const std::exception &) {
            run(g);  // no thread: this group runs after the others on the calling thread
        }
    }
    run(0);
    for (int g = 1; g < G; ++g)
        if (started[g]) th[g].join();
    (void)hipSetDevice(caller_dev);
    for (int g = 1; g < G; ++g) {
        HIP_TRY(c, hipEventRecord(c->grp_join[g], c->grp[g]->stream));
        HIP_TRY(c, hipStreamWaitEvent(c->stream, c->grp_join[g], 0));
    }
    forget_all(c);
    c->traj++;
    // a failure of the call itself first; then per-chain failures, a non-finite one before an
    // iteration cap (as a single context reports them)
    int worst = -1;
    for (int g = 0; g < G; ++g) {
        if (!rcs[g]) continue;
        const auto rank = [](int r) { return !chain_failure(r) ? 2 : r == HMC_E_NAN ? 1 : 0; };
        if (worst < 0 || rank(rcs[g]) > rank(rcs[worst])) worst = g;
    }
    if (worst < 0) return HMC_OK;
    c->err = c->grp[worst]->err;
    return rcs[worst];
}

int hmc_trajectory(hmc_ctx *c, int scheme, double tau, int n_outer, int n_inner, int prec,
                   hmc_traj_info *info) {
    CHECK_BOUND(c);
    int rc = check_md_args(c, scheme, tau, n_outer, n_inner, prec);
    if (rc) return rc;
    if (c->graph_on && !c->is_group) {
        // the whole trajectory as one graph when every solve is one persistent-solver kernel;
        // otherwise the solves' iteration slots run as captured chunks (solve)
        int vmax = 0;
        for (const ChainInfo &ci : c->chains) vmax = std::max(vmax, ci.V);
        if (vmax <= persistent_limit(c, prec == HMC_PREC_MIXED))
            return graph_trajectory(c, scheme, tau, n_outer, n_inner, prec, info);
    }
    if (c->groups > 1 && c->nchains > 1)
        return grouped_trajectory(c, scheme, tau, n_outer, n_inner, prec, info);
    MD md;
    init_md(md, c, prec);
    launch_set_u32(c->at<uint32_t>(c->off_trajc), c->traj, c->stream);
    rc = trajectory_body(c, md, scheme, tau, n_outer, n_inner);
    if (rc) return rc;
    rc = finish_traj_host(c, md, true, 0, info);
    c->traj++;
    return rc;
}

int hmc_trajectories_concurrent(hmc_ctx **ctxs, int n, int scheme, double tau, int n_outer,
                                int n_inner, int prec, hmc_traj_info **infos, int *rcs) {
    if (!ctxs || n < 1 || n > kMaxConcurrent) return HMC_E_INVAL;
    for (int k = 0; k < n; ++k) {
        if (!ctxs[k] || !ctxs[k]->ws) return HMC_E_INVAL;
        for (int j = 0; j < k; ++j)
            if (ctxs[j] == ctxs[k] || ctxs[j]->stream == ctxs[k]->stream) return HMC_E_INVAL;
    }
    std::vector<int> rc(n, HMC_OK);
    auto run = [&](int k) {
        if (hipSetDevice(ctxs[k]->device) != hipSuccess) {
            rc[k] = fail(ctxs[k], HMC_E_HIP, "hipSetDevice failed in a concurrent trajectory");
            return;
        }
        rc[k] = hmc_trajectory(ctxs[k], scheme, tau, n_outer, n_inner, prec, infos ? infos[k] : nullptr);
    };
    // the calling thread runs context 0; its current device is restored afterwards
    int caller_dev = 0;
    if (hipGetDevice(&caller_dev) != hipSuccess) return fail(ctxs[0], HMC_E_HIP, "hipGetDevice failed");
    std::vector<std::thread> th;
    for (int k = 1; k < n; ++k) {
        try {
            th.emplace_back(run, k);
        } catch (const std::exception &) {
            rc[k] = fail(ctxs[k], HMC_E_INVAL, "could not start a host thread for a concurrent trajectory");
        }
    }
    run(0);
    for (std::thread &t : th) t.join();
    (void)hipSetDevice(caller_dev);
    int first = HMC_OK;
    for (int k = 0; k < n; ++k) {
        if (rcs) rcs[k] = rc[k];
        if (first == HMC_OK) first = rc[k];
    }
    return first;
}

int hmc_set_graph(hmc_ctx *c, int on) {
    if (!c) return HMC_E_INVAL;
    c->graph_on = on != 0;
    return HMC_OK;
}

int hmc_integrate(hmc_ctx *c, int scheme, double tau, int n_outer, int n_inner, int prec,
                  hmc_traj_info *info) {
    CHECK_BOUND(c);
    int rc = check_md_args(c, scheme, tau, n_outer, n_inner, prec);
    if (rc) return rc;
    MD md;
    init_md(md, c, prec);
    launch_set_u32(c->at<uint32_t>(c->off_trajc), c->traj, c->stream);
    // energies before: refresh sums from the current p; zeta^dagger zeta is not known, so the
    // initial S_F is solved for (stored in the refresh slot)
    const Geo g = c->geo();
    const int C = c->nchains;
    copy_links(c, c->link(LQ), c->link(LQ0));
    copy_links(c, c->link(LP), c->link(LP0));
    double *rs = c->sums() + 7 * C;
    {
        // 1/2 sum p^2 and S_F(q0) = Re phi^dagger xi(q0)
        double *es = c->sums();
        if (!c->quenched) {
            ensure_links(c, c->link(LQ), prec == HMC_PREC_MIXED, c->q_version);
            rc = solve(c, c->spin(SPHI), c->spin(SXI), md.tol, md.max_iter, prec);
            if (rc) return rc;
        }
        launch_energy(g, c->link(LQ), c->link(LQ0), c->link(LP), c->link(LP0),
                      c->quenched ? nullptr : c->spin(SPHI), c->spin(SXI), c->partials(), es,
                      c->stream);
        std::vector<double> h(7 * C), r(2 * C);
        if ((rc = to_host(c, h.data(), es, sizeof(double) * 7 * C))) return rc;
        for (int k = 0; k < C; ++k) { r[k] = h[2 * C + k]; r[C + k] = h[5 * C + k]; }
        HIP_TRY(c, hipMemcpyAsync(rs, r.data(), sizeof(double) * 2 * C, hipMemcpyHostToDevice, c->stream));
        c->xi_version = c->chi_version = -1;
    }
    rc = run_md(md, scheme, tau, n_outer, n_inner);
    if (rc && !chain_failure(rc)) return rc;
    return finish_traj(c, md, false, info);
}

const char *hmc_last_error(const hmc_ctx *c) { return c ? c->err.c_str() : "null context"; }

int hmc_set_timing(hmc_ctx *c, int on) {
    if (!c) return HMC_E_INVAL;
    if (c->ws) {
        int rc = sync(c);
        if (rc) return rc;
    }
    KernelTimer &T = c->timer;
    if (on && !T.sums_host)
        HIP_TRY(c, hipHostMalloc((void **)&T.sums_host, sizeof(double) * 2 * (kMaxSamples + 1),
                                 hipHostMallocDefault));
    if (c->ws)  // rows of samples abandoned by an earlier error start from zero again
        HIP_TRY(c, hipMemsetAsync(c->at<double>(c->off_samples), 0,
                                  sizeof(double) * 2 * (kMaxSamples + 1) * c->nchains, c->stream));
    T.on = on != 0;
    c->graph_epoch++;  // captured chunks bake in whether slots record their bytes
    T.pending.clear();
    T.pool_used = 0;
    T.ms[0] = T.ms[1] = 0.0;
    T.bytes[0] = T.bytes[1] = 0.0;
    T.all_bytes[0] = T.all_bytes[1] = 0.0;
    T.timed[0] = T.timed[1] = 0;
    T.launches = 0;
    for (int g = 0; g < c->grp_n; ++g) {
        int rc = hmc_set_timing(c->grp[g], on);
        if (rc) return fail(c, rc, "chain group timing: %s", c->grp[g]->err.c_str());
    }
    return HMC_OK;
}

int hmc_get_kernel_stats(hmc_ctx *c, int which, hmc_kernel_stat *out) {
    if (!c || !out || which < 0 || which > 1) return HMC_E_INVAL;
    const KernelTimer &T = c->timer;
    out->launches = T.launches;
    out->timed_launches = T.timed[which];
    out->timed_ms = T.ms[which];
    out->timed_bytes = T.bytes[which];
    out->sample_every = T.sample_every;
    out->fused = T.fused ? 1 : 0;
    out->all_bytes = T.all_bytes[which];
    for (int g = 0; g < c->grp_n; ++g) {  // the chain groups' launches add up
        const KernelTimer &K = c->grp[g]->timer;
        out->launches += K.launches;
        out->timed_launches += K.timed[which];
        out->timed_ms += K.ms[which];
        out->timed_bytes += K.bytes[which];
        out->all_bytes += K.all_bytes[which];
        out->fused |= K.fused ? 1 : 0;
    }
    return HMC_OK;
}

int hmc_destroy(hmc_ctx *c) {
    if (!c) return HMC_E_INVAL;
    drop_groups(c);
    drop_chunks(c);
    for (hipStream_t st : c->grp_stream)
        if (st) (void)hipStreamDestroy(st);
    if (c->grp_fork) (void)hipEventDestroy(c->grp_fork);
    for (hipEvent_t e : c->grp_join)
        if (e) (void)hipEventDestroy(e);
    for (GraphEntry &g : c->graphs) drop_graph(g);
    for (hipEvent_t e : c->timer.pool) (void)hipEventDestroy(e);
    if (c->timer.sums_host) (void)hipHostFree(c->timer.sums_host);
    if (c->side) (void)hipStreamDestroy(c->side);
    if (c->fork_ev) (void)hipEventDestroy(c->fork_ev);
    if (c->join_ev) (void)hipEventDestroy(c->join_ev);
    if (c->pinned) (void)hipHostFree(c->pinned);
    delete c;
    return HMC_OK;
}

}  // extern "C"
