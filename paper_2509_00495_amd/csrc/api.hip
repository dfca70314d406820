// libjacobi host side: argument validation, workspace layout, stage
// sequencing and the C ABI.  Every arithmetic step runs in the kernels of
// kernels_*.hip; the host only launches, reads back one convergence scalar
// per sweep and decides when to stop.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <thread>
#include <tuple>
#include <vector>

#include "common.hpp"
#include "internal.hpp"

using namespace lj;

namespace {

thread_local hipError_t g_last_error = hipSuccess;

#define CK(x)                                                                  \
    do {                                                                       \
        hipError_t e_ = (x);                                                   \
        if (e_ != hipSuccess) {                                                \
            g_last_error = e_;                                                 \
            return JACOBI_DEVICE;                                              \
        }                                                                      \
    } while (0)

constexpr double U_D = 0x1p-53; // unit roundoff, double
constexpr double U_L = 0x1p-24; // unit roundoff, single
constexpr double U_H = 0x1p-11; // unit roundoff, binary16

// JACOBI_TRACE set in the environment: one line per block-path sweep on stderr
bool trace_on()
{
    static const bool on = std::getenv("JACOBI_TRACE") != nullptr;
    return on;
}

struct Opts {
    int max_sweeps, block, inner, ns_iters, check_sym, small_max_n, threads, timing, schedule,
        serial_v, tune, graph, pair_skip, gemm_slots, pair_v_split, orth, ladder;
    double c32;
};

// returns 0 or the (positive) index of the offending field
int resolve_opts(const jacobi_opts *o, Opts &r)
{
    r.max_sweeps = 30;
    r.block = 0;
    r.inner = 1;
    r.ns_iters = 0;
    r.check_sym = 0;
    r.small_max_n = 128;
    r.threads = 0;
    r.timing = 0;
    r.schedule = 0;
    r.serial_v = 0;
    r.tune = 0;
    r.graph = 0;
    r.pair_skip = 1;
    r.gemm_slots = 0;
    r.pair_v_split = 0;
    r.orth = 0;
    r.ladder = 0;
    // 0.1: the FP32 stage runs into its quadratic phase, to a few times its
    // rounding floor (off(Q_d^T A Q_d) settles near 0.05 n u_l ||A||_F), which
    // saves FP64 sweeps that cost more than the FP32 ones (measured on GOE and
    // geometric spectra, n = 1024 .. 4096)
    r.c32 = 0.1;
    if (!o)
        return 0;
    r.timing = o->timing != 0;
    if (o->schedule < 0 || o->schedule > 1)
        return 1;
    r.schedule = o->schedule;
    if (o->serial_v < 0 || o->serial_v > 2)
        return 1;
    r.serial_v = o->serial_v;
    if (o->tune < 0 || o->tune > 1)
        return 1;
    r.tune = o->tune;
    r.graph = o->graph != 0;
    r.pair_skip = o->no_pair_skip == 0;
    if (o->gemm_slots < 0 || o->gemm_slots > (1 << 16))
        return 1;
    r.gemm_slots = o->gemm_slots;
    if (o->pair_v_split < -1 || o->pair_v_split > (1 << 16))
        return 1;
    r.pair_v_split = o->pair_v_split;
    if (o->orth < 0 || o->orth > 2)
        return 1;
    r.orth = o->orth;
    if (o->ladder < 0 || o->ladder > 1)
        return 1;
    r.ladder = o->ladder;
    if (o->max_sweeps < 0 || o->max_sweeps > 1000)
        return 1;
    if (o->max_sweeps)
        r.max_sweeps = o->max_sweeps;
    if (o->block != 0 && o->block != 16 && o->block != 32)
        return 1;
    r.block = o->block;
    if (o->inner_sweeps < 0 || o->inner_sweeps > 16)
        return 1;
    if (o->inner_sweeps)
        r.inner = o->inner_sweeps;
    if (o->ns_iters < -1 || o->ns_iters > 8)
        return 1;
    r.ns_iters = o->ns_iters;
    if (std::isnan(o->c32) || o->c32 < 0.0)
        return 1;
    if (o->c32 > 0.0)
        r.c32 = o->c32;
    r.check_sym = o->check_symmetry != 0;
    if (o->small_max_n < -1 || o->small_max_n > 128)
        return 1;
    if (o->small_max_n == -1)
        r.small_max_n = 0;
    else if (o->small_max_n > 0)
        r.small_max_n = o->small_max_n;
    if (o->threads != 0 && o->threads != 256 && o->threads != 512 && o->threads != 1024)
        return 1;
    r.threads = o->threads;
    return 0;
}

struct DevInfo {
    int cus = 0;
    int lds_max = 0;
};

DevInfo dev_info()
{
    static DevInfo cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return DevInfo{};
    DevInfo &d = cache[dev];
    if (d.cus == 0) {
        int v = 0;
        hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev);
        d.cus = v;
        v = 0;
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
        d.lds_max = v;
    }
    return d;
}

// Bump allocator over the caller's workspace; with base == nullptr it only
// measures.
struct Bump {
    char *base;
    size_t off = 0;
    explicit Bump(void *b) : base((char *)b) {}
    template <typename T>
    T *take(size_t count)
    {
        off = (off + 255) & ~(size_t)255;
        T *p = base ? (T *)(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

// block size of the block path by order: 2b x 2b pair tiles of 32 up to
// n = 160, 64 above (measured, plain and mixed, n = 129 .. 512: b = 16 is
// faster at 129, b = 32 from 192 on by 6-16%)
int default_block(int64_t n) { return n <= 160 ? 16 : 32; }

constexpr int NPROBE = 4;           // Rademacher probes of the orthogonality estimate
constexpr int PROBE_BLOCKS = 64;    // workgroups of the probe's residual sums
constexpr double POLISH_FRAC = 0.2; // refresh V when the estimate exceeds this
                                    // fraction of 1e-14 n

struct Geometry {
    int b, N, M, npairs, nbt;
    int64_t npad;
};

Geometry geometry(int64_t n, int block)
{
    Geometry g;
    g.b = block ? block : default_block(n);
    int64_t N = (n + g.b - 1) / g.b;
    if (N < 2)
        N = 2;
    N += N % 2;
    g.N = (int)N;
    g.M = 2 * g.b;
    g.npairs = g.N / 2;
    g.nbt = g.npairs * (g.npairs - 1) / 2;
    g.npad = N * g.b;
    return g;
}

// Buffers of one block-path solve (plain or mixed).
struct BlockWs {
    double *B64, *V64, *U64, *X2, *R, *Vt, *A0, *probe;
    float *B32, *V32, *U32;
    double *partial, *scal, *wtmp, *sg, *cmax, *csq, *cinv;
    double *orth; // mixed: Cholesky block inverses / Householder factors and scratch
    int *flags, *perm, *cidx;
    int *prot; // per-pair rotation flags of a round, double-buffered like U
    int2 *pairs, *psmap;
};

size_t partial_count(const Geometry &g)
{
    // pair solve (one per wavefront) + update of B (one per wavefront and tile)
    size_t c = (size_t)g.npairs * pair_solve_waves(g.M) + (size_t)g.nbt * (g.M / 16);
    c = std::max(c, (size_t)2 * INGEST_BLOCKS); // ingest: sums of squares, then maxima
    c = std::max(c, (size_t)OFF_BLOCKS);
    return c;
}

BlockWs layout_block(Bump &bp, int64_t n, const Geometry &g, bool mixed)
{
    BlockWs w{};
    const size_t nn = (size_t)g.npad * g.npad;
    const size_t uu = (size_t)g.npairs * g.M * g.M;
    w.B64 = bp.take<double>(nn);
    w.V64 = bp.take<double>(nn);
    w.U64 = bp.take<double>(2 * uu); // double-buffered across rounds
    w.probe = bp.take<double>((size_t)g.npad * 2 * NPROBE + (size_t)16 * NPROBE * std::max<int64_t>(n, 1));
    if (!mixed) {
        w.Vt = bp.take<double>(nn);
        w.A0 = bp.take<double>(nn); // the scaled input, when ingest scales it
    }
    if (mixed) {
        w.X2 = bp.take<double>(nn);
        w.R = bp.take<double>(nn);
        w.B32 = bp.take<float>(nn);
        w.V32 = bp.take<float>(nn);
        w.U32 = bp.take<float>(2 * uu);
        // the Cholesky QR's diagonal-block inverses ((npad / CB + 1) CB^2) or
        // the Householder QR's compact factors ((npad / HB + 1) HB^2) and its
        // two HB x npad products, whichever is larger
        const size_t chol = (size_t)(g.npad + ORTH_CB) * ORTH_CB;
        const size_t house = (size_t)(g.npad + ORTH_HB) * ORTH_HB + 2 * (size_t)ORTH_HB * g.npad;
        w.orth = bp.take<double>(chol > house ? chol : house);
    }
    w.partial = bp.take<double>(partial_count(g));
    w.scal = bp.take<double>(8);
    w.flags = bp.take<int>(8);
    w.prot = bp.take<int>((size_t)2 * g.npairs * PROT_STRIDE);
    w.pairs = bp.take<int2>((size_t)(g.N - 1) * g.npairs);
    w.psmap = bp.take<int2>((size_t)g.b * (g.b + 1)); // circle map, then cross map
    w.perm = bp.take<int>((size_t)std::max<int64_t>(n, 1));
    w.wtmp = bp.take<double>((size_t)std::max<int64_t>(n, 1));
    w.sg = bp.take<double>((size_t)std::max<int64_t>(n, 1));
    w.cmax = bp.take<double>((size_t)SIGN_CHUNKS_HOST * std::max<int64_t>(n, 1));
    w.cidx = bp.take<int>((size_t)SIGN_CHUNKS_HOST * std::max<int64_t>(n, 1));
    w.csq = bp.take<double>((size_t)SIGN_CHUNKS_HOST * std::max<int64_t>(n, 1));
    w.cinv = bp.take<double>((size_t)g.npad);
    return w;
}

struct SmallWs {
    SmallDesc *desc;
    int *queue;
    double *vscratch, *info;
    int32_t *status;
};

SmallWs layout_small(Bump &bp, int64_t count, int64_t n_max, int64_t slots)
{
    SmallWs w{};
    w.desc = bp.take<SmallDesc>((size_t)std::max<int64_t>(count, 1));
    w.queue = bp.take<int>(4);
    w.vscratch = bp.take<double>((size_t)slots * small_vt_elems(n_max));
    w.info = bp.take<double>(8);
    w.status = bp.take<int32_t>((size_t)std::max<int64_t>(count, 1));
    return w;
}

// Workgroup size of the one-workgroup solver by the largest order (measured:
// 256 threads are fastest up to n = 64, 1024 from n = 80 on)
int small_threads(int64_t n_max, int req) { return req ? req : (n_max > 72 ? 1024 : 256); }

// LDS pool (doubles) of the one-workgroup solver: S of the largest matrix,
// plus its V when both fit the per-workgroup limit; otherwise as much as the
// limit allows (smaller matrices of a batch then still keep V in LDS).
// Returns 0 when S alone does not fit.
int small_pool(int64_t n_max, int lds_max)
{
    const int m = (int)((n_max + 3) & ~3);
    const int s = m * (m + 1);
    const int want = s + (int)small_vt_elems(n_max);
    if (lds_max <= 0 || small_smem_bytes(m, want) <= (size_t)lds_max)
        return want;
    const size_t fixed = small_smem_bytes(m, 0);
    if (fixed >= (size_t)lds_max)
        return 0;
    // even, so that the scratch after the pool stays 16-byte aligned without
    // growing the allocation
    const int fit = (int)((lds_max - fixed) / sizeof(double)) & ~1;
    return fit >= s ? fit : 0;
}

// Launch configuration of the one-workgroup solver: workgroup size, LDS pool
// (doubles) and persistent grid (resident workgroups, at most one per matrix).
struct SmallCfg {
    int threads, pool;
    int64_t slots;
};

size_t small_slots(int64_t n_max, int count, int threads, int pool)
{
    DevInfo d = dev_info();
    int cus = d.cus > 0 ? d.cus : 256;
    const int m = (int)((n_max + 3) & ~3);
    int per_cu = d.cus > 0 ? small_max_active(m, pool, threads) : 1;
    per_cu = std::max(per_cu, 1);
    return (size_t)std::min<int64_t>((int64_t)cus * per_cu, std::max(count, 1));
}

// The configurations the batched autotuner measures: 256, 512 and 1024
// threads, each with V beside S in LDS (when it fits) and with only S in LDS
// (V in the global scratch, which leaves room for more resident workgroups).
// With a fixed workgroup size (opts.threads) only that size; without tuning,
// the first candidate is the choice by n_max.
constexpr int SMALL_CANDS_MAX = 6;
int small_candidates_fixed(int64_t n_max, int count, int req_threads, int tune,
                           SmallCfg (&out)[SMALL_CANDS_MAX])
{
    int cnt = 0;
    const int lds = dev_info().lds_max;
    const int full = small_pool(n_max, lds);
    if (full == 0)
        return 0;
    const int m = (int)((n_max + 3) & ~3);
    const int s_only = m * (m + 1);
    const int first = small_threads(n_max, req_threads);
    int sizes[3] = {first, 0, 0};
    int nsz = 1;
    if (!req_threads && tune == 0)
        for (int t : {256, 512, 1024})
            if (t != first)
                sizes[nsz++] = t;
    for (int k = 0; k < nsz; ++k) {
        out[cnt++] = {sizes[k], full, (int64_t)small_slots(n_max, count, sizes[k], full)};
        if (tune == 0 && s_only < full)
            out[cnt++] = {sizes[k], s_only, (int64_t)small_slots(n_max, count, sizes[k], s_only)};
    }
    if (tune == 1 && cnt > 1)
        cnt = 1;
    return cnt;
}

void small_candidates(int64_t n_max, int count, int req_threads, int tune,
                      std::vector<SmallCfg> &out)
{
    SmallCfg c[SMALL_CANDS_MAX];
    const int k = small_candidates_fixed(n_max, count, req_threads, tune, c);
    out.assign(c, c + k);
}

size_t ws_small(int64_t count, int64_t n_max, int req_threads, int tune)
{
    std::vector<SmallCfg> c;
    small_candidates(n_max, (int)count, req_threads, tune, c);
    int64_t slots = 1;
    for (const SmallCfg &e : c)
        slots = std::max(slots, e.slots);
    Bump bp(nullptr);
    layout_small(bp, count, n_max, slots);
    return bp.off + 256;
}

// Autotuner cache of the batched path: the configuration measured fastest
// for a (device, largest order, batch size class = bit length of the count,
// requested workgroup size).  Only the workgroup size and the LDS pool are
// kept; the grid is recomputed for each call's count.
struct SmallKey {
    int dev, n_max, bclass, req_threads;
    bool operator<(const SmallKey &o) const
    {
        return std::tie(dev, n_max, bclass, req_threads) <
               std::tie(o.dev, o.n_max, o.bclass, o.req_threads);
    }
};

std::mutex g_small_mu;
std::map<SmallKey, SmallCfg> g_small_tuned;

bool small_tuned(const SmallKey &k, SmallCfg &out)
{
    std::lock_guard<std::mutex> lk(g_small_mu);
    auto it = g_small_tuned.find(k);
    if (it == g_small_tuned.end())
        return false;
    out = it->second;
    return true;
}

void small_tune_store(const SmallKey &k, const SmallCfg &c)
{
    std::lock_guard<std::mutex> lk(g_small_mu);
    g_small_tuned[k] = c;
}

// Graph cache of the batched path: one instantiated graph per distinct set of
// arguments, workspace and configuration.  A graph holds the queue and status
// resets (fill kernels, no memset nodes) and the persistent launch; the
// descriptor upload and the status read-back stay outside it.
struct SmallGraphKey {
    const void *A, *W, *V, *work;
    int64_t batch, layout; // layout: scratch slots the workspace was laid out for
    uint64_t nhash;
    double tol;
    int max_sweeps, threads, pool, slots, dev;
    bool operator<(const SmallGraphKey &o) const
    {
        return std::tie(A, W, V, work, batch, layout, nhash, tol, max_sweeps, threads, pool, slots, dev) <
               std::tie(o.A, o.W, o.V, o.work, o.batch, o.layout, o.nhash, o.tol, o.max_sweeps,
                        o.threads, o.pool, o.slots, o.dev);
    }
};

std::map<SmallGraphKey, hipGraphExec_t> g_small_graphs;
// graphs kept per process; a new key past this runs its launches directly
constexpr size_t SMALL_GRAPHS_MAX = 64;

// Replays the graph cached under `k` on `s`, capturing it first from
// `issue(capture_stream)` when the key is new (or issuing directly on `s`
// once the cache is full).
template <typename F> int small_graph_run(const SmallGraphKey &k, hipStream_t s, F issue)
{
    hipGraphExec_t exec = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_small_mu);
        auto it = g_small_graphs.find(k);
        if (it != g_small_graphs.end())
            exec = it->second;
        else if (g_small_graphs.size() >= SMALL_GRAPHS_MAX)
            return issue(s);
    }
    if (!exec) {
        hipStream_t cs = nullptr;
        CK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
        int bad = e != hipSuccess;
        if (!bad) {
            bad = issue(cs) != 0;
            e = hipStreamEndCapture(cs, &graph);
            bad = bad || e != hipSuccess;
        }
        if (!bad)
            bad = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess;
        if (graph)
            hipGraphDestroy(graph);
        hipStreamDestroy(cs);
        if (bad) {
            g_last_error = e != hipSuccess ? e : hipErrorUnknown;
            return JACOBI_DEVICE;
        }
        std::lock_guard<std::mutex> lk(g_small_mu);
        auto ins = g_small_graphs.emplace(k, exec);
        if (!ins.second) { // another thread stored the same graph meanwhile
            hipGraphExecDestroy(exec);
            exec = ins.first->second;
        }
    }
    CK(hipGraphLaunch(exec, s));
    return 0;
}

size_t ws_block(int64_t n, const Opts &o, bool mixed)
{
    Bump bp(nullptr);
    layout_block(bp, n, geometry(n, o.block), mixed);
    return bp.off + 256;
}

void fill_tables(const Geometry &g, std::vector<int2> &pairs)
{
    pairs.resize((size_t)(g.N - 1) * g.npairs);
    for (int r = 0; r < g.N - 1; ++r)
        for (int k = 0; k < g.npairs; ++k) {
            int p, q;
            rr_pair(k, r, g.N, p, q);
            pairs[(size_t)r * g.npairs + k] = make_int2(p, q);
        }
}

struct Readback {
    double scal[8];
    int flags[8];
};

int read_scalars(const BlockWs &w, hipStream_t s, Readback &rb)
{
    CK(hipMemcpyAsync(rb.scal, w.scal, sizeof(rb.scal), hipMemcpyDeviceToHost, s));
    CK(hipMemcpyAsync(rb.flags, w.flags, sizeof(rb.flags), hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    return 0;
}

// Kernel timing of the block path (opts->timing): every pair-solve, B-update
// and V-update launch records a start and an end event at the kernel itself
// (launched through hipExtLaunchKernel on its stream).  Events are read after
// the per-sweep readback.
struct RoundTimer {
    bool on = false;
    std::vector<hipEvent_t> ev; // 6 per round: pair solve, B update, V update
    double pair_ms = 0.0, apply_ms = 0.0, applyv_ms = 0.0;
    int npair = 0, napply = 0, napplyv = 0;
    int ensure(int rounds)
    {
        while ((int)ev.size() < 6 * rounds) {
            hipEvent_t e;
            CK(hipEventCreate(&e));
            ev.push_back(e);
        }
        return 0;
    }
    ~RoundTimer()
    {
        for (hipEvent_t e : ev)
            hipEventDestroy(e);
    }
    int collect(int rounds)
    {
        for (int r = 0; r < rounds; ++r) {
            float a = 0.f, b = 0.f, c = 0.f;
            CK(hipEventElapsedTime(&a, ev[6 * r], ev[6 * r + 1]));
            CK(hipEventElapsedTime(&b, ev[6 * r + 2], ev[6 * r + 3]));
            CK(hipEventElapsedTime(&c, ev[6 * r + 4], ev[6 * r + 5]));
            pair_ms += a;
            apply_ms += b;
            applyv_ms += c;
        }
        npair += rounds;
        napply += rounds;
        napplyv += rounds;
        return 0;
    }
    void store(jacobi_info *info, int idx) const
    {
        if (!info)
            return;
        info->t_pair_ms[idx] = pair_ms;
        info->t_apply_ms[idx] = apply_ms;
        info->t_applyv_ms[idx] = applyv_ms;
        info->n_pair[idx] = npair;
        info->n_apply[idx] = napply;
        info->n_applyv[idx] = napplyv;
    }
};

// Side stream for the V updates of the block path (overlapped mode, see
// run_sweeps).  Non-blocking and default priority.
struct SideStream {
    hipStream_t s2 = nullptr;
    hipEvent_t evU[2] = {nullptr, nullptr}, evV[2] = {nullptr, nullptr};
    bool recV[2] = {false, false}; // evV[j] recorded at least once (a stage on
                                   // one stream records none)
    int64_t round = 0;             // rounds issued so far (across stages)
    int init()
    {
        CK(hipStreamCreateWithFlags(&s2, hipStreamNonBlocking));
        for (int j = 0; j < 2; ++j) {
            CK(hipEventCreateWithFlags(&evU[j], hipEventDisableTiming));
            CK(hipEventCreateWithFlags(&evV[j], hipEventDisableTiming));
        }
        return 0;
    }
    ~SideStream()
    {
        for (int j = 0; j < 2; ++j) {
            if (evU[j])
                hipEventDestroy(evU[j]);
            if (evV[j])
                hipEventDestroy(evV[j]);
        }
        if (s2) {
            hipStreamSynchronize(s2);
            hipStreamDestroy(s2);
        }
    }
};

template <typename T>
int run_sweeps(const Geometry &g, int64_t n, const BlockWs &w, T *B, T *V, T *U, double tol,
               double eps, int max_sweeps, int inner, int schedule, int serial_v,
               bool pair_skip, int stage, int vsplit,
               hipStream_t s,
               SideStream &ss, int *sweeps_out, double *off_out, double *off0_out,
               RoundTimer *tm, int *skipped_out)
{
    Readback rb;
    if (tm && tm->on)
        if (int e = tm->ensure(g.N - 1))
            return e;
    CK(launch_off2_partial<T>(B, g.npad, w.partial, s));
    CK(launch_sum(w.partial, OFF_BLOCKS, w.scal + 1, s));
    if (int e = read_scalars(w, s, rb))
        return e;
    double off = std::sqrt(rb.scal[1]);
    if (off0_out)
        *off0_out = off;
    if (!std::isfinite(off))
        return JACOBI_NONFINITE; // the starting matrix (e.g. Q_d^T A Q_d) holds Inf or NaN
    int sweeps = 0;
    int status = JACOBI_OK;
    const double thr = n > 0 ? tol / (double)n : 0.0;
    const size_t ustride = (size_t)g.npairs * g.M * g.M;
    // The V update of round r needs only U_r.  Default: it rides in the launch
    // of round r + 1's pair solves, on the compute units they leave free (the
    // pair solves are latency-bound and take one unit per block pair); the
    // last round's update is launched on its own after the sweeps.  Without
    // it (and with per-launch timing, which times the kernels one by one) the
    // update runs after the B update on the same stream (serial_v = 1) or on a
    // side stream beside round r + 1 (serial_v = 2; U is double-buffered and
    // the pair solve of round r + 2, which overwrites U_r's buffer, waits for
    // it).  Measured at n = 4096: the shared launch is fastest in both
    // precisions; each cross-stream event adds a gap of several microseconds,
    // and a pair solve beside a running V update slows down.
    const bool side = serial_v == 2;
    const bool fuse = serial_v == 0;
    const int2 *vpend_pairs = nullptr; // V update waiting for the next launch
    const T *vpend_U = nullptr;
    const int *vpend_prot = nullptr;
    // Pair skipping (FP64 sweeps): a pair solve that applies no rotation
    // (every coupling passes the skip test of the rotation) leaves U = I
    // exactly; the B tiles of two such pairs and the V columns of such a pair
    // are then left out of the round's updates, which changes no result.
    // flags[3] counts the B tiles left out.  The FP32 stage runs without it
    // (null flags): there the flag store slows the pair solve, which sets the
    // pace of its rounds, by more than the skips return.
    while (off > tol) {
        if (sweeps >= max_sweeps) {
            status = JACOBI_NOCONV;
            break;
        }
        CK(launch_fill_i32(w.flags + 2, 1, 0, s));
        const bool timed = tm && tm->on;
        for (int r = 0; r < g.N - 1; ++r, ++ss.round) {
            const int j = (int)(ss.round & 1);
            T *Ub = U + j * ustride;
            int *pf = w.prot + (size_t)j * g.npairs * PROT_STRIDE; // written by FP64 solves
            const int *pfc = sizeof(T) == 8 && pair_skip ? pf : nullptr; // read by the updates
            const int2 *pr = w.pairs + (size_t)r * g.npairs;
            if (side && ss.recV[j])
                CK(hipStreamWaitEvent(s, ss.evV[j], 0));
            const int cross = schedule == 0 && r > 0;
            const int2 *map = w.psmap + (cross ? (size_t)g.b * (g.b + 1) / 2 : 0);
            if (vpend_pairs) {
                CK(launch_pair_solve_v<T>(B, g.npad, g.b, g.npairs, pr, map, Ub, eps, thr, inner,
                                          stage == 2, cross, w.partial, w.flags + 2, pf, V, g.npad,
                                          g.npad, vpend_pairs, vpend_U, vpend_prot, s, vsplit,
                                          timed ? tm->ev[6 * r] : nullptr,
                                          timed ? tm->ev[6 * r + 1] : nullptr));
                vpend_pairs = nullptr;
            } else {
                CK(launch_pair_solve<T>(B, g.npad, g.b, g.npairs, pr, map, Ub, eps, thr, inner,
                                        stage == 2, cross, w.partial, w.flags + 2, pf, s,
                                        timed ? tm->ev[6 * r] : nullptr,
                                        timed ? tm->ev[6 * r + 1] : nullptr));
            }
            if (side)
                CK(hipEventRecord(ss.evU[j], s));
            CK(launch_update_b<T>(B, g.npad, g.b, g.npairs, pr, Ub,
                                  w.partial + (size_t)g.npairs * pair_solve_waves(g.M),
                                  r == g.N - 2, stage == 2, pfc, w.flags + 3, s,
                                  timed ? tm->ev[6 * r + 2] : nullptr,
                                  timed ? tm->ev[6 * r + 3] : nullptr));
            if (fuse) {
                vpend_pairs = pr;
                vpend_U = Ub;
                vpend_prot = pfc;
                if (timed) { // this round's V update is timed inside the next launch
                    CK(hipEventRecord(tm->ev[6 * r + 4], s));
                    CK(hipEventRecord(tm->ev[6 * r + 5], s));
                }
                continue;
            }
            hipStream_t sv = side ? ss.s2 : s;
            if (side)
                CK(hipStreamWaitEvent(ss.s2, ss.evU[j], 0));
            CK(launch_update_v<T>(V, g.npad, g.npad, g.b, g.npairs, pr, Ub, pfc, sv,
                                  timed ? tm->ev[6 * r + 4] : nullptr,
                                  timed ? tm->ev[6 * r + 5] : nullptr));
            if (side) {
                CK(hipEventRecord(ss.evV[j], ss.s2));
                ss.recV[j] = true;
            }
        }
        // partials: one per wavefront of each pair solve, then one per
        // wavefront of each B tile
        CK(launch_sum(w.partial,
                      (int64_t)g.npairs * pair_solve_waves(g.M) + (int64_t)g.nbt * (g.M / 16),
                      w.scal + 1, s));
        if (int e = read_scalars(w, s, rb))
            return e;
        if (timed) {
            if (ss.s2)
                CK(hipStreamSynchronize(ss.s2));
            if (int e = tm->collect(g.N - 1))
                return e;
        }
        ++sweeps;
        const double prev = off;
        off = std::sqrt(rb.scal[1]);
        if (trace_on())
            std::fprintf(stderr, "jacobi: %s sweep %d off %.3e rotated %d\n",
                         stage == 2 ? "fp16" : (stage == 1 ? "fp32" : "fp64"), sweeps, off,
                         rb.flags[2]);
        if (!std::isfinite(off)) {
            status = JACOBI_NONFINITE;
            break;
        }
        if (!rb.flags[2])
            break; // no pair rotated: converged by the per-pair test
        if (stage == 1 && off >= prev)
            break; // the FP32 rounding floor
        if (stage == 2 && off > 0.9 * prev)
            break; // the binary16 rounding floor: a sweep lowers off by less than 10%
    }
    if (vpend_pairs)
        CK(launch_update_v<T>(V, g.npad, g.npad, g.b, g.npairs, vpend_pairs, vpend_U, vpend_prot,
                              s));
    // V is complete on the caller's stream from here on
    if (side && ss.round > 0 && ss.recV[(ss.round - 1) & 1])
        CK(hipStreamWaitEvent(s, ss.evV[(ss.round - 1) & 1], 0));
    *sweeps_out = sweeps;
    *off_out = off;
    if (skipped_out)
        *skipped_out = rb.flags[3]; // read after the last sweep
    return status;
}

int setup_block(const Geometry &g, const BlockWs &w, hipStream_t s)
{
    std::vector<int2> pairs;
    fill_tables(g, pairs);
    CK(hipMemcpyAsync(w.pairs, pairs.data(), pairs.size() * sizeof(int2), hipMemcpyHostToDevice,
                      s));
    const size_t nblk = (size_t)g.b * (g.b + 1) / 2;
    std::vector<int2> psmap(2 * nblk);
    pair_solve_map(g.M, 0, psmap.data());
    pair_solve_map(g.M, 1, psmap.data() + nblk);
    CK(hipMemcpyAsync(w.psmap, psmap.data(), psmap.size() * sizeof(int2), hipMemcpyHostToDevice,
                      s));
    CK(launch_fill_i32(w.flags, 8, 0, s));
    CK(launch_fill_i32(w.prot, (int64_t)2 * g.npairs * PROT_STRIDE, 0, s));
    CK(hipStreamSynchronize(s)); // the host tables go out of scope
    return 0;
}

int validate_common(const double *A, int64_t n, int64_t lda, double *W, double *V, int64_t ldv,
                    double tol, const jacobi_opts *opts, Opts &o)
{
    if (n < 0)
        return -2;
    if (n > 0 && !A)
        return -1;
    if (lda < std::max<int64_t>(1, n))
        return -3;
    if (n > 0 && !W)
        return -4;
    if (n > 0 && !V)
        return -5;
    if (ldv < std::max<int64_t>(1, n))
        return -6;
    if (std::isnan(tol) || std::isinf(tol))
        return -7;
    if (resolve_opts(opts, o))
        return -8;
    if (n > (int64_t)1 << 20)
        return -2;
    return 0;
}

struct WsGuard {
    void *p = nullptr;
    hipStream_t s = nullptr;
    ~WsGuard()
    {
        if (p) {
            hipStreamSynchronize(s);
            hipFree(p);
        }
    }
};

void fill_info(jacobi_info *info, int sweeps, int sweeps32, int ns, int path, int block,
               double normf, double tol, double off, double off32, double offc, double orth)
{
    if (!info)
        return;
    std::memset(info, 0, sizeof(*info));
    info->sweeps = sweeps;
    info->sweeps32 = sweeps32;
    info->ns_iters = ns;
    info->path = path;
    info->block = block;
    info->norm_f = normf;
    info->tol = tol;
    info->off_final = off;
    info->off32 = off32;
    info->off_cond = offc;
    info->orth_ns = orth;
}

// ---- one matrix on the one-workgroup solver
int eigh_small(const double *A, int64_t n, int64_t lda, double *W, double *V, int64_t ldv,
               double tol, const Opts &o, void *work, hipStream_t s, jacobi_info *info)
{
    // one matrix: the solve's latency is all that counts, so the whole
    // compute unit's 1024 threads (the batched default of 256 threads for
    // n <= 72 is for throughput, several workgroups per compute unit)
    const int threads = o.threads ? o.threads : 1024;
    Bump bp(work);
    SmallWs w = layout_small(bp, 1, n, 1);
    SmallDesc d{};
    d.a_off = 0;
    d.w_off = 0;
    d.v_off = 0;
    d.n = (int)n;
    d.lda = (int)lda;
    d.ldv = (int)ldv;
    d.orig = 0;
    d.info = w.info;
    CK(hipMemcpyAsync(w.desc, &d, sizeof(d), hipMemcpyHostToDevice, s));
    CK(launch_fill_i32(w.queue, 1, 0, s));
    const DevInfo dv = dev_info();
    const int m = (int)((n + 3) & ~3);
    const int pool = small_pool(n, dv.lds_max);
    CK(launch_small(A, W, V, w.desc, 1, w.queue, tol, o.max_sweeps, w.vscratch,
                    small_vt_elems(n), pool, m, threads, 1, w.status, s));
    double hinfo[4] = {0, 0, 0, 0};
    int32_t st = 0;
    CK(hipMemcpyAsync(hinfo, w.info, sizeof(hinfo), hipMemcpyDeviceToHost, s));
    CK(hipMemcpyAsync(&st, w.status, sizeof(st), hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    fill_info(info, (int)hinfo[0], 0, 0, 0, 0, hinfo[1], hinfo[2], hinfo[3], 0, 0, 0);
    return st;
}

// Output stage of the block path.  W is read off the diagonal of B.  The
// output columns are those of the accumulated V scaled to unit norm (the
// rounding of the rotations moves the column norms by a random walk, which is
// nearly all of V's departure from orthogonality; the columns stay orthogonal
// to each other far more closely).  The orthogonality of the normalized V is
// estimated from NPROBE Rademacher probes x (||D^-1 V^T V D^-1 x - x||, with
// D = diag of the column norms, O(n^2) work) and, when the estimate exceeds
// POLISH_FRAC * 1e-14 n, V gets one Newton-Schulz step
// V <- V + V (I - V^T V) / 2 (the paper's orthogonaliser, Section 4.3.4),
// which squares its departure from orthogonality, and the column statistics
// are taken again.  Rbuf and Vbuf are free npad x npad scratch buffers (Rbuf
// may alias B: the diagonal is extracted first).
// A_rq != nullptr: the eigenvalues are the Rayleigh quotients of the final
// normalized eigenvectors against the input (T = A V is formed in Rbuf)
// instead of the diagonal of B.  The plain FP64 path uses this: after its
// many sweeps of blockwise updates the rounding accumulated in the diagonal of
// B exceeds what the eigenvectors themselves allow.
// The output stage in two parts, so that a batch reads every matrix's
// estimate back at once: finalize_probe issues the diagonal, the column
// statistics and the probe (its sum lands in w.scal[3]); finalize_finish takes
// the estimate read back and issues the rest.
int finalize_probe(const Geometry &g, int64_t n, const BlockWs &w, const double *B,
                   const double *Vin, hipStream_t s)
{
    const int64_t np = g.npad;
    CK(launch_diag(B, np, n, w.wtmp, s));
    CK(launch_colstats(Vin, np, n, np, w.cmax, w.cidx, w.csq, w.cinv, s));
    double *X = w.probe, *Y = w.probe + np * NPROBE, *P = w.probe + 2 * np * NPROBE;
    CK(launch_rademacher(X, np, n, NPROBE, 0x5eedull, s));
    CK(launch_orth_probe(Vin, np, n, np, NPROBE, X, w.cinv, Y, P, w.partial, PROBE_BLOCKS, s));
    CK(launch_sum(w.partial, PROBE_BLOCKS, w.scal + 3, s));
    return 0;
}

int finalize_finish(const Geometry &g, int64_t n, const BlockWs &w, double probe_sum,
                    const double *Vin, double *Rbuf, double *Vbuf, double *W, double *V,
                    int64_t ldv, hipStream_t s, double *orth_est, int *polished,
                    const double *A_rq, int64_t lda)
{
    const int64_t np = g.npad;
    const double est = std::sqrt(probe_sum / NPROBE);
    *orth_est = est;
    *polished = 0;
    const double *Vf = Vin;
    if (!(est <= POLISH_FRAC * 1e-14 * (double)n)) {
        CK(launch_gemm64_sym(1, 0, np, np, -1.0, Vin, np, Vin, np, 0.0, nullptr, 0, 1.0, Rbuf,
                             np, s, Vbuf, np * np));
        CK(launch_gemm64(0, 0, np, np, np, 0.5, Vin, np, 0, Rbuf, np, 0, 1.0, Vin, np, 0, 0.0,
                         Vbuf, np, 0, 1, s));
        Vf = Vbuf;
        *polished = 1;
        CK(launch_colstats(Vf, np, n, np, w.cmax, w.cidx, w.csq, w.cinv, s));
    }
    if (A_rq) {
        CK(launch_gemm64(0, 0, n, n, n, 1.0, A_rq, lda, 0, Vf, np, 0, 0.0, nullptr, 0, 0, 0.0,
                         Rbuf, np, 0, 1, s));
        CK(launch_rayleigh(Vf, np, Rbuf, np, n, w.cinv, w.csq, w.wtmp, s));
    }
    CK(launch_fill_i32(w.perm, n, 0, s));
    CK(launch_finalize(w.wtmp, Vf, np, n, W, V, ldv, w.perm, w.sg, w.cmax, w.cidx, w.cinv, s));
    return 0;
}

int finalize_block(const Geometry &g, int64_t n, const BlockWs &w, const double *B,
                   const double *Vin, double *Rbuf, double *Vbuf, double *W, double *V,
                   int64_t ldv, hipStream_t s, double *orth_est, int *polished,
                   const double *A_rq = nullptr, int64_t lda = 0)
{
    if (int e = finalize_probe(g, n, w, B, Vin, s))
        return e;
    Readback rb;
    if (int e = read_scalars(w, s, rb))
        return e;
    return finalize_finish(g, n, w, rb.scal[3], Vin, Rbuf, Vbuf, W, V, ldv, s, orth_est,
                           polished, A_rq, lda);
}

// Exponent k of the exact scaling B <- 2^k B applied on ingest: inputs whose
// largest entry lies outside [2^-100, 2^100] are scaled so that it lands in
// [1, 2).  Jacobi rotations, the stopping rules and every product are
// invariant under a power-of-two scaling except for over- and underflow; the
// scaling keeps the sums of squares (||A||_F, off), the squared per-pair test
// and the FP32 stage of the mixed path in range.  Eigenvalues are scaled back
// by 2^-k, eigenvectors are unaffected.
int scale_exponent(double amax) { return scale_exp_of(amax); }

// Ingest of the block path: B = sym(A) zero-padded, the non-finite and
// symmetry checks, the scaling exponent ks (B, and copy when not null, then
// hold 2^ks sym(A)) and ||B||_F of the scaled matrix.
int ingest_norm(const double *A, int64_t lda, int64_t n, const Geometry &g, const BlockWs &w,
                double *B, double *copy, int check_sym, hipStream_t s, double &normf, int &ks,
                double *amax_out = nullptr)
{
    CK(launch_ingest<double>(A, lda, n, B, g.npad, w.partial, w.flags, check_sym, s));
    CK(launch_sum(w.partial, INGEST_BLOCKS, w.scal, s));
    CK(launch_max(w.partial + INGEST_BLOCKS, INGEST_BLOCKS, w.scal + 4, s));
    Readback rb;
    if (int e = read_scalars(w, s, rb))
        return e;
    if (rb.flags[0])
        return JACOBI_NONFINITE;
    if (check_sym && rb.flags[1])
        return JACOBI_NOTSYM;
    ks = scale_exponent(rb.scal[4]);
    if (amax_out)
        *amax_out = std::ldexp(rb.scal[4], ks);
    if (ks) {
        const int64_t nn = g.npad * g.npad;
        CK(launch_scale_pow2(B, nn, ks, copy, s));
        CK(launch_sq_partial(B, nn, w.partial, s));
        CK(launch_sum(w.partial, OFF_BLOCKS, w.scal, s));
        if (int e = read_scalars(w, s, rb))
            return e;
    }
    normf = std::sqrt(rb.scal[0]);
    return 0;
}

// info fields in the caller's scale: norm, tolerance and off values of a
// solve that ran on 2^ks sym(A)
void unscale_info(jacobi_info *info, int ks)
{
    if (!info || !ks)
        return;
    info->norm_f = std::ldexp(info->norm_f, -ks);
    info->tol = std::ldexp(info->tol, -ks);
    info->off_final = std::ldexp(info->off_final, -ks);
    info->off32 = std::ldexp(info->off32, -ks);
    info->off_cond = std::ldexp(info->off_cond, -ks);
}

int eigh_block(const double *A, int64_t n, int64_t lda, double *W, double *V, int64_t ldv,
               double tol_in, const Opts &o, void *work, hipStream_t s, jacobi_info *info)
{
    const Geometry g = geometry(n, o.block);
    Bump bp(work);
    BlockWs w = layout_block(bp, n, g, false);
    if (int e = setup_block(g, w, s))
        return e;
    double normf = 0.0;
    int ks = 0;
    if (int e = ingest_norm(A, lda, n, g, w, w.B64, w.A0, o.check_sym, s, normf, ks))
        return e;
    CK(launch_eye<double>(w.V64, g.npad, s));
    const double tol = tol_in > 0.0 ? std::ldexp(tol_in, ks) : 1e-15 * (double)n * normf;
    int sweeps = 0, skipped = 0;
    double off = 0.0;
    RoundTimer tm;
    tm.on = o.timing;
    SideStream ss; // its stream and events exist only for serial_v = 2
    if (o.serial_v == 2)
        if (int e = ss.init())
            return e;
    int st = run_sweeps<double>(g, n, w, w.B64, w.V64, w.U64, tol, U_D, o.max_sweeps, o.inner,
                                o.schedule, o.serial_v, o.pair_skip, 0, o.pair_v_split, s,
                                ss, &sweeps, &off, nullptr, &tm, &skipped);
    if (st == JACOBI_DEVICE || st == JACOBI_NONFINITE)
        return st;
    double est = 0.0;
    int pol = 0;
    // eigenvalues: Rayleigh quotients against the (scaled) symmetrised input
    if (int e = finalize_block(g, n, w, w.B64, w.V64, w.B64, w.Vt, W, V, ldv, s, &est, &pol,
                               ks ? w.A0 : A, ks ? g.npad : lda))
        return e;
    if (ks)
        CK(launch_scale_pow2(W, n, -ks, nullptr, s));
    CK(hipStreamSynchronize(s));
    fill_info(info, sweeps, 0, 0, 1, g.b, normf, tol, off, 0, 0, 0);
    unscale_info(info, ks);
    if (info) {
        info->orth_est = est;
        info->polished = pol;
        info->skipped_tiles = skipped;
    }
    tm.store(info, 0);
    return st;
}

int eigh_mixed_block(const double *A, int64_t n, int64_t lda, double *W, double *V,
                     int64_t ldv, double tol_in, const Opts &o, void *work, hipStream_t s,
                     jacobi_info *info)
{
    const Geometry g = geometry(n, o.block);
    Bump bp(work);
    BlockWs w = layout_block(bp, n, g, true);
    if (int e = setup_block(g, w, s))
        return e;
    const int64_t nn = g.npad * g.npad;
    // ingest: A64 = sym(A) (kept for the preconditioning product), B32 = fl32(A64)
    double *A64 = w.B64;
    double normf = 0.0, amax = 0.0;
    int ks = 0;
    if (int e = ingest_norm(A, lda, n, g, w, A64, nullptr, o.check_sym, s, normf, ks, &amax))
        return e;
    RoundTimer tm32, tm64, tm16;
    tm32.on = tm64.on = tm16.on = o.timing;
    SideStream ss; // its stream and events exist only for serial_v = 2
    if (o.serial_v == 2)
        if (int e = ss.init())
            return e;
    CK(launch_eye<float>(w.V32, g.npad, s));
    // stage 0 (ladder = 1): the binary16 stage.  Its matrix is fl16(2^kh A),
    // scaled by an exact power of two so that the largest entry lies in
    // [1, 2) (the entries of the iterates stay below ||A||_2 <= n max|a_ij|,
    // inside the binary16 range for n up to 2^14), every stored entry rounded to
    // binary16; V accumulates in FP32.  It stops when a sweep lowers off by
    // less than 10% (the binary16 rounding floor; early sweeps of a dense
    // matrix can lower it by only about a half) or at off <= 0.01 n u_h ||A||_F.  Then
    // B32 = fl32(Q_h^T A Q_h) (FP64 products) and the FP32 stage continues from
    // V = Q_h.
    int sw16 = 0;
    double off16 = 0.0;
    if (o.ladder == 1) {
        int e2 = 0;
        std::frexp(amax > 0.0 ? amax : 1.0, &e2);
        const int kh = 1 - e2;
        CK(launch_cast_f32_scaled(A64, w.B32, nn, kh, 1, s));
        const double tol16 = 0.01 * (double)n * U_H * std::ldexp(normf, kh);
        int st16 = run_sweeps<float>(g, n, w, w.B32, w.V32, w.U32, tol16, U_H, o.max_sweeps,
                                     o.inner, o.schedule, o.serial_v, o.pair_skip, 2,
                                     o.pair_v_split, s, ss, &sw16, &off16, nullptr, &tm16,
                                     nullptr);
        if (st16 == JACOBI_DEVICE || st16 == JACOBI_NONFINITE)
            return st16;
        off16 = std::ldexp(off16, -kh);
        double *Xh = w.V64, *T = w.R, *Bh = w.X2;
        CK(launch_widen_f64(w.V32, Xh, nn, s));
        CK(launch_gemm64(0, 0, g.npad, g.npad, g.npad, 1.0, A64, g.npad, 0, Xh, g.npad, 0, 0.0,
                         nullptr, 0, 0, 0.0, T, g.npad, 0, 1, s));
        CK(launch_gemm64_sym(1, 0, g.npad, g.npad, 1.0, Xh, g.npad, T, g.npad, 0.0, nullptr, 0,
                             0.0, Bh, g.npad, s));
        CK(launch_cast_f32(Bh, w.B32, nn, s));
    } else {
        CK(launch_cast_f32(A64, w.B32, nn, s));
    }
    // stage 1: FP32 Jacobi -> Q_l
    const double tol32 = o.c32 * (double)n * U_L * normf;
    int sw32 = 0;
    double off32 = 0.0;
    int st32 = run_sweeps<float>(g, n, w, w.B32, w.V32, w.U32, tol32, U_L, o.max_sweeps,
                                 o.inner, o.schedule, o.serial_v, o.pair_skip, 1,
                                 o.pair_v_split, s, ss, &sw32, &off32, nullptr, &tm32, nullptr);
    if (st32 == JACOBI_DEVICE || st32 == JACOBI_NONFINITE)
        return st32;
    // stage 2: Q_l -> Q_d.  Newton-Schulz (default): X <- X + X (I - X^T X) / 2
    // (= X (3I - X^T X) / 2); or the Q factor of a Householder or Cholesky QR
    // of Q_l.  Qd ends in one of V64 / X2 / R, T1 and T2 are the two others
    // (free n_pad^2 buffers for the products below).
    double *X = w.V64, *X2 = w.X2, *R = w.R;
    CK(launch_widen_f64(w.V32, X, nn, s));
    // ||Q_l^T Q_l - I||_F (stage diagnostic, into scal[6]): Newton-Schulz
    // computes I - X^T X in its first step anyway; for the QR orthogonalisers
    // it costs a product of its own, made only with opts.timing (R and X2 are
    // free until the factorisation starts)
    double orth_ql = 0.0;
    const bool ql_diag = o.orth == 0 || o.timing;
    if (o.orth != 0 && o.timing) {
        CK(launch_gemm64_sym(1, 0, g.npad, g.npad, -1.0, X, g.npad, X, g.npad, 0.0, nullptr, 0,
                             1.0, R, g.npad, s, X2, nn, o.gemm_slots));
        CK(launch_sq_partial(R, nn, w.partial, s));
        CK(launch_sum(w.partial, OFF_BLOCKS, w.scal + 6, s));
    }
    hipEvent_t eo0 = nullptr, eo1 = nullptr;
    if (o.timing) {
        CK(hipEventCreate(&eo0));
        CK(hipEventCreate(&eo1));
        CK(hipEventRecord(eo0, s));
    }
    double *Qd = X, *T1 = R, *T2 = X2;
    int ns = 0;
    double orth = 0.0;
    if (o.orth == 1) {
        double *Ts = w.orth, *Wb = Ts + (g.npad / ORTH_HB + 1) * ORTH_HB * ORTH_HB,
               *W2b = Wb + (size_t)ORTH_HB * g.npad;
        CK(householder_qr(X, X2, R, g.npad, g.npad, Ts, Wb, W2b, s));
        Qd = X2;
        T1 = R;
        T2 = X;
    } else if (o.orth == 2) {
        CK(launch_fill_i32(w.flags + 4, 1, 0, s));
        CK(cholesky_qr(X, R, R, X2, g.npad, g.npad, w.orth, w.flags + 4, s));
        Qd = R;
        T1 = X;
        T2 = X2;
    } else {
        const int fixed = o.ns_iters > 0 ? o.ns_iters : (n < 52000 ? 2 : 3);
        const bool adaptive = o.ns_iters == -1;
        const int max_it = adaptive ? 3 : fixed;
        for (int it = 0; it < max_it; ++it) {
            CK(launch_gemm64_sym(1, 0, g.npad, g.npad, -1.0, X, g.npad, X, g.npad, 0.0, nullptr,
                                 0, 1.0, R, g.npad, s, X2, nn, o.gemm_slots));
            if (it == 0) {
                CK(launch_sq_partial(R, nn, w.partial, s));
                CK(launch_sum(w.partial, OFF_BLOCKS, w.scal + 6, s));
            }
            if (adaptive || it == max_it - 1) {
                CK(launch_sq_partial(R, nn, w.partial, s));
                CK(launch_sum(w.partial, OFF_BLOCKS, w.scal + 2, s));
                Readback rb;
                if (int e = read_scalars(w, s, rb))
                    return e;
                orth = std::sqrt(rb.scal[2]);
                orth_ql = std::sqrt(rb.scal[6]);
                if (adaptive && orth <= (double)n * U_D)
                    break;
            }
            CK(launch_gemm64(0, 0, g.npad, g.npad, g.npad, 0.5, X, g.npad, 0, R, g.npad, 0, 1.0,
                             X, g.npad, 0, 0.0, X2, g.npad, 0, 1, s));
            std::swap(X, X2);
            ++ns;
        }
        Qd = X;
        T1 = R;
        T2 = X2;
    }
    double orth_qd = 0.0, t_orth = 0.0;
    if (o.timing) {
        CK(hipEventRecord(eo1, s));
        // ||Q_d^T Q_d - I||_F of the orthogonaliser's output (diagnostic)
        CK(launch_gemm64_sym(1, 0, g.npad, g.npad, -1.0, Qd, g.npad, Qd, g.npad, 0.0, nullptr, 0,
                             1.0, T1, g.npad, s, T2, nn, o.gemm_slots));
        CK(launch_sq_partial(T1, nn, w.partial, s));
        CK(launch_sum(w.partial, OFF_BLOCKS, w.scal + 5, s));
        Readback rb;
        if (int e = read_scalars(w, s, rb))
            return e;
        orth_qd = std::sqrt(rb.scal[5]);
        if (ql_diag)
            orth_ql = std::sqrt(rb.scal[6]);
        float ms = 0.0f;
        CK(hipEventElapsedTime(&ms, eo0, eo1));
        t_orth = ms;
        hipEventDestroy(eo0);
        hipEventDestroy(eo1);
    }
    if (o.orth == 2) {
        Readback rb;
        if (int e = read_scalars(w, s, rb))
            return e;
        if (rb.flags[4])
            return JACOBI_NONFINITE; // Q_l^T Q_l not positive definite
    }
    // stage 3: B = Q_d^T A Q_d, symmetric by construction (upper tiles of the
    // second product mirrored), then FP64 Jacobi from V = Q_d
    CK(launch_gemm64(0, 0, g.npad, g.npad, g.npad, 1.0, A64, g.npad, 0, Qd, g.npad, 0, 0.0,
                     nullptr, 0, 0, 0.0, T1, g.npad, 0, 1, s));
    CK(launch_gemm64_sym(1, 0, g.npad, g.npad, 1.0, Qd, g.npad, T1, g.npad, 0.0, nullptr, 0, 0.0,
                         A64, g.npad, s, T2, nn, o.gemm_slots));
    X = Qd;
    const double tol = tol_in > 0.0 ? std::ldexp(tol_in, ks) : 1e-15 * (double)n * normf;
    int sw64 = 0, skipped = 0;
    double off = 0.0, offc = 0.0;
    int st = run_sweeps<double>(g, n, w, A64, X, w.U64, tol, U_D, o.max_sweeps, o.inner,
                                o.schedule, o.serial_v, o.pair_skip, 0, o.pair_v_split, s,
                                ss, &sw64, &off, &offc, &tm64, &skipped);
    if (st == JACOBI_DEVICE || st == JACOBI_NONFINITE)
        return st;
    double est = 0.0;
    int pol = 0;
    if (int e = finalize_block(g, n, w, A64, X, A64, T1, W, V, ldv, s, &est, &pol))
        return e;
    if (ks)
        CK(launch_scale_pow2(W, n, -ks, nullptr, s));
    CK(hipStreamSynchronize(s));
    fill_info(info, sw64, sw32, ns, 1, g.b, normf, tol, off, off32, offc, orth);
    unscale_info(info, ks);
    if (info) {
        info->orth_qd = orth_qd;
        info->t_orth_ms = t_orth;
        info->sweeps16 = sw16;
        info->off16 = std::ldexp(off16, -ks);
        info->orth_ql = orth_ql;
    }
    if (info) {
        info->orth_est = est;
        info->polished = pol;
        info->skipped_tiles = skipped;
    }
    tm64.store(info, 0);
    tm32.store(info, 1);
    return st;
}

// ---- a batch of equal-order matrices on the block path (plain FP64)
// Every matrix gets a workspace region with the single-solve layout, all of
// one size R, so that one launch per step serves the whole batch (blockIdx.y
// = matrix, its pointers moved by m R); the pair tables live in region 0 and
// are shared.  Ingest and the output stage stay per matrix (O(n^2) launches)
// with one host synchronisation per phase for the whole batch.  Each matrix
// goes through the launches of a single solve (the same kernels, the same
// order of operations and the same stopping tests, its pending V update
// riding in the next sweep's first launch while it is active), so its results
// are bitwise those of jacobi_eigh on it; a matrix leaves the sweeps when its
// own tests say so (act = 0 from then on, its pending V update applied by one
// launch over the matrices leaving together).
// Streams of a batch's per-matrix ingest and output stages: their kernels
// are latency-bound (a few workgroups each), so the matrices' chains run on
// NPOOL streams side by side, forked from and joined back into the caller's
// stream by events.  The streams are created once per device (non-blocking,
// default priority) and kept until the process ends; the events belong to
// one call, so calls from several host threads can share the streams (a
// stream then also carries another call's work, which only adds waiting).
constexpr int NPOOL = 8;
int pool_streams(hipStream_t *&out)
{
    static hipStream_t pools[64][NPOOL] = {};
    static bool made[64] = {};
    static std::mutex mu;
    int dev = 0;
    CK(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64)
        return JACOBI_DEVICE;
    std::lock_guard<std::mutex> lk(mu);
    if (!made[dev]) {
        for (int k = 0; k < NPOOL; ++k)
            CK(hipStreamCreateWithFlags(&pools[dev][k], hipStreamNonBlocking));
        made[dev] = true;
    }
    out = pools[dev];
    return 0;
}

struct StreamPool {
    hipStream_t *st = nullptr;
    hipEvent_t fork = nullptr, join[NPOOL] = {};
    int init()
    {
        if (int e = pool_streams(st))
            return e;
        CK(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
        for (int k = 0; k < NPOOL; ++k)
            CK(hipEventCreateWithFlags(&join[k], hipEventDisableTiming));
        return 0;
    }
    ~StreamPool()
    {
        if (fork)
            hipEventDestroy(fork);
        for (int k = 0; k < NPOOL; ++k)
            if (join[k])
                hipEventDestroy(join[k]);
    }
};

// work on the pool streams after everything issued so far on s
int pool_fork(StreamPool &p, hipStream_t s)
{
    CK(hipEventRecord(p.fork, s));
    for (int k = 0; k < NPOOL; ++k)
        CK(hipStreamWaitEvent(p.st[k], p.fork, 0));
    return 0;
}

// s waits for everything issued on the pool streams
int pool_join(StreamPool &p, hipStream_t s)
{
    for (int k = 0; k < NPOOL; ++k) {
        CK(hipEventRecord(p.join[k], p.st[k]));
        CK(hipStreamWaitEvent(s, p.join[k], 0));
    }
    return 0;
}

// fn(m, stream) for every matrix m of a batch: matrix m's launches go to pool
// stream m mod NPOOL and are issued by host thread m mod NPOOL, so the
// per-matrix stages (many launches of a few microseconds of host time each)
// are issued side by side instead of one after another.  Returns the first
// failing matrix's code (its HIP error becomes this thread's last error).
template <typename F>
int pool_each(StreamPool &p, int64_t batch, F fn)
{
    int dev = 0;
    CK(hipGetDevice(&dev));
    const int nt = (int)std::min<int64_t>(NPOOL, batch);
    std::vector<int> err((size_t)nt, 0);
    std::vector<hipError_t> herr((size_t)nt, hipSuccess);
    auto body = [&](int k) {
        if (hipSetDevice(dev) != hipSuccess) {
            err[(size_t)k] = JACOBI_DEVICE;
            herr[(size_t)k] = hipErrorInvalidDevice;
            return;
        }
        for (int64_t m = k; m < batch; m += NPOOL)
            if (int e = fn(m, p.st[k])) {
                err[(size_t)k] = e;
                herr[(size_t)k] = g_last_error;
                return;
            }
    };
    std::vector<std::thread> th;
    for (int k = 1; k < nt; ++k)
        th.emplace_back(body, k);
    body(0);
    for (std::thread &t : th)
        t.join();
    for (int k = 0; k < nt; ++k)
        if (err[(size_t)k]) {
            g_last_error = herr[(size_t)k];
            return err[(size_t)k];
        }
    return 0;
}

size_t block_region_bytes(int64_t n, const Opts &o)
{
    Bump bp(nullptr);
    layout_block(bp, n, geometry(n, o.block), false);
    return (bp.off + 255) & ~(size_t)255;
}

size_t ws_block_batched(int64_t n, int64_t batch, const Opts &o)
{
    // the regions, then two sets of per-matrix flags and the thresholds
    const size_t per = ((size_t)std::max<int64_t>(batch, 1) * sizeof(double) + 255) & ~(size_t)255;
    return block_region_bytes(n, o) * (size_t)std::max<int64_t>(batch, 1) + 3 * per + 256;
}

int eigh_block_batched(const double *A, int64_t n, const int64_t *a_off, int64_t batch,
                       double *W, const int64_t *w_off, double *V, double tol_in, const Opts &o,
                       void *work, hipStream_t s, std::vector<int32_t> &st)
{
    const Geometry g = geometry(n, o.block);
    const size_t R = block_region_bytes(n, o);
    char *base = (char *)work;
    std::vector<BlockWs> ws((size_t)batch);
    for (int64_t m = 0; m < batch; ++m) {
        Bump bp(base + (size_t)m * R);
        ws[(size_t)m] = layout_block(bp, n, g, false);
    }
    Bump tail(base + (size_t)batch * R);
    int *act_d = tail.take<int>((size_t)batch);   // in the sweeps
    int *fin_d = tail.take<int>((size_t)batch);   // leaving the sweeps together
    double *thr_d = tail.take<double>((size_t)batch);
    const BlockWs &w0 = ws[0];
    const int64_t nn = g.npad * g.npad;
    auto aoff = [&](int64_t m) { return a_off ? a_off[m] : m * n * n; };
    auto woff = [&](int64_t m) { return w_off ? w_off[m] : m * n; };
    st.assign((size_t)batch, JACOBI_OK);
    if (int e = setup_block(g, w0, s))
        return e;
    const Batch all{batch, (int64_t)R, nullptr, nullptr};
    CK(launch_fill_batch_i32(w0.flags, 8, 0, all, s));
    CK(launch_fill_batch_i32(w0.prot, (int64_t)2 * g.npairs * PROT_STRIDE, 0, all, s));
    // Host side of the per-matrix transfers in pinned memory: every region's
    // scalars and flags come back in two strided copies (one synchronisation
    // per phase), the activity flags and thresholds go up from it.  (Strided
    // and upload copies from pageable memory were measured to return stale
    // data under a profiler that intercepts the runtime; pinned copies are
    // plain DMA on the stream.)
    struct Pinned {
        void *p = nullptr;
        ~Pinned()
        {
            if (p)
                hipHostFree(p);
        }
    } pin;
    CK(hipHostMalloc(&pin.p, (size_t)batch * (9 * sizeof(double) + 10 * sizeof(int)),
                     hipHostMallocDefault));
    double *sc = (double *)pin.p;            // 8 scalars per matrix
    double *thr = sc + (size_t)batch * 8;    // rotation thresholds
    int *fl = (int *)(thr + batch);          // 8 flags per matrix
    int *act = fl + (size_t)batch * 8;       // in the sweeps
    int *fin = act + batch;                  // leaving the sweeps together
    auto read_all = [&]() -> int {
        CK(hipMemcpy2DAsync(sc, 8 * sizeof(double), w0.scal, R, 8 * sizeof(double),
                            (size_t)batch, hipMemcpyDeviceToHost, s));
        CK(hipMemcpy2DAsync(fl, 8 * sizeof(int), w0.flags, R, 8 * sizeof(int), (size_t)batch,
                            hipMemcpyDeviceToHost, s));
        CK(hipStreamSynchronize(s));
        return 0;
    };
    // host flags to the device; the stream is synchronised after the copy, so
    // the host copy may be rewritten as soon as this returns
    auto upload = [&](void *dst, const void *src, size_t bytes) -> int {
        CK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s));
        CK(hipStreamSynchronize(s));
        return 0;
    };
    const auto t_start = std::chrono::steady_clock::now();
    auto ms_since = [](std::chrono::steady_clock::time_point t) {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t)
            .count();
    };
    StreamPool pool_obj;
    if (int e = pool_obj.init())
        return e;
    StreamPool *pool = &pool_obj;
    // ingest (ingest_norm per matrix)
    if (int e = pool_fork(*pool, s))
        return e;
    if (int e = pool_each(*pool, batch, [&](int64_t m, hipStream_t st) -> int {
            const BlockWs &w = ws[(size_t)m];
            CK(launch_ingest<double>(A + aoff(m), n, n, w.B64, g.npad, w.partial, w.flags,
                                     o.check_sym, st));
            CK(launch_sum(w.partial, INGEST_BLOCKS, w.scal, st));
            CK(launch_max(w.partial + INGEST_BLOCKS, INGEST_BLOCKS, w.scal + 4, st));
            return 0;
        }))
        return e;
    if (int e = pool_join(*pool, s))
        return e;
    if (int e = read_all())
        return e;
    std::vector<int> ks((size_t)batch, 0), sweeps((size_t)batch, 0);
    std::vector<double> tol((size_t)batch, 0.0);
    std::fill(act, act + batch, 0);
    std::fill(fin, fin + batch, 0);
    std::fill(thr, thr + batch, 0.0);
    bool rescaled = false;
    for (int64_t m = 0; m < batch; ++m) {
        const size_t i = (size_t)m;
        if (fl[8 * i]) {
            st[i] = JACOBI_NONFINITE;
            continue;
        }
        if (o.check_sym && fl[8 * i + 1]) {
            st[i] = JACOBI_NOTSYM;
            continue;
        }
        ks[i] = scale_exponent(sc[8 * i + 4]);
        if (ks[i]) {
            const BlockWs &w = ws[i];
            CK(launch_scale_pow2(w.B64, nn, ks[i], w.A0, s));
            CK(launch_sq_partial(w.B64, nn, w.partial, s));
            CK(launch_sum(w.partial, OFF_BLOCKS, w.scal, s));
            rescaled = true;
        }
        act[i] = 1;
    }
    if (rescaled)
        if (int e = read_all())
            return e;
    if (int e = pool_fork(*pool, s))
        return e;
    for (int64_t m = 0; m < batch; ++m) {
        const size_t i = (size_t)m;
        if (!act[i])
            continue;
        const double normf = std::sqrt(sc[8 * i]);
        tol[i] = tol_in > 0.0 ? std::ldexp(tol_in, ks[i]) : 1e-15 * (double)n * normf;
        thr[i] = tol[i] / (double)n;
    }
    if (int e = pool_each(*pool, batch, [&](int64_t m, hipStream_t st) -> int {
            if (!act[(size_t)m])
                return 0;
            CK(launch_eye<double>(ws[(size_t)m].V64, g.npad, st));
            CK(launch_off2_partial<double>(ws[(size_t)m].B64, g.npad, ws[(size_t)m].partial, st));
            return 0;
        }))
        return e;
    if (int e = pool_join(*pool, s))
        return e;
    if (int e = upload(act_d, act, (size_t)batch * sizeof(int)))
        return e;
    if (int e = upload(thr_d, thr, (size_t)batch * sizeof(double)))
        return e;
    const Batch bact{batch, (int64_t)R, act_d, nullptr};
    CK(launch_sum(w0.partial, OFF_BLOCKS, w0.scal + 1, s, bact));
    if (int e = read_all())
        return e;
    std::vector<int> solved((size_t)batch, 0); // outputs to write (OK or NOCONV)
    if (trace_on())
        std::fprintf(stderr, "jacobi: batch of %lld, n %lld: matrix 0 normf %.3e tol %.3e off %.3e\n",
                     (long long)batch, (long long)n, std::sqrt(sc[0]), tol[0], std::sqrt(sc[1]));
    for (int64_t m = 0; m < batch; ++m) {
        const size_t i = (size_t)m;
        if (!act[i])
            continue;
        const double off = std::sqrt(sc[8 * i + 1]);
        solved[i] = 1;
        if (!std::isfinite(off)) {
            st[i] = JACOBI_NONFINITE;
            solved[i] = 0;
            act[i] = 0;
        } else if (!(off > tol[i])) {
            act[i] = 0;
        }
    }
    // the sweeps (run_sweeps with the shared launch, per matrix)
    const double t_ingest = ms_since(t_start);
    const auto t_sweeps0 = std::chrono::steady_clock::now();
    int nsweeps = 0;
    const size_t ustride = (size_t)g.npairs * g.M * g.M;
    const int2 *vpend_pairs = nullptr;
    const double *vpend_U = nullptr;
    const int *vpend_prot = nullptr;
    int64_t round = 0;
    for (;;) {
        bool any_fin = false;
        for (int64_t m = 0; m < batch; ++m) {
            const size_t i = (size_t)m;
            if (act[i] && sweeps[i] >= o.max_sweeps) {
                st[i] = JACOBI_NOCONV;
                act[i] = 0;
                fin[i] = 1;
            }
            any_fin = any_fin || fin[i];
        }
        if (any_fin && vpend_pairs) {
            if (int e = upload(fin_d, fin, (size_t)batch * sizeof(int)))
                return e;
            const Batch bf{batch, (int64_t)R, fin_d, nullptr};
            CK(launch_update_v<double>(w0.V64, g.npad, g.npad, g.b, g.npairs, vpend_pairs,
                                       vpend_U, vpend_prot, s, nullptr, nullptr, bf));
        }
        std::fill(fin, fin + batch, 0);
        if (std::find(act, act + batch, 1) == act + batch)
            break;
        if (int e = upload(act_d, act, (size_t)batch * sizeof(int)))
            return e;
        const Batch bt{batch, (int64_t)R, act_d, thr_d};
        CK(launch_fill_batch_i32(w0.flags + 2, 1, 0, bt, s));
        for (int r = 0; r < g.N - 1; ++r, ++round) {
            const int j = (int)(round & 1);
            double *Ub = w0.U64 + j * ustride;
            int *pf = w0.prot + (size_t)j * g.npairs * PROT_STRIDE;
            const int *pfc = o.pair_skip ? pf : nullptr;
            const int2 *pr = w0.pairs + (size_t)r * g.npairs;
            const int cross = o.schedule == 0 && r > 0;
            const int2 *map = w0.psmap + (cross ? (size_t)g.b * (g.b + 1) / 2 : 0);
            if (vpend_pairs) {
                CK(launch_pair_solve_v<double>(w0.B64, g.npad, g.b, g.npairs, pr, map, Ub, U_D,
                                               0.0, o.inner, 0, cross, w0.partial, w0.flags + 2,
                                               pf, w0.V64, g.npad, g.npad, vpend_pairs, vpend_U,
                                               vpend_prot, s, o.pair_v_split, nullptr, nullptr,
                                               bt));
            } else {
                CK(launch_pair_solve<double>(w0.B64, g.npad, g.b, g.npairs, pr, map, Ub, U_D, 0.0,
                                             o.inner, 0, cross, w0.partial, w0.flags + 2, pf, s,
                                             nullptr, nullptr, bt));
            }
            CK(launch_update_b<double>(w0.B64, g.npad, g.b, g.npairs, pr, Ub,
                                       w0.partial + (size_t)g.npairs * pair_solve_waves(g.M),
                                       r == g.N - 2, 0, pfc, w0.flags + 3, s, nullptr, nullptr,
                                       bt));
            vpend_pairs = pr;
            vpend_U = Ub;
            vpend_prot = pfc;
        }
        CK(launch_sum(w0.partial,
                      (int64_t)g.npairs * pair_solve_waves(g.M) + (int64_t)g.nbt * (g.M / 16),
                      w0.scal + 1, s, bt));
        if (int e = read_all())
            return e;
        ++nsweeps;
        if (trace_on())
            std::fprintf(stderr, "jacobi: batch sweep, %lld matrices active, matrix 0 off %.3e\n",
                         (long long)std::count(act, act + batch, 1), std::sqrt(sc[1]));
        for (int64_t m = 0; m < batch; ++m) {
            const size_t i = (size_t)m;
            if (!act[i])
                continue;
            ++sweeps[i];
            const double off = std::sqrt(sc[8 * i + 1]);
            if (!std::isfinite(off)) {
                st[i] = JACOBI_NONFINITE;
                solved[i] = 0;
                act[i] = 0;
            } else if (!fl[8 * i + 2] || !(off > tol[i])) {
                act[i] = 0; // no pair rotated, or off <= tol
                fin[i] = 1;
            }
        }
    }
    // the output stage
    const double t_sweeps = ms_since(t_sweeps0);
    const auto t_out0 = std::chrono::steady_clock::now();
    if (int e = pool_fork(*pool, s))
        return e;
    if (int e = pool_each(*pool, batch, [&](int64_t m, hipStream_t st) -> int {
            if (!solved[(size_t)m])
                return 0;
            return finalize_probe(g, n, ws[(size_t)m], ws[(size_t)m].B64, ws[(size_t)m].V64, st);
        }))
        return e;
    if (int e = pool_join(*pool, s))
        return e;
    if (int e = read_all())
        return e;
    if (int e = pool_fork(*pool, s))
        return e;
    if (int e = pool_each(*pool, batch, [&](int64_t m, hipStream_t st) -> int {
            const size_t i = (size_t)m;
            if (!solved[i])
                return 0;
            const BlockWs &w = ws[i];
            double est = 0.0;
            int pol = 0;
            if (int e2 = finalize_finish(g, n, w, sc[8 * i + 3], w.V64, w.B64, w.Vt,
                                         W + woff(m), V + aoff(m), n, st, &est, &pol,
                                         ks[i] ? w.A0 : A + aoff(m), ks[i] ? g.npad : n))
                return e2;
            if (ks[i])
                CK(launch_scale_pow2(W + woff(m), n, -ks[i], nullptr, st));
            return 0;
        }))
        return e;
    if (int e = pool_join(*pool, s))
        return e;
    CK(hipStreamSynchronize(s));
    if (trace_on())
        std::fprintf(stderr,
                     "jacobi: batch of %lld, n %lld: ingest %.2f ms, %d sweeps %.2f ms, output "
                     "%.2f ms\n",
                     (long long)batch, (long long)n, t_ingest, nsweeps, t_sweeps, ms_since(t_out0));
    return 0;
}

} // namespace

// ======================================================================= ABI
extern "C" {

const char *jacobi_version(void) { return "libjacobi 0.1 (gfx950)"; }

const char *jacobi_status_string(int status)
{
    if (status < 0)
        return "invalid argument";
    switch (status) {
    case JACOBI_OK:
        return "ok";
    case JACOBI_NOCONV:
        return "not converged within max_sweeps";
    case JACOBI_NOTSYM:
        return "matrix is not symmetric";
    case JACOBI_NONFINITE:
        return "non-finite input";
    case JACOBI_DEGENERATE:
        return "degenerate eigenvalue gap in backward";
    case JACOBI_DEVICE:
        return "HIP runtime error";
    case JACOBI_WORKSPACE:
        return "workspace too small";
    default:
        return "unknown status";
    }
}

size_t jacobi_workspace_bytes(int op, int64_t n_max, int64_t batch, const jacobi_opts *opts)
{
    Opts o;
    if (resolve_opts(opts, o) || n_max < 0 || batch < 0)
        return 0;
    switch (op) {
    case 0: {
        size_t a = (n_max <= o.small_max_n) ? ws_small(1, std::max<int64_t>(n_max, 1),
                                                       o.threads, 1)
                                            : 0;
        size_t b = ws_block(std::max<int64_t>(n_max, 1), o, false);
        return std::max(a, b) + 256;
    }
    case 1:
        return ws_block(std::max<int64_t>(n_max, 1), o, true) + 256;
    case 2:
        if (n_max > 128) // a batch of one order on the block path
            return ws_block_batched(n_max, batch, o) + 256;
        return ws_small(std::max<int64_t>(batch, 1), std::max<int64_t>(n_max, 1), o.threads,
                        o.tune) +
               256;
    case 3: {
        size_t nn = (size_t)n_max * n_max * std::max<int64_t>(batch, 1);
        return 2 * nn * sizeof(double) + 1024;
    }
    default:
        return 0;
    }
}

static int eigh_entry(bool mixed, const double *A, int64_t n, int64_t lda, double *W, double *V,
                      int64_t ldv, double tol, const jacobi_opts *opts, void *work,
                      size_t work_bytes, void *stream, jacobi_info *info)
{
    Opts o;
    if (int e = validate_common(A, n, lda, W, V, ldv, tol, opts, o))
        return e;
    if (info)
        std::memset(info, 0, sizeof(*info));
    if (n == 0)
        return JACOBI_OK;
    hipStream_t s = (hipStream_t)stream;
    bool small = !mixed && n <= o.small_max_n;
    if (small && small_pool(n, dev_info().lds_max) == 0)
        small = false; // the matrix does not fit one workgroup's LDS

    const size_t need = jacobi_workspace_bytes(mixed ? 1 : 0, n, 1, opts);
    WsGuard guard;
    if (!work) {
        CK(hipMalloc(&guard.p, need));
        guard.s = s;
        work = guard.p;
    } else if (work_bytes < need) {
        return JACOBI_WORKSPACE;
    }
    void *aligned = (void *)(((uintptr_t)work + 255) & ~(uintptr_t)255);
    if (small)
        return eigh_small(A, n, lda, W, V, ldv, tol, o, aligned, s, info);
    if (mixed)
        return eigh_mixed_block(A, n, lda, W, V, ldv, tol, o, aligned, s, info);
    return eigh_block(A, n, lda, W, V, ldv, tol, o, aligned, s, info);
}

int jacobi_eigh(const double *A, int64_t n, int64_t lda, double *W, double *V, int64_t ldv,
                double tol, const jacobi_opts *opts, void *work, size_t work_bytes,
                void *stream, jacobi_info *info)
{
    return eigh_entry(false, A, n, lda, W, V, ldv, tol, opts, work, work_bytes, stream, info);
}

int jacobi_eigh_mixed(const double *A, int64_t n, int64_t lda, double *W, double *V,
                      int64_t ldv, double tol, const jacobi_opts *opts, void *work,
                      size_t work_bytes, void *stream, jacobi_info *info)
{
    return eigh_entry(true, A, n, lda, W, V, ldv, tol, opts, work, work_bytes, stream, info);
}

int jacobi_eigh_batched(const double *A, const int64_t *n, const int64_t *a_off, int64_t batch,
                        double *W, const int64_t *w_off, double *V, double tol, int mixed,
                        const jacobi_opts *opts, void *work, size_t work_bytes, void *stream,
                        int32_t *status)
{
    if (batch < 0)
        return -4;
    if (batch > 0 && !n)
        return -2;
    int64_t n_max = 0;
    bool uniform = true;
    for (int64_t i = 0; i < batch; ++i) {
        if (n[i] < 1 || n[i] > (int64_t)1 << 20)
            return -2;
        uniform = uniform && n[i] == n[0];
        n_max = std::max(n_max, n[i]);
        if (a_off && a_off[i] < 0)
            return -3;
        if (w_off && w_off[i] < 0)
            return -6;
    }
    // orders above 128 (one workgroup's LDS) only as a batch of one order,
    // which runs on the block path
    const bool block = n_max > 128;
    if (block && !uniform)
        return -2;
    if (block && batch > 65535)
        return -4; // the matrix index is the launches' second grid dimension
    if (batch > 0 && !A)
        return -1;
    if (batch > 0 && !W)
        return -5;
    if (batch > 0 && !V)
        return -7;
    if (std::isnan(tol) || std::isinf(tol))
        return -8;
    if (mixed != 0)
        return -9;
    Opts o;
    if (resolve_opts(opts, o))
        return -10;
    if (batch == 0)
        return JACOBI_OK;
    hipStream_t s = (hipStream_t)stream;
    const size_t need = jacobi_workspace_bytes(2, n_max, batch, opts);
    if (block) {
        // the block path synchronises with the host between sweeps, which a
        // stream being captured into a graph does not allow
        hipStreamCaptureStatus bcap = hipStreamCaptureStatusNone;
        CK(hipStreamIsCapturing(s, &bcap));
        if (bcap != hipStreamCaptureStatusNone) {
            g_last_error = hipErrorStreamCaptureUnsupported;
            return JACOBI_DEVICE;
        }
        WsGuard bguard;
        if (!work) {
            CK(hipMalloc(&bguard.p, need));
            bguard.s = s;
            work = bguard.p;
        } else if (work_bytes < need) {
            return JACOBI_WORKSPACE;
        }
        std::vector<int32_t> st;
        if (int e = eigh_block_batched(A, n_max, a_off, batch, W, w_off, V, tol, o,
                                       (void *)(((uintptr_t)work + 255) & ~(uintptr_t)255), s, st))
            return e;
        if (status) {
            CK(hipMemcpyAsync(status, st.data(), st.size() * sizeof(int32_t),
                              hipMemcpyHostToDevice, s));
            CK(hipStreamSynchronize(s));
        }
        int worst = 0;
        for (int32_t v : st)
            worst = std::max(worst, (int)v);
        return worst;
    }
    WsGuard guard;
    if (!work) {
        CK(hipMalloc(&guard.p, need));
        guard.s = s;
        work = guard.p;
    } else if (work_bytes < need) {
        return JACOBI_WORKSPACE;
    }
    void *aligned = (void *)(((uintptr_t)work + 255) & ~(uintptr_t)255);
    std::vector<SmallCfg> cands;
    small_candidates(n_max, (int)batch, o.threads, o.tune, cands);
    if (cands.empty()) {
        g_last_error = hipErrorInvalidConfiguration;
        return JACOBI_DEVICE; // the largest matrix does not fit one workgroup's LDS
    }
    int64_t slots_max = 1;
    for (const SmallCfg &c : cands)
        slots_max = std::max(slots_max, c.slots);
    Bump bp(aligned);
    SmallWs w = layout_small(bp, batch, n_max, slots_max);
    // descriptors: packed offsets in input order, queue order = n descending
    std::vector<SmallDesc> d((size_t)batch);
    int64_t ao = 0, wo = 0;
    uint64_t nhash = 1469598103934665603ull; // FNV-1a over the orders (graph key)
    for (int64_t i = 0; i < batch; ++i) {
        SmallDesc &e = d[(size_t)i];
        e.a_off = a_off ? a_off[i] : ao;
        e.v_off = e.a_off;
        e.w_off = w_off ? w_off[i] : wo;
        e.n = (int)n[i];
        e.lda = (int)n[i];
        e.ldv = (int)n[i];
        e.orig = (int)i;
        e.info = nullptr;
        ao += n[i] * n[i];
        wo += n[i];
        nhash = (nhash ^ (uint64_t)n[i]) * 1099511628211ull;
        nhash = (nhash ^ (uint64_t)e.a_off) * 1099511628211ull;
        nhash = (nhash ^ (uint64_t)e.w_off) * 1099511628211ull;
    }
    std::stable_sort(d.begin(), d.end(),
                     [](const SmallDesc &a, const SmallDesc &b) { return a.n > b.n; });
    CK(hipMemcpyAsync(w.desc, d.data(), d.size() * sizeof(SmallDesc), hipMemcpyHostToDevice, s));
    const int m = (int)((n_max + 3) & ~3);
    // one solve of the whole batch: reset the queue and the status, then the
    // persistent launch (the only stream operations, so a graph can hold them)
    auto issue = [&](const SmallCfg &c, hipStream_t st) -> int {
        CK(launch_fill_i32(w.queue, 1, 0, st));
        CK(launch_fill_i32(w.status, batch, 0, st));
        CK(launch_small(A, W, V, w.desc, (int)batch, w.queue, tol, o.max_sweeps, w.vscratch,
                        small_vt_elems(n_max), c.pool, m, c.threads, (int)c.slots, w.status, st));
        return 0;
    };
    // configuration: measured once per (device, n_max, batch size class);
    // not while the caller captures `s` (nothing runs then), nor stored
    int dev = 0;
    CK(hipGetDevice(&dev));
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    CK(hipStreamIsCapturing(s, &cap));
    SmallCfg cfg = cands[0];
    if (cands.size() > 1) {
        const int bclass = 64 - __builtin_clzll((unsigned long long)batch);
        const SmallKey key{dev, (int)n_max, bclass, o.threads};
        SmallCfg hit{};
        bool found = small_tuned(key, hit);
        if (found) {
            found = false;
            for (const SmallCfg &c : cands)
                if (c.threads == hit.threads && c.pool == hit.pool) {
                    cfg = c; // this call's grid, within the laid-out scratch
                    found = true;
                }
        }
        if (!found && cap == hipStreamCaptureStatusNone) {
            // every candidate solves the batch once; the outputs are
            // overwritten by the solve with the chosen one below
            hipEvent_t e0 = nullptr, e1 = nullptr;
            CK(hipEventCreate(&e0));
            CK(hipEventCreate(&e1));
            float best = 0.0f;
            int err = 0;
            for (size_t k = 0; k < cands.size() && !err; ++k) {
                err = hipEventRecord(e0, s) != hipSuccess || issue(cands[k], s) != 0 ||
                      hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess;
                float ms = 0.0f;
                if (!err && hipEventElapsedTime(&ms, e0, e1) == hipSuccess &&
                    (k == 0 || ms < best)) {
                    best = ms;
                    cfg = cands[k];
                }
            }
            hipEventDestroy(e0);
            hipEventDestroy(e1);
            if (err) {
                g_last_error = hipGetLastError();
                return JACOBI_DEVICE;
            }
            small_tune_store(key, cfg);
        }
    }
    if (o.graph && !guard.p && cap == hipStreamCaptureStatusNone) {
        const SmallGraphKey gk{A,   W,     V,   work, batch, slots_max, nhash, tol, o.max_sweeps,
                               cfg.threads, cfg.pool, (int)cfg.slots, dev};
        if (int e = small_graph_run(gk, s, [&](hipStream_t cs) { return issue(cfg, cs); }))
            return e;
    } else if (int e = issue(cfg, s)) {
        return e;
    }
    std::vector<int32_t> st((size_t)batch);
    CK(hipMemcpyAsync(st.data(), w.status, st.size() * sizeof(int32_t), hipMemcpyDeviceToHost,
                      s));
    if (status)
        CK(hipMemcpyAsync(status, w.status, st.size() * sizeof(int32_t),
                          hipMemcpyDeviceToDevice, s));
    CK(hipStreamSynchronize(s));
    int worst = 0;
    for (int32_t v : st)
        worst = std::max(worst, (int)v);
    return worst;
}

int jacobi_eigh_backward(const double *W, const double *V, const double *dW, const double *dV,
                         int64_t n, int64_t ld, int64_t batch, double *dA, double gap_tol,
                         void *work, size_t work_bytes, void *stream)
{
    if (n < 0)
        return -5;
    if (ld < std::max<int64_t>(1, n))
        return -6;
    if (batch < 0)
        return -7;
    if (n > 0 && batch > 0) {
        if (!W)
            return -1;
        if (!V)
            return -2;
        if (!dA)
            return -8;
    }
    if (std::isnan(gap_tol) || gap_tol < 0.0)
        return -9;
    if (n == 0 || batch == 0)
        return JACOBI_OK;
    hipStream_t s = (hipStream_t)stream;
    const size_t need = jacobi_workspace_bytes(3, n, batch, nullptr);
    WsGuard guard;
    if (!work) {
        CK(hipMalloc(&guard.p, need));
        guard.s = s;
        work = guard.p;
    } else if (work_bytes < need) {
        return JACOBI_WORKSPACE;
    }
    void *aligned = (void *)(((uintptr_t)work + 255) & ~(uintptr_t)255);
    Bump bp(aligned);
    const int64_t nn = n * n, sv = n * ld; // packed scratch; caller matrices n x ld apart
    double *Mb = bp.take<double>((size_t)(nn * batch));
    double *Tb = bp.take<double>((size_t)(nn * batch));
    int *flag = bp.take<int>(4);
    CK(launch_fill_i32(flag, 1, 0, s));
    if (dV)
        CK(launch_gemm64(1, 0, n, n, n, 1.0, V, ld, sv, dV, ld, sv, 0.0, nullptr, 0, 0, 0.0, Mb,
                         n, nn, batch, s));
    CK(launch_adjoint_mid(Mb, W, dW, n, batch, gap_tol, dV != nullptr, flag, s));
    CK(launch_gemm64(0, 0, n, n, n, 1.0, V, ld, sv, Mb, n, nn, 0.0, nullptr, 0, 0, 0.0, Tb, n,
                     nn, batch, s));
    CK(launch_gemm64(0, 1, n, n, n, 1.0, Tb, n, nn, V, ld, sv, 0.0, nullptr, 0, 0, 0.0, Mb, n,
                     nn, batch, s));
    CK(launch_sym_out(Mb, dA, n, ld, batch, s));
    int hflag = 0;
    CK(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    return hflag ? JACOBI_DEGENERATE : JACOBI_OK;
}

// ------------------------------------------------------------------
// Batched solve without any allocation.  The scratch of the batched path
// (descriptor table, work queue, per-matrix status, eigenvector scratch of
// the workgroups whose V does not fit LDS) lives in a fixed device array;
// the descriptors are built on the device from the caller's orders.  Each
// GPU holds its own copy of the array for the life of the process; calls on
// one GPU share it, so calls that overlap on one GPU race.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

}  // extern "C"

namespace {

std::mutex g_na_mu;
void *g_na_ptr[64] = {};

// Device address of `scratch` on the current device, looked up once per
// device with that device current (the array's name is only a host-side
// stand-in).
int noalloc_scratch(void **out)
{
    int dev = 0;
    CK(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) {
        g_last_error = hipErrorInvalidDevice;
        return JACOBI_DEVICE;
    }
    std::lock_guard<std::mutex> lk(g_na_mu);
    if (!g_na_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            g_last_error = e != hipSuccess ? e : hipErrorInvalidSymbol;
            return JACOBI_DEVICE;
        }
        g_na_ptr[dev] = p;
    }
    *out = g_na_ptr[dev];
    return 0;
}

// Descriptor table of a batch built on the device by one workgroup: orders
// n[i] (1..128), optional offsets aoff / woff (else packed: prefix sums of
// n_i^2 and n_i in input order), sorted by order, largest first (a counting
// sort; the order among equal orders is not fixed, which changes no result:
// each matrix is solved whole by one workgroup).
__global__ __launch_bounds__(1024) void na_build_desc_kernel(const int64_t *__restrict__ n,
                                                             const int64_t *__restrict__ aoff,
                                                             const int64_t *__restrict__ woff,
                                                             int64_t batch, SmallDesc *desc)
{
    __shared__ int hist[130];
    __shared__ int64_t sa[1024], sw[1024];
    const int tid = threadIdx.x;
    for (int i = tid; i < 130; i += 1024)
        hist[i] = 0;
    __syncthreads();
    const int64_t chunk = (batch + 1023) / 1024;
    const int64_t i0 = tid * chunk, i1 = i0 + chunk < batch ? i0 + chunk : batch;
    int64_t la = 0, lw = 0;
    for (int64_t i = i0; i < i1; ++i) {
        const int64_t m = n[i];
        atomicAdd(&hist[m], 1);
        la += m * m;
        lw += m;
    }
    sa[tid] = la;
    sw[tid] = lw;
    __syncthreads();
    if (tid == 0) {
        int64_t a = 0, w = 0;
        for (int t = 0; t < 1024; ++t) { // exclusive prefix sums of the chunks
            const int64_t ta = sa[t], tw = sw[t];
            sa[t] = a;
            sw[t] = w;
            a += ta;
            w += tw;
        }
        int pos = 0; // start of each order's run, largest order first
        for (int m = 128; m >= 1; --m) {
            const int c = hist[m];
            hist[m] = pos;
            pos += c;
        }
    }
    __syncthreads();
    int64_t a = sa[tid], w = sw[tid];
    for (int64_t i = i0; i < i1; ++i) {
        const int m = (int)n[i];
        const int p = atomicAdd(&hist[m], 1);
        SmallDesc d;
        d.a_off = aoff ? aoff[i] : a;
        d.v_off = d.a_off;
        d.w_off = woff ? woff[i] : w;
        d.n = m;
        d.lda = m;
        d.ldv = m;
        d.orig = (int)i;
        d.info = nullptr;
        desc[p] = d;
        a += (int64_t)m * m;
        w += m;
    }
}

// worst = max over the per-matrix status codes
__global__ __launch_bounds__(256) void na_status_max_kernel(const int32_t *__restrict__ st,
                                                            int64_t count, int *worst)
{
    __shared__ int red[4];
    int m = 0;
    for (int64_t i = threadIdx.x; i < count; i += 256)
        m = st[i] > m ? st[i] : m;
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1) {
        const int o = __shfl_xor(m, off, WAVE);
        m = o > m ? o : m;
    }
    if (threadIdx.x % WAVE == 0)
        red[threadIdx.x / WAVE] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        int r = red[0];
        for (int i = 1; i < 4; ++i)
            r = red[i] > r ? red[i] : r;
        *worst = r;
    }
}

} // namespace

extern "C" {

int jacobi_eigh_batched_noalloc(const double *A, const int64_t *n, const int64_t *a_off,
                                int64_t batch, double *W, const int64_t *w_off, double *V,
                                double tol, int mixed, const jacobi_opts *opts, void *stream,
                                int32_t *status)
{
    if (batch < 0)
        return -4;
    if (batch > 0 && !n)
        return -2;
    int64_t n_max = 0;
    for (int64_t i = 0; i < batch; ++i) {
        if (n[i] < 1 || n[i] > 128)
            return -2;
        n_max = std::max(n_max, n[i]);
        if (a_off && a_off[i] < 0)
            return -3;
        if (w_off && w_off[i] < 0)
            return -6;
    }
    if (batch > 0 && !A)
        return -1;
    if (batch > 0 && !W)
        return -5;
    if (batch > 0 && !V)
        return -7;
    if (std::isnan(tol) || std::isinf(tol))
        return -8;
    if (mixed != 0)
        return -9;
    Opts o;
    if (resolve_opts(opts, o))
        return -10;
    if (batch == 0)
        return JACOBI_OK;
    if (batch > (int64_t)1 << 30)
        return JACOBI_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    // launch configuration: the one the batched autotuner stored for this
    // (device, n_max, batch size class, workgroup size) if any, else the
    // fixed choice by n_max; nothing is measured here
    // (fixed-size candidate lists: no heap allocation on this path)
    const int cnt_b = (int)std::min<int64_t>(batch, 1 << 30);
    SmallCfg cands[SMALL_CANDS_MAX], all[SMALL_CANDS_MAX];
    if (small_candidates_fixed(n_max, cnt_b, o.threads, 1, cands) == 0) {
        g_last_error = hipErrorInvalidConfiguration;
        return JACOBI_DEVICE;
    }
    int dev = 0;
    CK(hipGetDevice(&dev));
    SmallCfg cfg = cands[0];
    {
        const int na = small_candidates_fixed(n_max, cnt_b, o.threads, 0, all);
        const int bclass = 64 - __builtin_clzll((unsigned long long)batch);
        SmallCfg hit{};
        if (small_tuned(SmallKey{dev, (int)n_max, bclass, o.threads}, hit))
            for (int k = 0; k < na; ++k)
                if (all[k].threads == hit.threads && all[k].pool == hit.pool)
                    cfg = all[k];
    }
    void *base = nullptr;
    if (int e = noalloc_scratch(&base))
        return e;
    // layout of the fixed scratch (the Bump rounds every piece to 256 bytes)
    Bump bp(base);
    int64_t *n_d = bp.take<int64_t>((size_t)batch);
    int64_t *ao_d = a_off ? bp.take<int64_t>((size_t)batch) : nullptr;
    int64_t *wo_d = w_off ? bp.take<int64_t>((size_t)batch) : nullptr;
    SmallWs w = layout_small(bp, batch, n_max, cfg.slots);
    int *worst = bp.take<int>(1);
    if (bp.off > NOALLOC_SCRATCH_BYTES)
        return JACOBI_WORKSPACE; // the batch needs more than the fixed scratch holds
    CK(hipMemcpyAsync(n_d, n, (size_t)batch * sizeof(int64_t), hipMemcpyHostToDevice, s));
    if (ao_d)
        CK(hipMemcpyAsync(ao_d, a_off, (size_t)batch * sizeof(int64_t), hipMemcpyHostToDevice,
                          s));
    if (wo_d)
        CK(hipMemcpyAsync(wo_d, w_off, (size_t)batch * sizeof(int64_t), hipMemcpyHostToDevice,
                          s));
    hipLaunchKernelGGL(na_build_desc_kernel, dim3(1), dim3(1024), 0, s, n_d, ao_d, wo_d, batch,
                       w.desc);
    CK(hipGetLastError());
    // the queue and the status start at zero on every call (fill kernels)
    CK(launch_fill_i32(w.queue, 1, 0, s));
    CK(launch_fill_i32(w.status, batch, 0, s));
    const int m = (int)((n_max + 3) & ~3);
    CK(launch_small(A, W, V, w.desc, (int)batch, w.queue, tol, o.max_sweeps, w.vscratch,
                    small_vt_elems(n_max), cfg.pool, m, cfg.threads, (int)cfg.slots, w.status,
                    s));
    hipLaunchKernelGGL(na_status_max_kernel, dim3(1), dim3(256), 0, s, w.status, batch, worst);
    CK(hipGetLastError());
    if (status)
        CK(hipMemcpyAsync(status, w.status, (size_t)batch * sizeof(int32_t),
                          hipMemcpyDeviceToDevice, s));
    int hworst = 0;
    CK(hipMemcpyAsync(&hworst, worst, sizeof(int), hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    return hworst;
}

int jacobi_device_summary(char *buf, size_t len)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return JACOBI_DEVICE;
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess)
        return JACOBI_DEVICE;
    int optin = 0;
    hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, dev);
    if (buf && len)
        std::snprintf(buf, len,
                      "%s arch=%s cus=%d lds_per_block=%zu lds_optin=%d clock_khz=%d "
                      "mem_clock_khz=%d bus_bits=%d l2=%d",
                      p.name, p.gcnArchName, p.multiProcessorCount, (size_t)p.sharedMemPerBlock,
                      optin, p.clockRate, p.memoryClockRate, p.memoryBusWidth, p.l2CacheSize);
    return 0;
}

const char *jacobi_last_hip_error(void) { return hipGetErrorString(g_last_error); }

} // extern "C"
