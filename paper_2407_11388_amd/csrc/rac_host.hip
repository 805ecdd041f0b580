// Host side of librac: the C ABI of rac.h, input validation, the CSR arc
// layout, device-side packing of relation rows, work items, and the launch of
// the per-step fixpoint kernels (directly, or as replayed HIP graphs of rounds of steps).
#include <algorithm>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "rac.h"
#include "rac_internal.h"
#include "rac_mfma.h"
#include "rac_tune.h"

using namespace rac;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------

static thread_local std::string g_last_error;

int rac::set_error(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

#define HIP_TRY(call)                                                                   \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess) {                                                         \
            if (e_ == hipErrorOutOfMemory)                                              \
                return set_error(RAC_ENOMEM, "%s: %s", #call, hipGetErrorString(e_));   \
            return set_error(RAC_EHIP, "%s: %s", #call, hipGetErrorString(e_));         \
        }                                                                               \
    } while (0)

extern "C" const char *rac_strerror(int code) {
    switch (code) {
    case RAC_OK: return "ok";
    case RAC_EINVAL: return "invalid argument";
    case RAC_ENOMEM: return "out of memory";
    case RAC_EHIP: return "HIP runtime error";
    case RAC_EUNSUPPORTED: return "unsupported by the selected path";
    case RAC_ENOTCONVERGED: return "max_sweeps reached before the fixpoint";
    case RAC_ENODEV: return "no usable gfx950 device";
    case RAC_ETIMEOUT: return "a batched state did not finish on the matrix-core path";
    default: return "unknown error";
    }
}

extern "C" const char *rac_last_error(void) { return g_last_error.c_str(); }

extern "C" void rac_default_options(rac_options *opt) {
    if (!opt) return;
    memset(opt, 0, sizeof(*opt));
    opt->mode = RAC_RUN_TO_FIXPOINT;
    opt->max_sweeps = 0;
    opt->path = RAC_PATH_AUTO;
    opt->use_graph = 1;
    opt->item_bytes = 0;
}

static int check_options(const rac_options *o) {
    if (o->mode != RAC_RUN_TO_FIXPOINT && o->mode != RAC_STOP_ON_WIPEOUT)
        return set_error(RAC_EINVAL, "options.mode must be 0 or 1");
    if (o->max_sweeps < 0) return set_error(RAC_EINVAL, "options.max_sweeps must be >= 0");
    if (o->path < RAC_PATH_AUTO || o->path > RAC_PATH_FUSED)
        return set_error(RAC_EINVAL, "options.path out of range");
    if (o->item_bytes < 0) return set_error(RAC_EINVAL, "options.item_bytes must be >= 0");
    if (o->profile != 0 && o->profile != 1) return set_error(RAC_EINVAL, "options.profile must be 0 or 1");
    if (o->tune < 0 || o->tune > 2) return set_error(RAC_EINVAL, "options.tune must be 0, 1 or 2");
    if (o->reserved != 0) return set_error(RAC_EINVAL, "options.reserved must be zero");
    return RAC_OK;
}

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------

#define RAC_TRY(expr)                  \
    do {                               \
        int rc_ = (expr);              \
        if (rc_ != RAC_OK) return rc_; \
    } while (0)

struct DeviceInfo {
    int device = -1;
    int num_cu = 0;
    std::vector<std::pair<size_t, int>> blocks_per_cu;   // (dynamic LDS bytes, resident sweep blocks)
    bool ok = false;
};

static std::mutex g_dev_mu;
static DeviceInfo g_dev[16];

static int device_info(int device, DeviceInfo **out) {
    std::lock_guard<std::mutex> lk(g_dev_mu);
    if (device < 0 || device >= 16) return set_error(RAC_ENODEV, "device ordinal %d", device);
    DeviceInfo &di = g_dev[device];
    if (!di.ok) {
        hipDeviceProp_t prop;
        HIP_TRY(hipGetDeviceProperties(&prop, device));
        if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
            return set_error(RAC_ENODEV, "device %d is %s, librac is built for gfx950", device,
                             prop.gcnArchName);
        di.device = device;
        di.num_cu = prop.multiProcessorCount;
        di.ok = true;
    }
    *out = &di;
    return RAC_OK;
}

// LDS bytes of one sweep wave: its scratch plus `vars` staged variables.
static size_t stage_bytes(int32_t vars) {
    return (size_t)kScratchWords * 8 + (vars > 0 ? (size_t)vars * 8 + ((size_t)vars / 32 + 2) * 4 : 0);
}

// Resident revise workgroups (= waves) on the whole device for a given LDS size.
static int sweep_slots(int device, size_t smem, int64_t *slots) {
    DeviceInfo *di;
    RAC_TRY(device_info(device, &di));
    std::lock_guard<std::mutex> lk(g_dev_mu);
    for (auto &e : di->blocks_per_cu)
        if (e.first == smem) {
            *slots = (int64_t)e.second * di->num_cu;
            return RAC_OK;
        }
    int nb = 0;
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, revise_kernel, kWave, smem));
    if (nb < 1) nb = 1;
    di->blocks_per_cu.push_back({smem, nb});
    *slots = (int64_t)nb * di->num_cu;
    return RAC_OK;
}

template <typename T> static int dalloc(T **p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    HIP_TRY(hipMalloc((void **)p, count * sizeof(T)));
    return RAC_OK;
}

template <typename T> static void dfree(T *&p) {
    if (p) (void)hipFree((void *)p);
    p = nullptr;
}


// ---------------------------------------------------------------------------
// networks
// ---------------------------------------------------------------------------

struct PathData {
    bool ready = false;
    int32_t kind = 0, dp = 0;
    void *rows = nullptr;
    size_t rows_bytes = 0;
    int32_t item_bytes = 0;
    int4 *items = nullptr;
    int32_t *pieces = nullptr;
    int32_t nitems = 0;
    NetDesc desc{};
    NetDesc *d_desc = nullptr;
};

constexpr int kProfSteps = 64;   // steps whose revise kernel is timed in profile mode
constexpr int kHist = kProfSteps + 2;

// One round of steps, captured as a HIP graph.
struct RoundGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

// Workspace + per-call buffers for up to `cap_probs` problems of one layout.
struct Runner {
    int32_t cap_probs = 0;
    int64_t cap_vars = 0;
    Workspace ws{};
    int32_t *hist = nullptr;        // [kHist] problems running at step k (profile mode)
    int32_t *prob_net = nullptr;
    int64_t *prob_off = nullptr;
    int64_t tables_key = -1;   // (B, nitems) the problem tables were last written for
    uint64_t *din = nullptr, *dout = nullptr;
    // per-problem results in one device block, read back with one copy:
    // checks [cap] | iters [cap] | status [cap] | rc
    uint8_t *res = nullptr;
    int32_t *iters = nullptr, *status = nullptr, *rc = nullptr;
    long long *checks = nullptr;
    uint8_t *h_res = nullptr;       // pinned mirror of res
    uint64_t *h_dom = nullptr;      // pinned staging of host-pointer domains [cap_vars]
    int64_t prefetched_vars = -1;   // >= 0: results (and that many domain words) already in
                                    // h_res / h_dom, copied by the last round of steps
    uint8_t *changed = nullptr;
    int32_t *count = nullptr;       // a device problem count (Launch::nprob_dev) of a caller
                                    // that decides it on the device
    int32_t *h_nact = nullptr;      // pinned: problems still running after a round
    hipEvent_t ev0 = nullptr, ev1 = nullptr, ev_round = nullptr;
    hipEvent_t kev[2 * kProfSteps] = {};
    bool profiled = false;
    bool fused = false;             // the last launch was small_fixpoint_kernel
    int32_t steps_launched = 0;
    // captured rounds, valid for graph_args / graph_grid
    std::vector<RoundGraph> rounds;
    Launch graph_args{};
    unsigned graph_grid[4] = {0, 0, 0, 0};
    size_t graph_smem = 0;
};

struct SearchWork;   // rac_search's device workspace, kept between searches

struct rac_net {
    int32_t n = 0, d = 0;
    int64_t m = 0, arcs = 0;
    rac_options opt{};
    int device = 0;
    hipStream_t stream = nullptr;
    std::vector<int32_t> h_row_ptr, h_deg, h_gptr;
    int32_t *row_ptr = nullptr, *nbr = nullptr, *deg = nullptr, *arc_src = nullptr;
    int32_t *gptr = nullptr, *nbrp = nullptr, *src_p = nullptr;   // 64-arc group layout
    int32_t *gown = nullptr;                                      // owner variable of each group
    int32_t *rpos = nullptr;   // [arcs] group-layout position of each arc's reverse arc
    int32_t max_deg = 0;
    int64_t groups = 0;
    uint64_t *rel = nullptr;   // [m][d] constraint rows, kept for lazily packed layouts
    PathData bits, i8;
    MfmaData mfma;
    uint64_t *mf_in = nullptr, *mf_out = nullptr;   // staging of host-pointer batch calls
    int32_t *mf_it = nullptr, *mf_st = nullptr;
    int32_t mf_cap = 0;
    Runner run;
    rac_stats last{};
    bool pending = false;      // a device-pointer call awaiting rac_sync_status
    int32_t tune_source = 0;   // of the last call (rac_stats.tune_source)
    SearchWork *search = nullptr;
};

struct rac_group {
    int32_t k = 0;
    std::vector<rac_net *> nets;
    rac_options opt{};
    int device = 0;
    hipStream_t stream = nullptr;
    NetDesc *d_nets = nullptr;
    int4 *items = nullptr;       // the group's own work-item tables of every net, back to back
    int32_t *pieces = nullptr;
    int4 *items_inc = nullptr;   // its tables for steps after a full first step (or null: the same)
    int32_t *pieces_inc = nullptr;
    std::vector<int64_t> h_off;
    std::vector<int32_t> paths;  // rows of each net (RAC_PATH_BITS / RAC_PATH_INT8)
    std::vector<NetDesc> descs;  // host copies of d_nets
    Runner run;
    rac_stats last{};
    int64_t total_vars = 0, total_items = 0, rel_bytes = 0, max_n = 0, max_nd = 0, max_groups = 0;
    int32_t item_target = 0;     // work-item bytes of the item tables of a step over every arc
    int32_t item_target_inc = 0; // ... of the steps that re-examine arcs into changed variables
    bool tuned = false;          // the item size is settled (given, measured or by rule)
    int32_t tune_source = 0;
    bool pending = false;
};

static int32_t round_up(int32_t v, int32_t m) { return (v + m - 1) / m * m; }

static void drop_graphs(Runner &r) {
    for (RoundGraph &g : r.rounds) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.graph) (void)hipGraphDestroy(g.graph);
    }
    r.rounds.clear();
}

static void release_runner(Runner &r) {
    drop_graphs(r);
    dfree(r.ws.dom[0]);
    dfree(r.ws.dom[1]);
    dfree(r.ws.chg[0]);
    dfree(r.ws.chg[1]);
    dfree(r.ws.failacc);
    dfree(r.ws.ctrl);
    dfree(r.ws.plan);
    dfree(r.ws.act);
    dfree(r.ws.act_off);
    dfree(r.ws.act_push);
    dfree(r.ws.clist[0]);
    dfree(r.ws.clist[1]);
    dfree(r.hist);
    dfree(r.prob_net);
    dfree(r.prob_off);
    r.tables_key = -1;
    dfree(r.din);
    dfree(r.dout);
    dfree(r.res);
    r.iters = r.status = r.rc = nullptr;
    r.checks = nullptr;
    if (r.h_res) (void)hipHostFree(r.h_res);
    if (r.h_dom) (void)hipHostFree(r.h_dom);
    r.h_res = nullptr;
    r.h_dom = nullptr;
    dfree(r.changed);
    dfree(r.count);
    if (r.h_nact) (void)hipHostFree(r.h_nact);
    r.h_nact = nullptr;
    if (r.ev0) (void)hipEventDestroy(r.ev0);
    if (r.ev1) (void)hipEventDestroy(r.ev1);
    if (r.ev_round) (void)hipEventDestroy(r.ev_round);
    r.ev0 = r.ev1 = r.ev_round = nullptr;
    for (hipEvent_t &e : r.kev) {
        if (e) (void)hipEventDestroy(e);
        e = nullptr;
    }
    r.cap_probs = 0;
    r.cap_vars = 0;
}

static size_t res_bytes(int32_t nprob) { return (size_t)nprob * 16 + 8; }

// Reads back B problems' domains (into dom, if not null) and results with two
// copies into pinned memory and one wait.
static int read_results(Runner &r, hipStream_t s, int32_t B, int64_t nvars, uint64_t *dom,
                        std::vector<long long> &checks, std::vector<int32_t> &iters,
                        std::vector<int32_t> &status, int32_t *rc) {
    if (r.prefetched_vars >= (dom ? nvars : 0)) {
        r.prefetched_vars = -1;   // the last round copied them and was waited for
    } else {
        r.prefetched_vars = -1;
        if (dom) HIP_TRY(hipMemcpyAsync(r.h_dom, r.dout, (size_t)nvars * 8, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(r.h_res, r.res, res_bytes(r.cap_probs), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    if (dom) memcpy(dom, r.h_dom, (size_t)nvars * 8);
    const size_t cap = (size_t)r.cap_probs;
    checks.assign(reinterpret_cast<const long long *>(r.h_res),
                  reinterpret_cast<const long long *>(r.h_res) + B);
    const int32_t *hi = reinterpret_cast<const int32_t *>(r.h_res + cap * 8);
    iters.assign(hi, hi + B);
    status.assign(hi + cap, hi + cap + B);
    *rc = hi[2 * cap];
    return RAC_OK;
}

static int ensure_runner(Runner &r, int32_t nprob, int64_t nvars) {
    if (nprob <= r.cap_probs && nvars <= r.cap_vars) return RAC_OK;
    release_runner(r);
    RAC_TRY(dalloc(&r.ws.dom[0], nvars));
    RAC_TRY(dalloc(&r.ws.dom[1], nvars));
    RAC_TRY(dalloc(&r.ws.chg[0], nvars));
    RAC_TRY(dalloc(&r.ws.chg[1], nvars));
    RAC_TRY(dalloc(&r.ws.failacc, nvars));
    RAC_TRY(dalloc(&r.ws.ctrl, nprob));
    RAC_TRY(dalloc(&r.ws.plan, 1));
    RAC_TRY(dalloc(&r.ws.act, nprob));
    RAC_TRY(dalloc(&r.ws.act_off, (size_t)nprob + 1));
    RAC_TRY(dalloc(&r.ws.act_push, nprob));
    RAC_TRY(dalloc(&r.ws.clist[0], nvars));
    RAC_TRY(dalloc(&r.ws.clist[1], nvars));
    RAC_TRY(dalloc(&r.hist, kHist));
    RAC_TRY(dalloc(&r.prob_net, nprob));
    RAC_TRY(dalloc(&r.prob_off, (size_t)nprob + 1));
    RAC_TRY(dalloc(&r.din, nvars));
    RAC_TRY(dalloc(&r.dout, nvars));
    RAC_TRY(dalloc(&r.res, res_bytes(nprob)));
    r.checks = reinterpret_cast<long long *>(r.res);
    r.iters = reinterpret_cast<int32_t *>(r.res + (size_t)nprob * 8);
    r.status = r.iters + nprob;
    r.rc = r.status + nprob;
    HIP_TRY(hipHostMalloc((void **)&r.h_res, res_bytes(nprob), hipHostMallocDefault));
    HIP_TRY(hipHostMalloc((void **)&r.h_dom, (size_t)nvars * 8, hipHostMallocDefault));
    RAC_TRY(dalloc(&r.changed, nvars));
    RAC_TRY(dalloc(&r.count, 1));
    HIP_TRY(hipHostMalloc((void **)&r.h_nact, 4, hipHostMallocDefault));
    HIP_TRY(hipEventCreate(&r.ev0));
    HIP_TRY(hipEventCreate(&r.ev1));
    HIP_TRY(hipEventCreateWithFlags(&r.ev_round, hipEventDisableTiming));
    for (hipEvent_t &e : r.kev) HIP_TRY(hipEventCreate(&e));
    r.cap_probs = nprob;
    r.cap_vars = nvars;
    return RAC_OK;
}

static void release_path(PathData &pd) {
    dfree(pd.rows);
    dfree(pd.items);
    dfree(pd.pieces);
    dfree(pd.d_desc);
    pd.ready = false;
    pd.nitems = 0;
}

// A device-pointer call still in flight on a net (or group) uses the net's
// workspace on the caller's stream: every call that touches that workspace
// waits for it first, and its device-side error code is reported then.
static int settle(rac_net *net) { return net->pending ? rac_sync_status(net) : RAC_OK; }
static int settle(rac_group *g) { return g->pending ? rac_group_sync_status(g) : RAC_OK; }

static void release_search(rac_net *net);

extern "C" void rac_destroy(rac_net *net) {
    if (!net) return;
    (void)hipSetDevice(net->device);
    (void)settle(net);
    if (net->stream) (void)hipStreamSynchronize(net->stream);
    release_search(net);
    release_runner(net->run);
    release_path(net->bits);
    release_path(net->i8);
    mfma_release(net->mfma);
    dfree(net->mf_in);
    dfree(net->mf_out);
    dfree(net->mf_it);
    dfree(net->mf_st);
    dfree(net->row_ptr);
    dfree(net->nbr);
    dfree(net->deg);
    dfree(net->arc_src);
    dfree(net->gptr);
    dfree(net->nbrp);
    dfree(net->gown);
    dfree(net->rpos);
    dfree(net->src_p);
    dfree(net->rel);
    if (net->stream) (void)hipStreamDestroy(net->stream);
    delete net;
}

static int current_device(int *dev) {
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count <= 0) return set_error(RAC_ENODEV, "no HIP device visible");
    HIP_TRY(hipGetDevice(dev));
    DeviceInfo *di;
    return device_info(*dev, &di);
}

// Work items over the arcs of one path (host tables): runs of whole variables
// up to about `target` relation bytes, and variables above that split into
// pieces.
static void build_items(const rac_net *net, const PathData &pd, int32_t target,
                        std::vector<int4> &items, std::vector<int32_t> &pieces) {
    // units: 64-arc groups for bit rows, single arcs for int8 rows
    const bool groups = pd.kind != ROWI8;
    const int64_t unit_bytes = groups ? (int64_t)pd.desc.qpa * 1024 : (int64_t)net->d * pd.dp;
    items.clear();
    pieces.clear();
    const int32_t n = net->n;
    const std::vector<int32_t> &rp = groups ? net->h_gptr : net->h_row_ptr;
    const int64_t per_var = 64;   // accounts for the domain read/write of a variable
    const int32_t max_vars = groups ? kItemVars : 256;   // bit rows: one variable per lane
    int32_t xb = 0;
    int64_t acc = 0;
    auto flush = [&](int32_t xe) {
        if (xe > xb) {
            items.push_back(make_int4(xb, xe, rp[xb], rp[xe]));
            pieces.push_back(0);
        }
        xb = xe;
        acc = 0;
    };
    for (int32_t x = 0; x < n; ++x) {
        const int64_t ux = rp[x + 1] - rp[x];
        const int64_t bx = ux * unit_bytes + per_var;
        int64_t np = (ux * unit_bytes + target - 1) / target;
        if (np > ux) np = ux;
        if (np >= 2) {
            flush(x);
            for (int64_t q = 0; q < np; ++q) {
                const int32_t lo = rp[x] + (int32_t)(ux * q / np);
                const int32_t hi = rp[x] + (int32_t)(ux * (q + 1) / np);
                items.push_back(make_int4(x, x + 1, lo, hi));
                pieces.push_back((int32_t)np);
            }
            xb = x + 1;
            acc = 0;
            continue;
        }
        if (x > xb && (acc + bx > target || x - xb >= max_vars)) flush(x);
        acc += bx;
    }
    flush(n);
}

// The net's own item tables for one path (used by calls on the net itself;
// groups build their own copies, so that a later rebuild here never leaves a
// group with freed tables).
static int make_items(rac_net *net, PathData &pd, int32_t target) {
    std::vector<int4> items;
    std::vector<int32_t> pieces;
    build_items(net, pd, target, items, pieces);
    dfree(pd.items);
    dfree(pd.pieces);
    RAC_TRY(dalloc(&pd.items, items.size()));
    RAC_TRY(dalloc(&pd.pieces, pieces.size()));
    HIP_TRY(hipMemcpy(pd.items, items.data(), items.size() * sizeof(int4), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(pd.pieces, pieces.data(), pieces.size() * sizeof(int32_t),
                      hipMemcpyHostToDevice));
    pd.nitems = (int32_t)items.size();
    pd.item_bytes = target;
    pd.desc.items = pd.items;
    pd.desc.pieces = pd.pieces;
    pd.desc.nitems = pd.nitems;
    pd.desc.items_inc = pd.items;   // one table for every step
    pd.desc.pieces_inc = pd.pieces;
    pd.desc.nitems_inc = pd.nitems;
    if (!pd.d_desc) RAC_TRY(dalloc(&pd.d_desc, 1));
    HIP_TRY(hipMemcpy(pd.d_desc, &pd.desc, sizeof(NetDesc), hipMemcpyHostToDevice));
    return RAC_OK;
}

// Default work-item size for a call that streams `total` relation bytes:
// about two items per resident wave, within [16 KiB, 4 MiB].
static int32_t default_item_bytes(int device, int64_t total) {
    int64_t slots = 0;
    if (sweep_slots(device, stage_bytes(kStageMax), &slots) != RAC_OK) return 65536;
    const char *e = getenv("RAC_ITEMS_PER_WAVE");
    const int64_t per = (e && atoi(e) > 0) ? atoi(e) : 2;
    int64_t t = total / (per * slots);
    t = std::max<int64_t>(16384, std::min<int64_t>(4 << 20, t));
    return (int32_t)t;
}

static int ensure_path(rac_net *net, int32_t path, int32_t item_bytes) {
    PathData &pd = path == RAC_PATH_INT8 ? net->i8 : net->bits;
    if (!pd.ready) {
        const int32_t d = net->d;
        if (path == RAC_PATH_INT8) {
            if (d > 32) return set_error(RAC_EUNSUPPORTED, "int8 rows need d <= 32 (d=%d)", d);
            pd.kind = ROWI8;
            pd.dp = round_up(d, 16);
            pd.rows_bytes = (size_t)net->arcs * d * pd.dp;
        } else if (d <= 32) {
            pd.kind = ROW32;
            pd.dp = round_up(d, 4);
            pd.desc.qpa = pd.dp / 4;
            pd.rows_bytes = (size_t)net->groups * pd.desc.qpa * 1024;
        } else {
            pd.kind = ROW64;
            pd.dp = round_up(d, 8);   // qpa = dp/2, a multiple of 4
            pd.desc.qpa = pd.dp / 2;
            pd.rows_bytes = (size_t)net->groups * pd.desc.qpa * 1024;
        }
        HIP_TRY(hipSetDevice(net->device));
        RAC_TRY(dalloc((uint8_t **)&pd.rows, pd.rows_bytes));
        if (net->arcs > 0) {
            if (pd.kind == ROWI8) {
                const int64_t threads = net->arcs * d * (pd.dp / 4);
                hipLaunchKernelGGL(pack_i8_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256),
                                   0, net->stream, net->rel, net->arc_src, net->arcs, d, d, pd.dp,
                                   (int8_t *)pd.rows);
            } else {
                const int64_t threads = net->groups * pd.desc.qpa * kGroup;
                hipLaunchKernelGGL(pack_bits_kernel, dim3((unsigned)((threads + 255) / 256)),
                                   dim3(256), 0, net->stream, net->rel, net->src_p, net->groups, d,
                                   pd.desc.qpa, pd.kind, (uint4 *)pd.rows);
            }
            HIP_TRY(hipGetLastError());
            HIP_TRY(hipStreamSynchronize(net->stream));
        }
        pd.desc.row_ptr = net->row_ptr;
        pd.desc.nbr = net->nbr;
        pd.desc.gptr = net->gptr;
        pd.desc.nbrp = net->nbrp;
        pd.desc.gown = net->gown;
        pd.desc.rpos = pd.kind == ROWI8 ? nullptr : net->rpos;
        pd.desc.pchunks = std::max<int32_t>(1, (net->max_deg + kGroup - 1) / kGroup);
        pd.desc.deg = net->deg;
        pd.desc.rows = pd.rows;
        pd.desc.n = net->n;
        pd.desc.d = net->d;
        pd.desc.dp = pd.dp;
        pd.desc.kind = pd.kind;
        pd.desc.arcs = net->arcs;
        pd.ready = true;
        pd.item_bytes = 0;
    }
    // item_bytes > 0: the caller's size; < 0: default for -item_bytes states
    const int32_t target = item_bytes > 0 ? item_bytes
                                          : default_item_bytes(net->device, (int64_t)pd.rows_bytes *
                                                               std::max<int32_t>(1, -item_bytes));
    if (target != pd.item_bytes || !pd.items) RAC_TRY(make_items(net, pd, target));
    return RAC_OK;
}

// Common creation from constraint rows rel[m][d] (uint64, bit b = allowed).
static int create_common(int32_t n, int32_t d, int64_t m, const int32_t *edges,
                         const uint64_t *rel, const rac_options *opt, rac_net **out) {
    if (!out) return set_error(RAC_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 1) return set_error(RAC_EINVAL, "n must be >= 1 (n=%d)", n);
    if (d < 1 || d > 64) return set_error(RAC_EINVAL, "d must be in 1..64 (d=%d)", d);
    if (m < 0) return set_error(RAC_EINVAL, "m must be >= 0");
    if (m > 0 && (!edges || !rel)) return set_error(RAC_EINVAL, "edges/relations are NULL");
    if (2 * m >= (int64_t)INT32_MAX) return set_error(RAC_EUNSUPPORTED, "too many constraints");
    rac_options o;
    rac_default_options(&o);
    if (opt) o = *opt;
    RAC_TRY(check_options(&o));

    // validate edges: in range, no self-loop, no duplicate unordered pair
    std::vector<int64_t> keys((size_t)m);
    for (int64_t e = 0; e < m; ++e) {
        const int32_t x = edges[2 * e], y = edges[2 * e + 1];
        if (x < 0 || x >= n || y < 0 || y >= n)
            return set_error(RAC_EINVAL, "edge %lld has a variable out of range", (long long)e);
        if (x == y) return set_error(RAC_EINVAL, "edge %lld is a self-loop", (long long)e);
        const int64_t lo = std::min(x, y), hi = std::max(x, y);
        keys[(size_t)e] = lo * (int64_t)n + hi;
    }
    std::sort(keys.begin(), keys.end());
    for (size_t i = 1; i < keys.size(); ++i)
        if (keys[i] == keys[i - 1])
            return set_error(RAC_EINVAL, "two constraints on the pair (%lld,%lld)",
                             (long long)(keys[i] / n), (long long)(keys[i] % n));
    const uint64_t bad = d >= 64 ? 0ull : ~((1ull << d) - 1ull);
    for (int64_t i = 0; i < m * d; ++i)
        if (rel[i] & bad)
            return set_error(RAC_EINVAL, "relation row %lld has bits >= d", (long long)i);

    int dev = 0;
    RAC_TRY(current_device(&dev));

    rac_net *net = new rac_net();
    net->n = n;
    net->d = d;
    net->m = m;
    net->arcs = 2 * m;
    net->opt = o;
    net->device = dev;
    int rc = RAC_OK;
    do {
        hipError_t e = hipStreamCreateWithFlags(&net->stream, hipStreamNonBlocking);
        if (e != hipSuccess) { rc = set_error(RAC_EHIP, "hipStreamCreate: %s", hipGetErrorString(e)); break; }
        // CSR of arcs grouped by source variable, in edge order
        net->h_deg.assign((size_t)n, 0);
        for (int64_t e2 = 0; e2 < m; ++e2) {
            net->h_deg[(size_t)edges[2 * e2]]++;
            net->h_deg[(size_t)edges[2 * e2 + 1]]++;
        }
        net->h_row_ptr.assign((size_t)n + 1, 0);
        for (int32_t x = 0; x < n; ++x) net->h_row_ptr[x + 1] = net->h_row_ptr[x] + net->h_deg[x];
        std::vector<int32_t> fill(net->h_row_ptr.begin(), net->h_row_ptr.end() - 1);
        std::vector<int32_t> nbr((size_t)net->arcs), src((size_t)net->arcs);
        for (int64_t e2 = 0; e2 < m; ++e2) {
            const int32_t x = edges[2 * e2], y = edges[2 * e2 + 1];
            int32_t j = fill[x]++;
            nbr[j] = y;
            src[j] = (int32_t)(2 * e2);
            j = fill[y]++;
            nbr[j] = x;
            src[j] = (int32_t)(2 * e2 + 1);
        }
        // the 64-arc group layout: each variable's arcs padded to whole groups
        net->h_gptr.assign((size_t)n + 1, 0);
        for (int32_t x = 0; x < n; ++x)
            net->h_gptr[x + 1] = net->h_gptr[x] + (net->h_deg[x] + kGroup - 1) / kGroup;
        net->groups = net->h_gptr[(size_t)n];
        std::vector<int32_t> nbrp((size_t)net->groups * kGroup, -1), srcp((size_t)net->groups * kGroup, -1);
        for (int32_t x = 0; x < n; ++x) {
            const int64_t pb = (int64_t)net->h_gptr[x] * kGroup;
            for (int32_t j = net->h_row_ptr[x]; j < net->h_row_ptr[x + 1]; ++j) {
                nbrp[(size_t)(pb + j - net->h_row_ptr[x])] = nbr[(size_t)j];
                srcp[(size_t)(pb + j - net->h_row_ptr[x])] = src[(size_t)j];
            }
        }
        std::vector<int32_t> gown((size_t)net->groups);
        for (int32_t x = 0; x < n; ++x)
            for (int32_t g = net->h_gptr[x]; g < net->h_gptr[x + 1]; ++g) gown[(size_t)g] = x;
        // the reverse of arc j (x -> y) is the arc of the same edge leaving y;
        // rpos[j] is that arc's position in the group layout
        std::vector<int32_t> apos((size_t)net->arcs), rpos((size_t)net->arcs);
        std::vector<int32_t> arc_of_src((size_t)net->arcs);
        for (int32_t x = 0; x < n; ++x)
            for (int32_t j = net->h_row_ptr[x]; j < net->h_row_ptr[x + 1]; ++j) {
                apos[(size_t)j] = net->h_gptr[x] * kGroup + (j - net->h_row_ptr[x]);
                arc_of_src[(size_t)src[(size_t)j]] = j;
            }
        for (int64_t j = 0; j < net->arcs; ++j)
            rpos[(size_t)j] = apos[(size_t)arc_of_src[(size_t)(src[(size_t)j] ^ 1)]];
        for (int32_t x = 0; x < n; ++x) net->max_deg = std::max(net->max_deg, net->h_deg[x]);
        if ((rc = dalloc(&net->rpos, std::max<size_t>(1, rpos.size())))) break;
        if (!rpos.empty() &&
            hipMemcpy(net->rpos, rpos.data(), rpos.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
            rc = set_error(RAC_EHIP, "hipMemcpy of the reverse-arc table failed");
            break;
        }
        if ((rc = dalloc(&net->gptr, (size_t)n + 1))) break;
        if ((rc = dalloc(&net->nbrp, nbrp.size()))) break;
        if ((rc = dalloc(&net->gown, gown.size()))) break;
        if (!gown.empty() &&
            hipMemcpy(net->gown, gown.data(), gown.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
            rc = set_error(RAC_EHIP, "hipMemcpy of the group owners failed");
            break;
        }
        if ((rc = dalloc(&net->src_p, srcp.size()))) break;
        if (hipMemcpy(net->gptr, net->h_gptr.data(), ((size_t)n + 1) * 4, hipMemcpyHostToDevice) != hipSuccess ||
            (!nbrp.empty() && hipMemcpy(net->nbrp, nbrp.data(), nbrp.size() * 4, hipMemcpyHostToDevice) != hipSuccess) ||
            (!srcp.empty() && hipMemcpy(net->src_p, srcp.data(), srcp.size() * 4, hipMemcpyHostToDevice) != hipSuccess)) {
            rc = set_error(RAC_EHIP, "hipMemcpy of the group layout failed");
            break;
        }
        if ((rc = dalloc(&net->row_ptr, (size_t)n + 1))) break;
        if ((rc = dalloc(&net->deg, (size_t)n))) break;
        if ((rc = dalloc(&net->nbr, (size_t)net->arcs))) break;
        if ((rc = dalloc(&net->arc_src, (size_t)net->arcs))) break;
        if ((rc = dalloc(&net->rel, (size_t)(m * d)))) break;
        if (hipMemcpy(net->row_ptr, net->h_row_ptr.data(), ((size_t)n + 1) * 4, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(net->deg, net->h_deg.data(), (size_t)n * 4, hipMemcpyHostToDevice) != hipSuccess ||
            (m > 0 && hipMemcpy(net->nbr, nbr.data(), (size_t)net->arcs * 4, hipMemcpyHostToDevice) != hipSuccess) ||
            (m > 0 && hipMemcpy(net->arc_src, src.data(), (size_t)net->arcs * 4, hipMemcpyHostToDevice) != hipSuccess) ||
            (m > 0 && hipMemcpy(net->rel, rel, (size_t)(m * d) * 8, hipMemcpyHostToDevice) != hipSuccess)) {
            rc = set_error(RAC_EHIP, "hipMemcpy of the network failed");
            break;
        }
        if ((rc = ensure_path(net, RAC_PATH_BITS, o.item_bytes > 0 ? o.item_bytes : -1))) break;
        if (o.path == RAC_PATH_INT8 &&
            (rc = ensure_path(net, RAC_PATH_INT8, o.item_bytes > 0 ? o.item_bytes : -1)))
            break;
    } while (0);
    if (rc != RAC_OK) {
        rac_destroy(net);
        return rc;
    }
    *out = net;
    return RAC_OK;
}

extern "C" int rac_create_bits(int32_t n, int32_t d, int64_t m, const int32_t *edges,
                               const uint64_t *rel_rows, const rac_options *opt, rac_net **out) {
    return create_common(n, d, m, edges, rel_rows, opt, out);
}

extern "C" int rac_create(int32_t n, int32_t d, int64_t m, const int32_t *edges,
                          const uint8_t *rel, const rac_options *opt, rac_net **out) {
    if (d < 1 || d > 64) return set_error(RAC_EINVAL, "d must be in 1..64 (d=%d)", d);
    if (m < 0) return set_error(RAC_EINVAL, "m must be >= 0");
    if (m > 0 && !rel) return set_error(RAC_EINVAL, "rel is NULL");
    std::vector<uint64_t> rows((size_t)(m * d));
    for (int64_t e = 0; e < m; ++e)
        for (int32_t a = 0; a < d; ++a) {
            uint64_t r = 0;
            const uint8_t *src = rel + ((size_t)e * d + a) * d;
            for (int32_t b = 0; b < d; ++b)
                if (src[b]) r |= 1ull << b;
            rows[(size_t)(e * d + a)] = r;
        }
    return create_common(n, d, m, edges, rows.data(), opt, out);
}

extern "C" int rac_create_dense(int32_t n, int32_t d, const uint8_t *R, int64_t m,
                                const int32_t *edges, const rac_options *opt, rac_net **out) {
    if (n < 1 || d < 1 || d > 64) return set_error(RAC_EINVAL, "bad n or d");
    if (!R) return set_error(RAC_EINVAL, "R is NULL");
    if (m < 0 || (m > 0 && !edges)) return set_error(RAC_EINVAL, "bad edge list");
    const size_t N = (size_t)n * d;
    std::vector<uint64_t> rows((size_t)(m * d));
    for (int64_t e = 0; e < m; ++e) {
        const int32_t x = edges[2 * e], y = edges[2 * e + 1];
        if (x < 0 || x >= n || y < 0 || y >= n || x == y)
            return set_error(RAC_EINVAL, "edge %lld is invalid", (long long)e);
        for (int32_t a = 0; a < d; ++a) {
            uint64_t r = 0;
            for (int32_t b = 0; b < d; ++b) {
                const uint8_t fwd = R[((size_t)x * d + a) * N + (size_t)y * d + b] != 0;
                const uint8_t rev = R[((size_t)y * d + b) * N + (size_t)x * d + a] != 0;
                if (fwd != rev)
                    return set_error(RAC_EINVAL,
                                     "R[%d,.,%d,.] is not the transpose of R[%d,.,%d,.]", y, x, x, y);
                if (fwd) r |= 1ull << b;
            }
            rows[(size_t)(e * d + a)] = r;
        }
    }
    return create_common(n, d, m, edges, rows.data(), opt, out);
}

extern "C" int rac_net_info(const rac_net *net, int32_t *n, int32_t *d, int64_t *m, int64_t *arcs) {
    if (!net) return set_error(RAC_EINVAL, "net is NULL");
    if (n) *n = net->n;
    if (d) *d = net->d;
    if (m) *m = net->m;
    if (arcs) *arcs = net->arcs;
    return RAC_OK;
}

// ---------------------------------------------------------------------------
// launching
// ---------------------------------------------------------------------------

static dim3 grid_init(int64_t nvars) {
    int64_t b = (nvars + 255) / 256;
    if (b > 4096) b = 4096;
    if (b < 1) b = 1;
    return dim3((unsigned)b);
}

// Steps per round of captured graphs: 4, 4, 8, 8, 16, 32, then 64 (one
// problem: 3, 4, 8, 8, ...). Steps past the fixpoint still launch (and return
// at once, about 7 µs a step), and each further round costs a host read
// (about 40 µs of a call), so the early rounds stay short: most calls end
// within their first 16 to 24 steps. For one problem, a first round of 3
// steps measured best overall: single-mid (1 step) 83 µs per call against 91
// with 4 and 68 with 2, calls of 3 steps 178 µs against 173 with 4 and 210
// with 2.
static int32_t round_steps(int round, bool single) {
    static const int32_t kSteps[6] = {4, 4, 8, 8, 16, 32};
    if (round == 0 && single) return 3;
    return round < 6 ? kSteps[round] : 64;
}
static int32_t round_first_step(int round, bool single) {
    int32_t k = 1;
    for (int i = 0; i < round; ++i) k += round_steps(i, single);
    return k;
}

struct StepGrids {
    dim3 init, revise, update;
    size_t smem;
};

// Kernel node of a round graph, chained after `prev` (if any).
static int add_node(hipGraph_t g, hipGraphNode_t *prev, const void *func, dim3 grid, dim3 block,
                    size_t smem, void **params) {
    hipKernelNodeParams kp;
    memset(&kp, 0, sizeof(kp));
    kp.func = const_cast<void *>(func);
    kp.gridDim = grid;
    kp.blockDim = block;
    kp.sharedMemBytes = (unsigned)smem;
    kp.kernelParams = params;
    kp.extra = nullptr;
    hipGraphNode_t node;
    HIP_TRY(hipGraphAddKernelNode(&node, g, *prev ? prev : nullptr, *prev ? 1 : 0, &kp));
    *prev = node;
    return RAC_OK;
}

// Round `round` as a graph: (round 0: init and the plan of step 1, then) for
// each of its steps k: revise(k), update(k), plan(k+1).
static int build_round(Runner &r, int round, const Launch &L, const StepGrids &sg) {
    RoundGraph rg;
    HIP_TRY(hipGraphCreate(&rg.graph, 0));
    Launch args = L;
    hipGraphNode_t prev = nullptr;
    int32_t one = 1;
    if (round == 0) {
        void *pi[1] = {&args};
        RAC_TRY(add_node(rg.graph, &prev, (const void *)init_kernel, sg.init, dim3(256), 0, pi));
        if (L.changed0)
            RAC_TRY(add_node(rg.graph, &prev, (const void *)list_changed0_kernel, sg.init, dim3(256),
                             0, pi));
        void *pp[2] = {&args, &one};
        RAC_TRY(add_node(rg.graph, &prev, (const void *)plan_kernel, dim3(1), dim3(1024), 0, pp));
    }
    const int32_t k0 = round_first_step(round, L.nprob == 1), K = round_steps(round, L.nprob == 1);
    std::vector<int32_t> ks((size_t)K + 1);
    for (int32_t i = 0; i <= K; ++i) ks[(size_t)i] = k0 + i;
    for (int32_t i = 0; i < K; ++i) {
        void *pk[2] = {&args, &ks[(size_t)i]};
        void *pn[2] = {&args, &ks[(size_t)i + 1]};
        if (L.shared_rows)
            RAC_TRY(add_node(rg.graph, &prev, (const void *)revise_shared_kernel, sg.revise,
                             dim3(kWave), 0, pk));
        else
            RAC_TRY(add_node(rg.graph, &prev, (const void *)revise_kernel, sg.revise, dim3(kWave),
                             sg.smem, pk));
        RAC_TRY(add_node(rg.graph, &prev, (const void *)update_kernel, sg.update, dim3(256), 0, pk));
        RAC_TRY(add_node(rg.graph, &prev, (const void *)plan_kernel, dim3(1), dim3(1024), 0, pn));
    }
    HIP_TRY(hipGraphInstantiate(&rg.exec, rg.graph, nullptr, nullptr, 0));
    if ((int)r.rounds.size() <= round) r.rounds.resize((size_t)round + 1);
    r.rounds[(size_t)round] = rg;
    return RAC_OK;
}

// Enqueues a whole enforcement on `stream`: init, then rounds of steps until
// the plan reports that no problem runs the next step (the host reads one
// counter per round), then finish. `nv` variables in all; `kcap` bounds the
// steps of every problem.
// rb_vars >= 0: after every round also run the finish kernel and copy the
// results and the first rb_vars words of L.dout to r.h_res / r.h_dom before the
// round's wait, so that a run that ends there needs no further wait.
static int launch_fixpoint(Runner &r, int device, hipStream_t stream, const Launch &L, int64_t nv,
                           int64_t total_items, int32_t kcap, bool use_graph, bool profile = false,
                           int64_t rb_vars = -1) {
    StepGrids sg;
    sg.smem = stage_bytes(L.stage_vars);
    int64_t g = 0;
    RAC_TRY(sweep_slots(device, sg.smem, &g));
    if (total_items < g) g = total_items;
    if (g < 1) g = 1;
    sg.init = grid_init(nv);
    sg.revise = dim3((unsigned)g);
    const int64_t ub = std::min<int64_t>(4096, std::max<int64_t>(1, (nv + 255) / 256));
    sg.update = dim3((unsigned)ub);
    if (getenv("RAC_DEBUG"))
        fprintf(stderr, "[rac] revise grid=%lld items=%lld lds=%zu stage_vars=%d nprob=%d\n",
                (long long)g, (long long)total_items, sg.smem, L.stage_vars, L.nprob);
    r.profiled = profile;
    r.fused = false;
    const bool graphs = use_graph && !profile;
    if (graphs) {
        const bool same = r.graph_grid[0] == sg.init.x && r.graph_grid[1] == sg.revise.x &&
                          r.graph_grid[2] == sg.update.x && r.graph_smem == sg.smem &&
                          memcmp(&r.graph_args, &L, sizeof(Launch)) == 0;
        if (!same) {
            drop_graphs(r);
            r.graph_args = L;
            r.graph_grid[0] = sg.init.x;
            r.graph_grid[1] = sg.revise.x;
            r.graph_grid[2] = sg.update.x;
            r.graph_smem = sg.smem;
        }
    }
    HIP_TRY(hipEventRecord(r.ev0, stream));
    int32_t k = 0;   // steps enqueued
    for (int round = 0;; ++round) {
        const int32_t K = round_steps(round, L.nprob == 1);
        if (graphs) {
            if ((int)r.rounds.size() <= round || !r.rounds[(size_t)round].exec)
                RAC_TRY(build_round(r, round, L, sg));
            HIP_TRY(hipGraphLaunch(r.rounds[(size_t)round].exec, stream));
        } else {
            if (round == 0) {
                hipLaunchKernelGGL(init_kernel, sg.init, dim3(256), 0, stream, L);
                if (L.changed0)
                    hipLaunchKernelGGL(list_changed0_kernel, sg.init, dim3(256), 0, stream, L);
                hipLaunchKernelGGL(plan_kernel, dim3(1), dim3(1024), 0, stream, L, 1);
            }
            for (int32_t i = 1; i <= K; ++i) {
                const int32_t kk = k + i;
                const bool timed = profile && kk <= kProfSteps;
                if (timed) HIP_TRY(hipEventRecord(r.kev[2 * (kk - 1)], stream));
                if (L.shared_rows)
                    hipLaunchKernelGGL(revise_shared_kernel, sg.revise, dim3(kWave), 0, stream, L, kk);
                else
                    hipLaunchKernelGGL(revise_kernel, sg.revise, dim3(kWave), sg.smem, stream, L, kk);
                if (timed) HIP_TRY(hipEventRecord(r.kev[2 * (kk - 1) + 1], stream));
                hipLaunchKernelGGL(update_kernel, sg.update, dim3(256), 0, stream, L, kk);
                hipLaunchKernelGGL(plan_kernel, dim3(1), dim3(1024), 0, stream, L, kk + 1);
                if (profile && kk + 1 < kHist)
                    HIP_TRY(hipMemcpyAsync(r.hist + kk + 1, &L.ws.plan->nact, 4,
                                           hipMemcpyDeviceToDevice, stream));
            }
            HIP_TRY(hipGetLastError());
        }
        k += K;
        HIP_TRY(hipMemcpyAsync(r.h_nact, &L.ws.plan->nact, 4, hipMemcpyDeviceToHost, stream));
        if (rb_vars >= 0) {
            hipLaunchKernelGGL(finish_kernel, sg.init, dim3(256), 0, stream, L);
            HIP_TRY(hipEventRecord(r.ev1, stream));
            if (rb_vars > 0)
                HIP_TRY(hipMemcpyAsync(r.h_dom, L.dout, (size_t)rb_vars * 8, hipMemcpyDeviceToHost,
                                       stream));
            HIP_TRY(hipMemcpyAsync(r.h_res, r.res, res_bytes(r.cap_probs), hipMemcpyDeviceToHost,
                                   stream));
        }
        HIP_TRY(hipEventRecord(r.ev_round, stream));
        HIP_TRY(hipEventSynchronize(r.ev_round));
        if (*r.h_nact == 0 || k >= kcap) break;
    }
    if (rb_vars >= 0) {
        HIP_TRY(hipGetLastError());
        r.prefetched_vars = rb_vars;
    } else {
        hipLaunchKernelGGL(finish_kernel, sg.init, dim3(256), 0, stream, L);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipEventRecord(r.ev1, stream));
        r.prefetched_vars = -1;
    }
    r.steps_launched = k;
    return RAC_OK;
}

// Every step of every problem in one launch (RAC_PATH_FUSED): one workgroup
// of small_fixpoint_kernel per problem with its domains in LDS; max_n and
// max_groups are the largest problem's variables and 64-arc groups. Waves
// per workgroup: up to 16 for one problem, fewer for many (measured: 8 for
// batches of states whose steps re-examine many arcs, 4 for search rounds
// whose children change few variables per step, where barriers dominate).
// Outputs and read-back as launch_fixpoint.
enum { kFusedWavesOne = 16, kFusedWavesBatch = 8, kFusedWavesSearch = 4 };
static int launch_fused(Runner &r, hipStream_t stream, const Launch &L, int32_t max_n,
                        int64_t max_groups, int max_waves, bool profile, int64_t rb_vars = -1,
                        int32_t grid = 0) {
    if (max_n > kSmallMaxN)
        return set_error(RAC_EUNSUPPORTED, "the fused path holds at most %d variables per state",
                         kSmallMaxN);
    HIP_TRY(hipEventRecord(r.ev0, stream));
    hipLaunchKernelGGL(clear_word_kernel, dim3(1), dim3(64), 0, stream, L.rc_out);
    if (profile) HIP_TRY(hipEventRecord(r.kev[0], stream));
    if (L.nprob > 0)
        hipLaunchKernelGGL(small_fixpoint_kernel,
                           dim3((unsigned)(grid > 0 ? std::min<int32_t>(grid, L.nprob) : L.nprob)),
                           dim3(small_threads(max_groups, max_waves)),
                           small_lds_bytes(max_n), stream, L);
    if (profile) HIP_TRY(hipEventRecord(r.kev[1], stream));
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipEventRecord(r.ev1, stream));
    r.profiled = profile;
    r.fused = true;
    r.steps_launched = 0;
    r.prefetched_vars = -1;
    if (rb_vars >= 0) {
        if (rb_vars > 0)
            HIP_TRY(hipMemcpyAsync(r.h_dom, L.dout, (size_t)rb_vars * 8, hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipMemcpyAsync(r.h_res, r.res, res_bytes(r.cap_probs), hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        r.prefetched_vars = rb_vars;
    }
    return RAC_OK;
}

// Profile mode: summed duration of the revise launches of steps that some
// problem executed, and their number.
static void revise_timing(Runner &r, double *ms, int64_t *launches, float *first_ms) {
    *ms = 0.0;
    *launches = 0;
    *first_ms = 0.f;
    if (!r.profiled) return;
    if (r.fused) {   // one launch ran every step
        float t = 0.f;
        if (hipEventElapsedTime(&t, r.kev[0], r.kev[1]) == hipSuccess) {
            *ms = t;
            *launches = 1;
            *first_ms = t;
        }
        return;
    }
    int32_t h[kHist] = {0};
    const int32_t n = std::min<int32_t>(r.steps_launched, kProfSteps);
    if (hipMemcpy(h, r.hist, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess) return;
    h[1] = 1;   // step 1 always runs
    for (int32_t k = 1; k <= n; ++k) {
        if (h[k] <= 0) continue;
        float t = 0.f;
        if (hipEventElapsedTime(&t, r.kev[2 * (k - 1)], r.kev[2 * (k - 1) + 1]) == hipSuccess) {
            if (k == 1) *first_ms = t;
            *ms += t;
            ++*launches;
        }
    }
}

// Steps k >= 2 that re-examine at most 1/ratio of a bit-row network's arcs go
// variable by variable (the changed variables' arcs) instead of scanning
// every group. RAC_PUSH_RATIO overrides the ratio (0: always scan).
static int32_t push_ratio() {
    const char *e = getenv("RAC_PUSH_RATIO");
    if (e && *e) return (int32_t)std::max(0L, std::min(strtol(e, nullptr, 10), 1L << 30));
    return 16;
}

static Launch base_launch(Runner &r, int32_t nprob, const rac_options &o) {
    Launch L;
    memset(&L, 0, sizeof(L));
    L.prob_net = r.prob_net;
    L.prob_off = r.prob_off;
    L.nprob = nprob;
    L.mode = o.mode;
    L.max_sweeps = o.max_sweeps;
    L.ws = r.ws;
    L.rc_out = r.rc;
    L.checks_out = r.checks;
    L.arcs1 = 0;
    L.push_ratio = push_ratio();
    return L;
}

// Step bound over the nets of a launch.
static int32_t step_cap(const rac_options &o, int64_t max_nd) {
    if (o.max_sweeps > 0) return o.max_sweeps;
    return (int32_t)std::min<int64_t>(max_nd + 1, INT32_MAX - 128);
}

static int rc_from_device(int32_t dev_rc) {
    if (dev_rc & 1) return set_error(RAC_ENOTCONVERGED, "max_sweeps reached before the fixpoint");
    return RAC_OK;
}

static int check_domains(const uint64_t *dom, int64_t count, int32_t d) {
    const uint64_t bad = d >= 64 ? 0ull : ~((1ull << d) - 1ull);
    for (int64_t i = 0; i < count; ++i)
        if (dom[i] & bad)
            return set_error(RAC_EINVAL, "domain word %lld has bits >= d", (long long)i);
    return RAC_OK;
}

// Prepare the runner of a net for B states sharing the net's path.
static int prepare_net_runner(rac_net *net, int32_t B, PathData &pd) {
    Runner &r = net->run;
    const int64_t nvars = (int64_t)B * net->n;
    RAC_TRY(ensure_runner(r, B, nvars));
    const int64_t key = (int64_t)B * 2147483648LL + pd.nitems;
    if (r.tables_key == key) return RAC_OK;
    std::vector<int32_t> pn((size_t)B, 0);
    std::vector<int64_t> off((size_t)B + 1);
    for (int32_t s = 0; s <= B; ++s) off[(size_t)s] = (int64_t)s * net->n;
    HIP_TRY(hipMemcpyAsync(r.prob_net, pn.data(), (size_t)B * 4, hipMemcpyHostToDevice, net->stream));
    HIP_TRY(hipMemcpyAsync(r.prob_off, off.data(), ((size_t)B + 1) * 8, hipMemcpyHostToDevice,
                           net->stream));
    HIP_TRY(hipStreamSynchronize(net->stream));
    r.tables_key = key;
    return RAC_OK;
}

static void fill_stats_bits(rac_stats &st, const std::vector<long long> &checks,
                            const std::vector<int32_t> &iters, int32_t path, const PathData &pd,
                            float ms) {
    memset(&st, 0, sizeof(st));
    for (size_t i = 0; i < checks.size(); ++i) {
        st.support_checks += checks[i];
        st.sweeps += iters[i];
    }
    st.path = path;
    st.item_bytes = pd.item_bytes;
    st.device_ms = ms;
    st.relation_bytes = 0;
}

// Item size argument of ensure_path for a call on B states of one net.
static int32_t call_target(const rac_net *net, int32_t B) {
    return net->opt.item_bytes > 0 ? net->opt.item_bytes : -std::max<int32_t>(1, B);
}

static int32_t stage_vars_for(int64_t max_n) {
    return (int32_t)std::min<int64_t>(max_n, kStageMax);
}


// Bit / int8 path for B states already in r.din (host waits between rounds).
// item_bytes > 0 fixes the work-item size (else the default for B states).
// d_count non-null: the first *d_count of the B states run (a device count,
// see Launch::nprob_dev); on the fused path count_bound (> 0) bounds the grid,
// whose workgroups stride over those states.
static int run_states(rac_net *net, int32_t B, int32_t path, const uint8_t *d_changed,
                      long long arcs1, bool allow_graph = true, bool readback = false,
                      int32_t item_bytes = 0, const int32_t *d_count = nullptr,
                      int32_t count_bound = 0) {
    const bool fused = path == RAC_PATH_FUSED;
    if (fused) path = RAC_PATH_BITS;
    PathData &pd = path == RAC_PATH_INT8 ? net->i8 : net->bits;
    RAC_TRY(ensure_path(net, path, item_bytes > 0 ? item_bytes : call_target(net, B)));
    Runner &r = net->run;
    Launch L = base_launch(r, B, net->opt);
    L.nets = pd.d_desc;
    L.uniform_n = net->n;   // every problem an instance of this net, at s*n
    L.stage_vars = stage_vars_for(net->n);
    L.din = r.din;
    L.dout = r.dout;
    L.iters_out = r.iters;
    L.status_out = r.status;
    L.changed0 = d_changed;
    L.arcs1 = arcs1;
    L.nprob_dev = d_count;
    if (fused)   // the grid strides over the states that run (at most count_bound)
        return launch_fused(r, net->stream, L, net->n, net->groups,
                            d_count ? kFusedWavesSearch : B == 1 ? kFusedWavesOne : kFusedWavesBatch,
                            net->opt.profile != 0, readback ? (int64_t)B * net->n : -1,
                            d_count ? count_bound : 0);
    RAC_TRY(launch_fixpoint(r, net->device, net->stream, L, (int64_t)B * net->n,
                            (int64_t)pd.nitems * B, step_cap(net->opt, (int64_t)net->n * net->d),
                            allow_graph && net->opt.use_graph != 0, net->opt.profile != 0,
                            readback ? (int64_t)B * net->n : -1));
    return RAC_OK;
}

static int collect_bits(rac_net *net, int32_t B, int32_t path, uint64_t *dom, int32_t *iters,
                        int32_t *status) {
    Runner &r = net->run;
    const int32_t used = path;
    if (path == RAC_PATH_FUSED) path = RAC_PATH_BITS;
    PathData &pd = path == RAC_PATH_INT8 ? net->i8 : net->bits;
    std::vector<int32_t> hi, hs;
    std::vector<long long> hc;
    int32_t hrc = 0;
    RAC_TRY(read_results(r, net->stream, B, (int64_t)B * net->n, dom, hc, hi, hs, &hrc));
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, r.ev0, r.ev1);
    fill_stats_bits(net->last, hc, hi, used, pd, ms);
    net->last.relation_bytes = (int64_t)pd.rows_bytes;
    revise_timing(r, &net->last.kernel_ms, &net->last.kernel_launches,
                 &net->last.first_kernel_ms);
    if (iters) memcpy(iters, hi.data(), (size_t)B * 4);
    if (status) memcpy(status, hs.data(), (size_t)B * 4);
    return rc_from_device(hrc);
}

// ---------------------------------------------------------------------------
// autotuner: path and work-item size per call
// ---------------------------------------------------------------------------

struct CallChoice {
    int32_t path = RAC_PATH_BITS;
    int32_t item_scale_log2 = 0;   // work items of 2^s times the default size
    int32_t handoff = -1;          // matrix-core path: -1 the default threshold
    int32_t source = kSourceRules;
};

static int effective_tune_mode(const rac_options &o) {
    if (o.tune == 1) return kTuneRules;
    if (o.tune == 2) return kTuneMeasure;
    return tune_mode();
}

// Relation bytes of one state's full sweep on a path (as ensure_path lays
// them out), for the default item size of a call.
static int64_t path_rows_bytes(const rac_net *net, int32_t path) {
    if (path == RAC_PATH_INT8) return net->arcs * net->d * round_up(net->d, 16);
    const int64_t qpa = net->d <= 32 ? round_up(net->d, 4) / 4 : round_up(net->d, 8) / 2;
    return net->groups * qpa * 1024;
}

// Fixed rule for the fused path (one workgroup per state, every step in one
// launch): networks whose bit rows fit the L2 caches many times over, where
// one workgroup's latency-bound sweep beats three launches per step. Bounds
// on the bit rows of one state, measured on MI355X: 512 KiB for a single
// state, 2 MiB for batches of states and for search rounds (whose children
// re-examine few arcs per step: model-B n = 500, 1.5 MiB of rows, searches
// 1.8x faster fused; n = 1000, 6 MiB, 2x slower).
enum { kFusedRuleOne = 512 << 10, kFusedRuleBatch = 2 << 20, kFusedRuleSearch = 2 << 20 };
static bool fused_rule(const rac_net *net, int64_t max_rows_bytes) {
    if (net->n > kSmallMaxN) return false;
    return path_rows_bytes(net, RAC_PATH_BITS) <= max_rows_bytes;
}

// The item size argument of ensure_path / run_states for B states.
static int32_t choice_items(const rac_net *net, const CallChoice &c, int32_t B) {
    if (net->opt.item_bytes > 0) return net->opt.item_bytes;
    if (c.item_scale_log2 == 0) return 0;   // the default for B states
    const int64_t t = (int64_t)default_item_bytes(net->device, path_rows_bytes(net, c.path) *
                                                   std::max<int32_t>(1, B));
    const int64_t sc = c.item_scale_log2 > 0 ? t << c.item_scale_log2 : t >> -c.item_scale_log2;
    return (int32_t)std::max<int64_t>(4096, std::min<int64_t>(sc, 16 << 20));
}

// The choice for a call: the caller's options, else the tuned table, else
// the fixed rules. *measure: the shape is not in the table and may be measured.
static CallChoice lookup_choice(rac_net *net, int kind, int32_t B, bool *measure) {
    CallChoice c;
    *measure = false;
    const int32_t req = net->opt.path;
    if (req != RAC_PATH_AUTO || net->opt.item_bytes > 0) {
        c.path = kind == kTuneSingle
                     ? (req == RAC_PATH_INT8 || req == RAC_PATH_FUSED ? req : RAC_PATH_BITS)
                     : (req == RAC_PATH_AUTO ? RAC_PATH_BITS : req);
        if (kind == kTuneBatch && req == RAC_PATH_AUTO)
            c.path = mfma_auto_choice(net->d, net->n, net->arcs, B) ? RAC_PATH_MFMA : RAC_PATH_BITS;
        return c;
    }
    // fixed rules: the fused path for small networks; else bit rows for one
    // state, the matrix cores for many states of a dense network with d <= 32
    c.path = kind == kTuneBatch && mfma_auto_choice(net->d, net->n, net->arcs, B) ? RAC_PATH_MFMA
                                                                                  : RAC_PATH_BITS;
    if (fused_rule(net, kind == kTuneBatch ? kFusedRuleBatch : kFusedRuleOne))
        c.path = RAC_PATH_FUSED;
    const int mode = effective_tune_mode(net->opt);
    if (mode == kTuneRules) return c;
    TuneChoice t;
    if (mode != kTuneMeasure && tune_lookup(tune_key(kind, net->n, net->d, net->arcs, B), &t) &&
        (t.path != RAC_PATH_MFMA || net->d <= 32) && (t.path != RAC_PATH_INT8 || net->d <= 32) &&
        (t.path != RAC_PATH_FUSED || net->n <= kSmallMaxN) &&
        (kind == kTuneBatch || t.path != RAC_PATH_MFMA)) {
        c.path = t.path;
        c.item_scale_log2 = t.item_scale_log2;
        c.handoff = t.handoff;
        c.source = t.source;
        return c;
    }
    // a call capped below the step bound (max_sweeps > 0) is no sample of
    // the shape's own runs: it takes the rules and stores nothing
    if (net->opt.max_sweeps > 0) return c;
    *measure = true;
    return c;
}

static std::vector<CallChoice> tune_candidates(const rac_net *net, int kind, int32_t B) {
    std::vector<CallChoice> v;
    auto add = [&](int32_t path, int32_t s, int32_t h) {
        CallChoice c;
        c.path = path;
        c.item_scale_log2 = s;
        c.handoff = h;
        c.source = kSourceMeasured;
        v.push_back(c);
    };
    add(RAC_PATH_BITS, 0, -1);
    add(RAC_PATH_BITS, 2, -1);
    if (kind == kTuneSingle) add(RAC_PATH_BITS, -2, -1);
    if (net->d <= 32) add(RAC_PATH_INT8, 0, -1);
    if (net->n <= kSmallMaxN) add(RAC_PATH_FUSED, 0, -1);
    if (kind == kTuneBatch && net->d <= 32 && B >= 8) {
        add(RAC_PATH_MFMA, 0, 32);
        add(RAC_PATH_MFMA, 0, 0);
    }
    return v;
}

static void remember(rac_net *net, int kind, int32_t B, const CallChoice &c, double ms) {
    TuneChoice t;
    t.path = c.path;
    t.item_scale_log2 = c.item_scale_log2;
    t.handoff = c.handoff;
    t.ms = ms;
    tune_store(tune_key(kind, net->n, net->d, net->arcs, B), t);
}

// One state on the bit or int8 path with a given choice (host buffers).
static int enforce_one(rac_net *net, const uint64_t *din, uint64_t *dout, const int32_t *changed,
                       int32_t n_changed, int32_t *iters, int32_t *status, const CallChoice &c) {
    const int32_t path = c.path == RAC_PATH_INT8 ? RAC_PATH_INT8 : RAC_PATH_BITS;   // rows used
    const int32_t run_path = c.path == RAC_PATH_FUSED ? RAC_PATH_FUSED : path;
    const int32_t items = choice_items(net, c, 1);
    RAC_TRY(ensure_path(net, path, items > 0 ? items : call_target(net, 1)));
    RAC_TRY(prepare_net_runner(net, 1, path == RAC_PATH_INT8 ? net->i8 : net->bits));
    Runner &r = net->run;
    memcpy(r.h_dom, din, (size_t)net->n * 8);
    HIP_TRY(hipMemcpyAsync(r.din, r.h_dom, (size_t)net->n * 8, hipMemcpyHostToDevice, net->stream));
    const uint8_t *d_changed = nullptr;
    long long arcs1 = 0;
    if (changed) {
        std::vector<uint8_t> mask((size_t)net->n, 0);
        long long degs = 0;
        for (int32_t i = 0; i < n_changed; ++i) {
            const int32_t x = changed[i];
            if (x < 0 || x >= net->n) return set_error(RAC_EINVAL, "changed[%d] out of range", i);
            if (!mask[(size_t)x]) degs += net->h_deg[(size_t)x];
            mask[(size_t)x] = 1;
        }
        HIP_TRY(hipMemcpyAsync(r.changed, mask.data(), (size_t)net->n, hipMemcpyHostToDevice,
                               net->stream));
        HIP_TRY(hipStreamSynchronize(net->stream));
        d_changed = r.changed;
        arcs1 = degs;
    }
    RAC_TRY(run_states(net, 1, run_path, d_changed, arcs1, true, true, items));
    RAC_TRY(collect_bits(net, 1, run_path, dout, iters, status));
    net->last.tune_source = c.source;
    return RAC_OK;
}

extern "C" int rac_enforce(rac_net *net, uint64_t *dom, const int32_t *changed, int32_t n_changed,
                           int32_t *iters, int32_t *status) {
    if (!net || !dom) return set_error(RAC_EINVAL, "net or dom is NULL");
    if (changed && n_changed < 0) return set_error(RAC_EINVAL, "n_changed < 0");
    RAC_TRY(check_domains(dom, net->n, net->d));
    HIP_TRY(hipSetDevice(net->device));
    RAC_TRY(settle(net));
    bool measure = false;
    CallChoice c = lookup_choice(net, kTuneSingle, 1, &measure);
    if (measure) {
        // every candidate on this call's own state (identical results): one
        // untimed run (packing, item tables), then the best of two timed ones
        std::vector<uint64_t> in(dom, dom + net->n), out((size_t)net->n);
        double best = 1e30;
        for (const CallChoice &cand : tune_candidates(net, kTuneSingle, 1)) {
            double t = 1e30;
            for (int rep = 0; rep < 3; ++rep) {
                const auto t0 = std::chrono::steady_clock::now();
                const int rc = enforce_one(net, in.data(), out.data(), changed, n_changed, nullptr,
                                           nullptr, cand);
                if (rc != RAC_OK && rc != RAC_ENOTCONVERGED) return rc;
                if (rep > 0)
                    t = std::min(t, std::chrono::duration<double, std::milli>(
                                        std::chrono::steady_clock::now() - t0).count());
            }
            if (t < best) {
                best = t;
                c = cand;
            }
        }
        remember(net, kTuneSingle, 1, c, best);
    }
    return enforce_one(net, dom, dom, changed, n_changed, iters, status, c);
}

// The hand-off's bit-row steps read each group's rows once for several
// states (revise_shared_kernel); RAC_SHARED_ROWS=0 revises state by state.
static bool shared_rows_on() {
    const char *e = getenv("RAC_SHARED_ROWS");
    return !(e && e[0] == '0');
}

// States still active when at most this many remain leave the matrix-core
// path and finish on the bit-row path, whose incremental steps
// touch only arcs into changed variables.
static int32_t mfma_handoff_threshold(int32_t tuned) {
    const char *e = getenv("RAC_MFMA_HANDOFF");
    if (e) return std::max(0, atoi(e));
    return tuned >= 0 ? tuned : 32;
}

// The batched matrix-core path: matrix-core steps while many states are
// active, then the stragglers on the bit-row path (continuing from D^(k)
// with @changed = the variables step k changed, Proposition 2).
static int run_mfma(rac_net *net, int32_t B, const uint64_t *d_in, uint64_t *d_out,
                    int32_t *d_it, int32_t *d_st, hipStream_t s, int32_t handoff) {
    RAC_TRY(mfma_ensure(net->mfma, net->n, net->d, net->arcs, net->row_ptr, net->nbr, net->deg,
                        net->rel, net->arc_src, net->h_row_ptr, net->stream));
    int32_t k = 0, P = 0;
    RAC_TRY(mfma_start(net->mfma, B, d_in, d_out, net->opt.mode, net->opt.max_sweeps,
                       net->opt.profile, handoff, s, &k, &P));
    if (P > 0) {
        RAC_TRY(ensure_path(net, RAC_PATH_BITS, call_target(net, P)));
        PathData &pd = net->bits;
        RAC_TRY(prepare_net_runner(net, P, pd));
        Runner &r = net->run;
        RAC_TRY(mfma_handoff(net->mfma, k, r.din, r.changed, s));
        Launch L = base_launch(r, P, net->opt);
        L.nets = pd.d_desc;
        L.uniform_n = net->n;   // every problem an instance of this net, at s*n
        L.stage_vars = stage_vars_for(net->n);
        L.din = r.din;
        L.dout = r.dout;
        L.iters_out = r.iters;
        L.status_out = r.status;
        L.changed0 = r.changed;
        L.arcs1 = 0;   // the matrix-core finaliser already counted step k+1
        const int32_t maxs = net->opt.max_sweeps > 0 ? net->opt.max_sweeps : net->n * net->d + 1;
        L.max_sweeps = maxs - k;
        // the states left are those with long, dense propagation: each step
        // reads every group's rows once for up to kSharedStates of them
        int64_t items = (int64_t)pd.nitems * P;
        if (shared_rows_on() && pd.desc.kind == ROW32) {
            L.shared_rows = 1;
            L.stage_vars = 0;
            items = net->groups * ((P + kSharedStates - 1) / kSharedStates);
        }
        RAC_TRY(launch_fixpoint(r, net->device, s, L, (int64_t)P * net->n, items, maxs - k, true,
                                false));
        RAC_TRY(mfma_merge(net->mfma, k, r.dout, r.iters, r.status, r.checks, r.rc, s));
    }
    RAC_TRY(mfma_finish(net->mfma, d_it, d_st, s));
    return RAC_OK;
}

// ---------------------------------------------------------------------------
// batched MAC search (Algorithm 2)
// ---------------------------------------------------------------------------

// Rounds the device-driven search enqueues between reads of its control block
// (1, 2, 4, then this many).
constexpr int32_t kSearchRoundsMax = 8;

// The search's device buffers: the node stack and the per-round lists, kept
// on the net and grown on demand, so that repeated searches allocate nothing.
struct SearchWork {
    uint64_t *stack = nullptr, *best = nullptr;
    int32_t *bvar = nullptr, *nchild = nullptr, *coff = nullptr, *has_best = nullptr;
    long long *stats = nullptr;
    int32_t *is_sol = nullptr, *is_open = nullptr, *sol_off = nullptr, *open_off = nullptr,
            *sol_list = nullptr;
    long long *h_stats = nullptr;   // pinned: a round's summary
    SearchCtl *ctl = nullptr;       // the search's control block (device)
    SearchCtl *h_ctl = nullptr;     // pinned mirror
    int64_t cap = 0;                // stack capacity in nodes
    int32_t cap_batch = 0, cap_children = 0, cap_n = 0;
    // captured batches of 1, 2, 4 and 8 device-driven rounds, valid for `key`
    hipGraph_t graph[4] = {};
    hipGraphExec_t exec[4] = {};
    std::vector<unsigned char> key;
    void drop_graphs() {
        for (int i = 0; i < 4; ++i) {
            if (exec[i]) (void)hipGraphExecDestroy(exec[i]);
            if (graph[i]) (void)hipGraphDestroy(graph[i]);
            exec[i] = nullptr;
            graph[i] = nullptr;
        }
        key.clear();
    }
    ~SearchWork() {
        drop_graphs();
        if (h_stats) (void)hipHostFree(h_stats);
        if (h_ctl) (void)hipHostFree(h_ctl);
        dfree(ctl);
        dfree(stack);
        dfree(best);
        dfree(bvar);
        dfree(nchild);
        dfree(coff);
        dfree(has_best);
        dfree(is_sol);
        dfree(is_open);
        dfree(sol_off);
        dfree(open_off);
        dfree(sol_list);
        dfree(stats);
    }
};

static void release_search(rac_net *net) {
    delete net->search;
    net->search = nullptr;
}

// Buffers for rounds of up to `batch` open nodes with up to `cmax` children
// on a network of n variables, and a stack of at least `min_cap` nodes.
static int ensure_search_work(rac_net *net, int32_t batch, int32_t cmax, int32_t n, int64_t min_cap) {
    SearchWork *w = net->search;
    if (w && w->cap_batch >= batch && w->cap_children >= cmax && w->cap_n == n && w->cap >= min_cap)
        return RAC_OK;
    release_search(net);
    w = net->search = new SearchWork();
    w->cap = min_cap;
    RAC_TRY(dalloc(&w->stack, (size_t)(w->cap * n)));
    RAC_TRY(dalloc(&w->best, (size_t)n));
    RAC_TRY(dalloc(&w->bvar, (size_t)batch));
    RAC_TRY(dalloc(&w->nchild, (size_t)batch));
    RAC_TRY(dalloc(&w->coff, (size_t)batch + 1));
    RAC_TRY(dalloc(&w->has_best, 1));
    RAC_TRY(dalloc(&w->is_sol, (size_t)cmax));
    RAC_TRY(dalloc(&w->is_open, (size_t)cmax));
    RAC_TRY(dalloc(&w->sol_off, (size_t)cmax + 1));
    RAC_TRY(dalloc(&w->open_off, (size_t)cmax + 1));
    RAC_TRY(dalloc(&w->sol_list, (size_t)cmax));
    RAC_TRY(dalloc(&w->stats, 8));
    HIP_TRY(hipHostMalloc((void **)&w->h_stats, 8 * sizeof(long long), hipHostMallocDefault));
    RAC_TRY(dalloc(&w->ctl, 1));
    HIP_TRY(hipHostMalloc((void **)&w->h_ctl, sizeof(SearchCtl), hipHostMallocDefault));
    w->cap_batch = batch;
    w->cap_children = cmax;
    w->cap_n = n;
    return RAC_OK;
}

// Everything the kernels of a device-driven round take as arguments.
struct SearchRoundArgs {
    Launch L;   // the fused enforcement of the round's children
    uint64_t *stack;
    int32_t batch, n, gnode, gc, gfused, threads;
    size_t lds;
    long long max_solutions, max_nodes;
};

// A graph of K device-driven rounds: begin, branch, offsets (which also
// clears the enforcement's flag word), expand, the fused enforcement, classify,
// lists, push, best, end (kernel arguments are copied into the nodes).
static int build_search_graph(SearchWork &b, Runner &r, const SearchRoundArgs &a, int32_t K,
                              hipGraph_t *graph, hipGraphExec_t *exec) {
    HIP_TRY(hipGraphCreate(graph, 0));
    hipGraphNode_t prev = nullptr;
    SearchRoundArgs v = a;
    SearchCtl *ctl = b.ctl;
    int32_t *count = r.count, *rc = r.rc;
    uint8_t *changed = r.changed;
    uint64_t *din = r.din, *dout = r.dout;
    int32_t *status = r.status, *iters = r.iters;
    void *p_begin[4] = {&ctl, &v.batch, &v.max_solutions, &v.max_nodes};
    void *p_branch[5] = {&v.stack, &ctl, &v.n, &b.bvar, &b.nchild};
    void *p_off[5] = {&b.nchild, &ctl, &b.coff, &count, &rc};
    void *p_expand[7] = {&v.stack, &ctl, &v.n, &b.bvar, &b.coff, &din, &changed};
    void *p_fused[1] = {&v.L};
    void *p_class[6] = {&dout, &status, &v.n, &count, &b.is_sol, &b.is_open};
    void *p_lists[8] = {&b.is_sol, &b.is_open, &iters, &count, &rc, &b.sol_off, &b.open_off, &b.stats};
    void *p_push[10] = {&dout, &v.n, &count, &b.is_sol, &b.is_open, &b.sol_off, &b.open_off,
                        &v.stack, &ctl, &b.sol_list};
    void *p_best[7] = {&dout, &v.n, &b.sol_list, &b.sol_off, &count, &b.best, &b.has_best};
    void *p_end[2] = {&ctl, &b.stats};
    for (int32_t i = 0; i < K; ++i) {
        RAC_TRY(add_node(*graph, &prev, (const void *)search_begin_kernel, dim3(1), dim3(64), 0, p_begin));
        RAC_TRY(add_node(*graph, &prev, (const void *)search_branch_kernel, dim3((unsigned)v.gnode),
                         dim3(64), 0, p_branch));
        RAC_TRY(add_node(*graph, &prev, (const void *)search_offsets_kernel, dim3(1), dim3(1024), 0, p_off));
        RAC_TRY(add_node(*graph, &prev, (const void *)search_expand_kernel, dim3((unsigned)v.gnode),
                         dim3(256), 0, p_expand));
        RAC_TRY(add_node(*graph, &prev, (const void *)small_fixpoint_kernel, dim3((unsigned)v.gfused),
                         dim3((unsigned)v.threads), v.lds, p_fused));
        RAC_TRY(add_node(*graph, &prev, (const void *)search_classify_kernel, dim3((unsigned)v.gc),
                         dim3(64), 0, p_class));
        RAC_TRY(add_node(*graph, &prev, (const void *)search_lists_kernel, dim3(1), dim3(1024), 0, p_lists));
        RAC_TRY(add_node(*graph, &prev, (const void *)search_push_kernel, dim3((unsigned)v.gc),
                         dim3(256), 0, p_push));
        RAC_TRY(add_node(*graph, &prev, (const void *)search_best_kernel, dim3(1), dim3(1024), 0, p_best));
        RAC_TRY(add_node(*graph, &prev, (const void *)search_end_kernel, dim3(1), dim3(64), 0, p_end));
    }
    HIP_TRY(hipGraphInstantiate(exec, *graph, nullptr, nullptr, 0));
    return RAC_OK;
}

namespace {
bool all_singletons(const uint64_t *dom, int32_t n) {
    for (int32_t x = 0; x < n; ++x)
        if (__builtin_popcountll(dom[x]) != 1) return false;
    return true;
}
}  // namespace

extern "C" int rac_search(rac_net *net, const uint64_t *dom, int64_t max_solutions,
                          int64_t max_nodes, int32_t batch, uint64_t *solution,
                          rac_search_result *out) {
    if (!net || !dom || !out) return set_error(RAC_EINVAL, "net, dom or out is NULL");
    if (batch < 0 || max_solutions < 0 || max_nodes < 0)
        return set_error(RAC_EINVAL, "negative batch or limit");
    const int32_t n = net->n, d = net->d;
    if (n >= (1 << 20)) return set_error(RAC_EUNSUPPORTED, "search supports n < 2^20");
    RAC_TRY(check_domains(dom, n, d));
    HIP_TRY(hipSetDevice(net->device));
    RAC_TRY(settle(net));
    const auto t0 = std::chrono::steady_clock::now();
    memset(out, 0, sizeof(*out));
    if (batch == 0) batch = 256;
    batch = std::min<int32_t>(batch, 1 << 16);
    const int32_t path = net->opt.path == RAC_PATH_INT8 ? RAC_PATH_INT8 : RAC_PATH_BITS;
    PathData &pd = path == RAC_PATH_INT8 ? net->i8 : net->bits;
    // the enforcements themselves: one fused launch per round when asked for,
    // or by the fixed rules on small networks (the root: one state's rule)
    const bool rules = net->opt.path == RAC_PATH_AUTO && net->opt.item_bytes == 0;
    const bool fused = net->opt.path == RAC_PATH_FUSED || (rules && fused_rule(net, kFusedRuleSearch));
    const bool fused_root = net->opt.path == RAC_PATH_FUSED || (rules && fused_rule(net, kFusedRuleOne));
    const int32_t run_path = fused ? RAC_PATH_FUSED : path;
    // a wipe-out anywhere ends a node: stop on the first one (same status as
    // running to the fixpoint, fewer steps)
    struct ModeGuard {
        rac_net *net;
        int32_t mode;
        ~ModeGuard() { net->opt.mode = mode; }
    } guard{net, net->opt.mode};
    net->opt.mode = RAC_STOP_ON_WIPEOUT;
    Runner &r = net->run;
    hipStream_t s = net->stream;

    // the root: full enforcement
    RAC_TRY(ensure_path(net, path, call_target(net, 1)));
    RAC_TRY(prepare_net_runner(net, 1, pd));
    HIP_TRY(hipMemcpyAsync(r.din, dom, (size_t)n * 8, hipMemcpyHostToDevice, s));
    RAC_TRY(run_states(net, 1, fused_root ? RAC_PATH_FUSED : path, nullptr, 0, false));
    std::vector<uint64_t> root((size_t)n);
    int32_t root_status = 0, hrc = 0, root_iters = 0;
    HIP_TRY(hipMemcpyAsync(root.data(), r.dout, (size_t)n * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&root_status, r.status, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&root_iters, r.iters, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&hrc, r.rc, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    RAC_TRY(rc_from_device(hrc));
    out->nodes = 1;
    out->sweeps = root_iters;
    auto finish = [&]() {
        out->search_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        return RAC_OK;
    };
    if (root_status == RAC_WIPEOUT) {
        out->failures = 1;
        out->complete = 1;
        return finish();
    }
    if (all_singletons(root.data(), n)) {
        out->solutions = 1;
        out->complete = 1;
        if (solution) memcpy(solution, root.data(), (size_t)n * 8);
        return finish();
    }

    // device buffers: the stack and the per-round lists (kept on the net).
    // On the fused path every round is one launch, so rounds follow each
    // other on the device (the control block decides each round's nodes):
    // the host enqueues 1, 2, 4, 8, 8, ... rounds and reads the control block
    // once per batch of rounds. The bit-row path's enforcement waits on the
    // host between its rounds of steps, so there the host reads it per round.
    const int32_t cmax = batch * d;
    const bool device_rounds = fused;
    const int64_t grow = (int64_t)kSearchRoundsMax * cmax;   // stack growth bound of a batch of rounds
    RAC_TRY(ensure_search_work(net, batch, cmax, n, std::max<int64_t>(grow + cmax, 1024)));
    SearchWork &b = *net->search;
    HIP_TRY(hipMemsetAsync(b.has_best, 0, 4, s));
    HIP_TRY(hipMemcpyAsync(b.stack, root.data(), (size_t)n * 8, hipMemcpyHostToDevice, s));
    {
        SearchCtl &c0 = *b.h_ctl;
        memset(&c0, 0, sizeof(c0));
        c0.ssize = 1;
        c0.nodes = 1;   // the root
        c0.sweeps = root_iters;
        HIP_TRY(hipMemcpyAsync(b.ctl, &c0, sizeof(SearchCtl), hipMemcpyHostToDevice, s));
    }
    RAC_TRY(ensure_path(net, path, call_target(net, cmax)));
    // one work-item size for every round (the one for cmax states), so that
    // rounds of different sizes reuse the item table
    const int32_t item_bytes = pd.item_bytes;
    // problem tables for cmax states once: a round with C <= cmax children uses
    // their prefix (problem s at s*n)
    RAC_TRY(prepare_net_runner(net, cmax, pd));
    // workgroups of the per-node and per-child kernels on the device-driven
    // path (they stride over the nodes and children; 4096 fused workgroups
    // of 4 waves measured best: 2048 leave CUs idle, one per child launches
    // tens of thousands that mostly return)
    const int32_t gchild = std::min<int32_t>(cmax, 4096);
    const int32_t gnodes = std::min<int32_t>(batch, 1024);
    int64_t ssize = 1;   // stack size after the last read of the control block
    for (int32_t batch_i = 0;; ++batch_i) {
        const int32_t K = device_rounds ? std::min(1 << std::min(batch_i, 3), kSearchRoundsMax) : 1;
        static_assert(kSearchRoundsMax == 8, "graphs of 1, 2, 4 and 8 rounds");
        // every round pops before it pushes, and pushes at most P * d nodes
        // above its base: grow the stack first (device copy of the live part)
        if (ssize + (int64_t)K * cmax > b.cap) {
            const int64_t ncap = std::max<int64_t>(2 * b.cap, ssize + (int64_t)K * cmax);
            uint64_t *ns = nullptr;
            RAC_TRY(dalloc(&ns, (size_t)(ncap * n)));
            HIP_TRY(hipMemcpyAsync(ns, b.stack, (size_t)(ssize * n) * 8, hipMemcpyDeviceToDevice, s));
            HIP_TRY(hipStreamSynchronize(s));
            dfree(b.stack);
            b.stack = ns;
            b.cap = ncap;
        }
        // the host knows P on the round-by-round path: exact grids there
        const int32_t P = (int32_t)std::min<int64_t>(ssize, batch);
        const int32_t gnode = device_rounds ? gnodes : std::max(P, 1);
        const int32_t gc = device_rounds ? gchild : std::max(P * d, 1);
        if (device_rounds && net->opt.use_graph != 0 && !net->opt.profile) {
            // K rounds as one captured graph (built once per network and shape)
            SearchRoundArgs a;
            memset(&a, 0, sizeof(a));
            a.L = base_launch(r, cmax, net->opt);
            a.L.nets = pd.d_desc;
            a.L.uniform_n = n;
            a.L.din = r.din;
            a.L.dout = r.dout;
            a.L.iters_out = r.iters;
            a.L.status_out = r.status;
            a.L.changed0 = r.changed;
            a.L.arcs1 = -1;
            a.L.nprob_dev = r.count;
            a.stack = b.stack;
            a.batch = batch;
            a.n = n;
            a.gnode = gnodes;
            a.gc = gchild;
            a.gfused = gchild;
            a.threads = small_threads(net->groups, kFusedWavesSearch);
            a.lds = small_lds_bytes(n);
            a.max_solutions = max_solutions;
            a.max_nodes = max_nodes;
            std::vector<unsigned char> key(sizeof(a));
            memcpy(key.data(), &a, sizeof(a));
            if (key != b.key) {
                b.drop_graphs();
                b.key = key;
            }
            const int gi = K >= 8 ? 3 : K >= 4 ? 2 : K >= 2 ? 1 : 0;
            if (!b.exec[gi]) RAC_TRY(build_search_graph(b, r, a, 1 << gi, &b.graph[gi], &b.exec[gi]));
            HIP_TRY(hipGraphLaunch(b.exec[gi], s));
        } else
        for (int32_t i = 0; i < K; ++i) {
            hipLaunchKernelGGL(search_begin_kernel, dim3(1), dim3(64), 0, s, b.ctl, batch,
                               (long long)max_solutions, (long long)max_nodes);
            hipLaunchKernelGGL(search_branch_kernel, dim3((unsigned)gnode), dim3(64), 0, s, b.stack,
                               b.ctl, n, b.bvar, b.nchild);
            // the child count C stays on the device (r.count): the kernels
            // below read it, and the host learns it with the round's summary
            hipLaunchKernelGGL(search_offsets_kernel, dim3(1), dim3(1024), 0, s, b.nchild, b.ctl,
                               b.coff, r.count, r.rc);
            hipLaunchKernelGGL(search_expand_kernel, dim3((unsigned)gnode), dim3(256), 0, s,
                               b.stack, b.ctl, n, b.bvar, b.coff, r.din, r.changed);
            HIP_TRY(hipGetLastError());
            // launched for cmax states with the count on the device: the same
            // arguments every round, so the captured step graphs are reused
            RAC_TRY(run_states(net, cmax, run_path, r.changed, -1, true, false, item_bytes, r.count,
                               gc));
            hipLaunchKernelGGL(search_classify_kernel, dim3((unsigned)gc), dim3(64), 0, s, r.dout,
                               r.status, n, r.count, b.is_sol, b.is_open);
            hipLaunchKernelGGL(search_lists_kernel, dim3(1), dim3(1024), 0, s, b.is_sol, b.is_open,
                               r.iters, r.count, r.rc, b.sol_off, b.open_off, b.stats);
            hipLaunchKernelGGL(search_push_kernel, dim3((unsigned)gc), dim3(256), 0, s, r.dout, n,
                               r.count, b.is_sol, b.is_open, b.sol_off, b.open_off, b.stack, b.ctl,
                               b.sol_list);
            hipLaunchKernelGGL(search_best_kernel, dim3(1), dim3(1024), 0, s, r.dout, n,
                               b.sol_list, b.sol_off, r.count, b.best, b.has_best);
            hipLaunchKernelGGL(search_end_kernel, dim3(1), dim3(64), 0, s, b.ctl, b.stats);
            HIP_TRY(hipGetLastError());
        }
        HIP_TRY(hipMemcpyAsync(b.h_ctl, b.ctl, sizeof(SearchCtl), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        const SearchCtl &c = *b.h_ctl;
        ssize = c.ssize;
        out->nodes = c.nodes;
        out->sweeps = c.sweeps;
        out->solutions = c.solutions;
        out->failures = c.failures;
        out->rounds = c.rounds;
        out->complete = c.complete;
        RAC_TRY(rc_from_device(c.rc));
        if (c.done) break;
        // what the next round's begin kernel would find, without launching it
        if (ssize == 0) {
            out->complete = 1;
            break;
        }
        if ((max_solutions > 0 && out->solutions >= max_solutions) ||
            (max_nodes > 0 && out->nodes >= max_nodes))
            break;
    }
    int32_t has = 0;
    HIP_TRY(hipMemcpyAsync(&has, b.has_best, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (has && solution)
        HIP_TRY(hipMemcpy(solution, b.best, (size_t)n * 8, hipMemcpyDeviceToHost));
    return finish();
}

// Enqueues B states of one net (device buffers) on stream s with a choice of
// path; the call is then pending on the net (rac_sync_status waits for it).
static int enqueue_batch(rac_net *net, int32_t B, const uint64_t *d_in, uint64_t *d_out,
                         int32_t *d_it, int32_t *d_st, hipStream_t s, const CallChoice &c) {
    net->tune_source = c.source;
    if (c.path == RAC_PATH_MFMA) {
        RAC_TRY(run_mfma(net, B, d_in, d_out, d_it, d_st, s, mfma_handoff_threshold(c.handoff)));
        net->pending = true;
        net->last.path = RAC_PATH_MFMA;
        return RAC_OK;
    }
    const int32_t items = choice_items(net, c, B);
    const int32_t rows = c.path == RAC_PATH_INT8 ? RAC_PATH_INT8 : RAC_PATH_BITS;
    RAC_TRY(ensure_path(net, rows, items > 0 ? items : call_target(net, B)));
    PathData &pd = rows == RAC_PATH_INT8 ? net->i8 : net->bits;
    RAC_TRY(prepare_net_runner(net, B, pd));
    Runner &r = net->run;
    Launch L = base_launch(r, B, net->opt);
    L.nets = pd.d_desc;
    L.uniform_n = net->n;   // every problem an instance of this net, at s*n
    L.stage_vars = stage_vars_for(net->n);
    L.din = d_in;
    L.dout = d_out;
    L.iters_out = d_it;
    L.status_out = d_st;
    if (c.path == RAC_PATH_FUSED)
        RAC_TRY(launch_fused(r, s, L, net->n, net->groups,
                             B == 1 ? kFusedWavesOne : kFusedWavesBatch, net->opt.profile != 0));
    else
        RAC_TRY(launch_fixpoint(r, net->device, s, L, (int64_t)B * net->n, (int64_t)pd.nitems * B,
                                step_cap(net->opt, (int64_t)net->n * net->d),
                                net->opt.use_graph != 0, net->opt.profile != 0));
    net->pending = true;
    net->last.path = c.path;
    net->last.item_bytes = pd.item_bytes;
    net->last.relation_bytes = (int64_t)pd.rows_bytes;
    return RAC_OK;
}

// Measures every candidate choice on B states already on the device (the
// results of all candidates are identical and land in d_out, d_it, d_st):
// one untimed run, then the best of two timed ones; returns the fastest.
static int measure_batch(rac_net *net, int32_t B, const uint64_t *d_in, uint64_t *d_out,
                         int32_t *d_it, int32_t *d_st, hipStream_t s, CallChoice *best_c) {
    double best = 1e30;
    for (const CallChoice &cand : tune_candidates(net, kTuneBatch, B)) {
        double t = 1e30;
        for (int rep = 0; rep < 3; ++rep) {
            HIP_TRY(hipStreamSynchronize(s));
            const auto t0 = std::chrono::steady_clock::now();
            RAC_TRY(enqueue_batch(net, B, d_in, d_out, d_it, d_st, s, cand));
            const int rc = rac_sync_status(net);
            if (rc != RAC_OK && rc != RAC_ENOTCONVERGED) return rc;
            if (rep > 0)
                t = std::min(t, std::chrono::duration<double, std::milli>(
                                    std::chrono::steady_clock::now() - t0).count());
        }
        if (t < best) {
            best = t;
            *best_c = cand;
        }
    }
    remember(net, kTuneBatch, B, *best_c, best);
    return RAC_OK;
}

static int ensure_mf_staging(rac_net *net, int32_t B) {
    if (B <= net->mf_cap) return RAC_OK;
    dfree(net->mf_in);
    dfree(net->mf_out);
    dfree(net->mf_it);
    dfree(net->mf_st);
    RAC_TRY(dalloc(&net->mf_in, (size_t)B * net->n));
    RAC_TRY(dalloc(&net->mf_out, (size_t)B * net->n));
    RAC_TRY(dalloc(&net->mf_it, (size_t)B));
    RAC_TRY(dalloc(&net->mf_st, (size_t)B));
    net->mf_cap = B;
    return RAC_OK;
}

extern "C" int rac_enforce_batch(rac_net *net, int32_t B, uint64_t *dom, int32_t *iters,
                                 int32_t *status) {
    if (!net || (!dom && B > 0)) return set_error(RAC_EINVAL, "net or dom is NULL");
    if (B < 0) return set_error(RAC_EINVAL, "B < 0");
    if (B == 0) return RAC_OK;
    RAC_TRY(check_domains(dom, (int64_t)B * net->n, net->d));
    HIP_TRY(hipSetDevice(net->device));
    RAC_TRY(settle(net));
    bool measure = false;
    CallChoice c = lookup_choice(net, kTuneBatch, B, &measure);
    if (measure) {
        RAC_TRY(ensure_mf_staging(net, B));
        HIP_TRY(hipMemcpyAsync(net->mf_in, dom, (size_t)B * net->n * 8, hipMemcpyHostToDevice,
                               net->stream));
        RAC_TRY(measure_batch(net, B, net->mf_in, net->mf_out, net->mf_it, net->mf_st, net->stream, &c));
    }
    if (c.path == RAC_PATH_MFMA) {
        RAC_TRY(ensure_mf_staging(net, B));
        HIP_TRY(hipMemcpyAsync(net->mf_in, dom, (size_t)B * net->n * 8, hipMemcpyHostToDevice,
                               net->stream));
        RAC_TRY(run_mfma(net, B, net->mf_in, net->mf_out, net->mf_it, net->mf_st, net->stream,
                         mfma_handoff_threshold(c.handoff)));
        HIP_TRY(hipMemcpyAsync(dom, net->mf_out, (size_t)B * net->n * 8, hipMemcpyDeviceToHost,
                               net->stream));
        if (iters)
            HIP_TRY(hipMemcpyAsync(iters, net->mf_it, (size_t)B * 4, hipMemcpyDeviceToHost, net->stream));
        if (status)
            HIP_TRY(hipMemcpyAsync(status, net->mf_st, (size_t)B * 4, hipMemcpyDeviceToHost,
                                   net->stream));
        HIP_TRY(hipStreamSynchronize(net->stream));
        const int rc = mfma_collect(net->mfma, &net->last);
        net->last.tune_source = c.source;
        return rc;
    }
    const int32_t items = choice_items(net, c, B);
    RAC_TRY(ensure_path(net, c.path == RAC_PATH_INT8 ? RAC_PATH_INT8 : RAC_PATH_BITS,
                        items > 0 ? items : call_target(net, B)));
    RAC_TRY(prepare_net_runner(net, B, c.path == RAC_PATH_INT8 ? net->i8 : net->bits));
    memcpy(net->run.h_dom, dom, (size_t)B * net->n * 8);
    HIP_TRY(hipMemcpyAsync(net->run.din, net->run.h_dom, (size_t)B * net->n * 8,
                           hipMemcpyHostToDevice, net->stream));
    RAC_TRY(run_states(net, B, c.path, nullptr, 0, true, true, items));
    const int rc = collect_bits(net, B, c.path, dom, iters, status);
    net->last.tune_source = c.source;
    return rc;
}

extern "C" int rac_enforce_batch_device(rac_net *net, int32_t B, const uint64_t *d_dom_in,
                                        uint64_t *d_dom_out, int32_t *d_iters, int32_t *d_status,
                                        void *stream) {
    if (!net || B < 0) return set_error(RAC_EINVAL, "bad net or B");
    if (B == 0) return RAC_OK;
    if (!d_dom_in || !d_dom_out) return set_error(RAC_EINVAL, "domain pointers are NULL");
    HIP_TRY(hipSetDevice(net->device));
    RAC_TRY(settle(net));
    hipStream_t s = (hipStream_t)stream;
    bool measure = false;
    CallChoice c = lookup_choice(net, kTuneBatch, B, &measure);
    if (measure) {
        if (d_dom_in == d_dom_out) {
            // the candidates must all start from the caller's input
            RAC_TRY(ensure_mf_staging(net, B));
            HIP_TRY(hipMemcpyAsync(net->mf_in, d_dom_in, (size_t)B * net->n * 8,
                                   hipMemcpyDeviceToDevice, s));
            RAC_TRY(measure_batch(net, B, net->mf_in, d_dom_out, d_iters, d_status, s, &c));
        } else {
            RAC_TRY(measure_batch(net, B, d_dom_in, d_dom_out, d_iters, d_status, s, &c));
        }
        // the call itself then runs the chosen path (from the caller's input,
        // restored if it was overwritten), so that the net's counters describe it
        if (d_dom_in == d_dom_out)
            HIP_TRY(hipMemcpyAsync(d_dom_out, net->mf_in, (size_t)B * net->n * 8,
                                   hipMemcpyDeviceToDevice, s));
    }
    RAC_TRY(enqueue_batch(net, B, d_dom_in, d_dom_out, d_iters, d_status, s, c));
    return RAC_OK;
}

extern "C" int rac_sync_status(rac_net *net) {
    if (!net) return set_error(RAC_EINVAL, "net is NULL");
    if (!net->pending) return RAC_OK;
    HIP_TRY(hipSetDevice(net->device));
    net->pending = false;
    if (net->last.path == RAC_PATH_MFMA) {
        const int rc = mfma_collect(net->mfma, &net->last);
        net->last.tune_source = net->tune_source;
        return rc;
    }
    net->last.tune_source = net->tune_source;
    int32_t hrc = 0;
    HIP_TRY(hipEventSynchronize(net->run.ev1));   // the end of the call on the caller's stream
    HIP_TRY(hipMemcpy(&hrc, net->run.rc, 4, hipMemcpyDeviceToHost));
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, net->run.ev0, net->run.ev1);
    net->last.device_ms = ms;
    revise_timing(net->run, &net->last.kernel_ms, &net->last.kernel_launches,
                 &net->last.first_kernel_ms);
    return rc_from_device(hrc);
}

extern "C" int rac_net_stats(const rac_net *net, rac_stats *out) {
    if (!net || !out) return set_error(RAC_EINVAL, "NULL argument");
    *out = net->last;
    return RAC_OK;
}

// ---------------------------------------------------------------------------
// batched states without allocation (workspace in a fixed device array)
// ---------------------------------------------------------------------------

// Workspace of rac_enforce_batch_noalloc: the bit-row path's double-buffered
// domains, change flags, failure accumulators, changed-variable lists and
// per-state control words, carved from one file-scope array per device. Host
// code never passes the array's name to a kernel (that is a host-side
// stand-in): it uses the device address fetched once per device below.
constexpr size_t kNoAllocBytes = (size_t)64 << 20;
static __device__ __align__(256) uint8_t scratch[kNoAllocBytes];

static std::mutex g_noalloc_mu;          // one call at a time per process (they share `scratch`)
static uint8_t *g_noalloc_ptr[16] = {};  // device address of `scratch`, per device

// Called with `device` current: fetches the array's device address on the
// first call on that device.
static int noalloc_scratch(int device, uint8_t **out) {
    if (device < 0 || device >= 16) return set_error(RAC_ENODEV, "device ordinal %d", device);
    if (!g_noalloc_ptr[device]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return set_error(RAC_EHIP, "hipGetSymbolAddress returned a null address");
        g_noalloc_ptr[device] = static_cast<uint8_t *>(p);
    }
    *out = g_noalloc_ptr[device];
    return RAC_OK;
}

// Byte offsets of the workspace parts for B states of n variables (each part
// 256-byte aligned); returns the total.
struct NoAllocLayout {
    size_t dom[2], chg[2], failacc, clist[2], ctrl, plan, act, act_off, act_push;
    size_t prob_net, prob_off, checks, rc, total;
};
static NoAllocLayout noalloc_layout(int64_t B, int64_t n) {
    NoAllocLayout o;
    size_t at = 0;
    auto take = [&](size_t bytes) {
        const size_t here = at;
        at += (bytes + 255) / 256 * 256;
        return here;
    };
    const size_t nv = (size_t)(B * n);
    o.dom[0] = take(nv * 8);
    o.dom[1] = take(nv * 8);
    o.chg[0] = take(nv * 4);
    o.chg[1] = take(nv * 4);
    o.failacc = take(nv * 8);
    o.clist[0] = take(nv * 4);
    o.clist[1] = take(nv * 4);
    o.ctrl = take((size_t)B * sizeof(Ctrl));
    o.plan = take(sizeof(Plan));
    o.act = take((size_t)B * 4);
    o.act_off = take(((size_t)B + 1) * 8);
    o.act_push = take((size_t)B * 4);
    o.prob_net = take((size_t)B * 4);
    o.prob_off = take(((size_t)B + 1) * 8);
    o.checks = take((size_t)B * 8);
    o.rc = take(4);
    o.total = at;
    return o;
}

// Problem tables of B instances of one net of n variables: problem p starts
// at variable p*n.
static __global__ void noalloc_tables_kernel(int64_t *prob_off, int32_t *prob_net, int32_t B, int32_t n) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = tid; p <= B; p += nth) {
        prob_off[p] = p * n;
        if (p < B) prob_net[p] = 0;
    }
}

extern "C" int rac_enforce_batch_noalloc(rac_net *net, int32_t B, const uint64_t *d_dom_in,
                                         uint64_t *d_dom_out, int32_t *d_iters, int32_t *d_status,
                                         void *stream) {
    if (!net || B < 0) return set_error(RAC_EINVAL, "bad net or B");
    if (B == 0) return RAC_OK;
    if (!d_dom_in || !d_dom_out) return set_error(RAC_EINVAL, "domain pointers are NULL");
    const NoAllocLayout lay = noalloc_layout(B, net->n);
    if (lay.total > kNoAllocBytes)
        return set_error(RAC_EINVAL,
                         "B*n = %lld variable states need %zu workspace bytes; the fixed "
                         "workspace of rac_enforce_batch_noalloc holds %zu (about %lld states "
                         "of this net)",
                         (long long)B * net->n, lay.total, kNoAllocBytes,
                         (long long)(kNoAllocBytes / std::max<size_t>(1, lay.total / (size_t)B)));
    PathData &pd = net->bits;
    if (!pd.ready || !pd.items || !pd.d_desc)
        return set_error(RAC_EINVAL, "the net's bit rows are not packed");
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    HIP_TRY(hipSetDevice(net->device));
    uint8_t *base = nullptr;
    RAC_TRY(noalloc_scratch(net->device, &base));
    hipStream_t s = (hipStream_t)stream;

    Launch L;
    memset(&L, 0, sizeof(L));
    L.nets = pd.d_desc;
    int32_t *prob_net = reinterpret_cast<int32_t *>(base + lay.prob_net);
    int64_t *prob_off = reinterpret_cast<int64_t *>(base + lay.prob_off);
    L.prob_net = prob_net;
    L.prob_off = prob_off;
    L.nprob = B;
    L.mode = net->opt.mode;
    L.max_sweeps = net->opt.max_sweeps;
    L.stage_vars = stage_vars_for(net->n);
    L.ws.dom[0] = reinterpret_cast<uint64_t *>(base + lay.dom[0]);
    L.ws.dom[1] = reinterpret_cast<uint64_t *>(base + lay.dom[1]);
    L.ws.chg[0] = reinterpret_cast<uint32_t *>(base + lay.chg[0]);
    L.ws.chg[1] = reinterpret_cast<uint32_t *>(base + lay.chg[1]);
    L.ws.failacc = reinterpret_cast<uint64_t *>(base + lay.failacc);
    L.ws.ctrl = reinterpret_cast<Ctrl *>(base + lay.ctrl);
    L.ws.plan = reinterpret_cast<Plan *>(base + lay.plan);
    L.ws.act = reinterpret_cast<int32_t *>(base + lay.act);
    L.ws.act_off = reinterpret_cast<int64_t *>(base + lay.act_off);
    L.ws.act_push = reinterpret_cast<int32_t *>(base + lay.act_push);
    L.ws.clist[0] = reinterpret_cast<int32_t *>(base + lay.clist[0]);
    L.ws.clist[1] = reinterpret_cast<int32_t *>(base + lay.clist[1]);
    L.din = d_dom_in;
    L.dout = d_dom_out;
    L.iters_out = d_iters;
    L.status_out = d_status;
    L.checks_out = reinterpret_cast<long long *>(base + lay.checks);
    L.rc_out = reinterpret_cast<int32_t *>(base + lay.rc);
    L.push_ratio = push_ratio();
    L.uniform_n = net->n;

    const int64_t nv = (int64_t)B * net->n;
    const size_t smem = stage_bytes(L.stage_vars);
    int64_t g = 0;
    RAC_TRY(sweep_slots(net->device, smem, &g));
    g = std::max<int64_t>(1, std::min<int64_t>(g, (int64_t)pd.nitems * B));
    const dim3 ginit = grid_init(nv);
    const dim3 gupd((unsigned)std::min<int64_t>(4096, std::max<int64_t>(1, (nv + 255) / 256)));
    const int32_t kcap = step_cap(net->opt, (int64_t)net->n * net->d);

    // every part the kernels read before writing is set here: the problem
    // tables, then (init) the domains, change flags, failure accumulators,
    // control words and the error word
    hipLaunchKernelGGL(noalloc_tables_kernel, dim3((unsigned)std::min<int64_t>(1024, (B + 256) / 256)),
                       dim3(256), 0, s, prob_off, prob_net, B, net->n);
    hipLaunchKernelGGL(init_kernel, ginit, dim3(256), 0, s, L);
    hipLaunchKernelGGL(plan_kernel, dim3(1), dim3(1024), 0, s, L, 1);
    int32_t k = 0;
    for (int round = 0;; ++round) {
        const int32_t K = round_steps(round, B == 1);
        for (int32_t i = 1; i <= K; ++i) {
            hipLaunchKernelGGL(revise_kernel, dim3((unsigned)g), dim3(kWave), smem, s, L, k + i);
            hipLaunchKernelGGL(update_kernel, gupd, dim3(256), 0, s, L, k + i);
            hipLaunchKernelGGL(plan_kernel, dim3(1), dim3(1024), 0, s, L, k + i + 1);
        }
        HIP_TRY(hipGetLastError());
        k += K;
        int32_t nact = 0;
        HIP_TRY(hipMemcpyAsync(&nact, &L.ws.plan->nact, 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (nact == 0 || k >= kcap) break;
    }
    hipLaunchKernelGGL(finish_kernel, ginit, dim3(256), 0, s, L);
    HIP_TRY(hipGetLastError());
    int32_t hrc = 0;
    HIP_TRY(hipMemcpyAsync(&hrc, L.rc_out, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return rc_from_device(hrc);
}

// ---------------------------------------------------------------------------
// groups of networks (one state each)
// ---------------------------------------------------------------------------

// (Re)builds the group's work-item tables for a target item size (the steps
// that re-examine every arc) and another for the later steps, and uploads
// them with the net descriptors.
static int group_items(rac_group *g, int32_t target, int32_t target_inc) {
    struct Tables {
        std::vector<int4> items;
        std::vector<int32_t> pieces;
        std::vector<size_t> off;
        std::vector<int32_t> count;
    };
    auto build = [&](int32_t t, Tables &T) {
        std::vector<int4> its;
        std::vector<int32_t> pcs;
        T.off.assign((size_t)g->k + 1, 0);
        T.count.assign((size_t)g->k, 0);
        for (int32_t i = 0; i < g->k; ++i) {
            rac_net *net = g->nets[(size_t)i];
            PathData &pd = g->paths[(size_t)i] == RAC_PATH_INT8 ? net->i8 : net->bits;
            build_items(net, pd, t, its, pcs);
            T.items.insert(T.items.end(), its.begin(), its.end());
            T.pieces.insert(T.pieces.end(), pcs.begin(), pcs.end());
            T.off[(size_t)i + 1] = T.items.size();
            T.count[(size_t)i] = (int32_t)its.size();
        }
    };
    Tables A, I;
    build(target, A);
    const bool two = target_inc != target;
    if (two) build(target_inc, I);
    if (g->stream) HIP_TRY(hipStreamSynchronize(g->stream));   // no launch still reads the old tables
    dfree(g->items);
    dfree(g->pieces);
    dfree(g->items_inc);
    dfree(g->pieces_inc);
    RAC_TRY(dalloc(&g->items, A.items.size()));
    RAC_TRY(dalloc(&g->pieces, A.pieces.size()));
    HIP_TRY(hipMemcpy(g->items, A.items.data(), A.items.size() * sizeof(int4), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(g->pieces, A.pieces.data(), A.pieces.size() * 4, hipMemcpyHostToDevice));
    if (two) {
        RAC_TRY(dalloc(&g->items_inc, I.items.size()));
        RAC_TRY(dalloc(&g->pieces_inc, I.pieces.size()));
        HIP_TRY(hipMemcpy(g->items_inc, I.items.data(), I.items.size() * sizeof(int4), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(g->pieces_inc, I.pieces.data(), I.pieces.size() * 4, hipMemcpyHostToDevice));
    }
    for (int32_t i = 0; i < g->k; ++i) {
        rac_net *net = g->nets[(size_t)i];
        NetDesc &D = g->descs[(size_t)i];
        D = (g->paths[(size_t)i] == RAC_PATH_INT8 ? net->i8 : net->bits).desc;
        D.items = g->items + A.off[(size_t)i];
        D.pieces = g->pieces + A.off[(size_t)i];
        D.nitems = A.count[(size_t)i];
        D.items_inc = two ? g->items_inc + I.off[(size_t)i] : D.items;
        D.pieces_inc = two ? g->pieces_inc + I.off[(size_t)i] : D.pieces;
        D.nitems_inc = two ? I.count[(size_t)i] : D.nitems;
    }
    if (!g->d_nets) RAC_TRY(dalloc(&g->d_nets, (size_t)g->k));
    HIP_TRY(hipMemcpy(g->d_nets, g->descs.data(), (size_t)g->k * sizeof(NetDesc), hipMemcpyHostToDevice));
    g->total_items = std::max<int64_t>((int64_t)A.items.size(), two ? (int64_t)I.items.size() : 0);
    g->item_target = target;
    g->item_target_inc = target_inc;
    return RAC_OK;
}

extern "C" void rac_group_destroy(rac_group *g) {
    if (!g) return;
    (void)hipSetDevice(g->device);
    (void)settle(g);
    if (g->stream) (void)hipStreamSynchronize(g->stream);
    release_runner(g->run);
    dfree(g->d_nets);
    dfree(g->items);
    dfree(g->pieces);
    dfree(g->items_inc);
    dfree(g->pieces_inc);
    if (g->stream) (void)hipStreamDestroy(g->stream);
    delete g;
}

extern "C" int rac_group_create(int32_t k, rac_net *const *nets, const rac_options *opt,
                                rac_group **out) {
    if (!out) return set_error(RAC_EINVAL, "out is NULL");
    *out = nullptr;
    if (k < 1 || !nets) return set_error(RAC_EINVAL, "k must be >= 1 with a net list");
    rac_options o;
    rac_default_options(&o);
    if (opt) o = *opt;
    RAC_TRY(check_options(&o));
    if (o.path == RAC_PATH_MFMA) return set_error(RAC_EUNSUPPORTED, "groups hold one state per net");
    for (int32_t i = 0; i < k; ++i) {
        if (!nets[i]) return set_error(RAC_EINVAL, "nets[%d] is NULL", i);
        if (nets[i]->device != nets[0]->device)
            return set_error(RAC_EINVAL, "nets of one group must share a device");
    }
    HIP_TRY(hipSetDevice(nets[0]->device));
    for (int32_t i = 0; i < k; ++i) RAC_TRY(settle(nets[i]));
    rac_group *g = new rac_group();
    g->k = k;
    g->nets.assign(nets, nets + k);
    g->opt = o;
    g->device = nets[0]->device;
    int rc = RAC_OK;
    do {
        if (hipSetDevice(g->device) != hipSuccess) { rc = set_error(RAC_EHIP, "hipSetDevice"); break; }
        if (hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking) != hipSuccess) {
            rc = set_error(RAC_EHIP, "hipStreamCreate");
            break;
        }
        std::vector<NetDesc> descs((size_t)k);
        g->h_off.assign((size_t)k + 1, 0);
        std::vector<int32_t> paths((size_t)k);
        int64_t total_bytes = 0;
        for (int32_t i = 0; i < k && rc == RAC_OK; ++i) {
            rac_net *net = nets[i];
            // per-net path: the int8 rows where they are asked for and fit, else
            // bit rows (a group's step streams every instance's rows at once, so
            // the fewest bytes win: single-instance measurements, latency-bound,
            // do not carry over)
            int32_t path = RAC_PATH_BITS;
            if (o.path == RAC_PATH_INT8 && net->d <= 32) path = RAC_PATH_INT8;
            paths[(size_t)i] = path;
            if ((rc = ensure_path(net, path, -1))) break;
            total_bytes += (int64_t)(path == RAC_PATH_INT8 ? net->i8 : net->bits).rows_bytes;
        }
        if (rc) break;
        // one item size for the whole group, from the group's total work (the
        // autotuner may measure smaller ones on the first call); the item
        // tables are the group's own (the nets' tables may be rebuilt by
        // calls on the nets themselves)
        g->descs = descs;
        for (int32_t i = 0; i < k; ++i) {
            rac_net *net = nets[i];
            g->h_off[(size_t)i + 1] = g->h_off[(size_t)i] + net->n;
            g->rel_bytes += (int64_t)(paths[(size_t)i] == RAC_PATH_INT8 ? net->i8 : net->bits).rows_bytes;
            g->max_n = std::max<int64_t>(g->max_n, net->n);
            g->max_groups = std::max<int64_t>(g->max_groups, net->groups);
        }
        g->total_vars = g->h_off[(size_t)k];
        g->paths = paths;
        {
            const int32_t t = o.item_bytes > 0 ? o.item_bytes : default_item_bytes(g->device, total_bytes);
            if ((rc = group_items(g, t, t))) break;
        }
        g->tuned = o.item_bytes > 0 || o.path != RAC_PATH_AUTO || effective_tune_mode(o) == kTuneRules;
        if ((rc = ensure_runner(g->run, k, g->total_vars))) break;
        std::vector<int32_t> pn((size_t)k);
        for (int32_t i = 0; i < k; ++i) {
            pn[(size_t)i] = i;
            g->max_nd = std::max<int64_t>(g->max_nd, (int64_t)nets[i]->n * nets[i]->d);
        }
        if (o.path == RAC_PATH_FUSED && g->max_n > kSmallMaxN) {
            rc = set_error(RAC_EUNSUPPORTED, "the fused path holds at most %d variables per net",
                           kSmallMaxN);
            break;
        }
        if (hipMemcpy(g->run.prob_net, pn.data(), (size_t)k * 4, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(g->run.prob_off, g->h_off.data(), ((size_t)k + 1) * 8, hipMemcpyHostToDevice) != hipSuccess) {
            rc = set_error(RAC_EHIP, "hipMemcpy of problem tables");
            break;
        }
    } while (0);
    if (rc != RAC_OK) {
        rac_group_destroy(g);
        return rc;
    }
    *out = g;
    return RAC_OK;
}

static Launch group_launch(rac_group *g, const uint64_t *din, uint64_t *dout, int32_t *it,
                           int32_t *st) {
    Launch L = base_launch(g->run, g->k, g->opt);
    L.nets = g->d_nets;
    L.stage_vars = stage_vars_for(g->max_n);
    L.din = din;
    L.dout = dout;
    L.iters_out = it;
    L.status_out = st;
    return L;
}

extern "C" int rac_group_enforce(rac_group *g, uint64_t *const *dom, int32_t *iters,
                                 int32_t *status) {
    if (!g || !dom) return set_error(RAC_EINVAL, "group or dom is NULL");
    HIP_TRY(hipSetDevice(g->device));
    RAC_TRY(settle(g));
    Runner &r = g->run;
    std::vector<uint64_t> h((size_t)g->total_vars);
    for (int32_t i = 0; i < g->k; ++i) {
        if (!dom[i]) return set_error(RAC_EINVAL, "dom[%d] is NULL", i);
        RAC_TRY(check_domains(dom[i], g->nets[(size_t)i]->n, g->nets[(size_t)i]->d));
        memcpy(r.h_dom + g->h_off[(size_t)i], dom[i], (size_t)g->nets[(size_t)i]->n * 8);
    }
    HIP_TRY(hipMemcpyAsync(r.din, r.h_dom, h.size() * 8, hipMemcpyHostToDevice, g->stream));
    std::vector<int32_t> hi, hs;
    std::vector<long long> hc;
    int32_t hrc = 0;
    auto run_once = [&]() -> int {
        Launch L = group_launch(g, r.din, r.dout, r.iters, r.status);
        if (g->opt.path == RAC_PATH_FUSED)
            RAC_TRY(launch_fused(r, g->stream, L, (int32_t)g->max_n, g->max_groups,
                                 g->k == 1 ? kFusedWavesOne : kFusedWavesBatch, g->opt.profile != 0,
                                 g->total_vars));
        else
            RAC_TRY(launch_fixpoint(r, g->device, g->stream, L, g->total_vars, g->total_items,
                                    step_cap(g->opt, g->max_nd), g->opt.use_graph != 0,
                                    g->opt.profile != 0, g->total_vars));
        return read_results(r, g->stream, g->k, g->total_vars, h.data(), hc, hi, hs, &hrc);
    };
    if (!g->tuned) {
        // the autotuner: the work-item size of the group's later steps,
        // measured on this call's own inputs (every size gives the same
        // results). Items sized from the group's total work suit the first
        // step, where every arc is re-examined, and keep that size; smaller
        // ones spread the later steps, where a few large instances run on,
        // over the chip.
        const int32_t t_all = g->item_target;
        std::vector<int32_t> cand = {t_all};
        for (int32_t t : {64 << 10, 16 << 10})
            if (t < t_all) cand.push_back(t);
        int32_t best_t = g->item_target_inc;
        double best = 1e30;
        for (int32_t t : cand) {
            if (t != g->item_target_inc) RAC_TRY(group_items(g, t_all, t));
            double tm = 1e30;
            for (int rep = 0; rep < 3; ++rep) {
                const auto t0 = std::chrono::steady_clock::now();
                const int rc = run_once();
                if (rc != RAC_OK) return rc;
                if (rep > 0)
                    tm = std::min(tm, std::chrono::duration<double, std::milli>(
                                          std::chrono::steady_clock::now() - t0).count());
            }
            if (tm < best) {
                best = tm;
                best_t = t;
            }
        }
        if (best_t != g->item_target_inc) RAC_TRY(group_items(g, t_all, best_t));
        g->tuned = true;
        g->tune_source = kSourceMeasured;
    }
    RAC_TRY(run_once());
    for (int32_t i = 0; i < g->k; ++i)
        memcpy(dom[i], h.data() + g->h_off[(size_t)i], (size_t)g->nets[(size_t)i]->n * 8);
    if (iters) memcpy(iters, hi.data(), (size_t)g->k * 4);
    if (status) memcpy(status, hs.data(), (size_t)g->k * 4);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, r.ev0, r.ev1);
    memset(&g->last, 0, sizeof(g->last));
    for (int32_t i = 0; i < g->k; ++i) {
        g->last.support_checks += hc[(size_t)i];
        g->last.sweeps += hi[(size_t)i];
    }
    g->last.device_ms = ms;
    g->last.path = g->opt.path == RAC_PATH_FUSED ? RAC_PATH_FUSED : RAC_PATH_BITS;
    g->last.relation_bytes = g->rel_bytes;
    g->last.item_bytes = g->item_target_inc;
    g->last.tune_source = g->tune_source;
    revise_timing(r, &g->last.kernel_ms, &g->last.kernel_launches,
                 &g->last.first_kernel_ms);
    return rc_from_device(hrc);
}

extern "C" int rac_group_enforce_device(rac_group *g, uint64_t *d_dom, int32_t *d_iters,
                                        int32_t *d_status, void *stream) {
    if (!g || !d_dom) return set_error(RAC_EINVAL, "group or dom is NULL");
    HIP_TRY(hipSetDevice(g->device));
    RAC_TRY(settle(g));
    Launch L = group_launch(g, d_dom, d_dom, d_iters, d_status);
    if (g->opt.path == RAC_PATH_FUSED)
        RAC_TRY(launch_fused(g->run, (hipStream_t)stream, L, (int32_t)g->max_n, g->max_groups,
                             g->k == 1 ? kFusedWavesOne : kFusedWavesBatch, g->opt.profile != 0));
    else
        RAC_TRY(launch_fixpoint(g->run, g->device, (hipStream_t)stream, L, g->total_vars,
                                g->total_items, step_cap(g->opt, g->max_nd),
                                g->opt.use_graph != 0, g->opt.profile != 0));
    g->pending = true;
    return RAC_OK;
}

extern "C" int rac_group_sync_status(rac_group *g) {
    if (!g) return set_error(RAC_EINVAL, "group is NULL");
    if (!g->pending) return RAC_OK;
    g->pending = false;
    HIP_TRY(hipSetDevice(g->device));
    HIP_TRY(hipEventSynchronize(g->run.ev1));   // the end of the call on the caller's stream
    int32_t hrc = 0;
    HIP_TRY(hipMemcpy(&hrc, g->run.rc, 4, hipMemcpyDeviceToHost));
    std::vector<long long> hc((size_t)g->k);
    HIP_TRY(hipMemcpy(hc.data(), g->run.checks, (size_t)g->k * 8, hipMemcpyDeviceToHost));
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, g->run.ev0, g->run.ev1);
    memset(&g->last, 0, sizeof(g->last));
    for (long long c : hc) g->last.support_checks += c;
    g->last.device_ms = ms;
    g->last.relation_bytes = g->rel_bytes;
    g->last.path = g->opt.path == RAC_PATH_FUSED ? RAC_PATH_FUSED : RAC_PATH_BITS;
    g->last.item_bytes = g->item_target_inc;
    g->last.tune_source = g->tune_source;
    revise_timing(g->run, &g->last.kernel_ms, &g->last.kernel_launches, &g->last.first_kernel_ms);
    return rc_from_device(hrc);
}

extern "C" int rac_group_stats(const rac_group *g, rac_stats *out) {
    if (!g || !out) return set_error(RAC_EINVAL, "NULL argument");
    *out = g->last;
    return RAC_OK;
}

extern "C" int rac_enforce_multi(int32_t k, rac_net *const *nets, uint64_t *const *dom,
                                 int32_t *iters, int32_t *status) {
    if (k < 1 || !nets || !dom) return set_error(RAC_EINVAL, "bad arguments");
    rac_options o = nets[0]->opt;
    if (o.path == RAC_PATH_MFMA) o.path = RAC_PATH_AUTO;
    rac_group *g = nullptr;
    RAC_TRY(rac_group_create(k, nets, &o, &g));
    g->tuned = true;   // one call: the item size from the group's total work, unmeasured
    const int rc = rac_group_enforce(g, dom, iters, status);
    rac_group_destroy(g);
    return rc;
}
