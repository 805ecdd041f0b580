// Host side of librac: the C ABI of rac.h, input validation, the CSR arc
// layout, device-side packing of relation rows, work items, and the launch of
// the persistent fixpoint kernel (directly or as a replayed HIP graph).
#include <algorithm>
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
    case RAC_ETIMEOUT: return "device scheduler wait expired";
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
    if (o->path < RAC_PATH_AUTO || o->path > RAC_PATH_MFMA)
        return set_error(RAC_EINVAL, "options.path out of range");
    if (o->item_bytes < 0) return set_error(RAC_EINVAL, "options.item_bytes must be >= 0");
    if (o->profile != 0 && o->profile != 1) return set_error(RAC_EINVAL, "options.profile must be 0 or 1");
    for (int i = 0; i < 2; ++i)
        if (o->reserved[i] != 0) return set_error(RAC_EINVAL, "options.reserved must be zero");
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

// LDS bytes the sweep kernel needs to stage `vars` variables.
static size_t stage_bytes(int32_t vars) {
    return vars > 0 ? (size_t)vars * 8 + ((size_t)vars / 32 + 2) * 4 : 0;
}

// Resident sweep workgroups (= waves) on the whole device for a given LDS size.
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
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sweep_kernel, kWave, smem));
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

// Workspace + per-call buffers for up to `cap_probs` problems of one layout.
struct Runner {
    int32_t cap_probs = 0;
    int64_t cap_vars = 0;
    Workspace ws{};
    int32_t *prob_net = nullptr;
    int64_t *prob_off = nullptr;
    int64_t *item_off = nullptr;
    int64_t tables_key = -1;   // (B, nitems) the problem tables were last written for
    uint64_t *din = nullptr, *dout = nullptr;
    int32_t *iters = nullptr, *status = nullptr, *rc = nullptr;
    long long *checks = nullptr;
    uint8_t *changed = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr, evk0 = nullptr, evk1 = nullptr;
    bool profiled = false;
    // graph of (init, sweep, finish)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t nodes[3] = {nullptr, nullptr, nullptr};
    Launch graph_args{};
    dim3 graph_grid[3];
    size_t graph_smem = 0;
    bool graph_valid = false;
};

struct rac_net {
    int32_t n = 0, d = 0;
    int64_t m = 0, arcs = 0;
    rac_options opt{};
    int device = 0;
    hipStream_t stream = nullptr;
    std::vector<int32_t> h_row_ptr, h_deg, h_gptr;
    int32_t *row_ptr = nullptr, *nbr = nullptr, *deg = nullptr, *arc_src = nullptr;
    int32_t *gptr = nullptr, *nbrp = nullptr, *src_p = nullptr;   // 64-arc group layout
    int64_t groups = 0;
    uint64_t *rel = nullptr;   // [m][d] constraint rows, kept for lazily packed layouts
    PathData bits, i8;
    MfmaData mfma;
    uint64_t *mf_in = nullptr, *mf_out = nullptr;   // staging of host-pointer batch calls
    int32_t *mf_it = nullptr, *mf_st = nullptr;
    int32_t mf_cap = 0;
    Runner run;
    rac_stats last{};
    int pending_rc = RAC_OK;   // device-pointer call awaiting rac_sync_status
    bool pending = false;
};

struct rac_group {
    int32_t k = 0;
    std::vector<rac_net *> nets;
    rac_options opt{};
    int device = 0;
    hipStream_t stream = nullptr;
    NetDesc *d_nets = nullptr;
    std::vector<int64_t> h_off;
    Runner run;
    rac_stats last{};
    int64_t total_vars = 0, total_items = 0, rel_bytes = 0, max_n = 0;
    bool pending = false;
};

static int32_t round_up(int32_t v, int32_t m) { return (v + m - 1) / m * m; }

static void release_runner(Runner &r) {
    if (r.exec) (void)hipGraphExecDestroy(r.exec);
    if (r.graph) (void)hipGraphDestroy(r.graph);
    r.exec = nullptr;
    r.graph = nullptr;
    r.graph_valid = false;
    dfree(r.ws.dom[0]);
    dfree(r.ws.dom[1]);
    dfree(r.ws.chg[0]);
    dfree(r.ws.chg[1]);
    dfree(r.ws.failacc);
    dfree(r.ws.xcnt);
    dfree(r.ws.ctrl);
    dfree(r.ws.lanes);
    dfree(r.ws.global);
    dfree(r.prob_net);
    dfree(r.prob_off);
    dfree(r.item_off);
    r.tables_key = -1;
    dfree(r.din);
    dfree(r.dout);
    dfree(r.iters);
    dfree(r.status);
    dfree(r.rc);
    dfree(r.checks);
    dfree(r.changed);
    if (r.ev0) (void)hipEventDestroy(r.ev0);
    if (r.ev1) (void)hipEventDestroy(r.ev1);
    if (r.evk0) (void)hipEventDestroy(r.evk0);
    if (r.evk1) (void)hipEventDestroy(r.evk1);
    r.ev0 = r.ev1 = r.evk0 = r.evk1 = nullptr;
    r.cap_probs = 0;
    r.cap_vars = 0;
}

static int ensure_runner(Runner &r, int32_t nprob, int64_t nvars) {
    if (nprob <= r.cap_probs && nvars <= r.cap_vars) return RAC_OK;
    release_runner(r);
    RAC_TRY(dalloc(&r.ws.dom[0], nvars));
    RAC_TRY(dalloc(&r.ws.dom[1], nvars));
    RAC_TRY(dalloc(&r.ws.chg[0], nvars));
    RAC_TRY(dalloc(&r.ws.chg[1], nvars));
    RAC_TRY(dalloc(&r.ws.failacc, nvars));
    RAC_TRY(dalloc(&r.ws.xcnt, nvars));
    RAC_TRY(dalloc(&r.ws.ctrl, nprob));
    RAC_TRY(dalloc(&r.ws.lanes, (size_t)std::max<int32_t>(nprob, 256)));
    RAC_TRY(dalloc(&r.ws.global, 1));
    RAC_TRY(dalloc(&r.prob_net, nprob));
    RAC_TRY(dalloc(&r.prob_off, (size_t)nprob + 1));
    RAC_TRY(dalloc(&r.item_off, (size_t)nprob + 1));
    RAC_TRY(dalloc(&r.din, nvars));
    RAC_TRY(dalloc(&r.dout, nvars));
    RAC_TRY(dalloc(&r.iters, nprob));
    RAC_TRY(dalloc(&r.status, nprob));
    RAC_TRY(dalloc(&r.rc, 1));
    RAC_TRY(dalloc(&r.checks, nprob));
    RAC_TRY(dalloc(&r.changed, nvars));
    HIP_TRY(hipEventCreate(&r.ev0));
    HIP_TRY(hipEventCreate(&r.ev1));
    HIP_TRY(hipEventCreate(&r.evk0));
    HIP_TRY(hipEventCreate(&r.evk1));
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

extern "C" void rac_destroy(rac_net *net) {
    if (!net) return;
    (void)hipSetDevice(net->device);
    if (net->stream) (void)hipStreamSynchronize(net->stream);
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

// Work items over the arcs of one path: runs of whole variables up to about
// `target` relation bytes, and variables above that split into pieces.
static int make_items(rac_net *net, PathData &pd, int32_t target) {
    // units: 64-arc groups for bit rows, single arcs for int8 rows
    const bool groups = pd.kind != ROWI8;
    const int64_t unit_bytes = groups ? (int64_t)pd.desc.qpa * 1024 : (int64_t)net->d * pd.dp;
    std::vector<int4> items;
    std::vector<int32_t> pieces;
    const int32_t n = net->n;
    const std::vector<int32_t> &rp = groups ? net->h_gptr : net->h_row_ptr;
    const int64_t per_var = 64;   // accounts for the domain read/write of a variable
    const int32_t max_vars = 256;
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
        if ((rc = dalloc(&net->gptr, (size_t)n + 1))) break;
        if ((rc = dalloc(&net->nbrp, nbrp.size()))) break;
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

static int spin_limit() {
    const char *s = getenv("RAC_SPIN_LIMIT");
    if (s && atoi(s) > 0) return atoi(s);
    return 4000000;
}

static dim3 grid_init(int64_t nvars) {
    int64_t b = (nvars + 255) / 256;
    if (b > 4096) b = 4096;
    if (b < 1) b = 1;
    return dim3((unsigned)b);
}

// Enqueues init + persistent sweep + finish on `stream`.
static int launch_fixpoint(Runner &r, int device, hipStream_t stream, const Launch &L,
                           int64_t total_items, bool use_graph, bool profile = false) {
    const size_t smem = stage_bytes(L.stage_vars);
    int64_t g = 0;
    RAC_TRY(sweep_slots(device, smem, &g));
    if (total_items < g) g = total_items;
    if (g < 1) g = 1;
    if (getenv("RAC_DEBUG"))
        fprintf(stderr, "[rac] sweep grid=%lld items=%lld lds=%zu stage_vars=%d lanes/prob=%d nprob=%d\n",
                (long long)g, (long long)total_items, smem, L.stage_vars, L.lanes_per_prob, L.nprob);
    dim3 grids[3] = {grid_init(r.cap_vars), dim3((unsigned)g), grid_init(r.cap_vars)};
    const void *funcs[3] = {(const void *)init_kernel, (const void *)sweep_kernel,
                            (const void *)finish_kernel};
    r.profiled = profile;
    if (!use_graph || profile) {
        HIP_TRY(hipEventRecord(r.ev0, stream));
        hipLaunchKernelGGL(init_kernel, grids[0], dim3(256), 0, stream, L);
        if (profile) HIP_TRY(hipEventRecord(r.evk0, stream));
        hipLaunchKernelGGL(sweep_kernel, grids[1], dim3(kWave), smem, stream, L);
        if (profile) HIP_TRY(hipEventRecord(r.evk1, stream));
        hipLaunchKernelGGL(finish_kernel, grids[2], dim3(256), 0, stream, L);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipEventRecord(r.ev1, stream));
        return RAC_OK;
    }
    Launch args = L;
    void *params[1] = {&args};
    hipKernelNodeParams kp[3];
    for (int i = 0; i < 3; ++i) {
        memset(&kp[i], 0, sizeof(kp[i]));
        kp[i].func = const_cast<void *>(funcs[i]);
        kp[i].gridDim = grids[i];
        kp[i].blockDim = dim3(i == 1 ? kWave : 256);
        kp[i].sharedMemBytes = i == 1 ? (unsigned)smem : 0u;
        kp[i].kernelParams = params;
        kp[i].extra = nullptr;
    }
    const bool same_grid = r.graph_valid && r.graph_grid[0].x == grids[0].x &&
                           r.graph_grid[1].x == grids[1].x && r.graph_grid[2].x == grids[2].x &&
                           r.graph_smem == smem;
    if (!same_grid) {
        if (r.exec) (void)hipGraphExecDestroy(r.exec);
        if (r.graph) (void)hipGraphDestroy(r.graph);
        r.exec = nullptr;
        r.graph = nullptr;
        r.graph_valid = false;
        HIP_TRY(hipGraphCreate(&r.graph, 0));
        HIP_TRY(hipGraphAddKernelNode(&r.nodes[0], r.graph, nullptr, 0, &kp[0]));
        HIP_TRY(hipGraphAddKernelNode(&r.nodes[1], r.graph, &r.nodes[0], 1, &kp[1]));
        HIP_TRY(hipGraphAddKernelNode(&r.nodes[2], r.graph, &r.nodes[1], 1, &kp[2]));
        HIP_TRY(hipGraphInstantiate(&r.exec, r.graph, nullptr, nullptr, 0));
        for (int i = 0; i < 3; ++i) r.graph_grid[i] = grids[i];
        r.graph_smem = smem;
        r.graph_args = args;
        r.graph_valid = true;
    } else if (memcmp(&r.graph_args, &args, sizeof(Launch)) != 0) {
        for (int i = 0; i < 3; ++i) HIP_TRY(hipGraphExecKernelNodeSetParams(r.exec, r.nodes[i], &kp[i]));
        r.graph_args = args;
    }
    HIP_TRY(hipEventRecord(r.ev0, stream));
    HIP_TRY(hipGraphLaunch(r.exec, stream));
    HIP_TRY(hipEventRecord(r.ev1, stream));
    return RAC_OK;
}

// Lane slots per problem: up to 64, with at most 256 lanes over all problems.
static int32_t lanes_per_problem(int32_t nprob) {
    int32_t lpp = 64;
    while (lpp > 1 && (int64_t)lpp * nprob > 256) lpp >>= 1;
    return lpp;
}

static Launch base_launch(Runner &r, int32_t nprob, const rac_options &o) {
    Launch L;
    memset(&L, 0, sizeof(L));
    L.prob_net = r.prob_net;
    L.prob_off = r.prob_off;
    L.item_off = r.item_off;
    L.nprob = nprob;
    L.mode = o.mode;
    L.max_sweeps = o.max_sweeps;
    L.spin_limit = spin_limit();
    L.lanes_per_prob = lanes_per_problem(nprob);
    L.ws = r.ws;
    L.rc_out = r.rc;
    L.checks_out = r.checks;
    L.checks1 = -1;
    return L;
}

static int rc_from_device(int32_t dev_rc) {
    if (dev_rc & 2) return set_error(RAC_ETIMEOUT, "device scheduler wait expired");
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
    std::vector<int64_t> off((size_t)B + 1), ioff((size_t)B + 1);
    for (int32_t s = 0; s <= B; ++s) {
        off[(size_t)s] = (int64_t)s * net->n;
        ioff[(size_t)s] = (int64_t)s * pd.nitems;
    }
    HIP_TRY(hipMemcpyAsync(r.prob_net, pn.data(), (size_t)B * 4, hipMemcpyHostToDevice, net->stream));
    HIP_TRY(hipMemcpyAsync(r.prob_off, off.data(), ((size_t)B + 1) * 8, hipMemcpyHostToDevice,
                           net->stream));
    HIP_TRY(hipMemcpyAsync(r.item_off, ioff.data(), ((size_t)B + 1) * 8, hipMemcpyHostToDevice,
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

static int pick_path(const rac_net *net, int32_t B, int32_t requested) {
    if (requested != RAC_PATH_AUTO) return requested;
    return mfma_auto_choice(net->d, net->n, net->arcs, B) ? RAC_PATH_MFMA : RAC_PATH_BITS;
}

// Bit / int8 path for B states already in r.din. Synchronous when `sync`.
static int run_states(rac_net *net, int32_t B, int32_t path, const uint8_t *d_changed,
                      long long checks1, bool sync) {
    PathData &pd = path == RAC_PATH_INT8 ? net->i8 : net->bits;
    RAC_TRY(ensure_path(net, path, call_target(net, B)));
    Runner &r = net->run;
    Launch L = base_launch(r, B, net->opt);
    L.nets = pd.d_desc;
    L.stage_vars = stage_vars_for(net->n);
    L.din = r.din;
    L.dout = r.dout;
    L.iters_out = r.iters;
    L.status_out = r.status;
    L.changed0 = d_changed;
    L.checks1 = checks1;
    RAC_TRY(launch_fixpoint(r, net->device, net->stream, L, (int64_t)pd.nitems * B,
                            net->opt.use_graph != 0, net->opt.profile != 0));
    (void)sync;
    return RAC_OK;
}

static int collect_bits(rac_net *net, int32_t B, int32_t path, uint64_t *dom, int32_t *iters,
                        int32_t *status) {
    Runner &r = net->run;
    PathData &pd = path == RAC_PATH_INT8 ? net->i8 : net->bits;
    std::vector<int32_t> hi((size_t)B), hs((size_t)B);
    std::vector<long long> hc((size_t)B);
    int32_t hrc = 0;
    HIP_TRY(hipMemcpyAsync(dom, r.dout, (size_t)B * net->n * 8, hipMemcpyDeviceToHost, net->stream));
    HIP_TRY(hipMemcpyAsync(hi.data(), r.iters, (size_t)B * 4, hipMemcpyDeviceToHost, net->stream));
    HIP_TRY(hipMemcpyAsync(hs.data(), r.status, (size_t)B * 4, hipMemcpyDeviceToHost, net->stream));
    HIP_TRY(hipMemcpyAsync(hc.data(), r.checks, (size_t)B * 8, hipMemcpyDeviceToHost, net->stream));
    HIP_TRY(hipMemcpyAsync(&hrc, r.rc, 4, hipMemcpyDeviceToHost, net->stream));
    HIP_TRY(hipStreamSynchronize(net->stream));
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, r.ev0, r.ev1);
    fill_stats_bits(net->last, hc, hi, path, pd, ms);
    net->last.relation_bytes = (int64_t)pd.rows_bytes;
    if (r.profiled) {
        float kms = 0.f;
        (void)hipEventElapsedTime(&kms, r.evk0, r.evk1);
        net->last.kernel_ms = kms;
        net->last.kernel_launches = 1;
    }
    if (iters) memcpy(iters, hi.data(), (size_t)B * 4);
    if (status) memcpy(status, hs.data(), (size_t)B * 4);
    return rc_from_device(hrc);
}

extern "C" int rac_enforce(rac_net *net, uint64_t *dom, const int32_t *changed, int32_t n_changed,
                           int32_t *iters, int32_t *status) {
    if (!net || !dom) return set_error(RAC_EINVAL, "net or dom is NULL");
    if (changed && n_changed < 0) return set_error(RAC_EINVAL, "n_changed < 0");
    RAC_TRY(check_domains(dom, net->n, net->d));
    HIP_TRY(hipSetDevice(net->device));
    int32_t path = net->opt.path;
    if (path == RAC_PATH_AUTO || path == RAC_PATH_MFMA) path = RAC_PATH_BITS;
    RAC_TRY(ensure_path(net, path, call_target(net, 1)));
    RAC_TRY(prepare_net_runner(net, 1, path == RAC_PATH_INT8 ? net->i8 : net->bits));
    Runner &r = net->run;
    HIP_TRY(hipMemcpyAsync(r.din, dom, (size_t)net->n * 8, hipMemcpyHostToDevice, net->stream));
    const uint8_t *d_changed = nullptr;
    long long checks1 = -1;
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
        checks1 = degs * net->d * net->d;
    }
    RAC_TRY(run_states(net, 1, path, d_changed, checks1, true));
    return collect_bits(net, 1, path, dom, iters, status);
}

// States still active when at most this many remain leave the matrix-core
// path and finish on the persistent bit-row path, whose incremental steps
// touch only arcs into changed variables.
static int32_t mfma_handoff_threshold() {
    const char *e = getenv("RAC_MFMA_HANDOFF");
    if (e) return std::max(0, atoi(e));
    return 32;
}

// The batched matrix-core path: matrix-core steps while many states are
// active, then the stragglers on the bit-row path (continuing from D^(k)
// with @changed = the variables step k changed, Proposition 2).
static int run_mfma(rac_net *net, int32_t B, const uint64_t *d_in, uint64_t *d_out,
                    int32_t *d_it, int32_t *d_st, hipStream_t s) {
    RAC_TRY(mfma_ensure(net->mfma, net->n, net->d, net->arcs, net->row_ptr, net->nbr, net->deg,
                        net->rel, net->arc_src, net->h_row_ptr, net->stream));
    int32_t k = 0, P = 0;
    RAC_TRY(mfma_start(net->mfma, B, d_in, net->opt.mode, net->opt.max_sweeps, net->opt.profile,
                       mfma_handoff_threshold(), s, &k, &P));
    if (P > 0) {
        RAC_TRY(ensure_path(net, RAC_PATH_BITS, call_target(net, P)));
        PathData &pd = net->bits;
        RAC_TRY(prepare_net_runner(net, P, pd));
        Runner &r = net->run;
        RAC_TRY(mfma_handoff(net->mfma, k, r.din, r.changed, s));
        Launch L = base_launch(r, P, net->opt);
        L.nets = pd.d_desc;
        L.stage_vars = stage_vars_for(net->n);
        L.din = r.din;
        L.dout = r.dout;
        L.iters_out = r.iters;
        L.status_out = r.status;
        L.changed0 = r.changed;
        L.checks1 = 0;   // the matrix-core finaliser already counted step k+1
        const int32_t maxs = net->opt.max_sweeps > 0 ? net->opt.max_sweeps : net->n * net->d + 1;
        L.max_sweeps = maxs - k;
        RAC_TRY(launch_fixpoint(r, net->device, s, L, (int64_t)pd.nitems * P, false, false));
        RAC_TRY(mfma_merge(net->mfma, k, r.dout, r.iters, r.status, r.checks, r.rc, s));
    }
    RAC_TRY(mfma_finish(net->mfma, d_out, d_it, d_st, s));
    return RAC_OK;
}

extern "C" int rac_enforce_batch(rac_net *net, int32_t B, uint64_t *dom, int32_t *iters,
                                 int32_t *status) {
    if (!net || (!dom && B > 0)) return set_error(RAC_EINVAL, "net or dom is NULL");
    if (B < 0) return set_error(RAC_EINVAL, "B < 0");
    if (B == 0) return RAC_OK;
    RAC_TRY(check_domains(dom, (int64_t)B * net->n, net->d));
    HIP_TRY(hipSetDevice(net->device));
    const int32_t path = pick_path(net, B, net->opt.path);
    if (path == RAC_PATH_MFMA) {
        if (B > net->mf_cap) {
            dfree(net->mf_in);
            dfree(net->mf_out);
            dfree(net->mf_it);
            dfree(net->mf_st);
            RAC_TRY(dalloc(&net->mf_in, (size_t)B * net->n));
            RAC_TRY(dalloc(&net->mf_out, (size_t)B * net->n));
            RAC_TRY(dalloc(&net->mf_it, (size_t)B));
            RAC_TRY(dalloc(&net->mf_st, (size_t)B));
            net->mf_cap = B;
        }
        HIP_TRY(hipMemcpyAsync(net->mf_in, dom, (size_t)B * net->n * 8, hipMemcpyHostToDevice,
                               net->stream));
        RAC_TRY(run_mfma(net, B, net->mf_in, net->mf_out, net->mf_it, net->mf_st, net->stream));
        HIP_TRY(hipMemcpyAsync(dom, net->mf_out, (size_t)B * net->n * 8, hipMemcpyDeviceToHost,
                               net->stream));
        if (iters)
            HIP_TRY(hipMemcpyAsync(iters, net->mf_it, (size_t)B * 4, hipMemcpyDeviceToHost, net->stream));
        if (status)
            HIP_TRY(hipMemcpyAsync(status, net->mf_st, (size_t)B * 4, hipMemcpyDeviceToHost,
                                   net->stream));
        HIP_TRY(hipStreamSynchronize(net->stream));
        return mfma_collect(net->mfma, &net->last);
    }
    RAC_TRY(ensure_path(net, path, call_target(net, B)));
    RAC_TRY(prepare_net_runner(net, B, path == RAC_PATH_INT8 ? net->i8 : net->bits));
    HIP_TRY(hipMemcpyAsync(net->run.din, dom, (size_t)B * net->n * 8, hipMemcpyHostToDevice,
                           net->stream));
    RAC_TRY(run_states(net, B, path, nullptr, -1, true));
    return collect_bits(net, B, path, dom, iters, status);
}

extern "C" int rac_enforce_batch_device(rac_net *net, int32_t B, const uint64_t *d_dom_in,
                                        uint64_t *d_dom_out, int32_t *d_iters, int32_t *d_status,
                                        void *stream) {
    if (!net || B < 0) return set_error(RAC_EINVAL, "bad net or B");
    if (B == 0) return RAC_OK;
    if (!d_dom_in || !d_dom_out) return set_error(RAC_EINVAL, "domain pointers are NULL");
    HIP_TRY(hipSetDevice(net->device));
    if (net->pending) {
        const int prc = rac_sync_status(net);
        if (prc != RAC_OK) return prc;
    }
    hipStream_t s = (hipStream_t)stream;
    const int32_t path = pick_path(net, B, net->opt.path);
    if (path == RAC_PATH_MFMA) {
        RAC_TRY(run_mfma(net, B, d_dom_in, d_dom_out, d_iters, d_status, s));
        net->pending = true;
        net->last.path = RAC_PATH_MFMA;
        return RAC_OK;
    }
    RAC_TRY(ensure_path(net, path, call_target(net, B)));
    RAC_TRY(prepare_net_runner(net, B, path == RAC_PATH_INT8 ? net->i8 : net->bits));
    PathData &pd = path == RAC_PATH_INT8 ? net->i8 : net->bits;
    Runner &r = net->run;
    Launch L = base_launch(r, B, net->opt);
    L.nets = pd.d_desc;
    L.stage_vars = stage_vars_for(net->n);
    L.din = d_dom_in;
    L.dout = d_dom_out;
    L.iters_out = d_iters;
    L.status_out = d_status;
    RAC_TRY(launch_fixpoint(r, net->device, s, L, (int64_t)pd.nitems * B, net->opt.use_graph != 0,
                            net->opt.profile != 0));
    net->pending = true;
    net->last.path = path;
    net->last.item_bytes = pd.item_bytes;
    net->last.relation_bytes = (int64_t)pd.rows_bytes;
    return RAC_OK;
}

extern "C" int rac_sync_status(rac_net *net) {
    if (!net) return set_error(RAC_EINVAL, "net is NULL");
    if (!net->pending) return RAC_OK;
    HIP_TRY(hipSetDevice(net->device));
    net->pending = false;
    if (net->last.path == RAC_PATH_MFMA) return mfma_collect(net->mfma, &net->last);
    int32_t hrc = 0;
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(&hrc, net->run.rc, 4, hipMemcpyDeviceToHost));
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, net->run.ev0, net->run.ev1);
    net->last.device_ms = ms;
    if (net->run.profiled) {
        float kms = 0.f;
        (void)hipEventElapsedTime(&kms, net->run.evk0, net->run.evk1);
        net->last.kernel_ms = kms;
        net->last.kernel_launches = 1;
    }
    return rc_from_device(hrc);
}

extern "C" int rac_net_stats(const rac_net *net, rac_stats *out) {
    if (!net || !out) return set_error(RAC_EINVAL, "NULL argument");
    *out = net->last;
    return RAC_OK;
}

// ---------------------------------------------------------------------------
// groups of networks (one state each)
// ---------------------------------------------------------------------------

extern "C" void rac_group_destroy(rac_group *g) {
    if (!g) return;
    (void)hipSetDevice(g->device);
    if (g->stream) (void)hipStreamSynchronize(g->stream);
    release_runner(g->run);
    dfree(g->d_nets);
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
            // per-net path: the int8 rows only where they are asked for and fit
            int32_t path = RAC_PATH_BITS;
            if (o.path == RAC_PATH_INT8 && net->d <= 32) path = RAC_PATH_INT8;
            paths[(size_t)i] = path;
            if ((rc = ensure_path(net, path, -1))) break;
            total_bytes += (int64_t)(path == RAC_PATH_INT8 ? net->i8 : net->bits).rows_bytes;
        }
        if (rc) break;
        // one item size for the whole group, from the group's total work
        const int32_t target = o.item_bytes > 0 ? o.item_bytes : default_item_bytes(g->device, total_bytes);
        for (int32_t i = 0; i < k; ++i) {
            rac_net *net = nets[i];
            if ((rc = ensure_path(net, paths[(size_t)i], target))) break;
            PathData &pd = paths[(size_t)i] == RAC_PATH_INT8 ? net->i8 : net->bits;
            descs[(size_t)i] = pd.desc;
            g->h_off[(size_t)i + 1] = g->h_off[(size_t)i] + net->n;
            g->total_items += pd.nitems;
            g->rel_bytes += (int64_t)pd.rows_bytes;
            g->max_n = std::max<int64_t>(g->max_n, net->n);
        }
        if (rc) break;
        g->total_vars = g->h_off[(size_t)k];
        if ((rc = dalloc(&g->d_nets, (size_t)k))) break;
        if (hipMemcpy(g->d_nets, descs.data(), (size_t)k * sizeof(NetDesc), hipMemcpyHostToDevice) != hipSuccess) {
            rc = set_error(RAC_EHIP, "hipMemcpy of descriptors");
            break;
        }
        if ((rc = ensure_runner(g->run, k, g->total_vars))) break;
        std::vector<int32_t> pn((size_t)k);
        std::vector<int64_t> ioff((size_t)k + 1, 0);
        for (int32_t i = 0; i < k; ++i) {
            pn[(size_t)i] = i;
            ioff[(size_t)i + 1] = ioff[(size_t)i] + descs[(size_t)i].nitems;
        }
        if (hipMemcpy(g->run.prob_net, pn.data(), (size_t)k * 4, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(g->run.item_off, ioff.data(), ((size_t)k + 1) * 8, hipMemcpyHostToDevice) != hipSuccess ||
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
    Runner &r = g->run;
    std::vector<uint64_t> h((size_t)g->total_vars);
    for (int32_t i = 0; i < g->k; ++i) {
        if (!dom[i]) return set_error(RAC_EINVAL, "dom[%d] is NULL", i);
        RAC_TRY(check_domains(dom[i], g->nets[(size_t)i]->n, g->nets[(size_t)i]->d));
        memcpy(h.data() + g->h_off[(size_t)i], dom[i], (size_t)g->nets[(size_t)i]->n * 8);
    }
    HIP_TRY(hipMemcpyAsync(r.din, h.data(), h.size() * 8, hipMemcpyHostToDevice, g->stream));
    Launch L = group_launch(g, r.din, r.dout, r.iters, r.status);
    RAC_TRY(launch_fixpoint(r, g->device, g->stream, L, g->total_items, g->opt.use_graph != 0,
                            g->opt.profile != 0));
    std::vector<int32_t> hi((size_t)g->k), hs((size_t)g->k);
    std::vector<long long> hc((size_t)g->k);
    int32_t hrc = 0;
    HIP_TRY(hipMemcpyAsync(h.data(), r.dout, h.size() * 8, hipMemcpyDeviceToHost, g->stream));
    HIP_TRY(hipMemcpyAsync(hi.data(), r.iters, (size_t)g->k * 4, hipMemcpyDeviceToHost, g->stream));
    HIP_TRY(hipMemcpyAsync(hs.data(), r.status, (size_t)g->k * 4, hipMemcpyDeviceToHost, g->stream));
    HIP_TRY(hipMemcpyAsync(hc.data(), r.checks, (size_t)g->k * 8, hipMemcpyDeviceToHost, g->stream));
    HIP_TRY(hipMemcpyAsync(&hrc, r.rc, 4, hipMemcpyDeviceToHost, g->stream));
    HIP_TRY(hipStreamSynchronize(g->stream));
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
    g->last.path = RAC_PATH_BITS;
    g->last.relation_bytes = g->rel_bytes;
    if (r.profiled) {
        float kms = 0.f;
        (void)hipEventElapsedTime(&kms, r.evk0, r.evk1);
        g->last.kernel_ms = kms;
        g->last.kernel_launches = 1;
    }
    return rc_from_device(hrc);
}

extern "C" int rac_group_enforce_device(rac_group *g, uint64_t *d_dom, int32_t *d_iters,
                                        int32_t *d_status, void *stream) {
    if (!g || !d_dom) return set_error(RAC_EINVAL, "group or dom is NULL");
    HIP_TRY(hipSetDevice(g->device));
    if (g->pending) {
        const int prc = rac_group_sync_status(g);
        if (prc != RAC_OK) return prc;
    }
    Launch L = group_launch(g, d_dom, d_dom, d_iters, d_status);
    RAC_TRY(launch_fixpoint(g->run, g->device, (hipStream_t)stream, L, g->total_items,
                            g->opt.use_graph != 0));
    g->pending = true;
    return RAC_OK;
}

extern "C" int rac_group_sync_status(rac_group *g) {
    if (!g) return set_error(RAC_EINVAL, "group is NULL");
    if (!g->pending) return RAC_OK;
    g->pending = false;
    HIP_TRY(hipSetDevice(g->device));
    HIP_TRY(hipDeviceSynchronize());
    int32_t hrc = 0;
    HIP_TRY(hipMemcpy(&hrc, g->run.rc, 4, hipMemcpyDeviceToHost));
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, g->run.ev0, g->run.ev1);
    g->last.device_ms = ms;
    g->last.relation_bytes = g->rel_bytes;
    g->last.path = RAC_PATH_BITS;
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
    const int rc = rac_group_enforce(g, dom, iters, status);
    rac_group_destroy(g);
    return rc;
}
