// rawalign_abi.cpp -- the C ABI of librawalign.so (declared in include/rawalign.h):
// argument checks, per-stream scratch, launch order, tuning cache, timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "dtw_path.h"
#include "internal.h"
#include "rawalign.h"

#define RAWALIGN_VERSION_STRING "rawalign-mi355x 0.6.0"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(RAWALIGN_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

struct DeviceInfo {
    int cus = 0;
    std::string name;
    std::string arch;
    bool ok = false;
};

std::mutex g_mu;
std::map<int, DeviceInfo> g_dev;
std::map<int, rawalign_opts> g_tuned;   // device -> tuned settings

// Per (device, user stream) state: planning scratch, edge slots of the
// multi-stripe kernel, internal streams for concurrent kernels, events.
struct StreamScratch {
    int32_t *words = nullptr;   // hist | counts | queue
    int32_t *list = nullptr;
    int64_t capacity = 0;
    float *edge = nullptr;
    int64_t edge_slots = 0;
    float *rowbuf = nullptr;    // anti-diagonal kernel only
    int64_t row_slots = 0;
    int32_t *tiny_words = nullptr;   // one-pair-per-lane planning: hist | counts | base
    ra::TinyRec *tiny_list = nullptr;
    int64_t tiny_capacity = 0;
    hipStream_t sub[3] = {nullptr, nullptr, nullptr};
    hipEvent_t fork = nullptr;
    hipEvent_t gap_planned = nullptr;   // global calls: the gap plan on sub[0] is done
    hipEvent_t join[3] = {nullptr, nullptr, nullptr};
    hipEvent_t ev[8] = {};      // timing: plan start/end, then start/end of lo, hi, long
};
std::map<std::pair<int, hipStream_t>, StreamScratch> g_scratch;

// Early-termination scratch, per (device, stream), grown on demand.
struct BnbStore {
    void *mem = nullptr;
    int64_t pairs = 0, reads = 0;
    ra::BnbScratch view;
};
std::map<std::pair<int, hipStream_t>, BnbStore> g_bnb;

// Alignment-start scratch, per (device, stream): the reverse pass's region
// lengths, scores and ends (12 bytes per pair), grown on demand.
struct SpanStore {
    void *mem = nullptr;
    int64_t pairs = 0;
};
std::map<std::pair<int, hipStream_t>, SpanStore> g_span;


struct TimingRecord {
    hipEvent_t ev[8] = {};
    bool valid = false;
};
TimingRecord g_last_timing;

int device_info(int &dev, DeviceInfo &info) {
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_dev.find(dev);
    if (it == g_dev.end()) {
        hipDeviceProp_t prop;
        e = hipGetDeviceProperties(&prop, dev);
        if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
        DeviceInfo d;
        d.cus = prop.multiProcessorCount;
        d.name = prop.name;
        d.arch = prop.gcnArchName;
        d.ok = d.arch.rfind("gfx950", 0) == 0;
        it = g_dev.emplace(dev, d).first;
    }
    info = it->second;
    if (!info.ok)
        return fail(RAWALIGN_ENODEV, "librawalign is built for gfx950; device " + std::to_string(dev) + " is " +
                                         info.arch);
    return RAWALIGN_OK;
}

int alloc_fail(hipError_t e) {
    return fail(RAWALIGN_ENOMEM, std::string("scratch allocation: ") + hipGetErrorString(e));
}

int get_scratch(int dev, hipStream_t stream, int64_t n_pairs, int64_t edge_slots, int64_t row_slots, bool timing,
                bool streams, StreamScratch *&out) {
    std::lock_guard<std::mutex> lk(g_mu);
    StreamScratch &s = g_scratch[{dev, stream}];
    hipError_t e;
    if (!s.words) {
        const size_t words = (size_t)ra::kNumRoutes * ra::kBuckets + 2 * ra::kNumRoutes;
        e = hipMalloc((void **)&s.words, words * sizeof(int32_t));
        if (e != hipSuccess) {
            s.words = nullptr;
            return alloc_fail(e);
        }
    }
    if (s.capacity < n_pairs) {
        int64_t cap = s.capacity ? s.capacity : 1024;
        while (cap < n_pairs) cap *= 2;
        if (s.list) (void)hipFree(s.list);
        s.list = nullptr;
        s.capacity = 0;
        e = hipMalloc((void **)&s.list, (size_t)cap * ra::kNumRoutes * sizeof(int32_t));
        if (e != hipSuccess) {
            s.list = nullptr;
            return alloc_fail(e);
        }
        s.capacity = cap;
    }
    if (s.edge_slots < edge_slots) {
        if (s.edge) (void)hipFree(s.edge);
        s.edge = nullptr;
        s.edge_slots = 0;
        e = hipMalloc((void **)&s.edge, (size_t)edge_slots * ra::kEdgeCap * sizeof(float));
        if (e != hipSuccess) {
            s.edge = nullptr;
            return alloc_fail(e);
        }
        s.edge_slots = edge_slots;
    }
    if (s.row_slots < row_slots) {
        if (s.rowbuf) (void)hipFree(s.rowbuf);
        s.rowbuf = nullptr;
        s.row_slots = 0;
        e = hipMalloc((void **)&s.rowbuf, (size_t)row_slots * ra::kMaxRegion * sizeof(float));
        if (e != hipSuccess) {
            s.rowbuf = nullptr;
            return alloc_fail(e);
        }
        s.row_slots = row_slots;
    }
    if (streams && !s.sub[0]) {
        for (int i = 0; i < 3; ++i) {
            e = hipStreamCreateWithFlags(&s.sub[i], hipStreamNonBlocking);
            if (e != hipSuccess) return hip_fail(e, "hipStreamCreateWithFlags");
            e = hipEventCreateWithFlags(&s.join[i], hipEventDisableTiming);
            if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
        }
        e = hipEventCreateWithFlags(&s.fork, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
        e = hipEventCreateWithFlags(&s.gap_planned, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    }
    if (timing && !s.ev[0]) {
        for (auto &ev : s.ev) {
            e = hipEventCreate(&ev);
            if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
        }
    }
    out = &s;
    return RAWALIGN_OK;
}

// Planning scratch of the one-pair-per-lane kernel (global calls only).
int get_tiny(StreamScratch &s, int64_t n_pairs) {
    std::lock_guard<std::mutex> lk(g_mu);
    hipError_t e;
    if (!s.tiny_words) {
        const size_t words = (size_t)ra::kTinyClasses * ra::kTinyBuckets + 2 * ra::kTinyClasses;
        e = hipMalloc((void **)&s.tiny_words, words * sizeof(int32_t));
        if (e != hipSuccess) {
            s.tiny_words = nullptr;
            return alloc_fail(e);
        }
    }
    if (s.tiny_capacity < n_pairs) {
        int64_t cap = s.tiny_capacity ? s.tiny_capacity : 1024;
        while (cap < n_pairs) cap *= 2;
        if (s.tiny_list) (void)hipFree(s.tiny_list);
        s.tiny_list = nullptr;
        s.tiny_capacity = 0;
        e = hipMalloc((void **)&s.tiny_list, (size_t)cap * sizeof(ra::TinyRec));
        if (e != hipSuccess) {
            s.tiny_list = nullptr;
            return alloc_fail(e);
        }
        s.tiny_capacity = cap;
    }
    return RAWALIGN_OK;
}

ra::TinyScratch tiny_view(StreamScratch &s) {
    ra::TinyScratch t;
    t.hist = s.tiny_words;
    t.counts = s.tiny_words + ra::kTinyClasses * ra::kTinyBuckets;
    t.base = t.counts + ra::kTinyClasses;
    t.list = s.tiny_list;
    t.capacity = s.tiny_capacity;
    return t;
}

ra::PlanScratch plan_view(StreamScratch &s) {
    ra::PlanScratch p;
    p.hist = s.words;
    p.counts = s.words + ra::kNumRoutes * ra::kBuckets;
    p.queue = p.counts + ra::kNumRoutes;
    p.list = s.list;
    p.capacity = s.capacity;
    p.edge = s.edge;
    p.rowbuf = s.rowbuf;
    return p;
}

int check_opts(const rawalign_opts &o) {
    if (o.mode != RAWALIGN_MODE_PLAIN && o.mode != RAWALIGN_MODE_PERSISTENT)
        return fail(RAWALIGN_EINVAL, "opts.mode must be RAWALIGN_MODE_PLAIN or RAWALIGN_MODE_PERSISTENT");
    if (o.long_kernel != RAWALIGN_LONG_STRIPED && o.long_kernel != RAWALIGN_LONG_ANTIDIAG &&
        o.long_kernel != RAWALIGN_LONG_PIPELINE)
        return fail(RAWALIGN_EINVAL,
                    "opts.long_kernel must be RAWALIGN_LONG_STRIPED, RAWALIGN_LONG_ANTIDIAG or RAWALIGN_LONG_PIPELINE");
    if (o.single_max != 0 && o.single_max != 2048 && o.single_max != 4096)
        return fail(RAWALIGN_EINVAL, "opts.single_max must be 0, 2048 or 4096");
    if (o.pipe_waves != 0 && o.pipe_waves != 2 && o.pipe_waves != 4 && o.pipe_waves != 8)
        return fail(RAWALIGN_EINVAL, "opts.pipe_waves must be 0, 2, 4 or 8");
    const int32_t w[3] = {o.lo_waves_per_cu, o.hi_waves_per_cu, o.long_waves_per_cu};
    for (int32_t v : w)
        if (v < 0 || v > 32) return fail(RAWALIGN_EINVAL, "opts.*_waves_per_cu must be in [0, 32]");
    if (o.streams != 1 && o.streams != 3) return fail(RAWALIGN_EINVAL, "opts.streams must be 1 or 3");
    if (o.flags & ~RAWALIGN_FLAG_TIMING) return fail(RAWALIGN_EINVAL, "opts.flags has unknown bits");
    return RAWALIGN_OK;
}

void defaults(rawalign_opts &o) {
    o.mode = RAWALIGN_MODE_PERSISTENT;
    o.long_kernel = RAWALIGN_LONG_STRIPED;
    o.lo_waves_per_cu = 0;
    o.hi_waves_per_cu = 0;
    o.long_waves_per_cu = 0;
    o.streams = 1;
    o.flags = 0;
    o.single_max = 0;
    o.pipe_waves = 0;
}

struct Call {
    const float *q;
    int64_t q_size;
    const int64_t *q_off;
    const int32_t *q_len;
    const float *r;
    int64_t r_size;
    const int64_t *r_off;
    const int32_t *r_len;
    int64_t n_pairs;
    float *out_score;
    int32_t *out_end;
    float *rows;
    int64_t rows_size;
    const int64_t *row_off;
    const uint8_t *first_chunk;
    hipStream_t stream;
    int bound = ra::kBoundSubseq;   // ra::BoundMode
    bool reverse = false;           // query and region read back to front
};

int check_call(const Call &c) {
    if (c.n_pairs < 0) return fail(RAWALIGN_EINVAL, "n_pairs must be >= 0");
    if (c.n_pairs >= (int64_t)1 << 31) return fail(RAWALIGN_EINVAL, "n_pairs must be < 2^31");
    if (c.q_size < 0 || c.r_size < 0) return fail(RAWALIGN_EINVAL, "q_size and r_size must be >= 0");
    if (c.q_size >= ((int64_t)1 << 40) || c.r_size >= ((int64_t)1 << 40))
        return fail(RAWALIGN_EINVAL, "q_size and r_size must be < 2^40");
    if (c.n_pairs == 0) return RAWALIGN_OK;
    if (!c.q_off || !c.q_len || !c.r_off || !c.r_len || !c.out_score ||
        (!c.out_end && c.bound != ra::kBoundGlobal))
        return fail(RAWALIGN_EINVAL, "null pointer argument");
    if ((c.q_size > 0 && !c.q) || (c.r_size > 0 && !c.r)) return fail(RAWALIGN_EINVAL, "null data pointer");
    if (c.rows && (!c.row_off || !c.first_chunk || c.rows_size < 0))
        return fail(RAWALIGN_EINVAL, "extend: rows, row_off and first_chunk are required");
    return RAWALIGN_OK;
}

int grid_of(int cus, int per_cu_opt, int occupancy) { return cus * (per_cu_opt ? per_cu_opt : occupancy); }

static_assert(RAWALIGN_NOALLOC_MAX_PAIRS == ra::kNoallocMaxPairs, "allocation-free pair limit");
static_assert(RAWALIGN_NOALLOC_EDGE_SLOTS == ra::kNoallocEdgeSlots, "allocation-free edge slots");
static_assert(RAWALIGN_NOALLOC_SCRATCH_BYTES == ra::kNoallocScratchBytes, "allocation-free scratch size");

// noalloc: take the planning lists and edge slots from the fixed device
// array (ra::noalloc_scratch) instead of the per-stream buffers; every
// kernel runs on c.stream, with no timing events and no allocation.
int run(const Call &c, const rawalign_opts &o, bool noalloc = false) {
    int rc = check_call(c);
    if (rc) return rc;
    rc = check_opts(o);
    if (rc) return rc;
    if (noalloc && (o.streams != 1 || (o.flags & RAWALIGN_FLAG_TIMING) || o.long_kernel != RAWALIGN_LONG_STRIPED ||
                    c.bound != ra::kBoundSubseq || c.rows))
        return fail(RAWALIGN_EINVAL, "allocation-free call: one stream, no timing, striped kernels, plain batch");
    if (noalloc && c.n_pairs > ra::kNoallocMaxPairs)
        return fail(RAWALIGN_EINVAL, "allocation-free call: n_pairs " + std::to_string(c.n_pairs) + " exceeds " +
                                         std::to_string(ra::kNoallocMaxPairs));
    if (c.rows && o.long_kernel == RAWALIGN_LONG_ANTIDIAG)
        return fail(RAWALIGN_EINVAL, "extend: opts.long_kernel must be RAWALIGN_LONG_STRIPED");
    if ((c.bound != ra::kBoundSubseq || c.reverse) && o.long_kernel == RAWALIGN_LONG_ANTIDIAG)
        return fail(RAWALIGN_EINVAL, "global alignment and alignment starts: opts.long_kernel must be "
                                     "RAWALIGN_LONG_STRIPED");
    if (c.n_pairs == 0) return RAWALIGN_OK;
    int dev = 0;
    DeviceInfo info;
    rc = device_info(dev, info);
    if (rc) return rc;

    const bool ext = c.rows != nullptr;
    // The pipelined kernel takes forward subsequence alignments (plain and
    // streaming); global and reversed passes keep the single-wave kernel.
    const bool pipeline = o.long_kernel == RAWALIGN_LONG_PIPELINE && c.bound == ra::kBoundSubseq && !c.reverse;
    const int pipe_waves = o.pipe_waves ? o.pipe_waves : 4;
    ra::LaunchCfg cfg;
    cfg.persistent = o.mode == RAWALIGN_MODE_PERSISTENT;
    cfg.single_max = o.single_max ? o.single_max : ra::kSingleMaxRegion;
    cfg.lo_grid = grid_of(info.cus, o.lo_waves_per_cu, ra::single_lo_blocks_per_cu(ext));
    cfg.hi_grid = grid_of(info.cus, o.hi_waves_per_cu, ra::single_hi_blocks_per_cu(ext));
    if (pipeline)   // workgroups of pipe_waves waves; long_waves_per_cu counts waves
        cfg.multi_grid = info.cus * (o.long_waves_per_cu ? std::max(1, o.long_waves_per_cu / pipe_waves)
                                                         : ra::pipe_blocks_per_cu(pipe_waves, ext));
    else
        cfg.multi_grid = grid_of(info.cus, o.long_waves_per_cu, ra::multi_blocks_per_cu(ext));
    // Anti-diagonal kernel: opts.long_waves_per_cu counts its workgroups per
    // CU; by default its occupancy limit (5: LDS and registers), each with a
    // 256 KiB row buffer.
    const int ad_occ = ra::antidiag_blocks_per_cu();
    cfg.antidiag_grid = info.cus * (o.long_waves_per_cu ? std::min(o.long_waves_per_cu, ad_occ) : ad_occ);
    // A persistent grid never needs more workgroups than the batch has pairs
    // (a small batch would otherwise launch thousands of waves that only
    // start and exit).
    {
        const int cap = (int)std::min<int64_t>(c.n_pairs, 1 << 30);
        cfg.lo_grid = std::min(cfg.lo_grid, cap);
        cfg.hi_grid = std::min(cfg.hi_grid, cap);
        cfg.multi_grid = std::min(cfg.multi_grid, cap);
        cfg.antidiag_grid = std::min(cfg.antidiag_grid, cap);
    }
    const bool antidiag = o.long_kernel == RAWALIGN_LONG_ANTIDIAG;

    const bool timing = (o.flags & RAWALIGN_FLAG_TIMING) != 0;
    const bool concurrent = o.streams == 3;
    StreamScratch *s = nullptr;
    ra::PlanScratch fixed;
    if (noalloc) {
        const hipError_t e = ra::noalloc_scratch(dev, fixed);
        if (e != hipSuccess) return hip_fail(e, "allocation-free scratch (hipGetSymbolAddress)");
        // One edge slot per resident multi-stripe wave.
        cfg.multi_grid = std::min(cfg.multi_grid, ra::kNoallocEdgeSlots);
    } else {
        rc = get_scratch(dev, c.stream, c.n_pairs, cfg.multi_grid, antidiag ? cfg.antidiag_grid : 0, timing,
                         concurrent, s);
        if (rc) return rc;
    }

    ra::PairArrays a;
    a.q = c.q;
    a.q_size = c.q_size;
    a.q_off = c.q_off;
    a.q_len = c.q_len;
    a.r = c.r;
    a.r_size = c.r_size;
    a.r_off = c.r_off;
    a.r_len = c.r_len;
    a.out_score = c.out_score;
    a.out_end = c.out_end;
    a.rows = c.rows;
    a.rows_size = c.rows_size;
    a.row_off = c.row_off;
    a.first_chunk = c.first_chunk;
    a.bound = c.bound;
    a.reverse = c.reverse ? 1 : 0;
    const ra::PlanScratch ps = noalloc ? fixed : plan_view(*s);
    const bool tiny = c.bound == ra::kBoundGlobal && !c.reverse;
    if (tiny) {
        rc = get_tiny(*s, c.n_pairs);
        if (rc) return rc;
    }

    // Global calls on three streams fork before planning: the gap plan runs
    // on sub[0] beside the main plan, the width classes then go round the
    // three sub-streams, and the striped routes follow the main plan on the
    // caller's stream, so four queues work at once. The two plans touch
    // disjoint pairs (the main plan skips every gap the one-lane kernel takes)
    // and separate scratch.
    const bool split = tiny && concurrent;
    hipError_t e;
    hipStream_t st[3] = {c.stream, c.stream, c.stream};
    auto fork = [&]() -> int {   // never with noalloc (checked above)
        if ((e = hipEventRecord(s->fork, c.stream)) != hipSuccess) return hip_fail(e, "hipEventRecord");
        for (int i = 0; i < 3; ++i) {
            st[i] = s->sub[i];
            if ((e = hipStreamWaitEvent(st[i], s->fork, 0)) != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
        }
        return RAWALIGN_OK;
    };
    if (timing && (e = hipEventRecord(s->ev[0], c.stream)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    if (split && (rc = fork()) != RAWALIGN_OK) return rc;
    e = ra::launch_plan(a, c.n_pairs, cfg, ps, c.stream);
    if (e != hipSuccess) return hip_fail(e, "plan kernels");
    if (tiny) {
        e = ra::launch_tiny_plan(a, c.n_pairs, tiny_view(*s), st[0]);
        if (e != hipSuccess) return hip_fail(e, "one-pair-per-lane planning");
    }
    if (timing) (void)hipEventRecord(s->ev[1], c.stream);   // split: the main plan only
    if (split) {
        if ((e = hipEventRecord(s->gap_planned, st[0])) != hipSuccess) return hip_fail(e, "hipEventRecord");
        for (int i = 1; i < 3; ++i)
            if ((e = hipStreamWaitEvent(st[i], s->gap_planned, 0)) != hipSuccess)
                return hip_fail(e, "hipStreamWaitEvent");
    } else if (concurrent && (rc = fork()) != RAWALIGN_OK) {
        return rc;
    }
    if (tiny) {
        e = ra::launch_tiny(a, c.n_pairs, tiny_view(*s), info.cus, st);
        if (e != hipSuccess) return hip_fail(e, "one-pair-per-lane kernels");
    }
    const hipStream_t route_st[3] = {split ? c.stream : st[0], split ? c.stream : st[1], split ? c.stream : st[2]};
    // Longest regions first: they bound the makespan.
    const char *names[3] = {antidiag ? "anti-diagonal kernel" : pipeline ? "pipelined multi-stripe kernel"
                                                                         : "multi-stripe kernel",
                            "single-stripe kernel (34-64 columns per lane)",
                            "single-stripe kernel (2-32 columns per lane)"};
    const int ev_slot[3] = {6, 4, 2};   // long, hi, lo
    for (int i = 0; i < 3; ++i) {
        const hipStream_t rs = route_st[i];
        if (timing) (void)hipEventRecord(s->ev[ev_slot[i]], rs);
        if (i == 0)
            e = antidiag ? ra::launch_antidiag(a, c.n_pairs, cfg, ps, rs)
                : pipeline ? ra::launch_pipe(pipe_waves, a, c.n_pairs, cfg, ps, rs)
                           : ra::launch_multi(a, c.n_pairs, cfg, ps, rs);
        else if (i == 1)
            e = ra::launch_single_hi(a, c.n_pairs, cfg, ps, rs);
        else
            e = ra::launch_single_lo(a, c.n_pairs, cfg, ps, rs);
        if (e != hipSuccess) return hip_fail(e, names[i]);
        if (timing) (void)hipEventRecord(s->ev[ev_slot[i] + 1], rs);
    }
    if (concurrent) {
        for (int i = 0; i < 3; ++i) {
            if ((e = hipEventRecord(s->join[i], st[i])) != hipSuccess) return hip_fail(e, "hipEventRecord");
            if ((e = hipStreamWaitEvent(c.stream, s->join[i], 0)) != hipSuccess)
                return hip_fail(e, "hipStreamWaitEvent");
        }
    }
    if (timing) {
        std::lock_guard<std::mutex> lk(g_mu);
        for (int i = 0; i < 8; ++i) g_last_timing.ev[i] = s->ev[i];
        g_last_timing.valid = true;
    }
    return RAWALIGN_OK;
}

// The caller's opts, else the device's tuned setting, else the defaults.
// The anti-diagonal kernel runs plain subsequence batches only; a call of
// another kind (antidiag_ok false) that inherits it from the tuned setting
// takes the striped kernel at its default grid instead (explicit opts are
// checked, not changed).
rawalign_opts effective_opts(const rawalign_opts *opts, bool antidiag_ok = false) {
    rawalign_opts o;
    if (opts) return *opts;
    defaults(o);
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_tuned.find(dev);
        if (it != g_tuned.end()) o = it->second;
    }
    if (!antidiag_ok && o.long_kernel == RAWALIGN_LONG_ANTIDIAG) {
        o.long_kernel = RAWALIGN_LONG_STRIPED;
        o.long_waves_per_cu = 0;
    }
    return o;
}

std::string json_escape(const std::string &s) {
    std::string o;
    for (char ch : s) {
        if (ch == '"' || ch == '\\') o += '\\';
        o += ch;
    }
    return o;
}

// Minimal reader for the flat JSON objects this library writes.
bool json_get(const std::string &doc, const std::string &key, std::string &val) {
    const std::string pat = "\"" + key + "\"";
    size_t k = doc.find(pat);
    if (k == std::string::npos) return false;
    k = doc.find(':', k + pat.size());
    if (k == std::string::npos) return false;
    ++k;
    while (k < doc.size() && (doc[k] == ' ' || doc[k] == '\t')) ++k;
    if (k < doc.size() && doc[k] == '"') {
        size_t e = doc.find('"', k + 1);
        if (e == std::string::npos) return false;
        val = doc.substr(k + 1, e - k - 1);
        return true;
    }
    size_t e = doc.find_first_of(",}\n", k);
    val = doc.substr(k, e == std::string::npos ? std::string::npos : e - k);
    return true;
}

constexpr int kNumOptFields = 8;
const char *kOptNames[kNumOptFields] = {"mode", "long_kernel", "lo_waves_per_cu", "hi_waves_per_cu",
                                        "long_waves_per_cu", "streams", "single_max", "pipe_waves"};

int32_t *opt_field(rawalign_opts &o, int i) {
    int32_t *f[kNumOptFields] = {&o.mode, &o.long_kernel, &o.lo_waves_per_cu, &o.hi_waves_per_cu,
                                 &o.long_waves_per_cu, &o.streams, &o.single_max, &o.pipe_waves};
    return f[i];
}

}  // namespace

extern "C" {

int rawalign_opts_default(rawalign_opts *opts) {
    if (!opts) return fail(RAWALIGN_EINVAL, "opts is null");
    defaults(*opts);
    return RAWALIGN_OK;
}

int rawalign_dtw_batch(const float *q, int64_t q_size, const int64_t *q_off, const int32_t *q_len,
                       const float *r, int64_t r_size, const int64_t *r_off, const int32_t *r_len,
                       int64_t n_pairs, float *out_score, int32_t *out_end, void *stream) {
    rawalign_opts o;
    defaults(o);
    o.mode = RAWALIGN_MODE_PLAIN;
    Call c{q, q_size, q_off, q_len, r, r_size, r_off, r_len, n_pairs, out_score, out_end,
           nullptr, 0, nullptr, nullptr, (hipStream_t)stream};
    return run(c, o);
}

int rawalign_dtw_batch_ex(const float *q, int64_t q_size, const int64_t *q_off, const int32_t *q_len,
                          const float *r, int64_t r_size, const int64_t *r_off, const int32_t *r_len,
                          int64_t n_pairs, float *out_score, int32_t *out_end, void *stream,
                          const rawalign_opts *opts) {
    Call c{q, q_size, q_off, q_len, r, r_size, r_off, r_len, n_pairs, out_score, out_end,
           nullptr, 0, nullptr, nullptr, (hipStream_t)stream};
    return run(c, effective_opts(opts, true));
}

int rawalign_dtw_batch_noalloc(const float *q, int64_t q_size, const int64_t *q_off, const int32_t *q_len,
                               const float *r, int64_t r_size, const int64_t *r_off, const int32_t *r_len,
                               int64_t n_pairs, float *out_score, int32_t *out_end, void *stream) {
    rawalign_opts o;
    defaults(o);   // persistent queues, striped kernels, one stream, no timing
    Call c{q, q_size, q_off, q_len, r, r_size, r_off, r_len, n_pairs, out_score, out_end,
           nullptr, 0, nullptr, nullptr, (hipStream_t)stream};
    return run(c, o, true);
}

int rawalign_dtw_extend(const float *q, int64_t q_size, const int64_t *q_off, const int32_t *q_len,
                        const float *r, int64_t r_size, const int64_t *r_off, const int32_t *r_len,
                        float *rows, int64_t rows_size, const int64_t *row_off,
                        const uint8_t *first_chunk, int64_t n_jobs,
                        float *out_score, int32_t *out_end, void *stream, const rawalign_opts *opts) {
    if (n_jobs > 0 && !rows) return fail(RAWALIGN_EINVAL, "extend: rows is null");
    Call c{q, q_size, q_off, q_len, r, r_size, r_off, r_len, n_jobs, out_score, out_end,
           rows, rows_size, row_off, first_chunk, (hipStream_t)stream};
    return run(c, effective_opts(opts));
}

int rawalign_map_bnb(const float *q, int64_t q_size, const int64_t *q_off, const int32_t *q_len,
                     const float *r, int64_t r_size, const int64_t *r_off, const int32_t *r_len, int64_t n_pairs,
                     const int64_t *cand_off, const int32_t *cand_cnt, const int32_t *n_events, int64_t n_reads,
                     double b_match, double threshold, int32_t max_query, int32_t block_rows,
                     float *rows, int64_t rows_size, const int64_t *row_off,
                     float *out_score, int32_t *out_end, int32_t *out_best, double *out_best_score,
                     uint8_t *out_mapped, void *stream, const rawalign_opts *opts) {
    if (n_reads < 0) return fail(RAWALIGN_EINVAL, "n_reads must be >= 0");
    if (n_reads >= (int64_t)1 << 31) return fail(RAWALIGN_EINVAL, "n_reads must be < 2^31");
    if (max_query < 0) return fail(RAWALIGN_EINVAL, "max_query must be >= 0");
    if (block_rows < 64 || block_rows > ra::kEdgeCap)
        return fail(RAWALIGN_EINVAL, "block_rows must be in [64, " + std::to_string(ra::kEdgeCap) + "]");
    if (!std::isfinite(b_match) || std::isnan(threshold))
        return fail(RAWALIGN_EINVAL, "b_match must be finite and threshold not NaN");
    if (n_reads > 0 && (!cand_off || !cand_cnt || !n_events || !out_best || !out_best_score || !out_mapped))
        return fail(RAWALIGN_EINVAL, "null pointer argument");
    if (n_pairs > 0 && (!rows || !row_off)) return fail(RAWALIGN_EINVAL, "rows and row_off are required");
    hipStream_t st = (hipStream_t)stream;
    if (n_pairs > 0) {
        int rc0 = check_call(Call{q, q_size, q_off, q_len, r, r_size, r_off, r_len, n_pairs, out_score, out_end,
                                  nullptr, 0, nullptr, nullptr, st});
        if (rc0) return rc0;
    } else if (n_pairs < 0) {
        return fail(RAWALIGN_EINVAL, "n_pairs must be >= 0");
    }
    rawalign_opts o = effective_opts(opts);
    o.flags = 0;
    int rc = check_opts(o);
    if (rc) return rc;
    if (n_pairs == 0 && n_reads == 0) return RAWALIGN_OK;
    int dev = 0;
    DeviceInfo info;
    rc = device_info(dev, info);
    if (rc) return rc;

    ra::BnbScratch sc;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        BnbStore &b = g_bnb[{dev, st}];
        const int64_t np = std::max<int64_t>(n_pairs, 1), nr = std::max<int64_t>(n_reads, 1);
        if (b.pairs < np || b.reads < nr) {
            if (b.mem) (void)hipFree(b.mem);
            b.mem = nullptr;
            b.pairs = b.reads = 0;
            const int64_t P = std::max(np, 2 * b.pairs), R = std::max(nr, 2 * b.reads);
            // 8-byte fields first, then 4-byte, then 1-byte: every field stays aligned.
            const size_t words = 2 * ra::kBuckets + 4;
            const size_t bytes = (size_t)R * 8 + (size_t)P * 8 + words * 4 + (size_t)P + 256;
            hipError_t e = hipMalloc(&b.mem, bytes);
            if (e != hipSuccess) {
                b.mem = nullptr;
                return alloc_fail(e);
            }
            char *m = (char *)b.mem;
            b.view.best = (uint64_t *)m;
            m += (size_t)R * 8;
            b.view.read_of = (int32_t *)m;
            m += (size_t)P * 4;
            b.view.list = (int32_t *)m;
            m += (size_t)P * 4;
            b.view.hist = (int32_t *)m;
            b.view.counts = b.view.hist + 2 * ra::kBuckets;
            b.view.queue = b.view.counts + 2;
            m += words * 4;
            b.view.status = (uint8_t *)m;
            b.pairs = P;
            b.reads = R;
        }
        sc = b.view;
    }

    ra::BnbArgs ba;
    ba.a.q = q;
    ba.a.q_size = q_size;
    ba.a.q_off = q_off;
    ba.a.q_len = q_len;
    ba.a.r = r;
    ba.a.r_size = r_size;
    ba.a.r_off = r_off;
    ba.a.r_len = r_len;
    ba.a.out_score = out_score;
    ba.a.out_end = out_end;
    ba.a.rows = rows;
    ba.a.rows_size = rows_size;
    ba.a.row_off = row_off;
    ba.a.first_chunk = nullptr;
    ba.n_pairs = n_pairs;
    ba.cand_off = cand_off;
    ba.cand_cnt = cand_cnt;
    ba.n_events = n_events;
    ba.n_reads = n_reads;
    ba.b_match = b_match;
    ba.max_query = max_query;
    ba.block_rows = block_rows;
    ba.s = sc;

    hipError_t e;
    if (n_pairs > 0) {
        // One persistent wave per resident slot, each with its own stripe edge slot.
        const int grid = (int)std::min<int64_t>(grid_of(info.cus, o.long_waves_per_cu, ra::bnb_blocks_per_cu()),
                                                n_pairs);
        StreamScratch *ss = nullptr;
        rc = get_scratch(dev, st, n_pairs, grid, 0, false, false, ss);
        if (rc) return rc;
        if ((e = ra::launch_bnb(ba, grid, ss->edge, st)) != hipSuccess) return hip_fail(e, "early-termination kernels");
    }
    if (n_reads > 0) {
        e = ra::launch_decide(out_score, n_pairs, cand_off, cand_cnt, n_events, n_reads, b_match, threshold, out_best,
                              out_best_score, out_mapped, false, st);
        if (e != hipSuccess) return hip_fail(e, "decide kernel");
    }
    return RAWALIGN_OK;
}

int rawalign_decide(const float *score, int64_t n_pairs, const int64_t *cand_off, const int32_t *cand_cnt,
                    const int32_t *n_events, int64_t n_reads, double b_match, double threshold,
                    int32_t *out_best, double *out_score, uint8_t *out_mapped, void *stream) {
    if (n_reads < 0 || n_pairs < 0) return fail(RAWALIGN_EINVAL, "n_reads and n_pairs must be >= 0");
    if (n_reads == 0) return RAWALIGN_OK;
    if (!cand_off || !cand_cnt || !n_events || !out_best || !out_score || !out_mapped ||
        (n_pairs > 0 && !score))
        return fail(RAWALIGN_EINVAL, "null pointer argument");
    if (!std::isfinite(b_match) || std::isnan(threshold))
        return fail(RAWALIGN_EINVAL, "b_match must be finite and threshold not NaN");
    int dev = 0;
    DeviceInfo info;
    int rc = device_info(dev, info);
    if (rc) return rc;
    hipError_t e = ra::launch_decide(score, n_pairs, cand_off, cand_cnt, n_events, n_reads, b_match, threshold,
                                     out_best, out_score, out_mapped, false, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "decide kernel");
    return RAWALIGN_OK;
}

int rawalign_dtw_global_batch(const float *q, int64_t q_size, const int64_t *q_off, const int32_t *q_len,
                              const float *r, int64_t r_size, const int64_t *r_off, const int32_t *r_len,
                              int64_t n_pairs, float *out_score, int32_t *out_end, void *stream,
                              const rawalign_opts *opts) {
    rawalign_opts o;
    defaults(o);
    // Defaults for anchor gaps: the width classes of the one-gap-per-lane
    // kernel overlap on three streams, and the routes above 2048 levels,
    // which such gaps hardly reach, get one persistent wave per CU instead
    // of a full grid that would mostly just start and exit.
    o.streams = 3;
    o.hi_waves_per_cu = 1;
    o.long_waves_per_cu = 1;
    if (opts) o = *opts;
    Call c{q, q_size, q_off, q_len, r, r_size, r_off, r_len, n_pairs, out_score, out_end,
           nullptr, 0, nullptr, nullptr, (hipStream_t)stream, ra::kBoundGlobal};
    return run(c, o);
}

int rawalign_dtw_span(const float *q, int64_t q_size, const int64_t *q_off, const int32_t *q_len,
                      const float *r, int64_t r_size, const int64_t *r_off, const int32_t *r_len,
                      int64_t n_pairs, float *out_score, int32_t *out_end, int32_t *out_start, void *stream,
                      const rawalign_opts *opts) {
    const rawalign_opts o = effective_opts(opts);
    if (o.long_kernel == RAWALIGN_LONG_ANTIDIAG)
        return fail(RAWALIGN_EINVAL, "alignment starts: opts.long_kernel must be RAWALIGN_LONG_STRIPED");
    if (n_pairs > 0 && !out_start) return fail(RAWALIGN_EINVAL, "null pointer argument: out_start");
    const hipStream_t st = (hipStream_t)stream;
    // Forward: cost and end column of every pair.
    Call fwd{q, q_size, q_off, q_len, r, r_size, r_off, r_len, n_pairs, out_score, out_end,
             nullptr, 0, nullptr, nullptr, st};
    int rc = run(fwd, o);
    if (rc || n_pairs == 0) return rc;
    int dev = 0;
    DeviceInfo info;
    rc = device_info(dev, info);
    if (rc) return rc;
    int32_t *rev_len, *rev_end;
    float *rev_score;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        SpanStore &sp = g_span[{dev, st}];
        if (sp.pairs < n_pairs) {
            int64_t cap = sp.pairs ? sp.pairs : 1024;
            while (cap < n_pairs) cap *= 2;
            if (sp.mem) (void)hipFree(sp.mem);
            sp.mem = nullptr;
            sp.pairs = 0;
            hipError_t e = hipMalloc(&sp.mem, (size_t)cap * 12);
            if (e != hipSuccess) {
                sp.mem = nullptr;
                return alloc_fail(e);
            }
            sp.pairs = cap;
        }
        rev_len = (int32_t *)sp.mem;
        rev_end = rev_len + sp.pairs;
        rev_score = (float *)(rev_end + sp.pairs);
    }
    hipError_t e = ra::launch_span_prep(out_end, n_pairs, rev_len, st);
    if (e != hipSuccess) return hip_fail(e, "span kernels");
    // Backward: the reversed query against the reversed prefix r[0 .. end],
    // anchored at the end cell, free to finish anywhere.
    Call bwd{q, q_size, q_off, q_len, r, r_size, r_off, rev_len, n_pairs, rev_score, rev_end,
             nullptr, 0, nullptr, nullptr, st, ra::kBoundAnchored, true};
    rc = run(bwd, o);
    if (rc) return rc;
    e = ra::launch_span_finish(out_end, rev_end, n_pairs, out_start, st);
    if (e != hipSuccess) return hip_fail(e, "span kernels");
    return RAWALIGN_OK;
}

int rawalign_dtw_path(const float *q, int64_t q_size, const int64_t *q_off, const int32_t *q_len,
                      const float *r, int64_t r_size, const int64_t *r_off, const int32_t *r_len,
                      int64_t n_pairs, const int64_t *dir_off, uint64_t *dirs, int64_t dir_size,
                      const int64_t *path_off, int32_t *path_lo, int32_t *path_hi, int64_t path_size,
                      float *out_score, int32_t *out_end, int32_t *out_start, void *stream,
                      const rawalign_opts *opts) {
    if (dir_size < 0 || path_size < 0) return fail(RAWALIGN_EINVAL, "dir_size and path_size must be >= 0");
    if (n_pairs > 0 && (!dir_off || !path_off || !path_lo || !path_hi))
        return fail(RAWALIGN_EINVAL, "null pointer argument: dir_off, path_off, path_lo and path_hi are required");
    if (n_pairs > 0 && dir_size > 0 && !dirs) return fail(RAWALIGN_EINVAL, "null pointer argument: dirs");
    // RAWALIGN_FLAG_SPAN_GIVEN belongs to this entry point alone: the span
    // passes (when run) see the other fields.
    const bool given = opts && (opts->flags & RAWALIGN_FLAG_SPAN_GIVEN);
    rawalign_opts o = effective_opts(opts);
    o.flags &= ~RAWALIGN_FLAG_SPAN_GIVEN;
    int rc;
    if (given) {
        // out_score / out_end / out_start hold a span result; the path
        // kernels check every interval against its pair before use.
        rc = check_opts(o);
        if (rc) return rc;
        rc = check_call(Call{q, q_size, q_off, q_len, r, r_size, r_off, r_len, n_pairs, out_score, out_end, nullptr,
                             0, nullptr, nullptr, (hipStream_t)stream});
        if (!rc && n_pairs > 0 && !out_start) rc = fail(RAWALIGN_EINVAL, "null pointer argument: out_start");
    } else {
        rc = rawalign_dtw_span(q, q_size, q_off, q_len, r, r_size, r_off, r_len, n_pairs, out_score, out_end,
                               out_start, stream, opts ? &o : nullptr);
    }
    if (rc || n_pairs == 0) return rc;
    ra::PathArgs pa;
    pa.q = q;
    pa.q_size = q_size;
    pa.q_off = q_off;
    pa.q_len = q_len;
    pa.r = r;
    pa.r_size = r_size;
    pa.r_off = r_off;
    pa.r_len = r_len;
    pa.start = out_start;
    pa.end = out_end;
    pa.n_pairs = n_pairs;
    pa.dir_off = dir_off;
    pa.dirs = dirs;
    pa.dir_size = dir_size;
    pa.path_off = path_off;
    pa.path_lo = path_lo;
    pa.path_hi = path_hi;
    pa.path_size = path_size;
    hipError_t e = ra::launch_path(pa, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "path kernels");
    return RAWALIGN_OK;
}

int rawalign_dtw_band(const float *q, int64_t q_size, const int64_t *q_off, const int32_t *q_len,
                      const float *r, int64_t r_size, const int64_t *r_off, const int32_t *r_len,
                      const int32_t *band, int64_t n_pairs, float *out_score, int32_t *out_end, void *stream) {
    Call c{q, q_size, q_off, q_len, r, r_size, r_off, r_len, n_pairs, out_score, out_end,
           nullptr, 0, nullptr, nullptr, (hipStream_t)stream};
    int rc = check_call(c);
    if (rc) return rc;
    if (n_pairs == 0) return RAWALIGN_OK;
    if (!band) return fail(RAWALIGN_EINVAL, "null pointer argument: band");
    int dev = 0;
    DeviceInfo info;
    rc = device_info(dev, info);
    if (rc) return rc;
    // Class 3 (striped band frames) gives each resident wave an edge slot.
    const int grid3 = (int)std::min<int64_t>((int64_t)info.cus * ra::band_blocks_per_cu(3), n_pairs);
    StreamScratch *s = nullptr;
    rc = get_scratch(dev, c.stream, n_pairs, grid3, 0, false, true, s);
    if (rc) return rc;
    ra::PairArrays a;
    a.q = q;
    a.q_size = q_size;
    a.q_off = q_off;
    a.q_len = q_len;
    a.r = r;
    a.r_size = r_size;
    a.r_off = r_off;
    a.r_len = r_len;
    a.out_score = out_score;
    a.out_end = out_end;
    a.rows = nullptr;
    a.rows_size = 0;
    a.row_off = nullptr;
    a.first_chunk = nullptr;
    a.bound = ra::kBoundSubseq;
    a.reverse = 0;
    const ra::PlanScratch ps = plan_view(*s);
    hipError_t e = ra::launch_band_plan(a, band, n_pairs, ps, c.stream);
    if (e != hipSuccess) return hip_fail(e, "banded planning");
    // The band classes run concurrently on the three internal streams (the
    // two whole-region classes share one) joined back to the caller's stream.
    if ((e = hipEventRecord(s->fork, c.stream)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    for (int i = 0; i < 3; ++i)
        if ((e = hipStreamWaitEvent(s->sub[i], s->fork, 0)) != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
    for (int cls = 0; cls < ra::kNumBandClasses; ++cls) {
        const int grid = cls == 3 ? grid3
                                  : (int)std::min<int64_t>((int64_t)info.cus * ra::band_blocks_per_cu(cls), n_pairs);
        e = ra::launch_band(cls, a, band, grid, ps, s->sub[cls < 3 ? cls : 2]);
        if (e != hipSuccess) return hip_fail(e, "banded kernel");
    }
    for (int i = 0; i < 3; ++i) {
        if ((e = hipEventRecord(s->join[i], s->sub[i])) != hipSuccess) return hip_fail(e, "hipEventRecord");
        if ((e = hipStreamWaitEvent(c.stream, s->join[i], 0)) != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
    }
    return RAWALIGN_OK;
}

int rawalign_chain_decide(const float *gap_cost, int64_t n_gaps, const int64_t *chain_gap_off,
                          const int32_t *chain_gap_cnt, const int32_t *chain_events, int64_t n_chains,
                          const int64_t *cand_off, const int32_t *cand_cnt, int64_t n_reads, double b_match,
                          double threshold, float *out_chain_cost, int32_t *out_best, double *out_best_score,
                          uint8_t *out_mapped, void *stream) {
    if (n_gaps < 0 || n_chains < 0 || n_reads < 0)
        return fail(RAWALIGN_EINVAL, "n_gaps, n_chains and n_reads must be >= 0");
    if (n_chains > 0 && (!chain_gap_off || !chain_gap_cnt || !chain_events || !out_chain_cost))
        return fail(RAWALIGN_EINVAL, "null chain pointer argument");
    if (n_gaps > 0 && !gap_cost) return fail(RAWALIGN_EINVAL, "null gap_cost");
    if (n_reads > 0 && (!cand_off || !cand_cnt || !out_best || !out_best_score || !out_mapped))
        return fail(RAWALIGN_EINVAL, "null read pointer argument");
    if (!std::isfinite(b_match) || std::isnan(threshold))
        return fail(RAWALIGN_EINVAL, "b_match must be finite and threshold not NaN");
    if (n_chains == 0 && n_reads == 0) return RAWALIGN_OK;
    int dev = 0;
    DeviceInfo info;
    int rc = device_info(dev, info);
    if (rc) return rc;
    const hipStream_t st = (hipStream_t)stream;
    hipError_t e;
    if (n_chains > 0) {
        e = ra::launch_chain_sum(gap_cost, n_gaps, chain_gap_off, chain_gap_cnt, n_chains, out_chain_cost, st);
        if (e != hipSuccess) return hip_fail(e, "chain sum kernel");
    }
    if (n_reads > 0) {
        e = ra::launch_decide(out_chain_cost, n_chains, cand_off, cand_cnt, chain_events, n_reads, b_match,
                              threshold, out_best, out_best_score, out_mapped, true, st);
        if (e != hipSuccess) return hip_fail(e, "decide kernel");
    }
    return RAWALIGN_OK;
}

int rawalign_last_timing(rawalign_timing *out) {
    if (!out) return fail(RAWALIGN_EINVAL, "out is null");
    TimingRecord t;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        t = g_last_timing;
    }
    if (!t.valid) return fail(RAWALIGN_EINVAL, "no call with RAWALIGN_FLAG_TIMING yet");
    for (int i = 0; i < 8; ++i) {
        hipError_t e = hipEventSynchronize(t.ev[i]);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    }
    float ms[4];
    for (int i = 0; i < 4; ++i) {
        hipError_t e = hipEventElapsedTime(&ms[i], t.ev[2 * i], t.ev[2 * i + 1]);
        if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
    }
    out->plan_ms = ms[0];
    out->lo_ms = ms[1];
    out->hi_ms = ms[2];
    out->long_ms = ms[3];
    float first_to_last = 0.0f;
    for (int i = 1; i < 8; ++i) {
        float d = 0.0f;
        if (hipEventElapsedTime(&d, t.ev[0], t.ev[i]) == hipSuccess && d > first_to_last) first_to_last = d;
    }
    out->total_ms = first_to_last;
    return RAWALIGN_OK;
}

int rawalign_autotune(const float *q, int64_t q_size, const int64_t *q_off, const int32_t *q_len,
                      const float *r, int64_t r_size, const int64_t *r_off, const int32_t *r_len,
                      int64_t n_pairs, float *out_score, int32_t *out_end, void *stream,
                      const char *cache_path, rawalign_opts *best_out) {
    int dev = 0;
    DeviceInfo info;
    int rc = device_info(dev, info);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    Call c{q, q_size, q_off, q_len, r, r_size, r_off, r_len, n_pairs, out_score, out_end,
           nullptr, 0, nullptr, nullptr, st};
    rc = check_call(c);
    if (rc) return rc;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return fail(RAWALIGN_EHIP, "hipEventCreate");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(RAWALIGN_EHIP, "hipEventCreate");
    }
    // Time each candidate: one warm-up call (which also grows the scratch),
    // then the mean of three.
    float best_ms = 1e30f;
    rawalign_opts best;
    defaults(best);
    auto measure = [&](const rawalign_opts &o, float &ms) -> int {
        int r = run(c, o);
        if (r) return r;
        const int reps = 3;
        (void)hipEventRecord(e0, st);
        for (int i = 0; i < reps && !r; ++i) r = run(c, o);
        (void)hipEventRecord(e1, st);
        if (r) return r;
        if (hipEventSynchronize(e1) != hipSuccess) return fail(RAWALIGN_EHIP, "hipEventSynchronize");
        float tot = 0.0f;
        (void)hipEventElapsedTime(&tot, e0, e1);
        ms = tot / reps;
        return RAWALIGN_OK;
    };
    auto consider = [&](const rawalign_opts &o) -> int {
        float ms = 0.0f;
        const int r = measure(o, ms);
        if (r) return r;
        if (ms < best_ms) {
            best_ms = ms;
            best = o;
        }
        return RAWALIGN_OK;
    };
    // Stage 1, the kernel shape at occupancy-sized grids on one stream: the
    // single-stripe cut-off (2049..4096-level regions on one stripe of
    // 34..64 columns per lane at two waves per SIMD, or on two stripes of
    // 17..32 at four) and the long-route kernel with its workgroup shape
    // (one wave per pair, 2, 4 or 8 waves sharing each pair, or the
    // anti-diagonal kernel's 256-thread workgroup; waves = 0 below).
    for (int single_max : {4096, 2048}) {
        for (int waves : {1, 2, 4, 8, 0}) {
            rawalign_opts o;
            defaults(o);
            o.single_max = single_max;
            if (waves > 1) {
                o.long_kernel = RAWALIGN_LONG_PIPELINE;
                o.pipe_waves = waves;
            } else if (waves == 0) {
                o.long_kernel = RAWALIGN_LONG_ANTIDIAG;
            }
            rc = consider(o);
            if (rc) break;
        }
        if (rc) break;
    }
    // Stage 2, at that shape: concurrent or sequential route kernels, and
    // persistent grids at or below each kernel's occupancy limit (waves per
    // CU; the pipelined kernel counts its waves, the anti-diagonal kernel
    // its workgroups).
    if (!rc) {
        const rawalign_opts shape = best;
        const bool pipe = shape.long_kernel == RAWALIGN_LONG_PIPELINE;
        const bool antidiag = shape.long_kernel == RAWALIGN_LONG_ANTIDIAG;
        const int pw = shape.pipe_waves ? shape.pipe_waves : 4;
        const int lo_occ = ra::single_lo_blocks_per_cu(false);
        const int hi_occ = ra::single_hi_blocks_per_cu(false);
        const int mu_occ = pipe       ? ra::pipe_blocks_per_cu(pw, false) * pw
                           : antidiag ? ra::antidiag_blocks_per_cu()
                                      : ra::multi_blocks_per_cu(false);
        const int mu_less = pipe ? mu_occ - pw : antidiag ? mu_occ - 1 : mu_occ - 4;
        std::vector<rawalign_opts> cands;
        for (int streams : {1, 3})
            for (int lo : {lo_occ, lo_occ > 4 ? lo_occ - 4 : lo_occ})
                for (int hi : {hi_occ, hi_occ > 4 ? hi_occ - 4 : hi_occ})
                    for (int mu : {mu_occ, mu_less > 0 ? mu_less : mu_occ}) {
                        rawalign_opts o = shape;
                        o.streams = streams;
                        o.lo_waves_per_cu = lo;
                        o.hi_waves_per_cu = hi;
                        o.long_waves_per_cu = mu;
                        bool dup = false;
                        for (const rawalign_opts &x : cands)
                            dup = dup || (x.streams == o.streams && x.lo_waves_per_cu == o.lo_waves_per_cu &&
                                          x.hi_waves_per_cu == o.hi_waves_per_cu &&
                                          x.long_waves_per_cu == o.long_waves_per_cu);
                        if (!dup) cands.push_back(o);
                    }
        for (const rawalign_opts &o : cands) {
            rc = consider(o);
            if (rc) break;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_tuned[dev] = best;
    }
    if (best_out) *best_out = best;
    if (cache_path) {
        std::ofstream f(cache_path);
        if (!f) return fail(RAWALIGN_EINVAL, std::string("cannot write ") + cache_path);
        f << "{\"device\": \"" << json_escape(info.name) << "\", \"arch\": \"" << json_escape(info.arch)
          << "\", \"version\": \"" << RAWALIGN_VERSION_STRING << "\"";
        for (int i = 0; i < kNumOptFields; ++i) f << ", \"" << kOptNames[i] << "\": " << *opt_field(best, i);
        f << ", \"ms\": " << best_ms << "}\n";
    }
    return RAWALIGN_OK;
}

int rawalign_load_tuning(const char *cache_path, rawalign_opts *out) {
    if (!cache_path) return fail(RAWALIGN_EINVAL, "cache_path is null");
    std::ifstream f(cache_path);
    if (!f) return fail(RAWALIGN_EINVAL, std::string("cannot read ") + cache_path);
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string doc = ss.str();
    int dev = 0;
    DeviceInfo info;
    int rc = device_info(dev, info);
    if (rc) return rc;
    std::string v;
    if (!json_get(doc, "arch", v) || v != info.arch) return fail(RAWALIGN_EINVAL, "tuning cache is for another device");
    if (!json_get(doc, "device", v) || v != info.name) return fail(RAWALIGN_EINVAL, "tuning cache is for another device");
    if (!json_get(doc, "version", v) || v != RAWALIGN_VERSION_STRING)
        return fail(RAWALIGN_EINVAL, "tuning cache is for another library version");
    rawalign_opts o;
    defaults(o);
    for (int i = 0; i < kNumOptFields; ++i) {
        if (!json_get(doc, kOptNames[i], v)) return fail(RAWALIGN_EINVAL, std::string("tuning cache lacks ") + kOptNames[i]);
        *opt_field(o, i) = (int32_t)std::strtol(v.c_str(), nullptr, 10);
    }
    rc = check_opts(o);
    if (rc) return rc;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_tuned[dev] = o;
    }
    if (out) *out = o;
    return RAWALIGN_OK;
}

const char *rawalign_last_error(void) { return g_err.c_str(); }

const char *rawalign_version(void) { return RAWALIGN_VERSION_STRING; }

}  // extern "C"
