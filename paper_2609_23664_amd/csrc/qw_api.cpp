// C ABI of libqw (include/qw.h): contexts, states, typed boundary
// snapshots, legality gates and the execution of pass plans on a HIP stream.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <map>
#include <set>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <sstream>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/qw.h"
#include "qw_internal.h"
#include "qw_kernels.h"
#include "qw_jit.h"

using namespace qw;

namespace {

const char *kVersion = "libqw 0.1 (gfx950)";

struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
};

struct ProfRec {
    int kind;
    double bytes;
    hipEvent_t e0, e1;
    uint32_t launches;  // back-to-back launches the two events bracket
};

struct PlanEntry {
    uint32_t n = 0;
    int tile_bits = 0;
    bool relabel = true;
    bool layout = true;
    bool in_place = false;
    bool fused_epilogue = true;
    uint64_t pingpong_cap = 16ull << 30;
    uint64_t mem_cap = 0;        // QW_OPT_DEVICE_MEM_CAP (0: none)
    uint64_t held = 0;           // bytes of the states and snapshot copies it allocated
    std::vector<char> gates;  // the gate records the plan was built from
    std::shared_ptr<const qw::Plan> plan;
};

struct KStats {
    uint64_t launches = 0;
    double ms = 0.0;
    double bytes = 0.0;
};

// State of a context while it records a graph (qw_graph_begin .. end): the
// device work of the calls goes into a stream capture, and every device
// buffer those calls use is kept for the graph's lifetime.
// One recorded task of a gate-running call: its plan and, per pass, where
// the graph keeps the pass's op records.
struct GraphSeg {
    uint32_t n = 0;
    std::shared_ptr<const qw::Plan> plan;
    std::vector<std::pair<void *, size_t>> ops;  // device address, bytes
};

// Where a recorded measured call's outcome bytes and zero-state flag live.
struct OutcomeRec {
    const uint8_t *outc;
    uint64_t count;
    const uint32_t *err;
};

struct GraphRec {
    std::vector<std::vector<GraphSeg>> calls;  // qw_apply_prefix / qw_run_suffix_batch, in order
    hipStream_t cap = nullptr;    // captured stream (non-blocking, default priority)
    hipStream_t up = nullptr;     // plan uploads, synchronous, outside the capture
    hipStream_t saved_stream = nullptr;
    DevBuf saved_plan, saved_scratch, saved_pingpong, saved_meas, saved_psync;
    std::vector<void *> owned;    // buffers replaced during the recording
    bool plan_used = false;       // ctx->plan already holds an uploaded blob
    std::vector<OutcomeRec> outcomes;  // measured calls: where a replay writes their outcomes
};

}  // namespace

struct qw_graph {
    qw_ctx *ctx = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<void *> owned;  // plan blobs and scratch the recorded nodes read
    uint64_t nodes = 0;
    std::vector<std::vector<GraphSeg>> calls;  // updatable op records per recorded task
    std::vector<OutcomeRec> outcomes;          // measured calls, in recording order
};

struct qw_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    int tile_bits = kMaxTileBits;
    bool profile = false;
    bool xcd_remap = true;
    int jit = 1;  // 0: interpreted kernels, 1: tiered, 2: always generated
    uint32_t n_cu = 256;
    DevBuf plan;     // uploaded descriptors/ops
    DevBuf scratch;  // partial sums, sampler buffers
    DevBuf pingpong; // second state buffers of tasks with relabelling passes
    DevBuf meas;     // measurement sums: slot pointers, qubits, partials, results
    DevBuf psync;    // persistent launches: claim counter, abandon flag, completion counters
    // persistent launches (QW_OPT_PERSISTENT): pinned host words, [0] set by
    // the host to abandon waits, [1] set by a launch that abandoned one
    uint32_t *host_flag = nullptr;
    bool persistent = false;
    uint32_t spin_limit = 1u << 20;  // QW_OPT_SPIN_LIMIT: microseconds per wait
    uint32_t persist_chunk = 8;      // QW_OPT_PERSIST_CHUNK: max tiles (rows) per claim
    std::vector<uint8_t> outcomes;  // outcome record of the last measured call
    std::unordered_map<std::string, uint64_t> jit_heat;  // task-tiles run per pass structure
    bool relabel = true;
    int layout = 1;              // QW_OPT_LAYOUT
    int tile_order = 1;          // QW_OPT_TILE_ORDER
    bool stream_loads = true;    // QW_OPT_STREAM_LOADS
    bool fused_epilogue = true;
    uint64_t pingpong_cap = 16ull << 30;
    uint64_t mem_cap = 0;        // QW_OPT_DEVICE_MEM_CAP (0: none)
    uint64_t held = 0;           // bytes of the states and snapshot copies it allocated
    void *staging = nullptr;
    size_t staging_cap = 0;
    hipEvent_t staging_ev = nullptr;
    std::vector<ProfRec> prof;
    std::vector<hipEvent_t> ev_pool;
    KStats stats[4];
    std::unordered_map<uint64_t, std::vector<PlanEntry>> plan_cache;
    size_t plan_cache_entries = 0;
    GraphRec *rec = nullptr;  // non-null while a graph is being recorded
};

struct qw_state {
    qw_ctx *ctx = nullptr;
    uint32_t n = 0, n_slots = 0;
    char *base = nullptr;
    bool owned = false;
    uint64_t slot_bytes = 0;
    std::vector<uint32_t> frozen;
};

struct qw_snap {
    qw_ctx *ctx = nullptr;
    qw_artifact art{};
    const void *data = nullptr;
    void *owned = nullptr;
    qw_state *fstate = nullptr;
    uint32_t fslot = 0;
    const qw_snap *parent = nullptr;
    int mode = QW_SNAP_COPY;
    uint64_t counted = 0;  // bytes of a COPY counted toward the context's cap
};

namespace {

int fail(qw_ctx *ctx, int code, const std::string &msg) {
    if (ctx) ctx->err = msg;
    return code;
}

// Calls that wait for the device or free memory cannot run while the
// context records a graph.
int recording_unsupported(qw_ctx *ctx, const char *what) {
    return fail(ctx, QW_E_UNSUPPORTED,
                std::string(what) + " is not available while a graph is being recorded");
}

int hip_fail(qw_ctx *ctx, hipError_t e, const char *what) {
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return fail(ctx, e == hipErrorOutOfMemory ? QW_E_OOM : QW_E_HIP, m);
}

#define HIP_TRY(ctx, call, what)                       \
    do {                                               \
        hipError_t _e = (call);                        \
        if (_e != hipSuccess) return hip_fail(ctx, _e, what); \
    } while (0)

// Device bytes the context holds: its states and snapshot copies (allocated
// by it or by the caller), and its plan, scratch,
// second-state and measurement buffers (buffers handed to a recorded graph
// belong to the graph).
uint64_t ctx_bytes(const qw_ctx *ctx) {
    return ctx->held + ctx->plan.cap + ctx->scratch.cap + ctx->pingpong.cap + ctx->meas.cap + ctx->psync.cap;
}

// QW_OPT_DEVICE_MEM_CAP: refuse an allocation of `want` bytes (replacing
// `released` bytes of the context's) that would take the context past its
// cap, before any device work of the call.
int cap_check(qw_ctx *ctx, uint64_t want, uint64_t released, const char *what) {
    if (!ctx->mem_cap) return QW_OK;
    const uint64_t now = ctx_bytes(ctx) - std::min(released, ctx_bytes(ctx));
    if (now + want <= ctx->mem_cap) return QW_OK;
    char b[256];
    std::snprintf(b, sizeof b, "%s: %llu bytes would take the context to %llu bytes, past its device "
                  "memory cap of %llu", what, (unsigned long long)want,
                  (unsigned long long)(now + want), (unsigned long long)ctx->mem_cap);
    return fail(ctx, QW_E_OOM, b);
}

// While recording, a buffer is never freed or rewritten behind the graph's
// back: a buffer that is too small (or a plan buffer that already holds an
// uploaded blob) is set aside for the graph and replaced by a new one.
int ensure_recording(qw_ctx *ctx, DevBuf &b, size_t bytes, const char *what) {
    const bool is_plan = &b == &ctx->plan;
    if (b.cap >= bytes && !(is_plan && ctx->rec->plan_used)) return QW_OK;
    {
        int rc = cap_check(ctx, (std::max<size_t>(bytes, 256) + 4095) & ~size_t(4095), b.cap, what);
        if (rc) return rc;
    }
    if (b.p) ctx->rec->owned.push_back(b.p);
    b.p = nullptr;
    b.cap = 0;
    const size_t want = (std::max<size_t>(bytes, 256) + 4095) & ~size_t(4095);
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) return hip_fail(ctx, e, what);
    b.p = p;
    b.cap = want;
    if (is_plan) ctx->rec->plan_used = false;
    return QW_OK;
}

int ensure(qw_ctx *ctx, DevBuf &b, size_t bytes, const char *what) {
    if (ctx->rec) return ensure_recording(ctx, b, bytes, what);
    if (b.cap >= bytes) return QW_OK;
    size_t want = std::max(bytes, b.cap * 2);
    want = (want + 4095) & ~size_t(4095);
    if (ctx->mem_cap && cap_check(ctx, want, b.cap, what) != QW_OK) {
        // doubling would pass the cap: try the size asked for
        want = (bytes + 4095) & ~size_t(4095);
        int rc = cap_check(ctx, want, b.cap, what);
        if (rc) return rc;
    }
    if (b.p) {
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream), "sync before regrow");
        HIP_TRY(ctx, hipFree(b.p), "free scratch");
        b.p = nullptr;
        b.cap = 0;
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) return hip_fail(ctx, e, what);
    b.p = p;
    b.cap = want;
    return QW_OK;
}

// Copy a host blob to ctx->plan (device) through the pinned staging buffer.
int upload(qw_ctx *ctx, const std::vector<uint8_t> &blob) {
    if (blob.empty()) return QW_OK;
    int rc = ensure(ctx, ctx->plan, blob.size(), "plan buffer");
    if (rc) return rc;
    if (ctx->rec) {
        // recording: the blob is copied now, once, into a buffer the graph
        // keeps (its nodes read it on every replay)
        HIP_TRY(ctx, hipMemcpyAsync(ctx->plan.p, blob.data(), blob.size(), hipMemcpyHostToDevice,
                                    ctx->rec->up),
                "plan upload (recording)");
        HIP_TRY(ctx, hipStreamSynchronize(ctx->rec->up), "plan upload (recording)");
        ctx->rec->plan_used = true;
        return QW_OK;
    }
    // the previous copy out of the staging buffer must have completed
    HIP_TRY(ctx, hipEventSynchronize(ctx->staging_ev), "staging wait");
    if (ctx->staging_cap < blob.size()) {
        if (ctx->staging) HIP_TRY(ctx, hipHostFree(ctx->staging), "free staging");
        ctx->staging = nullptr;
        size_t want = std::max(blob.size(), ctx->staging_cap * 2);
        HIP_TRY(ctx, hipHostMalloc(&ctx->staging, want, hipHostMallocDefault), "staging alloc");
        ctx->staging_cap = want;
    }
    std::memcpy(ctx->staging, blob.data(), blob.size());
    HIP_TRY(ctx, hipMemcpyAsync(ctx->plan.p, ctx->staging, blob.size(), hipMemcpyHostToDevice,
                                ctx->stream),
            "plan upload");
    HIP_TRY(ctx, hipEventRecord(ctx->staging_ev, ctx->stream), "staging event");
    return QW_OK;
}

// A blob built in place in the pinned staging buffer, which saves zeroing and
// copying a host vector (a batch of 512 tasks of about 14 passes has a 25 MB
// blob). stage_blob waits until the previous copy out of the buffer has
// completed and grows it; upload_staged copies it to ctx->plan. Nothing else
// may use the staging buffer in between. Padding between records is left as
// it is: no kernel reads it.
struct StagedBlob {
    uint8_t *p = nullptr;
    size_t n = 0;
    uint8_t *data() const { return p; }
    size_t size() const { return n; }
};

int stage_blob(qw_ctx *ctx, size_t bytes, StagedBlob *out) {
    HIP_TRY(ctx, hipEventSynchronize(ctx->staging_ev), "staging wait");
    if (ctx->staging_cap < bytes) {
        const size_t want = std::max(bytes, ctx->staging_cap * 2);
        if (ctx->staging) HIP_TRY(ctx, hipHostFree(ctx->staging), "free staging");
        ctx->staging = nullptr;
        ctx->staging_cap = 0;
        HIP_TRY(ctx, hipHostMalloc(&ctx->staging, want, hipHostMallocDefault), "staging alloc");
        ctx->staging_cap = want;
    }
    out->p = static_cast<uint8_t *>(ctx->staging);
    out->n = bytes;
    return QW_OK;
}

int upload_staged(qw_ctx *ctx, const StagedBlob &b) {
    if (b.n == 0) return QW_OK;
    if (ctx->rec) {
        // recording: copied now, once, into the buffer the graph keeps
        HIP_TRY(ctx, hipMemcpyAsync(ctx->plan.p, b.p, b.n, hipMemcpyHostToDevice, ctx->rec->up),
                "plan upload (recording)");
        HIP_TRY(ctx, hipStreamSynchronize(ctx->rec->up), "plan upload (recording)");
        ctx->rec->plan_used = true;
        return QW_OK;
    }
    HIP_TRY(ctx, hipMemcpyAsync(ctx->plan.p, b.p, b.n, hipMemcpyHostToDevice, ctx->stream), "plan upload");
    HIP_TRY(ctx, hipEventRecord(ctx->staging_ev, ctx->stream), "staging event");
    return QW_OK;
}

// Bump layout of a blob: offsets aligned to 64 bytes.
struct Layout {
    size_t size = 0;
    size_t take(size_t bytes, size_t align = 64) {
        size = (size + align - 1) & ~(align - 1);
        size_t off = size;
        size += bytes;
        return off;
    }
};

hipEvent_t get_event(qw_ctx *ctx) {
    if (!ctx->ev_pool.empty()) {
        hipEvent_t e = ctx->ev_pool.back();
        ctx->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Timing of launches with HIP events (QW_OPT_PROFILE): one pair of events
// around `launches` kernels of one kind that run back to back on the stream
// (an event pair per launch would put a timestamp between every two
// kernels of a batch).
struct ProfScope {
    qw_ctx *ctx;
    int kind;
    double bytes;
    uint32_t launches;
    hipEvent_t e0 = nullptr;
    ProfScope(qw_ctx *c, int k, double b, uint32_t n_launch = 1) : ctx(c), kind(k), bytes(b), launches(n_launch) {
        if (!ctx->profile || ctx->rec || launches == 0) return;
        e0 = get_event(ctx);
        if (e0) hipEventRecord(e0, ctx->stream);
    }
    ~ProfScope() {
        if (!ctx->profile || ctx->rec || !e0) return;
        hipEvent_t e1 = get_event(ctx);
        if (!e1) return;
        hipEventRecord(e1, ctx->stream);
        ctx->prof.push_back({kind, bytes, e0, e1, launches});
    }
};

const char *kind_name(uint32_t k) {
    switch (k) {
    case QW_KIND_STATEVECTOR: return "STATEVECTOR_BOUNDARY_STATE";
    case QW_KIND_TABLEAU: return "TABLEAU_BOUNDARY_STATE";
    default: return "UNKNOWN_KIND";
    }
}

const char *backend_name(uint32_t b) {
    switch (b) {
    case QW_BACKEND_SV: return "MI355X_SV_C64";
    case QW_BACKEND_STAB_ONLY: return "STABILIZER_ONLY";
    default: return "UNKNOWN";
    }
}

std::string json_escape(const std::string &s) {
    std::string o;
    for (char c : s) {
        if (c == '"' || c == '\\') o += '\\';
        o += c;
    }
    return o;
}

std::string refusal_json(const char *reason, const std::string &detail, uint32_t sk,
                         uint32_t tk, uint32_t sb, uint32_t tb, long task = -1) {
    std::ostringstream o;
    o << "{\"reason\": \"" << reason << "\", \"detail\": \"" << json_escape(detail)
      << "\", \"source_kind\": \"" << kind_name(sk) << "\", \"target_kind\": \"" << kind_name(tk)
      << "\", \"source_backend\": \"" << backend_name(sb) << "\", \"target_backend\": \""
      << backend_name(tb) << "\"";
    if (task >= 0) o << ", \"task\": " << task;
    o << "}";
    return o.str();
}

// The three gates of Sec. IV-B in order; Table II decides gate 3.
// Returns true if the continuation is EXACT; otherwise fills *json.
bool legal(const qw_artifact &a, uint32_t tk, uint32_t tb, std::string *json, long task = -1) {
    const uint32_t sk = a.kind, sb = a.backend;
    // gate 1: exactness validation
    if (a.exactness != QW_EXACT) {
        *json = refusal_json("NON_EXACT_ARTIFACT",
                             a.exactness == QW_APPROX ? "artifact exactness class is not EXACT."
                                                      : "artifact exactness class is unknown.",
                             sk, tk, sb, tb, task);
        return false;
    }
    // gate 2: backend-family validation
    const bool sb_known = (sb == QW_BACKEND_SV || sb == QW_BACKEND_STAB_ONLY);
    const bool tb_known = (tb == QW_BACKEND_SV || tb == QW_BACKEND_STAB_ONLY);
    const bool kinds_known = (sk == QW_KIND_STATEVECTOR || sk == QW_KIND_TABLEAU) &&
                             (tk == QW_KIND_STATEVECTOR || tk == QW_KIND_TABLEAU);
    if (!sb_known || !tb_known || !kinds_known) {
        *json = refusal_json("UNKNOWN_BACKEND", "producing or target backend family is unknown.",
                             sk, tk, sb, tb, task);
        return false;
    }
    // gate 3: conversion-rule lookup (Table II)
    if (sk == QW_KIND_TABLEAU && tk == QW_KIND_TABLEAU) {
        if (tb == QW_BACKEND_STAB_ONLY) return true;                 // STAB -> STAB
        *json = refusal_json("FORBIDDEN_CONVERSION", "tableau continuation needs a tableau backend.",
                             sk, tk, sb, tb, task);
        return false;
    }
    if (sk == QW_KIND_TABLEAU && tk == QW_KIND_STATEVECTOR) {
        if (tb == QW_BACKEND_SV) return true;                        // STAB -> SV (dense export)
        *json = refusal_json("FORBIDDEN_CONVERSION", "SV on stabilizer-only backend not supported.",
                             sk, tk, sb, tb, task);
        return false;
    }
    if (sk == QW_KIND_STATEVECTOR && tk == QW_KIND_TABLEAU) {      // SV -> STAB
        *json = refusal_json("FORBIDDEN_CONVERSION", "statevector to tableau handoff not supported.",
                             sk, tk, sb, tb, task);
        return false;
    }
    // SV -> SV: exact within a statevector-capable family only
    if (sb == QW_BACKEND_SV && tb == QW_BACKEND_SV) return true;
    *json = refusal_json("FORBIDDEN_CONVERSION", "SV on stabilizer-only backend not supported.",
                         sk, tk, sb, tb, task);
    return false;
}

bool slot_ok(const qw_state *st, uint32_t first, uint32_t count) {
    return (uint64_t)first + count <= st->n_slots;
}

char *slot_ptr(const qw_state *st, uint32_t s) { return st->base + (uint64_t)s * st->slot_bytes; }

// Plans of gate lists seen before on this context, keyed by the exact bytes
// of the gate records (and n, tile bits): resubmitting a gate list skips
// planning. Bounded; cleared when full. The hash only picks the bucket (a hit
// is confirmed by comparing the bytes), so it is a fast one: four independent
// 64-bit multiply-xorshift lanes over 8-byte words (a batch of 512 suffixes of
// 500 gates hashes 6 MB per call; one byte at a time that took about 9 ms).
uint64_t key_hash(const void *p, size_t len, uint64_t seed = 0xcbf29ce484222325ull) {
    const unsigned char *b = static_cast<const unsigned char *>(p);
    constexpr uint64_t K = 0x9E3779B97F4A7C15ull;
    uint64_t a[4] = {seed, seed ^ 0x243F6A8885A308D3ull, seed ^ 0x13198A2E03707344ull, seed ^ 0xA4093822299F31D0ull};
    size_t i = 0;
    for (; i + 32 <= len; i += 32)
        for (int l = 0; l < 4; ++l) {
            uint64_t w;
            std::memcpy(&w, b + i + 8 * l, 8);
            a[l] = (a[l] ^ w) * K;
            a[l] ^= a[l] >> 29;
        }
    uint64_t h = (uint64_t)len * K;
    for (int l = 0; l < 4; ++l) {
        h = (h ^ a[l]) * K;
        h ^= h >> 32;
    }
    for (; i < len; ++i) h = (h ^ b[i]) * 0x100000001b3ull;
    return h;
}

// Permuted index layouts between passes (QW_OPT_LAYOUT) make every pass
// that changes the layout run out of place, which doubles the memory a call
// sweeps. While a call's states fit the 256 MB last-level cache of the
// device (the MALL) in place, that costs more than the longer runs gain: a
// 24-qubit prefix state updated in place stays resident there for the 64
// suffix passes that then read it as their snapshot (measured: those passes
// took 3.87 instead of 4.20 ms when the prefix ran in place). Layouts are
// used when the states of the call exceed half of that cache (mode 1), or
// always (mode 2).
constexpr uint64_t kLayoutMinBytes = 128ull << 20;
bool layouts_pay(const qw_ctx *ctx, uint32_t n, uint64_t n_states) {
    return ctx->layout == 2 || (ctx->layout == 1 && n_states * (8ull << n) > kLayoutMinBytes);
}

// `in_place`: the plan's first pass loads its own destination (no snapshot
// or other source state). `layout`: permuted layouts allowed (layouts_pay).
std::string get_plan(qw_ctx *ctx, uint32_t n, const qw_gate *gates, uint64_t n_gates,
                     std::shared_ptr<const Plan> *out, bool in_place, bool layout, bool allow_dyn = false) {
    // the internal run-time operator of measured segments is never taken
    // from a caller's gate list (not even through the plan cache)
    if (!allow_dyn)
        for (uint64_t i = 0; i < n_gates; ++i)
            if (gates[i].kind == kGateDyn) return "gate " + std::to_string(i) + ": unknown kind 0x86";
    const size_t bytes = (size_t)n_gates * sizeof(qw_gate);
    const uint64_t opts[5] = {n, (uint64_t)ctx->tile_bits, (uint64_t)ctx->relabel, layout ? 1ull : 0ull,
                              in_place ? 1ull : 0ull};
    const uint64_t h = key_hash(gates, bytes, key_hash(opts, sizeof opts));
    auto &bucket = ctx->plan_cache[h];
    for (const auto &c : bucket) {
        if (c.n == n && c.tile_bits == ctx->tile_bits && c.relabel == ctx->relabel &&
            c.layout == layout && c.in_place == in_place &&
            c.gates.size() == bytes &&
            (bytes == 0 || std::memcmp(c.gates.data(), gates, bytes) == 0)) {
            *out = c.plan;
            return "";
        }
    }
    auto p = std::make_shared<Plan>();
    std::string e = build_plan((int)n, gates, (size_t)n_gates, ctx->tile_bits, p.get(), ctx->relabel, true,
                               allow_dyn, layout, in_place);
    if (!e.empty()) return e;
    if (ctx->plan_cache_entries >= 4096) {
        ctx->plan_cache.clear();
        ctx->plan_cache_entries = 0;
    }
    PlanEntry pe;
    pe.n = n;
    pe.tile_bits = ctx->tile_bits;
    pe.relabel = ctx->relabel;
    pe.layout = layout;
    pe.in_place = in_place;
    pe.gates.assign(reinterpret_cast<const char *>(gates), reinterpret_cast<const char *>(gates) + bytes);
    pe.plan = p;
    ctx->plan_cache[h].push_back(std::move(pe));
    ++ctx->plan_cache_entries;
    *out = p;
    return "";
}

// Tiered generated kernels: a pass structure not yet compiled is compiled
// when the launches of it on this context have run it over at least this
// many tiles (task-tiles, counted across calls: a structure that recurs in
// small groups, such as one error position of a batch, becomes hot too);
// until then, and for one-off structures, the interpreted kernels run
// (same results).
constexpr uint64_t kJitHotTiles = 4096;

// One task of an execution: its plan, source, destination.
struct Exec {
    std::shared_ptr<const Plan> planp;
    const Plan &plan_ref() const { return *planp; }
    const void *src = nullptr;  // first-pass source (snapshot) or nullptr
    void *dst = nullptr;
    // fused expectation epilogue of the last pass (generated kernels only)
    const RedPlan *epi = nullptr;
    const std::string *epi_key = nullptr;
    double *epi_part = nullptr;  // this task's [rows][epi_nt] partials
    uint32_t epi_nt = 0;
    // qw_run_tree: index (in the same execution) of the task whose final
    // state `src` is, or -1; such a task runs in a persistent launch
    int parent = -1;
};

// The plan has a pass that stores to other addresses than it loads (output
// relabelling or a change of index layout): its task needs a second buffer.
bool has_relabel(const Plan &p) {
    for (const HostPass &h : p.passes)
        if (h.moves()) return true;
    return false;
}

// `batch`: the call is a batch of tasks (qw_run_suffix_batch, qw_run_tree),
// which may run as one persistent launch (QW_OPT_PERSISTENT); the passes of
// a single state (qw_apply_prefix, measured segments) keep one launch per
// pass, since a lone state has no other tasks to fill the device between
// its dependent passes.
int execute_chunk(qw_ctx *ctx, uint32_t n, std::vector<Exec> &ex, bool batch);

int execute(qw_ctx *ctx, uint32_t n, std::vector<Exec> &ex, bool batch = false) {
    const uint64_t state_bytes = 8ull << n;
    // second state buffers of relabelling tasks are bounded by the
    // context's cap: larger batches run in chunks
    const uint64_t per = std::max<uint64_t>(1, ctx->pingpong_cap / state_bytes);
    uint64_t need = 0;
    for (const Exec &e : ex) need += has_relabel(*e.planp);
    if (need <= per) return execute_chunk(ctx, n, ex, batch);
    std::vector<Exec> part;
    uint64_t cnt = 0;
    for (size_t i = 0; i < ex.size(); ++i) {
        part.push_back(ex[i]);
        cnt += has_relabel(*ex[i].planp);
        if (cnt == per || i + 1 == ex.size()) {
            int rc = execute_chunk(ctx, n, part, batch);
            if (rc) return rc;
            part.clear();
            cnt = 0;
        }
    }
    return QW_OK;
}

// Buffers of one task's passes: 0 = the task's destination, 1 = its second
// buffer. A pass with output relabelling or a change of index layout stores
// to other addresses than it loads, so it never runs in place; the
// assignment ends in the destination.
// Returns the buffer pass 0 reads when the task has no external source, or
// 2 if the destination must first be copied to the second buffer.
int assign_buffers(const Plan &p, bool external_src, std::vector<int> *db) {
    const size_t P = p.passes.size();
    db->assign(P, 0);
    for (size_t k = P - 1; k >= 1; --k)
        (*db)[k - 1] = p.passes[k].moves() ? 1 - (*db)[k] : (*db)[k];
    if (external_src || !p.passes[0].moves() || (*db)[0] == 1) return 0;
    // pass 0 would relabel in place: make the first plain pass k >= 1 run
    // out of place (flips the buffers of passes 0..k-1)
    for (size_t k = 1; k < P; ++k)
        if (!p.passes[k].moves()) {
            for (size_t j = 0; j < k; ++j) (*db)[j] = 1 - (*db)[j];
            return 0;
        }
    return 2;
}

int execute_chunk(qw_ctx *ctx, uint32_t n, std::vector<Exec> &ex, bool batch) {
    if (ex.empty()) return QW_OK;
    const int m = ex[0].planp->m;
    const uint32_t tiles = (m >= kMinTileBits) ? (1u << (n - m)) : 1u;
    size_t steps = 0;
    for (Exec &e : ex) steps = std::max(steps, e.planp->passes.size());
    // tasks with a snapshot and no pass: plain copy of the boundary state
    const uint64_t state_bytes = 8ull << n;
    for (Exec &e : ex) {
        if (e.src && e.planp->passes.empty()) {
            ProfScope ps(ctx, 3, 2.0 * state_bytes);
            hipError_t er = launch_copy(ctx->stream, e.dst, e.src, state_bytes);
            if (er != hipSuccess) return hip_fail(ctx, er, "copy launch");
        }
    }
    if (steps == 0) return QW_OK;
    // scratch: per task norm partials [tiles] and one scale
    bool any_norm = false;
    for (Exec &e : ex)
        for (const HostPass &p : e.planp->passes) any_norm |= p.norm_out;
    const size_t norm_bytes = any_norm ? ex.size() * (tiles + 1) * sizeof(double) : 0;
    if (norm_bytes) {
        int rc = ensure(ctx, ctx->scratch, norm_bytes, "norm scratch");
        if (rc) return rc;
    }
    double *norm_base = static_cast<double *>(ctx->scratch.p);
    // one persistent launch for all passes (QW_OPT_PERSISTENT); a norm
    // finalisation between passes keeps the launches per pass structure
    const bool persist = batch && ctx->persistent && ctx->jit && m >= kMinTileBits && !any_norm;
    for (const Exec &e : ex)
        if (e.parent >= 0 && !persist)
            return fail(ctx, QW_E_INVALID_ARG, "in-call parents need a persistent launch");
    // second state buffers and per-pass buffer choice of relabelling tasks
    std::vector<std::vector<int>> bufsel(ex.size());
    std::vector<void *> second(ex.size(), nullptr);
    std::vector<char> precopy(ex.size(), 0);
    {
        uint64_t cnt = 0;
        for (Exec &e : ex) cnt += has_relabel(*e.planp);
        if (cnt) {
            const size_t want = (size_t)(cnt * state_bytes);
            if (ctx->rec && ctx->pingpong.cap < want) {
                int rc0 = ensure_recording(ctx, ctx->pingpong, want, "second state buffers");
                if (rc0) return rc0;
            }
            if (ctx->pingpong.cap < want) {
                int rc0 = cap_check(ctx, want, ctx->pingpong.cap, "second state buffers");
                if (rc0) return rc0;
                if (ctx->pingpong.p) {
                    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream), "sync before regrow");
                    HIP_TRY(ctx, hipFree(ctx->pingpong.p), "free second buffers");
                    ctx->pingpong.p = nullptr;
                    ctx->pingpong.cap = 0;
                }
                void *pp = nullptr;
                hipError_t er = hipMalloc(&pp, want);
                if (er != hipSuccess) return hip_fail(ctx, er, "second state buffers");
                ctx->pingpong.p = pp;
                ctx->pingpong.cap = want;
            }
            uint64_t i = 0;
            for (size_t t = 0; t < ex.size(); ++t) {
                if (!has_relabel(*ex[t].planp)) continue;
                second[t] = static_cast<char *>(ctx->pingpong.p) + (i++) * state_bytes;
                const int r = assign_buffers(*ex[t].planp, ex[t].src != nullptr, &bufsel[t]);
                if (r == 2) {
                    precopy[t] = 1;
                    ProfScope ps(ctx, 3, 2.0 * state_bytes);
                    hipError_t er = launch_copy(ctx->stream, second[t], ex[t].dst, state_bytes);
                    if (er != hipSuccess) return hip_fail(ctx, er, "copy launch");
                }
            }
        }
    }
    // blob layout
    Layout L;
    std::vector<size_t> step_off(steps), step_cnt(steps, 0);
    size_t n_desc = 0;
    for (size_t k = 0; k < steps; ++k) {
        for (Exec &e : ex) step_cnt[k] += (k < e.planp->passes.size());
        // (consecutive: the steps' descriptor arrays form one array)
        step_off[k] = L.take(step_cnt[k] * sizeof(PassDesc));
        n_desc += step_cnt[k];
    }
    // persistent launch: the descriptors again in claim order, at most one
    // segment per descriptor, one dependency each
    const size_t pdesc_off = persist ? L.take(n_desc * sizeof(PassDesc)) : 0;
    const size_t seg_off = persist ? L.take(n_desc * sizeof(PSeg)) : 0;
    const size_t dep_off = persist ? L.take(n_desc * sizeof(PDep)) : 0;
    std::vector<std::vector<std::pair<size_t, size_t>>> op_off(ex.size());
    std::vector<std::vector<size_t>> io_off(ex.size());
    for (size_t t = 0; t < ex.size(); ++t) {
        for (const HostPass &p : ex[t].planp->passes) {
            size_t oo = L.take(std::max<size_t>(1, p.dev_ops.size()) * sizeof(DevOp));
            size_t po = L.take(std::max<size_t>(1, p.dev_phases.size()) * sizeof(DevPhase));
            op_off[t].push_back({oo, po});
            io_off[t].push_back(L.take(2 * sizeof(IoRec)));
        }
    }
    // per distinct (local mask, load layout): the index of each tile's
    // origin in the state the pass loads
    std::vector<std::pair<const HostPass *, size_t>> tb_off;
    auto tile_table = [&](const HostPass &p) -> size_t {
        for (auto &e : tb_off)
            if (e.first->local_mask == p.local_mask && e.first->in_pos == p.in_pos) return e.second;
        size_t off = L.take((size_t)tiles * sizeof(uint32_t));
        tb_off.push_back({&p, off});
        return off;
    };
    std::vector<std::vector<size_t>> tb_of(ex.size());
    for (size_t t = 0; t < ex.size(); ++t)
        for (const HostPass &p : ex[t].planp->passes) tb_of[t].push_back(tile_table(p));
    // per distinct (local mask, relabelling, store layout): the index of
    // each tile's origin in the state the pass stores
    std::vector<std::pair<const HostPass *, size_t>> tbo_off;
    auto out_table = [&](const HostPass &p) -> size_t {
        for (auto &e : tbo_off)
            if (e.first->local_mask == p.local_mask && e.first->out_img == p.out_img &&
                e.first->out_pos == p.out_pos)
                return e.second;
        size_t off = L.take((size_t)tiles * sizeof(uint32_t));
        tbo_off.push_back({&p, off});
        return off;
    };
    std::vector<std::vector<size_t>> tbo_of(ex.size());
    for (size_t t = 0; t < ex.size(); ++t)
        for (const HostPass &p : ex[t].planp->passes)
            tbo_of[t].push_back(p.moves() ? out_table(p) : (size_t)-1);
    int rc = ensure(ctx, ctx->plan, L.size, "plan buffer");
    if (rc) return rc;
    uint8_t *dbase = static_cast<uint8_t *>(ctx->plan.p);
    StagedBlob blob;
    rc = stage_blob(ctx, L.size, &blob);
    if (rc) return rc;
    for (size_t t = 0; t < ex.size(); ++t) {
        for (size_t k = 0; k < ex[t].planp->passes.size(); ++k) {
            const HostPass &p = ex[t].planp->passes[k];
            std::memcpy(blob.data() + op_off[t][k].first, p.dev_ops.data(),
                        p.dev_ops.size() * sizeof(DevOp));
            std::memcpy(blob.data() + op_off[t][k].second, p.dev_phases.data(),
                        p.dev_phases.size() * sizeof(DevPhase));
            std::memcpy(blob.data() + io_off[t][k], &p.io_in, sizeof(IoRec));
            std::memcpy(blob.data() + io_off[t][k] + sizeof(IoRec), &p.io_out, sizeof(IoRec));
        }
    }
    {
        const uint64_t full = (1ull << n) - 1;
        // tile ti is the ti-th value of the non-local qubits in counting
        // order, whatever the layouts (so results do not depend on them)
        for (auto &e : tb_off) {
            uint32_t *tb = reinterpret_cast<uint32_t *>(blob.data() + e.second);
            const uint64_t nl = full & ~e.first->local_mask;
            const std::vector<uint8_t> &pos = e.first->in_pos;
            uint64_t g = 0;
            for (uint32_t ti = 0; ti < tiles; ++ti, g = next_in_mask(g, nl))
                tb[ti] = (uint32_t)to_layout(g, pos);
        }
        for (auto &e : tbo_off) {
            uint32_t *tb = reinterpret_cast<uint32_t *>(blob.data() + e.second);
            const uint64_t nl = full & ~e.first->local_mask;
            const std::vector<uint64_t> &img = e.first->out_img;
            const std::vector<uint8_t> &pos = e.first->out_pos;
            uint64_t g = 0;
            for (uint32_t ti = 0; ti < tiles; ++ti, g = next_in_mask(g, nl)) {
                uint64_t o = img.empty() ? g : 0;
                if (!img.empty())
                    for (uint64_t r = g; r; r &= r - 1) o ^= img[__builtin_ctzll(r)];
                tb[ti] = (uint32_t)to_layout(o, pos);
            }
        }
    }
    // Order of the tasks in each step's descriptor array. With generated
    // kernels, the tasks of one pass structure are consecutive and form one
    // launch (groups[k]: kernel, first descriptor, count).
    struct Group {
        const JitKernel *k;  // nullptr: interpreted kernels for this group
        uint32_t first, count;
        bool lds;
        uint32_t req;        // generated kernels: its request
    };
    std::vector<std::vector<size_t>> order(steps);
    std::vector<std::vector<Group>> groups(steps);
    const bool use_jit = ctx->jit && m >= kMinTileBits;
    std::vector<JitReq> reqs;
    if (use_jit) {
        std::vector<std::vector<std::pair<size_t, std::vector<size_t>>>> members(steps);
        for (size_t k = 0; k < steps; ++k) {
            std::map<std::string, size_t> gi;
            for (size_t t = 0; t < ex.size(); ++t) {
                if (k >= ex[t].planp->passes.size()) continue;
                const HostPass &p = ex[t].planp->passes[k];
                const bool with_epi = ex[t].epi && k + 1 == ex[t].planp->passes.size();
                const bool lds = p.norm_out || p.dev_phases.size() > 1 || with_epi;
                // a first pass that reads a boundary snapshot keeps the
                // default load policy (other tasks read the same snapshot)
                const bool stream = ctx->stream_loads && !(k == 0 && ex[t].src);
                if (p.jit_key.empty()) p.jit_key = jit_pass_key((int)n, m, p, p.norm_out || p.dev_phases.size() > 1);
                const std::string key = (with_epi ? jit_pass_key((int)n, m, p, true) + *ex[t].epi_key : p.jit_key) +
                                        (stream ? "S" : "T");
                auto it = gi.find(key);
                if (it == gi.end()) {
                    it = gi.emplace(key, members[k].size()).first;
                    members[k].push_back({reqs.size(), {}});
                    JitReq r;
                    r.key = key;
                    r.pass = &p;
                    r.epi = with_epi ? ex[t].epi : nullptr;
                    r.n = (int)n;
                    r.m = m;
                    r.use_lds = lds;
                    r.stream_loads = stream;
                    reqs.push_back(std::move(r));
                }
                members[k][it->second].second.push_back(t);
            }
        }
        // tiered: generate a kernel when it is available without compiling,
        // or when its structure has run enough work on this context to pay
        // for compiling it
        std::vector<char> want(reqs.size(), 1);
        if (ctx->jit == 1 && !persist) {
            std::vector<uint64_t> work(reqs.size(), 0);
            for (size_t k = 0; k < steps; ++k)
                for (auto &gm : members[k]) work[gm.first] += (uint64_t)gm.second.size() * tiles;
            for (size_t i = 0; i < reqs.size(); ++i) {
                uint64_t &heat = ctx->jit_heat[reqs[i].key];
                heat += work[i];
                want[i] = reqs[i].epi || heat >= kJitHotTiles || jit_available(ctx->device, reqs[i]);
            }
            if (ctx->jit_heat.size() > 65536) ctx->jit_heat.clear();
        }
        std::vector<JitReq> sel;
        std::vector<size_t> sel_of(reqs.size(), (size_t)-1);
        for (size_t i = 0; i < reqs.size(); ++i)
            if (want[i]) {
                sel_of[i] = sel.size();
                sel.push_back(reqs[i]);
            }
        std::vector<const JitKernel *> kern(sel.size(), nullptr);
        if (!persist) {
            const std::string err = jit_get(ctx->device, sel, &kern);
            if (!err.empty()) return fail(ctx, QW_E_HIP, err);
        }
        for (size_t k = 0; k < steps; ++k) {
            for (auto &gm : members[k]) {
                const JitKernel *kk = sel_of[gm.first] == (size_t)-1 ? nullptr : kern[sel_of[gm.first]];
                groups[k].push_back({kk, (uint32_t)order[k].size(), (uint32_t)gm.second.size(),
                                     reqs[gm.first].use_lds, (uint32_t)gm.first});
                for (size_t t : gm.second) order[k].push_back(t);
            }
        }
    } else {
        for (size_t k = 0; k < steps; ++k)
            for (size_t t = 0; t < ex.size(); ++t)
                if (k < ex[t].planp->passes.size()) order[k].push_back(t);
    }
    std::vector<char> step_norm(steps, 0), step_lds(steps, 0);
    for (size_t k = 0; k < steps; ++k) {
        size_t c = 0;
        for (size_t t : order[k]) {
            Exec &e = ex[t];
            const HostPass &p = e.planp->passes[k];
            PassDesc d{};
            if (second[t]) {
                void *buf[2] = {e.dst, second[t]};
                const std::vector<int> &db = bufsel[t];
                d.dst = buf[db[k]];
                d.src = k > 0 ? buf[db[k - 1]] : (e.src ? e.src : buf[precopy[t] ? 1 : 0]);
            } else {
                d.src = (k == 0 && e.src) ? e.src : e.dst;
                d.dst = e.dst;
            }
            if (p.moves()) {
                d.tile_base_out = reinterpret_cast<const uint32_t *>(dbase + tbo_of[t][k]);
                d.flags |= PD_REMAP_OUT;
            }
            if (e.epi && k + 1 == e.planp->passes.size()) {
                d.red_part = e.epi_part;
                d.red_nt = e.epi_nt;
            }
            d.ops = reinterpret_cast<const DevOp *>(dbase + op_off[t][k].first);
            d.phases = reinterpret_cast<const DevPhase *>(dbase + op_off[t][k].second);
            d.local_mask = p.local_mask;
            double *nb = norm_base ? norm_base + t * (tiles + 1) : nullptr;
            d.scale_in = nb ? nb + tiles : nullptr;
            d.norm_part = nb;
            d.scale_out = nb ? nb + tiles : nullptr;
            d.tile_base = reinterpret_cast<const uint32_t *>(dbase + tb_of[t][k]);
            d.io_in = reinterpret_cast<const IoRec *>(dbase + io_off[t][k]);
            d.io_out = reinterpret_cast<const IoRec *>(dbase + io_off[t][k] + sizeof(IoRec));
            d.n_ops = (uint32_t)p.dev_ops.size();
            d.n_phases = (uint32_t)p.dev_phases.size();
            d.flags |= (p.scale_in ? PD_SCALE_IN : 0u) | (p.norm_out ? PD_NORM_OUT : 0u);
            if (p.norm_out) step_norm[k] = 1;
            if (p.norm_out || p.dev_phases.size() > 1) step_lds[k] = 1;
            std::memcpy(blob.data() + step_off[k] + c * sizeof(PassDesc), &d, sizeof d);
            ++c;
        }
    }
    // persistent launch: its kernel (every pass structure of the call), the
    // segments (one per level and pass structure, in claim order) and each
    // descriptor's dependency
    const JitKernel *pk = nullptr;
    std::vector<PersistPart> parts;
    uint32_t n_segs = 0, n_claims = 0, pgrid = 0;
    if (persist) {
        std::vector<uint32_t> kind_of(reqs.size(), kNoDep);
        for (size_t k = 0; k < steps; ++k)
            for (const Group &g : groups[k]) {
                if (kind_of[g.req] != kNoDep) continue;
                kind_of[g.req] = (uint32_t)parts.size();
                PersistPart q;
                q.pass = reqs[g.req].pass;
                q.epi = reqs[g.req].epi;
                q.epi_key = ex[order[k][g.first]].epi_key;
                q.n = (int)n;
                q.m = m;
                q.stream_loads = reqs[g.req].stream_loads;
                parts.push_back(q);
            }
        JitReq pr;
        pr.key = jit_persist_key(parts);
        pr.persist = &parts;
        pr.n = (int)n;
        pr.m = m;
        pr.use_lds = true;
        std::vector<const JitKernel *> kk;
        const std::string err = jit_get(ctx->device, {pr}, &kk);
        if (!err.empty()) return fail(ctx, QW_E_HIP, err);
        pk = kk[0];
        pgrid = ctx->n_cu * (uint32_t)pk->blocks_per_cu;
        // the claim schedule (levels, segments, dependencies)
        std::vector<int> par(ex.size());
        std::vector<uint32_t> npass(ex.size());
        for (size_t t = 0; t < ex.size(); ++t) {
            par[t] = ex[t].parent;
            npass[t] = (uint32_t)ex[t].planp->passes.size();
        }
        std::vector<PersistDesc> pds;
        std::vector<uint32_t> from;  // index in the per-step descriptor arrays
        pds.reserve(n_desc);
        for (size_t k = 0; k < steps; ++k) {
            const uint32_t d0 = (uint32_t)(step_off[k] / sizeof(PassDesc));
            const PassDesc *hd = reinterpret_cast<const PassDesc *>(blob.data() + step_off[k]);
            for (const Group &g : groups[k]) {
                const uint32_t units = reqs[g.req].epi ? tiles / red_row_tiles(tiles) : tiles;
                for (uint32_t i = 0; i < g.count; ++i) {
                    const size_t t = order[k][g.first + i];
                    PersistDesc d;
                    d.t = (uint32_t)t;
                    d.k = (uint32_t)k;
                    d.kind = kind_of[g.req];
                    d.units = units;
                    d.src = reinterpret_cast<uint64_t>(hd[g.first + i].src);
                    d.relabel = !ex[t].planp->passes[k].out_img.empty();
                    pds.push_back(d);
                    from.push_back(d0 + g.first + i);
                }
            }
        }
        PersistSchedule sch;
        const std::string se = persist_schedule(par, npass, pds, ctx->tile_order, ctx->persist_chunk, pgrid, &sch);
        if (!se.empty()) return fail(ctx, QW_E_INVALID_ARG, se);
        PassDesc *pd = reinterpret_cast<PassDesc *>(blob.data() + pdesc_off);
        const PassDesc *sd = reinterpret_cast<const PassDesc *>(blob.data() + step_off[0]);
        for (uint32_t i = 0; i < (uint32_t)sch.order.size(); ++i) pd[i] = sd[from[sch.order[i]]];
        std::memcpy(blob.data() + seg_off, sch.segs.data(), sch.segs.size() * sizeof(PSeg));
        std::memcpy(blob.data() + dep_off, sch.deps.data(), sch.deps.size() * sizeof(PDep));
        n_segs = (uint32_t)sch.segs.size();
        n_claims = sch.claims;
    }
    if (ctx->rec && !ctx->rec->calls.empty()) {
        // where each task's op records live in the graph (qw_graph_update_gates)
        for (size_t t = 0; t < ex.size(); ++t) {
            GraphSeg sg;
            sg.n = n;
            sg.plan = ex[t].planp;
            for (size_t k = 0; k < ex[t].planp->passes.size(); ++k)
                sg.ops.push_back({dbase + op_off[t][k].first,
                                  ex[t].planp->passes[k].dev_ops.size() * sizeof(DevOp)});
            ctx->rec->calls.back().push_back(std::move(sg));
        }
    }
    rc = upload_staged(ctx, blob);
    if (rc) return rc;
    // one event pair around all pass launches of the call when they run back
    // to back (no norm finalisation between them), else one per launch
    uint32_t n_launch = 0;
    double all_bytes = 0.0;
    for (size_t k = 0; k < steps; ++k) {
        n_launch += use_jit ? (uint32_t)groups[k].size() : 1u;
        all_bytes += (double)step_cnt[k] * 2.0 * (double)state_bytes;
    }
    if (persist) {
        const size_t words = kSyncCounters + n_desc;
        int rc2 = ensure(ctx, ctx->psync, words * sizeof(uint32_t), "persistent sync area");
        if (rc2) return rc2;
        uint32_t *sync = static_cast<uint32_t *>(ctx->psync.p);
        hipError_t er = launch_zero_words(ctx->stream, sync, words);
        if (er != hipSuccess) return hip_fail(ctx, er, "sync clear launch");
        ProfScope ps(ctx, 0, all_bytes, 1u);
        er = jit_launch_persist(ctx->stream, *pk, reinterpret_cast<const PSeg *>(dbase + seg_off), n_segs,
                                reinterpret_cast<const PassDesc *>(dbase + pdesc_off),
                                reinterpret_cast<const PDep *>(dbase + dep_off), sync, n_claims,
                                std::min(pgrid, n_claims), ctx->spin_limit, ctx->host_flag);
        if (er != hipSuccess) return hip_fail(ctx, er, "persistent launch");
        return QW_OK;
    }
    ProfScope ps_all(ctx, 0, all_bytes, any_norm ? 0u : n_launch);
    for (size_t k = 0; k < steps; ++k) {
        const PassDesc *dd = reinterpret_cast<const PassDesc *>(dbase + step_off[k]);
        if (use_jit) {
            for (const Group &g : groups[k]) {
                ProfScope ps(ctx, 0, (double)g.count * 2.0 * (double)state_bytes, any_norm ? 1u : 0u);
                // item order (QW_OPT_TILE_ORDER); descriptor-major whenever
                // every task of the group reads one source
                bool tile_major = false;
                {
                    const PassDesc *hd = reinterpret_cast<const PassDesc *>(blob.data() + step_off[k]);
                    bool shared_src = true;
                    for (uint32_t i = 1; i < g.count && shared_src; ++i)
                        shared_src = hd[g.first + i].src == hd[g.first].src;
                    const bool relabel = !ex[order[k][g.first]].planp->passes[k].out_img.empty();
                    tile_major = !shared_src && (ctx->tile_order == 2 || (ctx->tile_order == 1 && relabel));
                }
                hipError_t er = g.k ? jit_launch(ctx->stream, *g.k, dd + g.first, g.count, tiles,
                                                 ctx->xcd_remap ? 1 : 0, ctx->n_cu, tile_major)
                                    : launch_pass(ctx->stream, dd + g.first, g.count, n, (uint32_t)m,
                                                  ctx->xcd_remap ? 1 : 0, g.lds);
                if (er != hipSuccess) return hip_fail(ctx, er, "pass launch");
            }
        } else {
            ProfScope ps(ctx, 0, (double)step_cnt[k] * 2.0 * (double)state_bytes, any_norm ? 1u : 0u);
            hipError_t er = launch_pass(ctx->stream, dd, (uint32_t)step_cnt[k], n, (uint32_t)m,
                                        ctx->xcd_remap ? 1 : 0, step_lds[k] != 0);
            if (er != hipSuccess) return hip_fail(ctx, er, "pass launch");
        }
        if (step_norm[k]) {
            hipError_t er = launch_norm_finalize(ctx->stream, dd, (uint32_t)step_cnt[k], tiles);
            if (er != hipSuccess) return hip_fail(ctx, er, "norm finalize launch");
        }
    }
    return QW_OK;
}

// Pauli string (X/Y support x, Z/Y support z, Y where both) conjugated by
// CNOT(c, t): P -> C P C. The update of the support and of the sign is the
// tableau rule of Aaronson and Gottesman (Phys. Rev. A 70, 052328, 2004).
void conj_cnot(uint64_t *x, uint64_t *z, int *neg, int c, int t) {
    const int xc = (int)((*x >> c) & 1ull), zc = (int)((*z >> c) & 1ull);
    const int xt = (int)((*x >> t) & 1ull), zt = (int)((*z >> t) & 1ull);
    *neg ^= xc & zt & (xt ^ zc ^ 1);
    *x ^= (uint64_t)xc << t;
    *z ^= (uint64_t)zt << c;
}

struct FusedEpi {
    bool active = false;
    std::vector<char> fused;  // per term: reduced in the last pass
    RedPlan rplan;
    std::string key;
};

void plan_fused_last(int n, int m, const HostPass &lp, const uint64_t *x, const uint64_t *z,
                     uint32_t n_terms, FusedEpi *fe);

// Decides the fused epilogue of a batch: every task's last pass must have
// the same local set and relabelling, no pass may renormalize, the last
// passes must run as generated kernels, and the terms left for the reducer
// must need fewer sweeps than all of them.
void plan_fused(qw_ctx *ctx, uint32_t n, const std::vector<Exec> &ex, const uint64_t *x,
                const uint64_t *z, uint32_t n_terms, FusedEpi *fe) {
    if (!ctx->fused_epilogue || ex.empty() || ctx->jit == 0) return;
    const int m = ex[0].planp->m;
    if (m < kMinTileBits || (int)n <= m) return;
    const HostPass *last = nullptr;
    for (const Exec &e : ex) {
        const Plan &p = *e.planp;
        if (p.passes.empty()) return;
        for (const HostPass &h : p.passes)
            if (h.norm_out || h.scale_in) return;
        const HostPass &l = p.passes.back();
        if (!last) last = &l;
        else if (l.local_mask != last->local_mask || l.out_cx != last->out_cx || l.in_pos != last->in_pos)
            return;
    }
    const uint64_t tiles = 1ull << (n - m);
    if (ctx->jit == 1 && (uint64_t)ex.size() * tiles < kJitHotTiles) return;
    plan_fused_last((int)n, m, *last, x, z, n_terms, fe);
}

// The fused epilogue of a last pass: its terms (conjugated through the
// pass's relabelling CNOTs) and their reducer plan, if that saves a sweep.
void plan_fused_last(int n, int m, const HostPass &lp, const uint64_t *x, const uint64_t *z,
                     uint32_t n_terms, FusedEpi *fe) {
    const HostPass *last = &lp;
    std::vector<uint64_t> xc(x, x + n_terms), zc(z, z + n_terms);
    std::vector<int> neg(n_terms, 0);
    std::vector<char> fused(n_terms, 0);
    TermGroup g{last->local_mask, {}};
    for (uint32_t j = 0; j < n_terms; ++j) {
        for (size_t i = last->out_cx.size(); i-- > 0;)
            conj_cnot(&xc[j], &zc[j], &neg[j], last->out_cx[i].first, last->out_cx[i].second);
        if ((xc[j] & ~last->local_mask) == 0 && g.terms.size() < (size_t)kMaxGroupTerms) {
            fused[j] = 1;
            g.terms.push_back(j);
        }
    }
    if (g.terms.empty()) return;
    std::vector<uint64_t> rest;
    for (uint32_t j = 0; j < n_terms; ++j)
        if (!fused[j]) rest.push_back(x[j]);
    const size_t before = group_terms(n, m, x, n_terms).size();
    const size_t after = rest.empty() ? 0 : group_terms(n, m, rest.data(), rest.size()).size();
    if (after >= before) return;
    // the diagonal terms are evaluated in the layout the pass ends in
    fe->rplan = plan_reduce_group(n, m, g, xc.data(), zc.data(),
                                  last->dev_phases.empty() ? nullptr : last->dev_phases.back().reg);
    for (TermDev &t : fe->rplan.terms) {
        if (neg[fe->rplan.cols[t.col]]) t.neg ^= 1;
        t.zg = to_layout(t.zg, last->in_pos);   // read from the tile origin
    }
    fe->fused = fused;
    fe->key = jit_epilogue_key(n, m, *last, fe->rplan);
    fe->active = true;
}

// Expectations for a list of slot pointers of one n-qubit layout.
int expect_slots(qw_ctx *ctx, uint32_t n, const std::vector<const void *> &slots,
                 const uint64_t *x, const uint64_t *z, const double *c, uint32_t n_terms,
                 double *out, int out_is_host, const std::vector<char> *fused = nullptr) {
    const uint32_t ns = (uint32_t)slots.size();
    if (ns == 0) return QW_OK;
    const uint64_t full = (1ull << n) - 1;
    for (uint32_t j = 0; j < n_terms; ++j)
        if ((x[j] & ~full) || (z[j] & ~full))
            return fail(ctx, QW_E_INVALID_ARG, "Pauli mask has bits >= n");
    if (ctx->rec && (out_is_host || n_terms == 0))
        return recording_unsupported(ctx, out_is_host ? "a host output" : "an empty term list");
    if (n_terms == 0) {
        std::vector<double> zero(ns, 0.0);
        if (out_is_host) {
            std::memcpy(out, zero.data(), ns * sizeof(double));
            return QW_OK;
        }
        HIP_TRY(ctx, hipMemcpyAsync(out, zero.data(), ns * sizeof(double), hipMemcpyHostToDevice,
                                    ctx->stream), "zero out");
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream), "sync");
        return QW_OK;
    }
    const int m = tile_bits_for((int)n, ctx->tile_bits);
    const bool small = m < kMinTileBits;
    const uint32_t tiles = small ? 1u : (1u << (n - m));
    const uint32_t rows = tiles / red_row_tiles(tiles);   // partial rows per slot
    // terms whose partials a fused pass epilogue already wrote are left out
    std::vector<TermGroup> groups;
    if (fused && !small) {
        std::vector<uint32_t> idx;
        std::vector<uint64_t> xs;
        for (uint32_t j = 0; j < n_terms; ++j)
            if (!(*fused)[j]) {
                idx.push_back(j);
                xs.push_back(x[j]);
            }
        if (!idx.empty()) groups = group_terms((int)n, m, xs.data(), xs.size());
        for (TermGroup &g : groups)
            for (uint32_t &t : g.terms) t = idx[t];
    } else {
        groups = group_terms((int)n, m, x, n_terms);
    }
    std::vector<RedPlan> rplans;
    if (!small)
        for (const TermGroup &g : groups) rplans.push_back(plan_reduce_group((int)n, m, g, x, z));
    Layout L;
    std::vector<size_t> t_off(groups.size()), p_off(groups.size()), c_off(groups.size());
    size_t small_terms_off = 0;
    if (small) {
        small_terms_off = L.take(n_terms * sizeof(TermSmall));
    } else {
        for (size_t g = 0; g < groups.size(); ++g) {
            t_off[g] = L.take(rplans[g].terms.size() * sizeof(TermDev));
            p_off[g] = L.take(rplans[g].phases.size() * sizeof(RedPhase));
            c_off[g] = L.take(rplans[g].cols.size() * sizeof(uint32_t));
        }
    }
    bool use_jit = ctx->jit && !small;
    if (use_jit && ctx->jit == 1 && (uint64_t)ns * tiles < kJitHotTiles) {
        // tiered: small one-off reductions use the interpreted reducer unless
        // every group's kernel is available without compiling
        for (size_t g = 0; g < groups.size() && use_jit; ++g) {
            JitReq r;
            r.key = jit_reduce_key((int)n, m, groups[g], rplans[g]);
            r.group = &groups[g];
            r.rplan = &rplans[g];
            r.n = (int)n;
            r.m = m;
            use_jit = jit_available(ctx->device, r);
        }
    }
    std::vector<size_t> tb_off(groups.size(), 0);
    if (use_jit)
        for (size_t g = 0; g < groups.size(); ++g) tb_off[g] = L.take((size_t)tiles * sizeof(uint32_t));
    const size_t coeff_off = L.take(n_terms * sizeof(double));
    const size_t n_desc = small ? ns : ns * groups.size();
    const size_t desc_off = L.take(n_desc * (small ? sizeof(ReduceDescSmall) : sizeof(ReduceDesc)));
    int rc = ensure(ctx, ctx->plan, L.size, "plan buffer");
    if (rc) return rc;
    const size_t part_bytes = (size_t)ns * rows * n_terms * sizeof(double);
    const size_t out_bytes = ns * sizeof(double);
    rc = ensure(ctx, ctx->scratch, part_bytes + out_bytes + 256, "reduce scratch");
    if (rc) return rc;
    uint8_t *dbase = static_cast<uint8_t *>(ctx->plan.p);
    double *part = static_cast<double *>(ctx->scratch.p);
    double *dout = out_is_host ? reinterpret_cast<double *>(
                                     static_cast<uint8_t *>(ctx->scratch.p) +
                                     ((part_bytes + 255) & ~size_t(255)))
                               : out;
    std::vector<uint8_t> blob(L.size, 0);
    std::memcpy(blob.data() + coeff_off, c, n_terms * sizeof(double));
    if (small) {
        for (uint32_t j = 0; j < n_terms; ++j) {
            TermSmall t{};
            t.x = (uint32_t)x[j];
            t.z = (uint32_t)z[j];
            t.ny_mod4 = (uint32_t)(popc64(x[j] & z[j]) & 3);
            t.out_index = j;
            std::memcpy(blob.data() + small_terms_off + j * sizeof(TermSmall), &t, sizeof t);
        }
        for (uint32_t s = 0; s < ns; ++s) {
            ReduceDescSmall d{};
            d.psi = slots[s];
            d.terms = reinterpret_cast<const TermSmall *>(dbase + small_terms_off);
            d.part = part + (size_t)s * n_terms;
            d.n_terms = n_terms;
            std::memcpy(blob.data() + desc_off + s * sizeof(ReduceDescSmall), &d, sizeof d);
        }
    } else {
        for (size_t g = 0; g < groups.size(); ++g) {
            const RedPlan &rp = rplans[g];
            std::memcpy(blob.data() + t_off[g], rp.terms.data(), rp.terms.size() * sizeof(TermDev));
            std::memcpy(blob.data() + p_off[g], rp.phases.data(), rp.phases.size() * sizeof(RedPhase));
            std::memcpy(blob.data() + c_off[g], rp.cols.data(), rp.cols.size() * sizeof(uint32_t));
        }
        for (size_t g = 0; g < groups.size() && use_jit; ++g) {
            uint32_t *tb = reinterpret_cast<uint32_t *>(blob.data() + tb_off[g]);
            const uint64_t nl = full & ~groups[g].local_mask;
            uint64_t gb = 0;
            for (uint32_t ti = 0; ti < tiles; ++ti, gb = next_in_mask(gb, nl)) tb[ti] = (uint32_t)gb;
        }
        for (uint32_t s = 0; s < ns; ++s) {
            for (size_t g = 0; g < groups.size(); ++g) {
                // generated reducers: one launch per group, descriptors [group][slot]
                const size_t di = use_jit ? g * ns + s : (size_t)s * groups.size() + g;
                ReduceDesc d{};
                d.psi = slots[s];
                d.terms = reinterpret_cast<const TermDev *>(dbase + t_off[g]);
                d.phases = reinterpret_cast<const RedPhase *>(dbase + p_off[g]);
                d.cols = reinterpret_cast<const uint32_t *>(dbase + c_off[g]);
                d.part = part + (size_t)s * rows * n_terms;
                d.local_mask = groups[g].local_mask;
                d.n_phases = (uint32_t)rplans[g].phases.size();
                d.n_terms = (uint32_t)rplans[g].terms.size();
                d.n_terms_total = n_terms;
                d.tile_base = use_jit ? reinterpret_cast<const uint32_t *>(dbase + tb_off[g]) : nullptr;
                std::memcpy(blob.data() + desc_off + di * sizeof(ReduceDesc), &d, sizeof d);
            }
        }
    }
    std::vector<const JitKernel *> rk;
    if (use_jit) {
        std::vector<JitReq> reqs(groups.size());
        for (size_t g = 0; g < groups.size(); ++g) {
            reqs[g].key = jit_reduce_key((int)n, m, groups[g], rplans[g]);
            reqs[g].group = &groups[g];
            reqs[g].rplan = &rplans[g];
            reqs[g].n = (int)n;
            reqs[g].m = m;
        }
        const std::string err = jit_get(ctx->device, reqs, &rk);
        if (!err.empty()) return fail(ctx, QW_E_HIP, err);
    }
    rc = upload(ctx, blob);
    if (rc) return rc;
    if (use_jit) {
        const ReduceDesc *dd = reinterpret_cast<const ReduceDesc *>(dbase + desc_off);
        ProfScope ps(ctx, 1, (double)ns * groups.size() * (double)(8ull << n), (uint32_t)groups.size());
        for (size_t g = 0; g < groups.size(); ++g) {
            hipError_t er = jit_launch_reduce(ctx->stream, *rk[g], dd + g * ns, ns, tiles, ctx->n_cu,
                                              ctx->tile_order == 2);
            if (er != hipSuccess) return hip_fail(ctx, er, "generated reduce launch");
        }
    } else if (small || !groups.empty()) {
        ProfScope ps(ctx, 1, (double)ns * groups.size() * (double)(8ull << n));
        hipError_t er = small
            ? launch_reduce_small(ctx->stream, reinterpret_cast<const ReduceDescSmall *>(dbase + desc_off),
                                  ns, n)
            : launch_reduce(ctx->stream, reinterpret_cast<const ReduceDesc *>(dbase + desc_off),
                            (uint32_t)n_desc, n, (uint32_t)m);
        if (er != hipSuccess) return hip_fail(ctx, er, "reduce launch");
    }
    hipError_t er = launch_expect_finalize(ctx->stream, part,
                                           reinterpret_cast<const double *>(dbase + coeff_off),
                                           n_terms, rows, ns, dout);
    if (er != hipSuccess) return hip_fail(ctx, er, "finalize launch");
    if (out_is_host) {
        HIP_TRY(ctx, hipMemcpyAsync(out, dout, out_bytes, hipMemcpyDeviceToHost, ctx->stream),
                "result copy");
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream), "sync");
    }
    return QW_OK;
}

bool is_measure(uint32_t kind) { return kind == QW_GATE_MEASURE || kind == QW_GATE_RESET; }

bool has_measure(const qw_gate *g, uint64_t n) {
    for (uint64_t i = 0; i < n; ++i)
        if (is_measure(g[i].kind)) return true;
    return false;
}

// One task of a measured execution.
struct MeasTask {
    std::vector<qw_gate> rest;   // gates not yet run
    const void *src = nullptr;   // the first segment's source (a snapshot), or null
    void *dst = nullptr;
    std::vector<qw_gate> head;   // projectors (and X) that open the next segment
    std::vector<qw_gate> cluster;  // measurements decided after this round's segment
    std::vector<uint8_t> outc;
    bool done = false;
};

// Largest number of measurements decided jointly (2^k outcome bins).
constexpr size_t kMaxJoint = 12;
// Joint decisions need every measured qubit >= this (a 256-amplitude chunk
// then lies in one outcome bin).
constexpr uint32_t kJointMinQubit = 8;

uint64_t gate_qubits(const qw_gate &g) {
    if (g.kind == QW_GATE_RENORM) return 0;
    uint64_t m = 1ull << g.q0;
    if (g.kind == QW_GATE_CNOT || g.kind == QW_GATE_CZ) m |= 1ull << g.q1;
    return m;
}

// Splits off the next segment of a task: the gates up to its next
// measurement, plus every later gate that touches none of the qubits
// measured so far (a measurement commutes with gates on other qubits, so it
// is decided after them), collecting the measurements met on the way; stops
// at a gate on a measured qubit, a second measurement of one, a RENORM after
// a measurement, kMaxJoint measurements, or (for a joint decision) a
// measurement of a qubit below kJointMinQubit.
void next_segment(MeasTask &t, std::vector<qw_gate> *seg) {
    *seg = t.head;
    t.head.clear();
    t.cluster.clear();
    uint64_t pend = 0;
    bool low = false;
    size_t i = 0;
    for (; i < t.rest.size(); ++i) {
        const qw_gate &g = t.rest[i];
        if (is_measure(g.kind)) {
            const bool q_low = g.q0 < kJointMinQubit;
            if ((pend >> g.q0) & 1ull) break;
            if (!t.cluster.empty() && (low || q_low)) break;
            t.cluster.push_back(g);
            pend |= 1ull << g.q0;
            low = low || q_low;
            if (t.cluster.size() == kMaxJoint) {
                ++i;
                break;
            }
            continue;
        }
        if (g.kind == QW_GATE_RENORM && !t.cluster.empty()) break;
        if (gate_qubits(g) & pend) break;
        seg->push_back(g);
    }
    t.rest.erase(t.rest.begin(), t.rest.begin() + (std::ptrdiff_t)i);
}

// The outcomes of a cluster from its outcome-bin masses (bin bits = the
// measured qubits in ascending order): measurement j (gate order) takes
// b_j = (u_j < M(bit = 1 | earlier outcomes) / M(earlier outcomes)), FP64
// sums in ascending bin order; then the bins are halved along that bit.
// Returns the mass of the chosen bin.
double decide_cluster(MeasTask &t, std::vector<double> mass, std::vector<uint32_t> *outs) {
    std::vector<uint32_t> qs;
    for (const qw_gate &g : t.cluster) qs.push_back(g.q0);
    std::vector<uint32_t> asc = qs;
    std::sort(asc.begin(), asc.end());
    std::vector<uint32_t> alive = asc;  // qubits still bits of `mass`, ascending
    outs->clear();
    for (const qw_gate &g : t.cluster) {
        const uint32_t p = (uint32_t)(std::find(alive.begin(), alive.end(), g.q0) - alive.begin());
        double tot = 0.0, one = 0.0;
        for (size_t b = 0; b < mass.size(); ++b) {
            tot += mass[b];
            if ((b >> p) & 1u) one += mass[b];
        }
        const uint32_t bit = g.param < one / tot ? 1u : 0u;
        outs->push_back(bit);
        std::vector<double> half(mass.size() / 2);
        for (size_t b = 0, h = 0; b < mass.size(); ++b)
            if (((b >> p) & 1u) == bit) half[h++] = mass[b];
        mass.swap(half);
        alive.erase(alive.begin() + p);
    }
    return mass[0];
}

// Gate lists with MEASURE / RESET gates run in rounds. A round runs every
// unfinished task's next segment (next_segment) as one batch (the first
// round reads the tasks' snapshots, later rounds run in place). The
// measurements collected with the segments are then decided: a single one
// from its FP64 sums S and S1, a cluster from the FP64 masses of its 2^k
// outcome bins (decide_cluster), with the caller's draws; the next segment
// opens with the projectors (the first one carrying 1 / sqrt of the chosen
// mass) and an X for each RESET with outcome 1. Outcomes are recorded per
// task in gate order (qw_outcomes).
int run_measured(qw_ctx *ctx, uint32_t n, std::vector<MeasTask> &mt) {
    uint64_t total_meas = 0;
    std::vector<uint32_t> outc_base(mt.size()), outc_next(mt.size());
    for (size_t k = 0; k < mt.size(); ++k) {
        outc_base[k] = outc_next[k] = (uint32_t)total_meas;
        for (size_t i = 0; i < mt[k].rest.size(); ++i) {
            const qw_gate &q = mt[k].rest[i];
            if (!is_measure(q.kind)) continue;
            if (q.q0 >= n || q.reserved != 0 || !(q.param >= 0.0 && q.param < 1.0)) {
                char buf[160];
                snprintf(buf, sizeof buf, "task %zu gate %zu: a measurement needs a qubit < n and u in [0, 1)",
                         k, i);
                return fail(ctx, QW_E_INVALID_ARG, buf);
            }
            ++total_meas;
        }
    }
    const uint32_t T = (uint32_t)mt.size();
    const uint32_t kStride = 1u << kMaxJoint;
    const uint64_t chunks_max = 1ull << (n > kJointMinQubit ? n - kJointMinQubit : 0);
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t part_doubles = std::max<size_t>((size_t)2 * T * chunks_max, 2 * (size_t)T);
    const size_t out_doubles = (size_t)T * kStride;
    const size_t dyn_off = al((part_doubles + out_doubles) * sizeof(double));
    const size_t outc_off = dyn_off + al((size_t)total_meas * 4 * sizeof(float));
    const size_t err_off = outc_off + al((size_t)total_meas);
    // a recorded graph keeps each measured call's buffer (its outcomes stay
    // readable after a replay)
    if (ctx->rec && ctx->meas.p) {
        ctx->rec->owned.push_back(ctx->meas.p);
        ctx->meas = DevBuf{};
    }
    int rc = ensure(ctx, ctx->meas, err_off + 256, "measure buffer");
    if (rc) return rc;
    char *mb = static_cast<char *>(ctx->meas.p);
    double *part = reinterpret_cast<double *>(mb);
    double *dout = part + part_doubles;
    float *dyn = reinterpret_cast<float *>(mb + dyn_off);
    uint8_t *outc = reinterpret_cast<uint8_t *>(mb + outc_off);
    uint32_t *err = reinterpret_cast<uint32_t *>(mb + err_off);
    {
        hipError_t e = launch_meas_clear(ctx->stream, err);
        if (e != hipSuccess) return hip_fail(ctx, e, "measure launch");
    }
    uint32_t dyn_next = 0;
    bool first = true;
    std::vector<std::vector<qw_gate>> segs(mt.size());
    while (true) {
        std::vector<Exec> ex;
        for (size_t k = 0; k < mt.size(); ++k) {
            MeasTask &t = mt[k];
            if (t.done) continue;
            next_segment(t, &segs[k]);
            Exec x;
            x.src = first ? t.src : nullptr;
            std::string err_s = get_plan(ctx, n, segs[k].data(), segs[k].size(), &x.planp, x.src == nullptr,
                                         layouts_pay(ctx, n, mt.size()), true);
            if (!err_s.empty()) return fail(ctx, QW_E_INVALID_ARG, "task " + std::to_string(k) + ": " + err_s);
            x.dst = t.dst;
            ex.push_back(x);
            if (t.cluster.empty() && t.rest.empty()) t.done = true;
        }
        first = false;
        if (ex.empty()) break;
        rc = execute(ctx, n, ex);
        if (rc) return rc;
        // decision groups: single measurements (bit split, any qubit), and
        // joint clusters by chunk size C (the lowest measured qubit, <= 14)
        std::map<uint32_t, std::vector<size_t>> groups;  // C (0 = single) -> tasks
        for (size_t k = 0; k < mt.size(); ++k) {
            const MeasTask &t = mt[k];
            if (t.done || t.cluster.empty()) continue;
            uint32_t C = 0;
            if (t.cluster.size() > 1) {
                C = std::min<uint32_t>(14, n);
                for (const qw_gate &g : t.cluster) C = std::min(C, g.q0);
            }
            groups[C].push_back(k);
        }
        if (groups.empty()) break;
        for (auto &gr : groups) {
            const uint32_t C = gr.first;
            const std::vector<size_t> &who = gr.second;
            const uint32_t M = (uint32_t)who.size();
            // uploaded with the group: slot pointers, qubits (single) or
            // measured masks >> C (joint), per-task decision ranges, decisions
            std::vector<const void *> ptrs(M);
            std::vector<uint64_t> qs(M);
            std::vector<uint32_t> tfirst(M), tcount(M);
            std::vector<MeasDec> dec;
            for (uint32_t i = 0; i < M; ++i) {
                MeasTask &t = mt[who[i]];
                ptrs[i] = t.dst;
                uint64_t msk = 0;
                for (const qw_gate &g : t.cluster) msk |= 1ull << g.q0;
                qs[i] = C ? (msk >> C) : (uint64_t)t.cluster[0].q0;
                tfirst[i] = (uint32_t)dec.size();
                tcount[i] = (uint32_t)t.cluster.size();
                // bin bit of each measurement at its turn: its rank among the
                // qubits still open (ascending), the decided ones removed
                std::vector<uint32_t> alive;
                for (const qw_gate &g : t.cluster) alive.push_back(g.q0);
                std::sort(alive.begin(), alive.end());
                for (const qw_gate &g : t.cluster) {
                    const auto it = std::find(alive.begin(), alive.end(), g.q0);
                    MeasDec d{};
                    d.u = g.param;
                    d.reset = g.kind == QW_GATE_RESET ? 1u : 0u;
                    d.pos = (uint32_t)(it - alive.begin());
                    d.dyn = dyn_next++;
                    d.outc = outc_next[who[i]]++;
                    alive.erase(it);
                    dec.push_back(d);
                    // the next segment opens with the operator the decision writes
                    qw_gate pg{};
                    pg.kind = kGateDyn;
                    pg.q0 = g.q0;
                    pg.param = dyn_param(dyn + 4ull * d.dyn);
                    t.head.push_back(pg);
                }
                t.cluster.clear();
            }
            const size_t o_ptr = 0, o_q = al(M * sizeof(void *)), o_tf = o_q + al(M * sizeof(uint64_t));
            const size_t o_tc = o_tf + al(M * sizeof(uint32_t)), o_dec = o_tc + al(M * sizeof(uint32_t));
            std::vector<uint8_t> blob(o_dec + dec.size() * sizeof(MeasDec));
            std::memcpy(blob.data() + o_ptr, ptrs.data(), M * sizeof(void *));
            if (C == 0) {
                std::vector<uint32_t> q32(M);
                for (uint32_t i = 0; i < M; ++i) q32[i] = (uint32_t)qs[i];
                std::memcpy(blob.data() + o_q, q32.data(), M * sizeof(uint32_t));
            } else {
                std::memcpy(blob.data() + o_q, qs.data(), M * sizeof(uint64_t));
            }
            std::memcpy(blob.data() + o_tf, tfirst.data(), M * sizeof(uint32_t));
            std::memcpy(blob.data() + o_tc, tcount.data(), M * sizeof(uint32_t));
            std::memcpy(blob.data() + o_dec, dec.data(), dec.size() * sizeof(MeasDec));
            rc = upload(ctx, blob);
            if (rc) return rc;
            const char *ub = static_cast<const char *>(ctx->plan.p);
            {
                ProfScope ps(ctx, 1, (double)M * (double)(8ull << n));
                hipError_t er = C == 0
                    ? launch_measure_sums(ctx->stream, reinterpret_cast<const float2 *const *>(ub + o_ptr),
                                          reinterpret_cast<const uint32_t *>(ub + o_q), M, n, part, dout)
                    : launch_joint_masses(ctx->stream, reinterpret_cast<const float2 *const *>(ub + o_ptr),
                                          reinterpret_cast<const uint64_t *>(ub + o_q), M, n, C, part,
                                          kStride, dout);
                if (er != hipSuccess) return hip_fail(ctx, er, "measure launch");
                er = launch_meas_decide(ctx->stream, reinterpret_cast<const uint32_t *>(ub + o_tf),
                                        reinterpret_cast<const uint32_t *>(ub + o_tc),
                                        reinterpret_cast<const MeasDec *>(ub + o_dec), M, C != 0, dout, kStride,
                                        dyn, outc, err);
                if (er != hipSuccess) return hip_fail(ctx, er, "measure decision launch");
            }
        }
    }
    if (ctx->rec) {
        // a replay writes the outcomes where qw_graph_outcomes reads them
        ctx->rec->outcomes.push_back({outc, total_meas, err});
        ctx->outcomes.clear();
        return QW_OK;
    }
    std::vector<uint8_t> host(total_meas + sizeof(uint32_t));
    uint32_t herr = 0;
    if (total_meas)
        HIP_TRY(ctx, hipMemcpyAsync(host.data(), outc, total_meas, hipMemcpyDeviceToHost, ctx->stream),
                "outcome copy");
    HIP_TRY(ctx, hipMemcpyAsync(&herr, err, sizeof herr, hipMemcpyDeviceToHost, ctx->stream), "outcome copy");
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream), "sync");
    ctx->outcomes.assign(host.begin(), host.begin() + (std::ptrdiff_t)total_meas);
    if (herr) return fail(ctx, QW_E_INVALID_ARG, "measurement of a zero state");
    (void)outc_base;
    return QW_OK;
}

}  // namespace

// ================================================================= ABI
extern "C" {

const char *qw_version(void) { return kVersion; }

int qw_ctx_create(int device, void *hip_stream, qw_ctx **out) {
    if (!out) return QW_E_INVALID_ARG;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
        return QW_E_INVALID_ARG;
    if (hipSetDevice(device) != hipSuccess) return QW_E_HIP;
    qw_ctx *c = new (std::nothrow) qw_ctx();
    if (!c) return QW_E_OOM;
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    {
        int ncu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess &&
            ncu > 0)
            c->n_cu = (uint32_t)ncu;
    }
    if (hipEventCreateWithFlags(&c->staging_ev, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(c->staging_ev, c->stream) != hipSuccess || kernels_init() != hipSuccess) {
        delete c;
        return QW_E_HIP;
    }
    if (hipHostMalloc(reinterpret_cast<void **>(&c->host_flag), 2 * sizeof(uint32_t), hipHostMallocDefault) !=
        hipSuccess) {
        hipEventDestroy(c->staging_ev);
        delete c;
        return QW_E_OOM;
    }
    __atomic_store_n(&c->host_flag[0], 0u, __ATOMIC_RELAXED);
    __atomic_store_n(&c->host_flag[1], 0u, __ATOMIC_RELAXED);
    *out = c;
    return QW_OK;
}

int qw_ctx_destroy(qw_ctx *ctx) {
    if (!ctx) return QW_E_INVALID_ARG;
    if (ctx->rec) {
        qw_graph *g = nullptr;
        (void)qw_graph_end(ctx, &g);
        if (g) (void)qw_graph_free(g);
    }
    hipStreamSynchronize(ctx->stream);
    for (ProfRec &r : ctx->prof) {
        hipEventDestroy(r.e0);
        hipEventDestroy(r.e1);
    }
    for (hipEvent_t e : ctx->ev_pool) hipEventDestroy(e);
    if (ctx->plan.p) (void)hipFree(ctx->plan.p);
    if (ctx->scratch.p) hipFree(ctx->scratch.p);
    if (ctx->pingpong.p) hipFree(ctx->pingpong.p);
    if (ctx->meas.p) hipFree(ctx->meas.p);
    if (ctx->psync.p) hipFree(ctx->psync.p);
    if (ctx->host_flag) hipHostFree(ctx->host_flag);
    if (ctx->staging) hipHostFree(ctx->staging);
    if (ctx->staging_ev) hipEventDestroy(ctx->staging_ev);
    delete ctx;
    return QW_OK;
}

const char *qw_last_error(const qw_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int qw_ctx_sync(qw_ctx *ctx) {
    if (!ctx) return QW_E_INVALID_ARG;
    if (ctx->rec) return recording_unsupported(ctx, "qw_ctx_sync");
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream), "stream sync");
    if (__atomic_load_n(&ctx->host_flag[1], __ATOMIC_ACQUIRE) != 0u) {
        __atomic_store_n(&ctx->host_flag[0], 0u, __ATOMIC_RELAXED);
        __atomic_store_n(&ctx->host_flag[1], 0u, __ATOMIC_RELEASE);
        return fail(ctx, QW_E_ABANDONED,
                    "a persistent launch abandoned a wait (spin limit reached or qw_ctx_abandon); "
                    "the states it was computing are undefined");
    }
    __atomic_store_n(&ctx->host_flag[0], 0u, __ATOMIC_RELAXED);
    return QW_OK;
}

int qw_ctx_abandon(qw_ctx *ctx) {
    if (!ctx) return QW_E_INVALID_ARG;
    __atomic_store_n(&ctx->host_flag[0], 1u, __ATOMIC_RELEASE);
    return QW_OK;
}

int qw_ctx_set_option(qw_ctx *ctx, int key, int64_t value) {
    if (!ctx) return QW_E_INVALID_ARG;
    switch (key) {
    case QW_OPT_TILE_BITS:
        if (value < kMinTileBits || value > kMaxTileBits)
            return fail(ctx, QW_E_INVALID_ARG, "tile bits must be 10..14");
        ctx->tile_bits = (int)value;
        return QW_OK;
    case QW_OPT_PROFILE: ctx->profile = value != 0; return QW_OK;
    case QW_OPT_XCD_REMAP: ctx->xcd_remap = value != 0; return QW_OK;
    case QW_OPT_JIT:
        if (value < 0 || value > 2) return fail(ctx, QW_E_INVALID_ARG, "jit mode must be 0, 1 or 2");
        ctx->jit = (int)value;
        return QW_OK;
    case QW_OPT_RELABEL: ctx->relabel = value != 0; return QW_OK;
    case QW_OPT_LAYOUT:
        if (value < 0 || value > 2) return fail(ctx, QW_E_INVALID_ARG, "layout mode must be 0, 1 or 2");
        ctx->layout = (int)value;
        return QW_OK;
    case QW_OPT_FUSED_EPILOGUE: ctx->fused_epilogue = value != 0; return QW_OK;
    case QW_OPT_PERSISTENT: ctx->persistent = value != 0; return QW_OK;
    case QW_OPT_PERSIST_CHUNK:
        if (value < 1 || value > 1024 || (value & (value - 1)))
            return fail(ctx, QW_E_INVALID_ARG, "claim size must be a power of two in 1..1024");
        ctx->persist_chunk = (uint32_t)value;
        return QW_OK;
    case QW_OPT_SPIN_LIMIT:
        if (value < 0 || value > 0xFFFFFFFFll) return fail(ctx, QW_E_INVALID_ARG, "spin limit must be 0..2^32-1");
        ctx->spin_limit = (uint32_t)value;
        return QW_OK;
    case QW_OPT_STREAM_LOADS: ctx->stream_loads = value != 0; return QW_OK;
    case QW_OPT_TILE_ORDER:
        if (value < 0 || value > 2) return fail(ctx, QW_E_INVALID_ARG, "tile order must be 0, 1 or 2");
        ctx->tile_order = (int)value;
        return QW_OK;
    case QW_OPT_SECOND_BUFFER_CAP:
        if (value <= 0) return fail(ctx, QW_E_INVALID_ARG, "second buffer cap must be > 0");
        ctx->pingpong_cap = (uint64_t)value;
        return QW_OK;
    case QW_OPT_DEVICE_MEM_CAP:
        if (value < 0) return fail(ctx, QW_E_INVALID_ARG, "device memory cap must be >= 0");
        if (ctx->rec) return recording_unsupported(ctx, "a new device memory cap");
        // the context's buffers are released, to grow again within the cap
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream), "stream sync");
        for (DevBuf *b : {&ctx->plan, &ctx->scratch, &ctx->pingpong, &ctx->meas, &ctx->psync}) {
            if (b->p) HIP_TRY(ctx, hipFree(b->p), "free buffer");
            b->p = nullptr;
            b->cap = 0;
        }
        ctx->mem_cap = (uint64_t)value;
        return QW_OK;
    default: return fail(ctx, QW_E_INVALID_ARG, "unknown option");
    }
}

int qw_ctx_kernel_stats(qw_ctx *ctx, int kernel, uint64_t *launches, double *total_ms,
                        double *total_bytes, int reset) {
    if (!ctx || kernel < 0 || kernel > 3) return QW_E_INVALID_ARG;
    if (ctx->rec) return recording_unsupported(ctx, "qw_ctx_kernel_stats");
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream), "stream sync");
    for (ProfRec &r : ctx->prof) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, r.e0, r.e1) == hipSuccess) {
            KStats &s = ctx->stats[r.kind];
            s.launches += r.launches;
            s.ms += ms;
            s.bytes += r.bytes;
        }
        ctx->ev_pool.push_back(r.e0);
        ctx->ev_pool.push_back(r.e1);
    }
    ctx->prof.clear();
    KStats &s = ctx->stats[kernel];
    if (launches) *launches = s.launches;
    if (total_ms) *total_ms = s.ms;
    if (total_bytes) *total_bytes = s.bytes;
    if (reset) s = KStats{};
    return QW_OK;
}

int qw_state_alloc(qw_ctx *ctx, uint32_t n, uint32_t n_slots, void *dev_buf,
                   uint64_t dev_buf_bytes, qw_state **out) {
    if (!ctx || !out) return QW_E_INVALID_ARG;
    *out = nullptr;
    if (n < 1 || n > (uint32_t)kMaxQubits) return fail(ctx, QW_E_INVALID_ARG, "n_qubits must be 1..30");
    if (n_slots < 1) return fail(ctx, QW_E_INVALID_ARG, "n_slots must be >= 1");
    const uint64_t slot_bytes = 8ull << n;
    const uint64_t need = slot_bytes * n_slots;
    if (dev_buf) {
        if (dev_buf_bytes < need) return fail(ctx, QW_E_INVALID_ARG, "dev_buf too small");
        if (reinterpret_cast<uintptr_t>(dev_buf) & 255u)
            return fail(ctx, QW_E_INVALID_ARG, "dev_buf must be 256-byte aligned");
    }
    std::unique_ptr<qw_state> st(new (std::nothrow) qw_state());
    if (!st) return fail(ctx, QW_E_OOM, "host allocation");
    st->ctx = ctx;
    st->n = n;
    st->n_slots = n_slots;
    st->slot_bytes = slot_bytes;
    st->frozen.assign(n_slots, 0);
    {
        // a caller buffer counts toward the cap like the library's own
        int rc = cap_check(ctx, need, 0, dev_buf ? "state" : "state allocation");
        if (rc) return rc;
    }
    if (dev_buf) {
        st->base = static_cast<char *>(dev_buf);
        ctx->held += need;
    } else {
        void *p = nullptr;
        hipError_t e = hipMalloc(&p, need);
        if (e != hipSuccess) return hip_fail(ctx, e, "state allocation");
        st->base = static_cast<char *>(p);
        st->owned = true;
        ctx->held += need;
    }
    hipError_t e = launch_init(ctx->stream, st->base, n, n_slots);
    if (e != hipSuccess) {
        if (st->owned) hipFree(st->base);
        ctx->held -= need;
        return hip_fail(ctx, e, "init launch");
    }
    *out = st.release();
    return QW_OK;
}

int qw_state_free(qw_state *st) {
    if (!st) return QW_E_INVALID_ARG;
    if (st->ctx->rec) return recording_unsupported(st->ctx, "qw_state_free");
    for (uint32_t f : st->frozen)
        if (f) return fail(st->ctx, QW_E_INVALID_ARG, "state has frozen slots (free the snapshots first)");
    if (st->owned) {
        hipStreamSynchronize(st->ctx->stream);
        hipFree(st->base);
    }
    st->ctx->held -= st->slot_bytes * st->n_slots;
    delete st;
    return QW_OK;
}

int qw_state_reset(qw_state *st, uint32_t first, uint32_t count) {
    if (!st) return QW_E_INVALID_ARG;
    if (!slot_ok(st, first, count)) return fail(st->ctx, QW_E_INVALID_ARG, "slot range out of bounds");
    for (uint32_t s = first; s < first + count; ++s)
        if (st->frozen[s]) return fail(st->ctx, QW_E_INVALID_ARG, "slot is frozen by a snapshot");
    if (count == 0) return QW_OK;
    hipError_t e = launch_init(st->ctx->stream, slot_ptr(st, first), st->n, count);
    if (e != hipSuccess) return hip_fail(st->ctx, e, "init launch");
    return QW_OK;
}

int qw_state_slot_ptr(const qw_state *st, uint32_t slot, void **dev_ptr) {
    if (!st || !dev_ptr || slot >= st->n_slots) return QW_E_INVALID_ARG;
    *dev_ptr = slot_ptr(st, slot);
    return QW_OK;
}

int qw_apply_prefix(qw_state *st, uint32_t slot, const qw_gate *gates, uint64_t n_gates) {
    if (!st) return QW_E_INVALID_ARG;
    qw_ctx *ctx = st->ctx;
    if (slot >= st->n_slots) return fail(ctx, QW_E_INVALID_ARG, "slot out of range");
    if (st->frozen[slot]) return fail(ctx, QW_E_INVALID_ARG, "slot is frozen by a snapshot");
    if (n_gates && !gates) return fail(ctx, QW_E_INVALID_ARG, "gates == NULL");
    ctx->outcomes.clear();
    if (has_measure(gates, n_gates)) {
        std::vector<MeasTask> mt(1);
        mt[0].rest.assign(gates, gates + n_gates);
        mt[0].dst = slot_ptr(st, slot);
        if (ctx->rec) ctx->rec->calls.emplace_back();
        const int rc = run_measured(ctx, st->n, mt);
        if (ctx->rec) ctx->rec->calls.back().clear();  // a measured call's gates cannot be updated
        return rc;
    }
    std::vector<Exec> ex(1);
    std::string e = get_plan(ctx, st->n, gates, n_gates, &ex[0].planp, true, layouts_pay(ctx, st->n, 1));
    if (!e.empty()) return fail(ctx, QW_E_INVALID_ARG, e);
    ex[0].dst = slot_ptr(st, slot);
    if (ctx->rec) ctx->rec->calls.emplace_back();
    return execute(ctx, st->n, ex);
}

int qw_snapshot(qw_state *st, uint32_t slot, const uint8_t provenance[32], int mode,
                const qw_snap *parent, void *copy_buf, uint64_t copy_buf_bytes,
                qw_snap **out) {
    if (!st || !out || !provenance) return st ? fail(st->ctx, QW_E_INVALID_ARG, "null argument") : QW_E_INVALID_ARG;
    qw_ctx *ctx = st->ctx;
    *out = nullptr;
    if (slot >= st->n_slots) return fail(ctx, QW_E_INVALID_ARG, "slot out of range");
    if (mode != QW_SNAP_COPY && mode != QW_SNAP_FREEZE) return fail(ctx, QW_E_INVALID_ARG, "bad mode");
    if (parent && parent->art.n_qubits != st->n)
        return fail(ctx, QW_E_INVALID_ARG, "parent snapshot has another qubit count");
    std::unique_ptr<qw_snap> s(new (std::nothrow) qw_snap());
    if (!s) return fail(ctx, QW_E_OOM, "host allocation");
    s->ctx = ctx;
    s->art.kind = QW_KIND_STATEVECTOR;
    s->art.exactness = QW_EXACT;
    s->art.backend = QW_BACKEND_SV;
    s->art.n_qubits = st->n;
    s->art.bytes = st->slot_bytes;
    std::memcpy(s->art.provenance, provenance, 32);
    s->parent = parent;
    s->mode = mode;
    if (mode == QW_SNAP_FREEZE) {
        s->data = slot_ptr(st, slot);
        s->fstate = st;
        s->fslot = slot;
        st->frozen[slot] += 1;
    } else {
        void *dst = copy_buf;
        if (dst) {
            if (copy_buf_bytes < st->slot_bytes) return fail(ctx, QW_E_INVALID_ARG, "copy_buf too small");
            if (reinterpret_cast<uintptr_t>(dst) & 255u)
                return fail(ctx, QW_E_INVALID_ARG, "copy_buf must be 256-byte aligned");
        }
        {
            // a caller copy buffer counts toward the cap like the library's own
            int rc = cap_check(ctx, st->slot_bytes, 0, dst ? "snapshot copy" : "snapshot allocation");
            if (rc) return rc;
        }
        if (!dst) {
            hipError_t e = hipMalloc(&dst, st->slot_bytes);
            if (e != hipSuccess) return hip_fail(ctx, e, "snapshot allocation");
            s->owned = dst;
        }
        ctx->held += st->slot_bytes;
        s->counted = st->slot_bytes;
        ProfScope ps(ctx, 3, 2.0 * (double)st->slot_bytes);
        hipError_t e = launch_copy(ctx->stream, dst, slot_ptr(st, slot), st->slot_bytes);
        if (e != hipSuccess) {
            if (s->owned) hipFree(s->owned);
            ctx->held -= st->slot_bytes;
            return hip_fail(ctx, e, "snapshot copy");
        }
        s->data = dst;
    }
    *out = s.release();
    return QW_OK;
}

int qw_snapshot_free(qw_snap *s) {
    if (!s) return QW_E_INVALID_ARG;
    if (s->ctx->rec) return recording_unsupported(s->ctx, "qw_snapshot_free");
    if (s->fstate && s->fstate->frozen[s->fslot] > 0) s->fstate->frozen[s->fslot] -= 1;
    if (s->owned) {
        hipStreamSynchronize(s->ctx->stream);
        hipFree(s->owned);
    }
    s->ctx->held -= s->counted;
    delete s;
    return QW_OK;
}

int qw_snapshot_info(const qw_snap *s, qw_artifact *out) {
    if (!s || !out) return QW_E_INVALID_ARG;
    *out = s->art;
    return QW_OK;
}

int qw_run_suffix_batch(qw_ctx *ctx, const qw_snap *const *src, const qw_task *tasks,
                        uint32_t n_tasks, qw_state *dst, const qw_reduce *epi) {
    if (!ctx || !dst) return ctx ? fail(ctx, QW_E_INVALID_ARG, "null state") : QW_E_INVALID_ARG;
    if (dst->ctx != ctx) return fail(ctx, QW_E_INVALID_ARG, "state belongs to another context");
    if (n_tasks > 0 && !tasks) return fail(ctx, QW_E_INVALID_ARG, "tasks == NULL");
    std::vector<char> seen(dst->n_slots, 0);
    for (uint32_t k = 0; k < n_tasks; ++k) {
        const uint32_t s = tasks[k].dst_slot;
        char buf[128];
        if (s >= dst->n_slots) {
            snprintf(buf, sizeof buf, "task %u: dst_slot %u out of range", k, s);
            return fail(ctx, QW_E_INVALID_ARG, buf);
        }
        if (seen[s]) {
            snprintf(buf, sizeof buf, "task %u: dst_slot %u used twice", k, s);
            return fail(ctx, QW_E_INVALID_ARG, buf);
        }
        if (dst->frozen[s]) {
            snprintf(buf, sizeof buf, "task %u: dst_slot %u is frozen by a snapshot", k, s);
            return fail(ctx, QW_E_INVALID_ARG, buf);
        }
        if (tasks[k].reserved != 0) return fail(ctx, QW_E_INVALID_ARG, "task reserved field must be 0");
        seen[s] = 1;
    }
    // legality gates before any device work (Sec. IV-B)
    for (uint32_t k = 0; k < n_tasks; ++k) {
        const qw_snap *sn = src ? src[k] : nullptr;
        if (!sn) continue;
        std::string js;
        if (!legal(sn->art, QW_KIND_STATEVECTOR, QW_BACKEND_SV, &js, k))
            return fail(ctx, QW_E_REFUSED, js);
        if (sn->art.n_qubits != dst->n)
            return fail(ctx, QW_E_REFUSED,
                        refusal_json("QUBIT_COUNT_MISMATCH", "artifact qubit count differs from the target state.",
                                     sn->art.kind, QW_KIND_STATEVECTOR, sn->art.backend, QW_BACKEND_SV, k));
        if (std::memcmp(sn->art.provenance, tasks[k].expect_prov, 32) != 0)
            return fail(ctx, QW_E_REFUSED,
                        refusal_json("PROVENANCE_MISMATCH", "artifact provenance hash differs from the task's prefix fingerprint.",
                                     sn->art.kind, QW_KIND_STATEVECTOR, sn->art.backend, QW_BACKEND_SV, k));
        if (sn->ctx != ctx) return fail(ctx, QW_E_INVALID_ARG, "snapshot belongs to another context");
    }
    if (epi) {
        if (epi->n_terms > 0 && (!epi->x_mask || !epi->z_mask || !epi->coeff))
            return fail(ctx, QW_E_INVALID_ARG, "epilogue arrays are NULL");
        if (!epi->out) return fail(ctx, QW_E_INVALID_ARG, "epilogue out is NULL");
        const uint64_t full = (1ull << dst->n) - 1;
        for (uint32_t j = 0; j < epi->n_terms; ++j)
            if ((epi->x_mask[j] & ~full) || (epi->z_mask[j] & ~full))
                return fail(ctx, QW_E_INVALID_ARG, "Pauli mask has bits >= n");
    }
    ctx->outcomes.clear();
    bool measured = false;
    for (uint32_t k = 0; k < n_tasks && !measured; ++k) {
        if (tasks[k].n_gates && !tasks[k].gates) return fail(ctx, QW_E_INVALID_ARG, "task gates == NULL");
        measured = has_measure(tasks[k].gates, tasks[k].n_gates);
    }
    if (ctx->rec && epi && epi->out_is_host) return recording_unsupported(ctx, "a host output");
    if (measured) {
        // segments between measurements; the expectations after the last one
        std::vector<MeasTask> mt(n_tasks);
        for (uint32_t k = 0; k < n_tasks; ++k) {
            if (tasks[k].n_gates) mt[k].rest.assign(tasks[k].gates, tasks[k].gates + tasks[k].n_gates);
            mt[k].src = (src && src[k]) ? src[k]->data : nullptr;
            mt[k].dst = slot_ptr(dst, tasks[k].dst_slot);
        }
        if (ctx->rec) ctx->rec->calls.emplace_back();
        int rc = run_measured(ctx, dst->n, mt);
        if (ctx->rec) ctx->rec->calls.back().clear();  // a measured call's gates cannot be updated
        if (rc || !epi) return rc;
        std::vector<const void *> slots(n_tasks);
        for (uint32_t k = 0; k < n_tasks; ++k) slots[k] = slot_ptr(dst, tasks[k].dst_slot);
        return expect_slots(ctx, dst->n, slots, epi->x_mask, epi->z_mask, epi->coeff, epi->n_terms,
                            epi->out, epi->out_is_host, nullptr);
    }
    std::vector<Exec> ex(n_tasks);
    for (uint32_t k = 0; k < n_tasks; ++k) {
        ex[k].src = (src && src[k]) ? src[k]->data : nullptr;
        std::string e = get_plan(ctx, dst->n, tasks[k].gates, tasks[k].n_gates, &ex[k].planp, ex[k].src == nullptr,
                                 layouts_pay(ctx, dst->n, n_tasks));
        if (!e.empty()) return fail(ctx, QW_E_INVALID_ARG, "task " + std::to_string(k) + ": " + e);
        ex[k].dst = slot_ptr(dst, tasks[k].dst_slot);
    }
    // Fused expectation epilogue: terms that the last pass can evaluate on
    // its own tile (after conjugation through its output relabelling) are
    // reduced inside that pass, which saves a reducer sweep when the others
    // then need fewer term groups.
    FusedEpi fe;
    if (epi && epi->n_terms > 0)
        plan_fused(ctx, dst->n, ex, epi->x_mask, epi->z_mask, epi->n_terms, &fe);
    if (fe.active) {
        const int m = ex[0].planp->m;
        const uint32_t tiles = 1u << (dst->n - m);
        const uint32_t rows = tiles / red_row_tiles(tiles);
        const size_t part_bytes = (size_t)n_tasks * rows * epi->n_terms * sizeof(double);
        int rc0 = ensure(ctx, ctx->scratch, part_bytes + n_tasks * sizeof(double) + 256, "reduce scratch");
        if (rc0) return rc0;
        double *part = static_cast<double *>(ctx->scratch.p);
        for (uint32_t k = 0; k < n_tasks; ++k) {
            ex[k].epi = &fe.rplan;
            ex[k].epi_key = &fe.key;
            ex[k].epi_part = part + (size_t)k * rows * epi->n_terms;
            ex[k].epi_nt = epi->n_terms;
        }
    }
    if (ctx->rec) ctx->rec->calls.emplace_back();
    int rc = execute(ctx, dst->n, ex, true);
    if (rc) return rc;
    if (epi) {
        std::vector<const void *> slots(n_tasks);
        for (uint32_t k = 0; k < n_tasks; ++k) slots[k] = slot_ptr(dst, tasks[k].dst_slot);
        return expect_slots(ctx, dst->n, slots, epi->x_mask, epi->z_mask, epi->coeff,
                            epi->n_terms, epi->out, epi->out_is_host, fe.active ? &fe.fused : nullptr);
    }
    return QW_OK;
}

int qw_run_tree(qw_ctx *ctx, const qw_snap *const *src, const qw_task *tasks, const int32_t *parent,
                const uint8_t *out_prov, uint32_t n_tasks, qw_state *dst) {
    if (!ctx || !dst) return ctx ? fail(ctx, QW_E_INVALID_ARG, "null state") : QW_E_INVALID_ARG;
    if (dst->ctx != ctx) return fail(ctx, QW_E_INVALID_ARG, "state belongs to another context");
    if (n_tasks > 0 && (!tasks || !parent)) return fail(ctx, QW_E_INVALID_ARG, "tasks or parent == NULL");
    std::vector<char> seen(dst->n_slots, 0);
    bool any_parent = false;
    for (uint32_t k = 0; k < n_tasks; ++k) {
        const uint32_t s = tasks[k].dst_slot;
        char buf[128];
        if (s >= dst->n_slots || seen[s] || dst->frozen[s]) {
            snprintf(buf, sizeof buf, "task %u: dst_slot %u out of range, used twice or frozen", k, s);
            return fail(ctx, QW_E_INVALID_ARG, buf);
        }
        if (tasks[k].reserved != 0) return fail(ctx, QW_E_INVALID_ARG, "task reserved field must be 0");
        if (tasks[k].n_gates && !tasks[k].gates) return fail(ctx, QW_E_INVALID_ARG, "task gates == NULL");
        if (has_measure(tasks[k].gates, tasks[k].n_gates))
            return fail(ctx, QW_E_UNSUPPORTED, "qw_run_tree: gates may not measure or reset");
        seen[s] = 1;
        if (parent[k] >= 0) {
            if ((uint32_t)parent[k] >= k) {
                snprintf(buf, sizeof buf, "task %u: parent %d does not come before it", k, parent[k]);
                return fail(ctx, QW_E_INVALID_ARG, buf);
            }
            if (src && src[k]) return fail(ctx, QW_E_INVALID_ARG, "a task has both a parent and a snapshot");
            if (tasks[k].n_gates == 0) return fail(ctx, QW_E_INVALID_ARG, "a task with a parent must have gates");
            any_parent = true;
        } else if (parent[k] != -1) {
            return fail(ctx, QW_E_INVALID_ARG, "parent must be -1 or an earlier task");
        }
    }
    if (any_parent && !out_prov) return fail(ctx, QW_E_INVALID_ARG, "out_prov is required with parents");
    // legality gates before any device work (Sec. IV-B): snapshot sources as
    // in qw_run_suffix_batch; an in-call parent's state is an exact
    // statevector of this context, so only its provenance is checked
    for (uint32_t k = 0; k < n_tasks; ++k) {
        if (parent[k] >= 0) {
            if (std::memcmp(out_prov + 32ull * (uint32_t)parent[k], tasks[k].expect_prov, 32) != 0)
                return fail(ctx, QW_E_REFUSED,
                            refusal_json("PROVENANCE_MISMATCH", "parent state provenance differs from the task's prefix fingerprint.",
                                         QW_KIND_STATEVECTOR, QW_KIND_STATEVECTOR, QW_BACKEND_SV, QW_BACKEND_SV, k));
            continue;
        }
        const qw_snap *sn = src ? src[k] : nullptr;
        if (!sn) continue;
        std::string js;
        if (!legal(sn->art, QW_KIND_STATEVECTOR, QW_BACKEND_SV, &js, k)) return fail(ctx, QW_E_REFUSED, js);
        if (sn->art.n_qubits != dst->n)
            return fail(ctx, QW_E_REFUSED,
                        refusal_json("QUBIT_COUNT_MISMATCH", "artifact qubit count differs from the target state.",
                                     sn->art.kind, QW_KIND_STATEVECTOR, sn->art.backend, QW_BACKEND_SV, k));
        if (std::memcmp(sn->art.provenance, tasks[k].expect_prov, 32) != 0)
            return fail(ctx, QW_E_REFUSED,
                        refusal_json("PROVENANCE_MISMATCH", "artifact provenance hash differs from the task's prefix fingerprint.",
                                     sn->art.kind, QW_KIND_STATEVECTOR, sn->art.backend, QW_BACKEND_SV, k));
        if (sn->ctx != ctx) return fail(ctx, QW_E_INVALID_ARG, "snapshot belongs to another context");
    }
    ctx->outcomes.clear();
    std::vector<Exec> ex(n_tasks);
    for (uint32_t k = 0; k < n_tasks; ++k) {
        ex[k].parent = parent[k];
        ex[k].dst = slot_ptr(dst, tasks[k].dst_slot);
        ex[k].src = parent[k] >= 0 ? slot_ptr(dst, tasks[(uint32_t)parent[k]].dst_slot)
                                   : ((src && src[k]) ? src[k]->data : nullptr);
        std::string e = get_plan(ctx, dst->n, tasks[k].gates, tasks[k].n_gates, &ex[k].planp, ex[k].src == nullptr,
                                 layouts_pay(ctx, dst->n, n_tasks));
        if (!e.empty()) return fail(ctx, QW_E_INVALID_ARG, "task " + std::to_string(k) + ": " + e);
    }
    // one persistent launch when it applies to the whole tree (every task in
    // one execution: no norm passes, generated kernels, second buffers within
    // the cap, every parent with passes)
    bool one = ctx->persistent && ctx->jit && n_tasks > 0 && ex[0].planp->m >= kMinTileBits;
    {
        const uint64_t state_bytes = 8ull << dst->n;
        uint64_t relabels = 0;
        for (const Exec &e : ex) {
            relabels += has_relabel(*e.planp);
            for (const HostPass &p : e.planp->passes) one = one && !p.norm_out;
            if (e.parent >= 0) one = one && !ex[(size_t)e.parent].planp->passes.empty();
        }
        one = one && relabels <= std::max<uint64_t>(1, ctx->pingpong_cap / state_bytes);
    }
    if (ctx->rec) ctx->rec->calls.emplace_back();
    if (one || !any_parent) {
        if (one) return execute_chunk(ctx, dst->n, ex, true);
        return execute(ctx, dst->n, ex, true);
    }
    // level by level: a task runs in the execution after its parent's
    std::vector<uint32_t> depth(n_tasks, 0);
    uint32_t levels = 0;
    for (uint32_t k = 0; k < n_tasks; ++k) {
        if (parent[k] >= 0) depth[k] = depth[(uint32_t)parent[k]] + 1;
        levels = std::max(levels, depth[k] + 1);
    }
    std::vector<GraphSeg> by_task(n_tasks);  // recorded op positions, in task order
    for (uint32_t d = 0; d < levels; ++d) {
        std::vector<Exec> lev;
        std::vector<uint32_t> lev_k;
        for (uint32_t k = 0; k < n_tasks; ++k)
            if (depth[k] == d) {
                lev.push_back(ex[k]);
                lev.back().parent = -1;
                lev_k.push_back(k);
            }
        int rc = execute(ctx, dst->n, lev, true);
        if (rc) return rc;
        if (ctx->rec) {
            std::vector<GraphSeg> &got = ctx->rec->calls.back();
            for (size_t i = 0; i < got.size() && i < lev_k.size(); ++i) by_task[lev_k[i]] = std::move(got[i]);
            got.clear();
        }
    }
    if (ctx->rec) ctx->rec->calls.back() = std::move(by_task);
    return QW_OK;
}

int qw_expect_pauli(const qw_state *st, uint32_t first, uint32_t count, const uint64_t *x,
                    const uint64_t *z, const double *c, uint32_t n_terms, double *out,
                    int out_is_host) {
    if (!st) return QW_E_INVALID_ARG;
    qw_ctx *ctx = st->ctx;
    if (!slot_ok(st, first, count)) return fail(ctx, QW_E_INVALID_ARG, "slot range out of bounds");
    if (n_terms > 0 && (!x || !z || !c)) return fail(ctx, QW_E_INVALID_ARG, "term arrays are NULL");
    if (!out && count > 0) return fail(ctx, QW_E_INVALID_ARG, "out is NULL");
    std::vector<const void *> slots(count);
    for (uint32_t k = 0; k < count; ++k) slots[k] = slot_ptr(st, first + k);
    return expect_slots(ctx, st->n, slots, x, z, c, n_terms, out, out_is_host);
}

int qw_sample(const qw_state *st, uint32_t first, uint32_t count, uint64_t seed,
              uint64_t task_base, uint32_t shots, uint32_t *out, int out_is_host) {
    if (!st) return QW_E_INVALID_ARG;
    qw_ctx *ctx = st->ctx;
    if (!slot_ok(st, first, count)) return fail(ctx, QW_E_INVALID_ARG, "slot range out of bounds");
    if (count == 0 || shots == 0) return QW_OK;
    if (!out) return fail(ctx, QW_E_INVALID_ARG, "out is NULL");
    if (ctx->rec && out_is_host) return recording_unsupported(ctx, "a host output");
    const uint32_t n = st->n;
    const uint32_t C = sample_chunk_bits(n);
    const uint64_t chunks = 1ull << (n - C);
    std::vector<const void *> ptrs(count);
    for (uint32_t k = 0; k < count; ++k) ptrs[k] = slot_ptr(st, first + k);
    std::vector<uint8_t> blob(count * sizeof(void *));
    std::memcpy(blob.data(), ptrs.data(), blob.size());
    int rc = upload(ctx, blob);
    if (rc) return rc;
    const size_t cs = (size_t)count * chunks * sizeof(double);
    const size_t tot = (size_t)count * sizeof(double);
    const size_t ob = (size_t)count * shots * sizeof(uint32_t);
    const size_t ss = (size_t)count * ((size_t)1 << (n - sample_sub_bits(n))) * sizeof(double);
    const size_t a1 = (cs + 255) & ~size_t(255), a2 = (tot + 255) & ~size_t(255);
    const size_t a3 = (ss + 255) & ~size_t(255);
    rc = ensure(ctx, ctx->scratch, 2 * a1 + a2 + a3 + (out_is_host ? ob : 0) + 256, "sample scratch");
    if (rc) return rc;
    uint8_t *sb = static_cast<uint8_t *>(ctx->scratch.p);
    double *csum = reinterpret_cast<double *>(sb);
    double *cpre = reinterpret_cast<double *>(sb + a1);
    double *total = reinterpret_cast<double *>(sb + 2 * a1);
    double *ssum = reinterpret_cast<double *>(sb + 2 * a1 + a2);
    uint32_t *dout = out_is_host ? reinterpret_cast<uint32_t *>(sb + 2 * a1 + a2 + a3) : out;
    {
        ProfScope ps(ctx, 2, (double)count * (double)(8ull << n));
        hipError_t e = launch_sample(ctx->stream, reinterpret_cast<const float2 *const *>(ctx->plan.p),
                                     count, n, csum, cpre, ssum, total, seed, task_base, shots, dout);
        if (e != hipSuccess) return hip_fail(ctx, e, "sample launch");
    }
    if (out_is_host) {
        HIP_TRY(ctx, hipMemcpyAsync(out, dout, ob, hipMemcpyDeviceToHost, ctx->stream), "result copy");
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream), "sync");
    }
    return QW_OK;
}

int qw_sample_noalloc(const qw_state *st, uint32_t first, uint32_t count, uint64_t seed,
                      uint64_t task_base, uint32_t shots, uint32_t *out, int out_is_host) {
    if (!st) return QW_E_INVALID_ARG;
    qw_ctx *ctx = st->ctx;
    if (!slot_ok(st, first, count)) return fail(ctx, QW_E_INVALID_ARG, "slot range out of bounds");
    if (count == 0 || shots == 0) return QW_OK;
    if (!out) return fail(ctx, QW_E_INVALID_ARG, "out is NULL");
    if (ctx->rec) return recording_unsupported(ctx, "qw_sample_noalloc");
    const uint32_t n = st->n;
    const uint32_t C = sample_chunk_bits(n);
    const uint64_t chunks = 1ull << (n - C);
    auto al = [](uint64_t b) { return (b + 255) & ~uint64_t(255); };
    // scratch layout: slot pointers, chunk sums, chunk prefixes, totals,
    // sub-chunk sums, then the indices when they go to host memory
    const uint64_t ap = al((uint64_t)count * sizeof(void *));
    const uint64_t a1 = al((uint64_t)count * chunks * sizeof(double));
    const uint64_t a2 = al((uint64_t)count * sizeof(double));
    const uint64_t a3 = al((uint64_t)count * (1ull << (n - sample_sub_bits(n))) * sizeof(double));
    const uint64_t ob = (uint64_t)count * shots * sizeof(uint32_t);
    const uint64_t need = ap + 2 * a1 + a2 + a3 + (out_is_host ? al(ob) : 0);
    if (need > kNoAllocScratchBytes) {
        char b[200];
        std::snprintf(b, sizeof b,
                      "qw_sample_noalloc needs %llu bytes of scratch for %u slots of %u qubits "
                      "and %u shots; its fixed scratch holds %llu",
                      (unsigned long long)need, count, n, shots,
                      (unsigned long long)kNoAllocScratchBytes);
        return fail(ctx, QW_E_INVALID_ARG, b);
    }
    void *sp = nullptr;
    HIP_TRY(ctx, noalloc_scratch(ctx->device, &sp), "scratch symbol lookup");
    uint8_t *sb = static_cast<uint8_t *>(sp);
    const float2 **ptrs = reinterpret_cast<const float2 **>(sb);
    double *csum = reinterpret_cast<double *>(sb + ap);
    double *cpre = reinterpret_cast<double *>(sb + ap + a1);
    double *total = reinterpret_cast<double *>(sb + ap + 2 * a1);
    double *ssum = reinterpret_cast<double *>(sb + ap + 2 * a1 + a2);
    uint32_t *dout = out_is_host ? reinterpret_cast<uint32_t *>(sb + ap + 2 * a1 + a2 + a3) : out;
    hipError_t e = launch_slot_ptrs(ctx->stream, ptrs, slot_ptr(st, first), st->slot_bytes, count);
    if (e != hipSuccess) return hip_fail(ctx, e, "slot pointer launch");
    e = launch_sample(ctx->stream, ptrs, count, n, csum, cpre, ssum, total, seed, task_base, shots,
                      dout);
    if (e != hipSuccess) return hip_fail(ctx, e, "sample launch");
    if (out_is_host) {
        HIP_TRY(ctx, hipMemcpyAsync(out, dout, ob, hipMemcpyDeviceToHost, ctx->stream), "result copy");
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream), "sync");
    }
    return QW_OK;
}

struct qw_tableau {
    qw::Tableau t;
    explicit qw_tableau(int n) : t(n) {}
};

int qw_tableau_create(uint32_t n_qubits, qw_tableau **out) {
    if (!out || n_qubits < 1 || n_qubits > 30) return QW_E_INVALID_ARG;
    *out = new qw_tableau((int)n_qubits);
    return QW_OK;
}

int qw_tableau_free(qw_tableau *tb) {
    if (!tb) return QW_E_INVALID_ARG;
    delete tb;
    return QW_OK;
}

int qw_tableau_apply(qw_tableau *tb, const qw_gate *gates, uint64_t n_gates) {
    if (!tb || (n_gates && !gates)) return QW_E_INVALID_ARG;
    qw::Tableau t = tb->t;  // unchanged on error
    const std::string e = t.apply(gates, n_gates);
    if (!e.empty()) return e.find("Clifford") != std::string::npos ? QW_E_UNSUPPORTED : QW_E_INVALID_ARG;
    tb->t = std::move(t);
    return QW_OK;
}

int qw_tableau_rows(const qw_tableau *tb, uint64_t *x, uint64_t *z, uint8_t *r) {
    if (!tb || !x || !z || !r) return QW_E_INVALID_ARG;
    for (int i = 0; i < 2 * tb->t.n; ++i) {
        x[i] = tb->t.x[i];
        z[i] = tb->t.z[i];
        r[i] = tb->t.r[i];
    }
    return QW_OK;
}

int qw_tableau_artifact(const qw_tableau *tb, const uint8_t provenance[32], qw_artifact *out) {
    if (!tb || !provenance || !out) return QW_E_INVALID_ARG;
    qw_artifact a{};
    a.kind = QW_KIND_TABLEAU;
    a.exactness = QW_EXACT;
    a.backend = QW_BACKEND_STAB_ONLY;
    a.n_qubits = (uint32_t)tb->t.n;
    a.bytes = (uint64_t)tb->t.n * 2 * (2 * sizeof(uint64_t) + 1);
    std::memcpy(a.provenance, provenance, 32);
    *out = a;
    return QW_OK;
}

int qw_tableau_export(const qw_tableau *tb, qw_state *st, uint32_t slot) {
    if (!tb || !st) return QW_E_INVALID_ARG;
    qw_ctx *ctx = st->ctx;
    if (slot >= st->n_slots) return fail(ctx, QW_E_INVALID_ARG, "slot out of range");
    if (st->frozen[slot]) return fail(ctx, QW_E_INVALID_ARG, "slot is frozen by a snapshot");
    if ((uint32_t)tb->t.n != st->n) return fail(ctx, QW_E_INVALID_ARG, "tableau and state qubit counts differ");
    // the conversion rule of Table II (tableau -> statevector, exact export)
    qw_artifact a{};
    uint8_t prov[32] = {0};
    qw_tableau_artifact(tb, prov, &a);
    std::string js;
    if (!legal(a, QW_KIND_STATEVECTOR, QW_BACKEND_SV, &js)) return fail(ctx, QW_E_REFUSED, js);
    const qw::StabExport e = tb->t.export_form();
    const uint32_t r = (uint32_t)e.x.size();
    std::vector<uint8_t> blob(r * (2 * sizeof(uint64_t) + 2 * sizeof(uint32_t)) + 64);
    uint64_t *hx = reinterpret_cast<uint64_t *>(blob.data());
    uint64_t *hz = hx + r;
    uint32_t *hp = reinterpret_cast<uint32_t *>(hz + r);
    uint32_t *hv = hp + r;
    for (uint32_t i = 0; i < r; ++i) {
        hx[i] = e.x[i];
        hz[i] = e.z[i];
        hp[i] = e.phase[i];
        hv[i] = e.pivot[i];
    }
    int rc = upload(ctx, blob);
    if (rc) return rc;
    const char *d = static_cast<const char *>(ctx->plan.p);
    const uint64_t *dx = reinterpret_cast<const uint64_t *>(d);
    const uint64_t *dz = dx + r;
    const uint32_t *dp = reinterpret_cast<const uint32_t *>(dz + r);
    const uint32_t *dv = dp + r;
    const double nd = std::pow(2.0, -0.5 * (double)r);
    ProfScope ps(ctx, 3, (double)(8ull << st->n));
    hipError_t er = launch_stab_export(ctx->stream, reinterpret_cast<float2 *>(slot_ptr(st, slot)), st->n, e.x0, r,
                                       dx, dz, dp, dv, (float)nd);
    if (er != hipSuccess) return hip_fail(ctx, er, "export launch");
    return QW_OK;
}

int qw_legality_check(const qw_artifact *src, uint32_t target_kind, uint32_t target_backend,
                      char *json_out, uint64_t cap) {
    if (!src) return QW_E_INVALID_ARG;
    std::string js;
    if (legal(*src, target_kind, target_backend, &js)) {
        if (json_out && cap) json_out[0] = 0;
        return QW_OK;
    }
    if (json_out && cap) {
        size_t k = std::min<size_t>(js.size(), cap - 1);
        std::memcpy(json_out, js.data(), k);
        json_out[k] = 0;
    }
    return QW_E_REFUSED;
}

uint64_t qw_mlp_workspace_floats(uint32_t batch) { return mlp_workspace_floats(batch); }

int qw_mlp_forward(qw_ctx *ctx, const float *params, const float *x, uint32_t batch, float *work,
                   float *y) {
    if (!ctx || !params || (batch && (!x || !work || !y))) return QW_E_INVALID_ARG;
    hipError_t e = launch_mlp_forward(ctx->stream, params, x, nullptr, batch, work, y);
    return e == hipSuccess ? QW_OK : hip_fail(ctx, e, "mlp forward");
}

int qw_mlp_backward(qw_ctx *ctx, const float *params, const float *x, const float *target,
                    uint32_t batch, float *work, float *grad) {
    if (!ctx || !params || !grad || (batch && (!x || !target || !work))) return QW_E_INVALID_ARG;
    if (batch == 0) return fail(ctx, QW_E_INVALID_ARG, "batch must be >= 1");
    hipError_t e = launch_mlp_backward(ctx->stream, params, x, target, nullptr, batch, work, grad);
    return e == hipSuccess ? QW_OK : hip_fail(ctx, e, "mlp backward");
}

int qw_mlp_backward_rows(qw_ctx *ctx, const float *params, const float *x, const float *target,
                         uint32_t n_rows, const uint32_t *rows, uint32_t batch, float *work,
                         float *grad) {
    if (!ctx || !params || !grad || !x || !target || !work || !rows) return QW_E_INVALID_ARG;
    if (batch == 0) return fail(ctx, QW_E_INVALID_ARG, "batch must be >= 1");
    for (uint32_t b = 0; b < batch; ++b)
        if (rows[b] >= n_rows)
            return fail(ctx, QW_E_INVALID_ARG,
                        "row " + std::to_string(rows[b]) + " of batch entry " + std::to_string(b) +
                            " is not below n_rows = " + std::to_string(n_rows));
    std::vector<uint8_t> blob(batch * sizeof(uint32_t));
    std::memcpy(blob.data(), rows, blob.size());
    int rc = upload(ctx, blob);
    if (rc) return rc;
    hipError_t e = launch_mlp_backward(ctx->stream, params, x, target,
                                       static_cast<const uint32_t *>(ctx->plan.p), batch, work, grad);
    return e == hipSuccess ? QW_OK : hip_fail(ctx, e, "mlp backward (rows)");
}

int qw_mlp_loss(qw_ctx *ctx, const float *params, const float *x, const float *target,
                uint32_t batch, float *work, double *loss) {
    if (!ctx || !params || !x || !target || !work || !loss) return QW_E_INVALID_ARG;
    if (batch == 0) return fail(ctx, QW_E_INVALID_ARG, "batch must be >= 1");
    hipError_t e = launch_mlp_loss(ctx->stream, params, x, target, nullptr, batch, work, loss);
    return e == hipSuccess ? QW_OK : hip_fail(ctx, e, "mlp loss");
}

int qw_mlp_adam(qw_ctx *ctx, float *params, const float *grad, float *m, float *v, uint32_t step,
                float lr, float beta1, float beta2, float eps) {
    if (!ctx || !params || !grad || !m || !v || step == 0) return QW_E_INVALID_ARG;
    hipError_t e = launch_mlp_adam(ctx->stream, params, grad, m, v, step, lr, beta1, beta2, eps);
    return e == hipSuccess ? QW_OK : hip_fail(ctx, e, "mlp adam");
}

int qw_outcomes(const qw_ctx *ctx, uint8_t *out, uint64_t cap, uint64_t *count) {
    if (!ctx || (cap && !out)) return QW_E_INVALID_ARG;
    const uint64_t m = std::min<uint64_t>(cap, ctx->outcomes.size());
    if (m) std::memcpy(out, ctx->outcomes.data(), m);
    if (count) *count = ctx->outcomes.size();
    return QW_OK;
}

int qw_plan_cost(uint32_t n, const qw_gate *gates, uint64_t n_gates, uint32_t tile_bits,
                 uint64_t *n_passes, double *bytes) {
    if (n_gates && !gates) return QW_E_INVALID_ARG;
    // segments between measurements are planned alone; each measurement
    // reads the state once and leaves a projector for the next segment
    uint64_t passes = 0, reads = 0;
    std::vector<qw_gate> seg;
    for (uint64_t i = 0; i <= n_gates; ++i) {
        if (i < n_gates && !is_measure(gates[i].kind)) {
            seg.push_back(gates[i]);
            continue;
        }
        if (i < n_gates && (gates[i].q0 >= n || !(gates[i].param >= 0.0 && gates[i].param < 1.0)))
            return QW_E_INVALID_ARG;
        Plan p;
        if (!build_plan((int)n, seg.data(), seg.size(), (int)tile_bits, &p, true, false).empty())
            return QW_E_INVALID_ARG;
        passes += p.passes.size();
        if (i == n_gates) break;
        ++reads;
        seg.clear();
        qw_gate pg{};
        pg.kind = QW_GATE_PROJ0;
        pg.q0 = gates[i].q0;
        pg.param = 1.0;
        seg.push_back(pg);
    }
    const double sb = 8.0 * std::ldexp(1.0, (int)n);
    if (n_passes) *n_passes = passes;
    if (bytes) *bytes = (double)passes * 2.0 * sb + (double)reads * sb;
    return QW_OK;
}

int qw_jit_precompile(uint32_t n, const qw_gate *gates, uint64_t n_gates, uint32_t tile_bits,
                      char *log, uint64_t cap) {
    auto put = [&](const std::string &msg) {
        if (log && cap) {
            size_t k = std::min<size_t>(msg.size(), cap - 1);
            std::memcpy(log, msg.data(), k);
            log[k] = 0;
        }
    };
    // the plans from a separate source and in place, with and without
    // permuted layouts (calls choose by where the first pass loads from and
    // by the size of their states)
    Plan pv[4];
    std::string e;
    for (int v = 0; v < 4 && e.empty(); ++v)
        e = build_plan((int)n, gates, (size_t)n_gates, (int)tile_bits, &pv[v], true, true, false, v >= 2, v & 1);
    if (!e.empty()) {
        put(e);
        return QW_E_INVALID_ARG;
    }
    put("");
    if (pv[0].m < kMinTileBits) return QW_OK;
    std::vector<JitReq> reqs;
    std::set<std::string> seen;
    for (const Plan &p : pv)
        for (size_t k = 0; k < p.passes.size(); ++k) {
            const HostPass &h = p.passes[k];
            // both load policies (QW_OPT_STREAM_LOADS, snapshot-reading first passes)
            for (int stream = 1; stream >= 0; --stream) {
                JitReq r;
                r.use_lds = h.norm_out || h.dev_phases.size() > 1;
                r.key = jit_pass_key((int)n, p.m, h, r.use_lds) + (stream ? "S" : "T");
                if (!seen.insert(r.key).second) continue;
                r.pass = &h;
                r.n = (int)n;
                r.m = p.m;
                r.stream_loads = stream != 0;
                reqs.push_back(std::move(r));
            }
        }
    e = jit_precompile(reqs);
    if (!e.empty()) {
        put(e);
        return QW_E_HIP;
    }
    return QW_OK;
}

int qw_jit_precompile_terms(uint32_t n, const uint64_t *x, const uint64_t *z, uint32_t n_terms,
                            uint32_t tile_bits, char *log, uint64_t cap) {
    auto put = [&](const std::string &msg) {
        if (log && cap) {
            size_t k = std::min<size_t>(msg.size(), cap - 1);
            std::memcpy(log, msg.data(), k);
            log[k] = 0;
        }
    };
    put("");
    if (n < 1 || n > (uint32_t)kMaxQubits || tile_bits < (uint32_t)kMinTileBits ||
        tile_bits > (uint32_t)kMaxTileBits || (n_terms && (!x || !z))) {
        put("bad arguments");
        return QW_E_INVALID_ARG;
    }
    const uint64_t full = (1ull << n) - 1;
    for (uint32_t j = 0; j < n_terms; ++j)
        if ((x[j] & ~full) || (z[j] & ~full)) {
            put("Pauli mask has bits >= n");
            return QW_E_INVALID_ARG;
        }
    const int m = tile_bits_for((int)n, (int)tile_bits);
    if (m < kMinTileBits || n_terms == 0) return QW_OK;
    std::vector<TermGroup> groups = group_terms((int)n, m, x, n_terms);
    std::vector<RedPlan> rplans;
    for (const TermGroup &g : groups) rplans.push_back(plan_reduce_group((int)n, m, g, x, z));
    std::vector<JitReq> reqs(groups.size());
    for (size_t g = 0; g < groups.size(); ++g) {
        reqs[g].key = jit_reduce_key((int)n, m, groups[g], rplans[g]);
        reqs[g].group = &groups[g];
        reqs[g].rplan = &rplans[g];
        reqs[g].n = (int)n;
        reqs[g].m = m;
    }
    const std::string e = jit_precompile(reqs);
    if (!e.empty()) {
        put(e);
        return QW_E_HIP;
    }
    return QW_OK;
}

int qw_jit_precompile_suffix(uint32_t n, const qw_gate *gates, uint64_t n_gates, const uint64_t *x,
                             const uint64_t *z, uint32_t n_terms, uint32_t tile_bits, char *log,
                             uint64_t cap) {
    auto put = [&](const std::string &msg) {
        if (log && cap) {
            size_t k = std::min<size_t>(msg.size(), cap - 1);
            std::memcpy(log, msg.data(), k);
            log[k] = 0;
        }
    };
    put("");
    if (n_terms && (!x || !z)) {
        put("term arrays are NULL");
        return QW_E_INVALID_ARG;
    }
    // the plans from a snapshot and in place, with and without permuted
    // layouts (calls choose by where the first pass loads from and by the
    // size of their states)
    Plan pv[4];
    std::string e;
    for (int v = 0; v < 4 && e.empty(); ++v)
        e = build_plan((int)n, gates, (size_t)n_gates, (int)tile_bits, &pv[v], true, true, false, v >= 2, v & 1);
    if (!e.empty()) {
        put(e);
        return QW_E_INVALID_ARG;
    }
    const Plan &p = pv[0];
    if (p.m < kMinTileBits) return QW_OK;
    const uint64_t full = (1ull << n) - 1;
    for (uint32_t j = 0; j < n_terms; ++j)
        if ((x[j] & ~full) || (z[j] & ~full)) {
            put("Pauli mask has bits >= n");
            return QW_E_INVALID_ARG;
        }
    FusedEpi fev[4];
    std::vector<JitReq> reqs;
    std::set<std::string> seen;
    for (int v = 0; v < 4; ++v) {
        const Plan &pp = pv[v];
        FusedEpi &fe = fev[v];
        bool norm = false;
        for (const HostPass &h : pp.passes) norm |= h.norm_out || h.scale_in;
        if (n_terms && !pp.passes.empty() && !norm && (int)n > pp.m)
            plan_fused_last((int)n, pp.m, pp.passes.back(), x, z, n_terms, &fe);
        for (size_t k = 0; k < pp.passes.size(); ++k) {
            const HostPass &h = pp.passes[k];
            const bool with_epi = fe.active && k + 1 == pp.passes.size();
            // both load policies (QW_OPT_STREAM_LOADS, snapshot-reading first passes)
            for (int stream = 0; stream <= 1; ++stream) {
                JitReq r;
                r.use_lds = h.norm_out || h.dev_phases.size() > 1 || with_epi;
                r.key = jit_pass_key((int)n, pp.m, h, r.use_lds) + (with_epi ? fe.key : std::string()) +
                        (stream ? "S" : "T");
                if (!seen.insert(r.key).second) continue;
                r.pass = &h;
                r.epi = with_epi ? &fe.rplan : nullptr;
                r.n = (int)n;
                r.m = pp.m;
                r.stream_loads = stream != 0;
                reqs.push_back(std::move(r));
            }
        }
    }
    // the persistent kernels of such a batch (QW_OPT_PERSISTENT): its pass
    // structures in pass order, the first reading the snapshot
    std::vector<std::vector<PersistPart>> pparts;
    for (int v = 0; v < 4; ++v)
        for (int stream = 0; stream <= 1; ++stream) {
            const Plan &pp = pv[v];
            bool norm = false;
            for (const HostPass &h : pp.passes) norm |= h.norm_out;
            if (pp.passes.empty() || norm) continue;
            std::vector<PersistPart> parts;
            for (size_t k = 0; k < pp.passes.size(); ++k) {
                PersistPart q;
                q.pass = &pp.passes[k];
                const bool with_epi = fev[v].active && k + 1 == pp.passes.size();
                q.epi = with_epi ? &fev[v].rplan : nullptr;
                q.epi_key = with_epi ? &fev[v].key : nullptr;
                q.n = (int)n;
                q.m = pp.m;
                q.stream_loads = stream != 0 && k > 0;
                parts.push_back(q);
            }
            pparts.push_back(std::move(parts));
        }
    for (const auto &parts : pparts) {
        JitReq r;
        r.key = jit_persist_key(parts);
        if (!seen.insert(r.key).second) continue;
        r.persist = &parts;
        r.n = (int)n;
        r.m = p.m;
        r.use_lds = true;
        reqs.push_back(std::move(r));
    }
    const FusedEpi &fe = fev[0];
    // the reducer groups of the remaining terms, built as expect_slots builds them
    std::vector<uint32_t> idx;
    std::vector<uint64_t> xs;
    for (uint32_t j = 0; j < n_terms; ++j)
        if (!fe.active || !fe.fused[j]) {
            idx.push_back(j);
            xs.push_back(x[j]);
        }
    std::vector<TermGroup> groups;
    if (!xs.empty()) groups = group_terms((int)n, p.m, xs.data(), xs.size());
    for (TermGroup &g : groups)
        for (uint32_t &t : g.terms) t = idx[t];
    std::vector<RedPlan> rplans;
    for (const TermGroup &g : groups) rplans.push_back(plan_reduce_group((int)n, p.m, g, x, z));
    for (size_t g = 0; g < groups.size(); ++g) {
        JitReq r;
        r.key = jit_reduce_key((int)n, p.m, groups[g], rplans[g]);
        r.group = &groups[g];
        r.rplan = &rplans[g];
        r.n = (int)n;
        r.m = p.m;
        reqs.push_back(std::move(r));
    }
    e = jit_precompile(reqs);
    if (!e.empty()) {
        put(e);
        return QW_E_HIP;
    }
    return QW_OK;
}

int qw_jit_stats(uint64_t *compiled, uint64_t *disk_hits, double *compile_seconds) {
    jit_stats(compiled, disk_hits, compile_seconds);
    return QW_OK;
}

int qw_persist_schedule(uint32_t n_tasks, const int32_t *parent, const uint32_t *n_passes, const uint32_t *kinds,
                        const uint32_t *units, uint32_t chunk_max, uint32_t grid, char *json_out, uint64_t cap) {
    if (n_tasks && (!parent || !n_passes)) return QW_E_INVALID_ARG;
    if (grid == 0) return QW_E_INVALID_ARG;
    std::vector<int> par(n_tasks);
    std::vector<uint32_t> np(n_tasks);
    std::vector<PersistDesc> ds;
    for (uint32_t t = 0; t < n_tasks; ++t) {
        par[t] = parent[t];
        np[t] = n_passes[t];
        if (par[t] < -1) return QW_E_INVALID_ARG;
    }
    uint64_t total = 0;
    for (uint32_t t = 0; t < n_tasks; ++t) total += np[t];
    if (total && (!kinds || !units)) return QW_E_INVALID_ARG;
    uint64_t i = 0;
    for (uint32_t t = 0; t < n_tasks; ++t)
        for (uint32_t k = 0; k < np[t]; ++k, ++i) {
            PersistDesc d;
            d.t = t;
            d.k = k;
            d.kind = kinds[i];
            d.units = units[i];
            // the first pass loads its parent's final state (shared by
            // siblings), any other pass the task's own
            d.src = (k == 0 && par[t] >= 0) ? (uint64_t)par[t] : (1ull << 32) + t;
            ds.push_back(d);
        }
    PersistSchedule sch;
    const std::string e = persist_schedule(par, np, ds, 1, chunk_max, grid, &sch);
    if (!e.empty()) {
        if (json_out && cap) std::snprintf(json_out, cap, "%s", e.c_str());
        return QW_E_INVALID_ARG;
    }
    std::string js = "{\"claims\": " + std::to_string(sch.claims) + ", \"segments\": [";
    for (size_t q = 0; q < sch.segs.size(); ++q) {
        const PSeg &g = sch.segs[q];
        js += (q ? ", [" : "[") + std::to_string(g.claim0) + ", " + std::to_string(g.n_claims) + ", " +
              std::to_string(g.desc0) + ", " + std::to_string(g.n_descs) + ", " + std::to_string(g.chunk) + ", " +
              std::to_string(g.kind) + ", " + std::to_string(g.tmaj) + ", " + std::to_string(g.units) + "]";
    }
    js += "], \"deps\": [";
    for (size_t q = 0; q < sch.deps.size(); ++q)
        js += (q ? ", [" : "[") + std::to_string((int64_t)(sch.deps[q].dep == kNoDep ? -1 : (int64_t)sch.deps[q].dep)) +
              ", " + std::to_string(sch.deps[q].need) + "]";
    js += "], \"descs\": [";
    for (size_t q = 0; q < sch.order.size(); ++q)
        js += (q ? ", [" : "[") + std::to_string(ds[sch.order[q]].t) + ", " + std::to_string(ds[sch.order[q]].k) + "]";
    js += "]}";
    if (!json_out || cap <= js.size()) return QW_E_INVALID_ARG;
    std::memcpy(json_out, js.c_str(), js.size() + 1);
    return QW_OK;
}

int qw_plan_describe(uint32_t n, const qw_gate *gates, uint64_t n_gates, uint32_t tile_bits,
                     char *json_out, uint64_t cap) {
    Plan p;
    std::string e = build_plan((int)n, gates, (size_t)n_gates, (int)tile_bits, &p);
    std::string js = e.empty() ? plan_json(p) : ("{\"error\": \"" + json_escape(e) + "\"}");
    if (json_out && cap) {
        size_t k = std::min<size_t>(js.size(), cap - 1);
        std::memcpy(json_out, js.data(), k);
        json_out[k] = 0;
    }
    if (!e.empty()) return QW_E_INVALID_ARG;
    return js.size() + 1 > cap ? QW_E_INVALID_ARG : QW_OK;
}

// ------------------------------------------------------------ graphs
namespace {

// Leave recording mode: the capture ends, the context gets its own buffers
// and stream back, and the buffers of the recording are returned.
void end_recording(qw_ctx *ctx, hipGraph_t *graph, std::vector<void *> *owned,
                   std::vector<std::vector<GraphSeg>> *calls = nullptr,
                   std::vector<OutcomeRec> *outcomes = nullptr) {
    GraphRec *r = ctx->rec;
    if (calls) *calls = std::move(r->calls);
    if (outcomes) *outcomes = std::move(r->outcomes);
    hipGraph_t gr = nullptr;
    hipError_t e = hipStreamEndCapture(r->cap, &gr);
    if (e != hipSuccess) gr = nullptr;
    *graph = gr;
    *owned = std::move(r->owned);
    for (DevBuf *b : {&ctx->plan, &ctx->scratch, &ctx->pingpong, &ctx->meas, &ctx->psync})
        if (b->p) owned->push_back(b->p);
    ctx->plan = r->saved_plan;
    ctx->scratch = r->saved_scratch;
    ctx->pingpong = r->saved_pingpong;
    ctx->meas = r->saved_meas;
    ctx->psync = r->saved_psync;
    ctx->stream = r->saved_stream;
    (void)hipStreamDestroy(r->cap);
    (void)hipStreamDestroy(r->up);
    delete r;
    ctx->rec = nullptr;
}

void free_owned(std::vector<void *> &owned) {
    for (void *p : owned) (void)hipFree(p);
    owned.clear();
}

}  // namespace

int qw_graph_begin(qw_ctx *ctx) {
    if (!ctx) return QW_E_INVALID_ARG;
    if (ctx->rec) return fail(ctx, QW_E_INVALID_ARG, "a graph is already being recorded");
    // earlier work of the context's stream, and the staging buffer, are done
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream), "stream sync");
    std::unique_ptr<GraphRec> r(new (std::nothrow) GraphRec());
    if (!r) return fail(ctx, QW_E_OOM, "host allocation");
    HIP_TRY(ctx, hipStreamCreateWithFlags(&r->cap, hipStreamNonBlocking), "capture stream");
    hipError_t e = hipStreamCreateWithFlags(&r->up, hipStreamNonBlocking);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(r->cap);
        return hip_fail(ctx, e, "upload stream");
    }
    e = hipStreamBeginCapture(r->cap, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(r->cap);
        (void)hipStreamDestroy(r->up);
        return hip_fail(ctx, e, "begin capture");
    }
    r->saved_stream = ctx->stream;
    r->saved_plan = ctx->plan;
    r->saved_scratch = ctx->scratch;
    r->saved_pingpong = ctx->pingpong;
    r->saved_meas = ctx->meas;
    r->saved_psync = ctx->psync;
    ctx->plan = DevBuf{};
    ctx->scratch = DevBuf{};
    ctx->pingpong = DevBuf{};
    ctx->meas = DevBuf{};
    ctx->psync = DevBuf{};
    ctx->stream = r->cap;
    ctx->rec = r.release();
    return QW_OK;
}

int qw_graph_end(qw_ctx *ctx, qw_graph **out) {
    if (!ctx || !out) return QW_E_INVALID_ARG;
    *out = nullptr;
    if (!ctx->rec) return fail(ctx, QW_E_INVALID_ARG, "no graph is being recorded");
    hipGraph_t gr = nullptr;
    std::vector<void *> owned;
    std::vector<std::vector<GraphSeg>> calls;
    std::vector<OutcomeRec> outcomes;
    end_recording(ctx, &gr, &owned, &calls, &outcomes);
    if (!gr) {
        free_owned(owned);
        return fail(ctx, QW_E_HIP, "stream capture ended without a graph (a recorded call failed)");
    }
    std::unique_ptr<qw_graph> g(new (std::nothrow) qw_graph());
    if (!g) {
        (void)hipGraphDestroy(gr);
        free_owned(owned);
        return fail(ctx, QW_E_OOM, "host allocation");
    }
    size_t nn = 0;
    (void)hipGraphGetNodes(gr, nullptr, &nn);
    hipError_t e = hipGraphInstantiate(&g->exec, gr, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(gr);
        free_owned(owned);
        return hip_fail(ctx, e, "graph instantiate");
    }
    g->ctx = ctx;
    g->graph = gr;
    g->owned = std::move(owned);
    g->calls = std::move(calls);
    g->outcomes = std::move(outcomes);
    g->nodes = nn;
    *out = g.release();
    return QW_OK;
}

int qw_graph_outcomes(qw_graph *g, uint8_t *out, uint64_t cap, uint64_t *count) {
    if (!g || (cap && !out)) return QW_E_INVALID_ARG;
    qw_ctx *ctx = g->ctx;
    if (ctx->rec) return recording_unsupported(ctx, "qw_graph_outcomes");
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream), "stream sync");
    uint64_t total = 0;
    bool zero = false;
    for (const OutcomeRec &r : g->outcomes) {
        const uint64_t m = total < cap ? std::min<uint64_t>(cap - total, r.count) : 0;
        if (m) HIP_TRY(ctx, hipMemcpy(out + total, r.outc, m, hipMemcpyDeviceToHost), "outcome copy");
        uint32_t e = 0;
        HIP_TRY(ctx, hipMemcpy(&e, r.err, sizeof e, hipMemcpyDeviceToHost), "outcome copy");
        zero = zero || e != 0;
        total += r.count;
    }
    if (count) *count = total;
    if (zero) return fail(ctx, QW_E_INVALID_ARG, "measurement of a zero state");
    return QW_OK;
}

int qw_graph_launch(qw_graph *g) {
    if (!g) return QW_E_INVALID_ARG;
    qw_ctx *ctx = g->ctx;
    if (ctx->rec) return recording_unsupported(ctx, "qw_graph_launch");
    HIP_TRY(ctx, hipGraphLaunch(g->exec, ctx->stream), "graph launch");
    return QW_OK;
}

int qw_graph_nodes(const qw_graph *g, uint64_t *nodes) {
    if (!g || !nodes) return QW_E_INVALID_ARG;
    *nodes = g->nodes;
    return QW_OK;
}

int qw_graph_update_gates(qw_graph *g, uint32_t call, uint32_t task, const qw_gate *gates,
                          uint64_t n_gates) {
    if (!g) return QW_E_INVALID_ARG;
    qw_ctx *ctx = g->ctx;
    if (ctx->rec) return recording_unsupported(ctx, "qw_graph_update_gates");
    if (call >= g->calls.size() || task >= g->calls[call].size())
        return fail(ctx, QW_E_INVALID_ARG, "no such recorded call or task");
    if (n_gates && !gates) return fail(ctx, QW_E_INVALID_ARG, "gates == NULL");
    for (uint64_t i = 0; i < n_gates; ++i)
        if (is_measure(gates[i].kind)) return fail(ctx, QW_E_INVALID_ARG, "measurement gates cannot be updated");
    GraphSeg &sg = g->calls[call][task];
    std::shared_ptr<const Plan> np;
    std::string e = get_plan(ctx, sg.n, gates, n_gates, &np, sg.plan->in_place, sg.plan->layout);
    if (!e.empty()) return fail(ctx, QW_E_INVALID_ARG, e);
    // the pass structure (kernel identity, record counts, phases, I/O and
    // relabelling) must be the recorded one; only op-record values change
    const Plan &a = *sg.plan, &b = *np;
    bool same = a.m == b.m && a.passes.size() == b.passes.size();
    for (size_t k = 0; same && k < a.passes.size(); ++k) {
        const HostPass &pa = a.passes[k], &pb = b.passes[k];
        const bool la = pa.norm_out || pa.dev_phases.size() > 1, lb = pb.norm_out || pb.dev_phases.size() > 1;
        same = pa.dev_ops.size() == pb.dev_ops.size() && pa.dev_phases.size() == pb.dev_phases.size() &&
               std::memcmp(pa.dev_phases.data(), pb.dev_phases.data(),
                           pa.dev_phases.size() * sizeof(DevPhase)) == 0 &&
               std::memcmp(&pa.io_in, &pb.io_in, sizeof(IoRec)) == 0 &&
               std::memcmp(&pa.io_out, &pb.io_out, sizeof(IoRec)) == 0 &&
               pa.scale_in == pb.scale_in && pa.norm_out == pb.norm_out && pa.out_img == pb.out_img &&
               pa.in_pos == pb.in_pos && pa.out_pos == pb.out_pos &&
               jit_pass_key((int)sg.n, a.m, pa, la) == jit_pass_key((int)sg.n, b.m, pb, lb);
    }
    if (!same)
        return fail(ctx, QW_E_INVALID_ARG,
                    "the gates plan to another pass structure than the recorded ones (gate kinds, "
                    "qubits or context options differ)");
    // replays already enqueued read the old records
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream), "stream sync");
    for (size_t k = 0; k < b.passes.size(); ++k)
        if (sg.ops[k].second)
            HIP_TRY(ctx, hipMemcpy(sg.ops[k].first, b.passes[k].dev_ops.data(), sg.ops[k].second,
                                   hipMemcpyHostToDevice),
                    "op record update");
    sg.plan = np;
    return QW_OK;
}

int qw_graph_free(qw_graph *g) {
    if (!g) return QW_E_INVALID_ARG;
    qw_ctx *ctx = g->ctx;
    if (ctx->rec) return recording_unsupported(ctx, "qw_graph_free");
    // replays in flight still read the graph's buffers
    hipStreamSynchronize(ctx->stream);
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    free_owned(g->owned);
    delete g;
    return QW_OK;
}

}  // extern "C"
