// Internal: the context object behind the opaque phg_context handle, shared by
// the single-request ABI (phg_host.cpp) and the serving engine (phg_server.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <map>
#include <string>
#include <vector>

#include "../../include/phg.h"
#include "phg_internal.h"

namespace phg {

// Workspace plan: byte offsets of every device buffer inside one arena.
struct Plan {
    size_t codes, part, expo, eloc, P64, dP64, P32, dP32, PB32, PB64, dPB32, dPB64, vsum, TT64, dTT64, TT32, dTT32, b, V, Vinv, lam, rates, cw,
        pi, pw, sll, lpart, gpart, out, sched, desc, ch_parent, ch_kids, heights, trates, set_ptr, set_idx,
        qitems, qdep, qdone, qctr, total;
};
// table_slots = 0: P(t) tables for every branch; else a pool of that many
// (branch) tables, rebuilt per launch chunk (17..255-state kernels only).
Plan make_plan(int N, int C, int S, int R, phg_precision prec, int table_slots);
// Table slots a context of these sizes uses under a table-memory budget:
// 0 (every branch's tables) when they fit, else the pool that fits (>= 2).
int table_slots_for(int N, int S, int R, phg_precision prec, size_t budget);
constexpr size_t kDefaultTableBudget = size_t{16} << 30;

enum InputBit : unsigned {
    kTopo = 1u << 0,
    kB = 1u << 1,
    kEig = 1u << 2,
    kPi = 1u << 3,
    kCat = 1u << 4,
    kTips = 1u << 5,
    kPw = 1u << 6,
    kTime = 1u << 7,   // node heights + branch rate scalars (time tree)
    kSets = 1u << 8,   // branch sets
    kDesc = 1u << 9,   // descriptor fields changed (no input of its own)
    kTipVec = 1u << 10,  // general tip partial vectors
    kRequired = kTopo | kB | kEig | kPi | kCat | kTips,
};

constexpr int kProfEvents = PHG_PROF_CLASSES + 1;

// Doubles in the output region (device) and its pinned host mirror:
// logL, gradient [E], d/d heights [2N-1], d/d rates [E], set sums [<= E].
inline size_t out_doubles(int N) {
    const size_t E = 2 * static_cast<size_t>(N) - 2;
    return 1 + E + (E + 1) + E + E;
}

}  // namespace phg

struct phg_context {
    int N = 0, C = 0, S = 0, R = 0, device = 0;
    phg_precision prec = PHG_FP64;
    int Cpad = 0, tiles = 0, S4 = 0;
    std::string err;

    // host mirrors of every input
    std::vector<int32_t> parent;
    std::vector<int32_t> kids;   // [N-1][2] children of internal node N + k
    std::vector<double> b, V, Vinv, lam, pi, rates, cw, pw;
    std::vector<double> vsum;    // [models][S] row sums of Vinv (uploaded with the eigensystem)
    std::vector<uint8_t> codes;  // [N][Cpad], padding = S
    bool eig_cat = false;        // V, Vinv, lam hold one model per category
    // time tree (heights [2N-1], rate scalars [2N-2]) and branch sets (CSR)
    std::vector<double> heights, trates;
    std::vector<int32_t> set_ptr, set_idx;
    int n_sets = 0;
    // general tip partials: tip -> C x S values (pattern-major); on the device
    // in the partials layout of the level kernels, one slot per such tip in
    // ascending tip order, in memory the context allocates itself
    std::map<int, std::vector<double>> tip_vectors;
    void* d_tipvec = nullptr;
    size_t d_tipvec_bytes = 0;
    int32_t* d_tslot = nullptr;
    unsigned have = 0;           // inputs set at least once
    unsigned dirty = 0;          // inputs changed since the last upload
    unsigned sdirty = 0;         // inputs changed since the FP64 twin was last synchronised

    // FP32 precision guard: an FP32 context whose tree is more saturated
    // than fp32_guard (phg::fp32_saturation) evaluates on an FP64 twin
    // context holding copies of the same inputs; fp32_guard <= 0 disables.
    double fp32_guard = phg::kDefaultFp32Guard;
    uint64_t uid = 0;            // unique per context of this process
    size_t table_budget = phg::kDefaultTableBudget;   // bytes of P(t) tables before per-chunk tables
    int table_slots = 0;         // 0: tables for every branch; else the per-chunk pool (set at device init)
    bool static_ws = false;      // workspace is the static scratch array (phg_gradient_async_noalloc)
    phg_context* twin = nullptr;
    int last_prec = -1;          // precision of the last evaluation issued (-1: none)

    // schedule (host copy; uploaded to the sched region): NodeTriple records
    // (level schedule) or BlockRec records (blocked schedule), as raw words
    int sched_mode = PHG_SCHEDULE_AUTO;
    bool blocked = false;
    std::vector<int32_t> sched;
    // levels in execution order: (first record, record count)
    std::vector<std::pair<int, int>> post_lv, pre_lv;
    // work-queue traversal of the blocked schedule (phg::QueueArgs): items
    // [n][2] (post-order items first), dependencies [B][16]
    bool queue = false;
    std::vector<int32_t> qitems, qdep;
    int q_post = 0, q_blocks = 0;

    // device state
    bool dev_init = false;
    bool own_arena = false;
    char* arena = nullptr;
    char* bound_ws = nullptr;
    size_t bound_ws_bytes = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    double* host_out = nullptr;  // pinned, out_doubles(N)
    phg::Plan plan{};
    phg::ReqDesc rd{};           // host copy of this request's descriptor

    // library-owned HIP graphs of one whole evaluation (gradient, and
    // log-likelihood only) for the synchronous calls: captured on first use,
    // replayed while only device data changes (branch lengths, model, tips,
    // weights are uploaded before the replay); dropped when the launch
    // sequence changes (topology, schedule, descriptor, device binding)
    bool graph_on = true;
    hipGraphExec_t graph_exec[2] = {nullptr, nullptr};   // [0] gradient, [1] log-likelihood only
    uint64_t graph_captures = 0, graph_replays = 0;

    // profiling: kProfEvents events per recorded evaluation
    bool prof_on = false;
    std::vector<hipEvent_t> prof_pool;
    size_t prof_used = 0;

    phg_status fail(phg_status s, const char* fmt, ...) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        err = buf;
        return s;
    }
};

#define PHG_HIP(ctx, call)                                                                  \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return (ctx)->fail(e_ == hipErrorOutOfMemory ? PHG_ERR_OOM : PHG_ERR_DEVICE,    \
                               "%s failed: %s", #call, hipGetErrorString(e_));              \
    } while (0)

#define PHG_TRY(expr)                \
    do {                             \
        phg_status s_ = (expr);      \
        if (s_ != PHG_OK) return s_; \
    } while (0)

namespace phg {

// Validate required inputs, allocate / bind device memory on first use and
// upload whatever changed (on the context's stream).
phg_status ctx_ready(phg_context* ctx);
// Device pointer of this context's descriptor and of its output region.
ReqDesc* ctx_desc_dev(phg_context* ctx);
double* ctx_out_dev(phg_context* ctx);
// Allocate the pinned host mirror of the output region on first use.
phg_status ctx_host_out(phg_context* ctx);
// Enqueue one whole evaluation of this context alone.
phg_status ctx_enqueue_eval(phg_context* ctx, double* d_logl, double* d_grad);
// Saturation statistic of the FP32 precision guard for the context's current
// tree, branch lengths, eigensystem and rates (host only).
double fp32_saturation(const phg_context* ctx);
// The context that evaluates ctx's next request: ctx itself, or its FP64 twin
// (created and synchronised here) when the guard routes it.  Records the
// precision in ctx->last_prec.  Sets *st and returns nullptr on failure.
phg_context* eval_target(phg_context* ctx, phg_status* st);
// Copy the twin's error message into ctx when a routed call failed.
phg_status from_twin(phg_context* ctx, phg_context* t, phg_status s);
// The static scratch array of phg_gradient_async_noalloc (phg_static.hip):
// its device address on ctx's device, and whether another context used it
// since ctx did (recording ctx as its user).
phg_status scratch_address(phg_context* ctx, void** out);
bool scratch_claim(const phg_context* ctx);
// Destroy the context's captured evaluation graphs (they are captured again
// on next use).
void ctx_drop_graphs(phg_context* ctx);
// Forget the device binding (workspace, pinned output) so the context can be
// bound to new memory later; every input is uploaded again on next use.  The
// caller guarantees no device work of this context is pending.
void ctx_drop_device(phg_context* ctx);

}  // namespace phg
