// Host runtime behind include/phg.h: input validation and host mirrors,
// topology -> level schedule, workspace plan, device upload and the kernel
// sequence of one log-likelihood / gradient evaluation.
//
// Every phg_set_* call validates and copies its input on the host only; the
// device is first touched by a compute call (or phg_prepare), which allocates
// the workspace (or uses a caller-bound one), uploads whatever changed and
// enqueues: pmat -> post-order levels (height 1..H, the root last) ->
// pre-order levels (depth 0..D) -> finalize.
#include <dlfcn.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <tuple>
#include <cmath>
#include <cstring>
#include <limits>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "phg_context.h"

using phg::BlockRec;
using phg::NodeTriple;
using phg::ReqDesc;
using phg::SegTable;

namespace phg {

namespace {
constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
}  // namespace

namespace {
size_t gl_table_bytes_per_branch(int S, int R, bool fp32) {
    return static_cast<size_t>(R) * (2 * gl_mat_rows(S) + 2 * gl_back_rows(S)) * gl_row(S) * (fp32 ? 4 : 8);
}
// Vector-ALU kernels: forward P, dP [SP][SP] and backward P, dP [SP + 1][SP].
size_t vs_table_bytes_per_branch(int S, int R, bool fp32) {
    const size_t SP = vs_padded_states(S);
    return static_cast<size_t>(R) * (2 * SP * SP + 2 * (SP + 1) * SP) * (fp32 ? 4 : 8);
}
}  // namespace

int table_slots_for(int N, int S, int R, phg_precision prec, size_t budget) {
    const bool fp32 = prec == PHG_FP32_SCALED;
    const bool vs = uses_vs_kernels(S, R, fp32);
    if (!vs && !uses_gl_kernels(S, R, fp32)) return 0;
    const size_t E = 2 * static_cast<size_t>(N) - 2;
    const size_t per = vs ? vs_table_bytes_per_branch(S, R, fp32) : gl_table_bytes_per_branch(S, R, fp32);
    if (E * per <= budget) return 0;
    const size_t fit = budget / per;
    return static_cast<int>(std::max<size_t>(2, std::min(fit, E) & ~size_t{1}));
}

Plan make_plan(int N, int C, int S, int R, phg_precision prec, int table_slots) {
    const int Cpad = (C + kLanes - 1) / kLanes * kLanes;
    const int tp = tile_patterns(S, R, prec == PHG_FP32_SCALED);
    const int tiles = Cpad / tp;
    const size_t E = 2 * static_cast<size_t>(N) - 2;
    const size_t I = static_cast<size_t>(N) - 1;
    const size_t tsz = prec == PHG_FP32_SCALED ? 4 : 8;
    Plan p{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    const bool fp32 = prec == PHG_FP32_SCALED;
    p.codes = take(static_cast<size_t>(N) * Cpad * code_bytes(S));
    p.expo = take(I * Cpad * sizeof(int32_t));
    if (uses_vs_kernels(S, R, fp32)) {
        // vector-ALU kernels: zero-padded tables of the path's own type
        const size_t SP = vs_padded_states(S);
        const size_t T = table_slots > 0 ? static_cast<size_t>(table_slots) : E;   // tables held
        const size_t mat = T * R * SP * SP;
        const size_t back = T * R * (SP + 1) * SP;
        p.part = take(I * tiles * R * SP * tp * tsz);
        p.eloc = take(0);
        p.P64 = take(fp32 ? 0 : mat * 8);
        p.dP64 = take(fp32 ? 0 : mat * 8);
        p.PB64 = take(fp32 ? 0 : back * 8);
        p.dPB64 = take(fp32 ? 0 : back * 8);
        p.P32 = take(fp32 ? mat * 4 : 0);
        p.dP32 = take(fp32 ? mat * 4 : 0);
        p.PB32 = take(fp32 ? back * 4 : 0);
        p.dPB32 = take(fp32 ? back * 4 : 0);
    } else if (uses_gl_kernels(S, R, fp32)) {
        // MFMA operand order: one forward table per matrix and a backward
        // copy of P, in the path's own type only
        const size_t T = table_slots > 0 ? static_cast<size_t>(table_slots) : E;   // tables held
        const size_t mat = T * R * gl_mat_rows(S) * gl_row(S);
        const size_t back = T * R * gl_back_rows(S) * gl_row(S);
        p.part = take(I * tiles * R * tp * gl_row(S) * tsz);
        p.eloc = take(I * Cpad * sizeof(int32_t));
        p.P64 = take(fp32 ? 0 : mat * 8);
        p.dP64 = take(fp32 ? 0 : mat * 8);
        p.PB64 = take(fp32 ? 0 : back * 8);
        p.dPB64 = take(fp32 ? 0 : back * 8);
        p.P32 = take(fp32 ? mat * 4 : 0);
        p.dP32 = take(fp32 ? mat * 4 : 0);
        p.PB32 = take(fp32 ? back * 4 : 0);
        p.dPB32 = take(fp32 ? back * 4 : 0);
    } else {
        p.part = take(I * tiles * R * S * tp * tsz);
        p.eloc = take(0);
        p.P64 = take(E * R * S * S * 8);
        p.dP64 = take(E * R * S * S * 8);
        p.P32 = take(fp32 ? E * R * S * S * 4 : 0);
        p.dP32 = take(fp32 ? E * R * S * S * 4 : 0);
        p.PB64 = take(0);
        p.PB32 = take(0);
        p.dPB64 = take(0);
        p.dPB32 = take(0);
    }
    p.vsum = take(static_cast<size_t>(R) * S * 8);
    const size_t tt = S == 4 ? E * R * 20 : 0;
    p.TT64 = take(tt * 8);
    p.dTT64 = take(tt * 8);
    p.TT32 = take(prec == PHG_FP32_SCALED ? tt * 4 : 0);
    p.dTT32 = take(prec == PHG_FP32_SCALED ? tt * 4 : 0);
    p.b = take(E * 8);
    p.V = take(static_cast<size_t>(R) * S * S * 8);       // room for one model per category
    p.Vinv = take(static_cast<size_t>(R) * S * S * 8);
    p.lam = take(static_cast<size_t>(R) * S * 8);
    p.rates = take(R * 8);
    p.cw = take(R * 8);
    p.pi = take(S * 8);
    p.pw = take(static_cast<size_t>(Cpad) * 8);
    p.sll = take(static_cast<size_t>(Cpad) * 8);
    p.lpart = take(static_cast<size_t>(tiles) * 8);
    p.gpart = take(E * tiles * 8);
    p.out = take(out_doubles(N) * 8);
    p.sched = take(I * sizeof(BlockRec));   // >= 2 I NodeTriples or I block records
    p.desc = take(sizeof(ReqDesc));
    p.ch_parent = take((E + 1) * 4);
    p.ch_kids = take(2 * I * 4);
    p.heights = take((E + 1) * 8);
    p.trates = take(E * 8);
    p.set_ptr = take((E + 1) * 4);
    p.set_idx = take(E * 4);
    // work-queue traversal (blocks <= internal nodes)
    const bool queue = queue_supported(S, R, fp32);
    p.qitems = take(queue ? 2 * I * tiles * 2 * sizeof(int32_t) : 0);
    p.qdep = take(queue ? I * 16 * sizeof(int32_t) : 0);
    p.qdone = take(queue ? 2 * I * tiles * sizeof(uint32_t) : 0);
    p.qctr = take(queue ? kQueueWords * sizeof(uint32_t) : 0);
    p.total = off;
    return p;
}

}  // namespace phg

using namespace phg;

namespace {

thread_local std::string g_create_error;

// Tip code i (tip-major, Cpad per tip) in the host mirror: a byte, or a
// little-endian 16-bit value above 255 states.
void put_code(phg_context* ctx, size_t i, int v) {
    if (code_bytes(ctx->S) == 1) {
        ctx->codes[i] = static_cast<uint8_t>(v);
    } else {
        ctx->codes[2 * i] = static_cast<uint8_t>(v & 0xff);
        ctx->codes[2 * i + 1] = static_cast<uint8_t>(v >> 8);
    }
}

// ---- tuning table (phg_set_tuning, tuning file)
struct TuneKey {
    int S, R, fp32, param;
    bool operator<(const TuneKey& o) const {
        return std::tie(S, R, fp32, param) < std::tie(o.S, o.R, o.fp32, o.param);
    }
};
std::mutex g_tune_mu;
std::map<TuneKey, int> g_tune;
std::once_flag g_tune_once;

bool tune_value_ok(int S, int R, bool fp32, int param, int value) {
    if (value < 0) return false;
    if (value == 0) return true;
    if (param == PHG_TUNE_ROW_BLOCKS)
        return S > 16 && phg::gl_row_blocks_allowed(S, fp32, value);   // read by the MFMA kernels only
    if (param == PHG_TUNE_NARROW_UNITS) return S == 4 && fp32;
    if (param == PHG_TUNE_QUEUE_LAUNCHES) return S == 4 && fp32 && value <= 2;
    if (param == PHG_TUNE_QUEUE_WAIT_US) return phg::queue_supported(S, R, fp32);
    return false;
}

void tune_load_file() {
    const char* off = std::getenv("PHG_TUNE");
    if (off && std::strcmp(off, "off") == 0) return;
    std::string path;
    if (const char* f = std::getenv("PHG_TUNE_FILE")) {
        path = f;
    } else {
        Dl_info info;
        if (dladdr(reinterpret_cast<void*>(&tune_load_file), &info) && info.dli_fname) {
            path = info.dli_fname;
            const size_t slash = path.rfind('/');
            path = (slash == std::string::npos ? std::string(".") : path.substr(0, slash)) + "/tune_cache.txt";
        }
    }
    if (path.empty()) return;
    FILE* fp = std::fopen(path.c_str(), "r");
    if (!fp) return;
    char line[256];
    while (std::fgets(line, sizeof line, fp)) {
        char arch[32];
        int S, R, prec, param, value;
        if (line[0] == '#') continue;
        if (std::sscanf(line, "%31s %d %d %d %d %d", arch, &S, &R, &prec, &param, &value) != 6) continue;
        if (std::strcmp(arch, "gfx950") != 0) continue;
        if (param < 0 || param >= PHG_TUNE_PARAMS || (prec != 0 && prec != 1)) continue;
        if (!tune_value_ok(S, R, prec == 1, param, value)) continue;
        g_tune[TuneKey{S, R, prec, param}] = value;
    }
    std::fclose(fp);
}

bool finite_all(const double* x, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(x[i])) return false;
    return true;
}

phg_status check_sizes(int n_tips, int n_patterns, int n_states, int n_categories, int prec,
                       std::string* why) {
    if (n_tips < 2) return *why = "n_tips must be >= 2", PHG_ERR_ARG;
    if (n_tips > (1 << 24)) return *why = "n_tips too large", PHG_ERR_ARG;
    if (n_patterns < 1) return *why = "n_patterns must be >= 1", PHG_ERR_ARG;
    if (n_patterns > (1 << 28)) return *why = "n_patterns too large", PHG_ERR_ARG;
    // S itself is the ambiguous code: bytes up to 255 states, 16 bits above
    if (n_states < 2 || n_states > 256) return *why = "n_states must be in [2, 256]", PHG_ERR_ARG;
    if (n_categories < 1 || n_categories > 64)
        return *why = "n_categories must be in [1, 64]", PHG_ERR_ARG;
    if (prec != PHG_FP64 && prec != PHG_FP32_SCALED) return *why = "unknown precision", PHG_ERR_ARG;
    return PHG_OK;
}

// Build post-order (by height) and pre-order (by depth) levels.
void build_schedule(phg_context* ctx) {
    const int N = ctx->N, n = 2 * N - 1, root = n - 1;
    std::vector<int> c0(n, -1), c1(n, -1);
    for (int v = 0; v < n; ++v) {
        const int p = ctx->parent[v];
        if (p < 0) continue;
        if (c0[p] < 0)
            c0[p] = v;
        else
            c1[p] = v;
    }
    for (int v = N; v < n; ++v)
        if (c0[v] > c1[v]) std::swap(c0[v], c1[v]);
    ctx->kids.resize(2 * static_cast<size_t>(N - 1));
    for (int v = N; v < n; ++v) {
        ctx->kids[2 * (v - N)] = c0[v];
        ctx->kids[2 * (v - N) + 1] = c1[v];
    }
    // depth by walking down from the root (iterative)
    std::vector<int> depth(n, 0), order;
    order.reserve(n);
    order.push_back(root);
    for (size_t h = 0; h < order.size(); ++h) {
        const int v = order[h];
        if (v >= N) {
            depth[c0[v]] = depth[v] + 1;
            depth[c1[v]] = depth[v] + 1;
            order.push_back(c0[v]);
            order.push_back(c1[v]);
        }
    }
    std::vector<int> height(n, 0);
    for (int h = static_cast<int>(order.size()) - 1; h >= 0; --h) {
        const int v = order[h];
        if (v >= N) height[v] = 1 + std::max(height[c0[v]], height[c1[v]]);
    }
    const int H = height[root];
    int D = 0;
    for (int v = N; v < n; ++v) D = std::max(D, depth[v]);
    ctx->sched.clear();
    ctx->post_lv.clear();
    ctx->pre_lv.clear();
    ctx->queue = false;
    ctx->qitems.clear();
    ctx->qdep.clear();
    const bool fp32 = ctx->prec == PHG_FP32_SCALED;
    // the blocked kernels take tips by their codes only
    ctx->blocked = ctx->sched_mode == PHG_SCHEDULE_BLOCKS ||
                   (ctx->sched_mode == PHG_SCHEDULE_QUEUE && phg::blocked_supported(ctx->S, ctx->R, fp32)) ||
                   (ctx->sched_mode == PHG_SCHEDULE_AUTO && phg::blocked_supported(ctx->S, ctx->R, fp32) &&
                    ctx->tip_vectors.empty());
    if (ctx->blocked) {
        // block roots: internal nodes at depths 0, 3, 6, ...; records grouped
        // by block depth m (depth / 3), shallowest first
        const int M = D / phg::kBlockDepth;
        std::vector<std::vector<int>> bylev(M + 1);
        for (int v = N; v < n; ++v)
            if (depth[v] % phg::kBlockDepth == 0) bylev[depth[v] / phg::kBlockDepth].push_back(v);
        std::vector<int> start(M + 2, 0);
        for (int m = 0; m <= M; ++m) {
            start[m] = static_cast<int>(ctx->sched.size() / 16);
            for (int v : bylev[m]) {
                int32_t heap[16];
                std::fill(heap, heap + 16, -1);
                heap[0] = 0;
                heap[1] = v;
                for (int pos = 1; pos < 8; ++pos) {
                    const int k = heap[pos];
                    if (k >= N) {
                        heap[2 * pos] = c0[k];
                        heap[2 * pos + 1] = c1[k];
                    }
                }
                ctx->sched.insert(ctx->sched.end(), heap, heap + 16);
            }
        }
        start[M + 1] = static_cast<int>(ctx->sched.size() / 16);
        for (int m = M; m >= 0; --m) ctx->post_lv.emplace_back(start[m], start[m + 1] - start[m]);
        for (int m = 0; m <= M; ++m) ctx->pre_lv.emplace_back(start[m], start[m + 1] - start[m]);
        const int B = start[M + 1];
        ctx->queue = ctx->sched_mode == PHG_SCHEDULE_QUEUE && ctx->S == 4 && phg::queue_supported(ctx->S, ctx->R, fp32) &&
                     static_cast<int64_t>(2) * B * ctx->tiles * phg::kLanes * ctx->R < (int64_t{1} << 31);
        if (ctx->queue) {
            // dependencies: the records of the blocks rooted at each frontier
            // position, and each block's parent record
            std::vector<int> rec_of(n, -1);
            for (int r = 0; r < B; ++r) rec_of[ctx->sched[16 * r + 1]] = r;
            ctx->qdep.assign(static_cast<size_t>(B) * 16, -1);
            for (int r = 0; r < B; ++r)
                for (int j = 0; j < 8; ++j) {
                    const int c = ctx->sched[16 * r + 8 + j];
                    if (c < N) continue;                     // tip or absent
                    ctx->qdep[16 * r + j] = rec_of[c];
                    ctx->qdep[16 * rec_of[c] + 8] = r;
                }
            // items: post-order levels deepest first, then pre-order levels
            // from the root's; block-major within a level (a block's tiles
            // together: its matrices and tip-code rows are read by
            // neighbouring workgroups)
            ctx->qitems.clear();
            ctx->qitems.reserve(static_cast<size_t>(4) * B * ctx->tiles);
            for (int pass = 0; pass < 2; ++pass) {
                for (const auto& lv : pass == 0 ? ctx->post_lv : ctx->pre_lv)
                    for (int r = lv.first; r < lv.first + lv.second; ++r)
                        for (int t = 0; t < ctx->tiles; ++t) {
                            ctx->qitems.push_back(r | (pass << 30));
                            ctx->qitems.push_back(t);
                        }
                if (pass == 0) ctx->q_post = static_cast<int>(ctx->qitems.size() / 2);
            }
            ctx->q_blocks = B;
        }
        return;
    }
    // kernel families that fold, with tables for every branch: fold the
    // internal nodes (but the root) whose two children are tips given by
    // codes -- no post-order launch; the parent forms the partial from the
    // tips (and, with folds_pre_order, the tips' gradient sums from the
    // node's pre-order vector, so no pre-order launch either)
    std::vector<char> folded(n, 0);
    if (phg::folds_tip_pairs(ctx->S, ctx->R, fp32) &&
        table_slots_for(N, ctx->S, ctx->R, ctx->prec, ctx->table_budget) == 0) {
        for (int v = N; v < root; ++v)
            folded[v] = c0[v] < N && c1[v] < N && !ctx->tip_vectors.count(c0[v]) && !ctx->tip_vectors.count(c1[v]);
    }
    std::vector<std::vector<int>> by(H + 1);
    for (int v = N; v < n; ++v)
        if (!folded[v]) by[height[v]].push_back(v);
    auto put = [&](int v) {
        const int32_t rec[4] = {v, c0[v], c1[v], (folded[c0[v]] ? 1 : 0) | (folded[c1[v]] ? 2 : 0)};
        ctx->sched.insert(ctx->sched.end(), rec, rec + 4);
    };
    for (int h = 1; h <= H; ++h) {
        if (by[h].empty()) continue;   // height 1 when every node there is folded
        const int a = static_cast<int>(ctx->sched.size() / 4);
        for (int v : by[h]) put(v);
        ctx->post_lv.emplace_back(a, static_cast<int>(ctx->sched.size() / 4) - a);
    }
    std::vector<std::vector<int>> bd(D + 1);
    const bool fold_pre = phg::folds_pre_order(ctx->S, ctx->R, fp32);
    for (int v = N; v < n; ++v)
        if (!(fold_pre && folded[v])) bd[depth[v]].push_back(v);   // else the parent forms its tip gradients
    for (int d = 0; d <= D; ++d) {
        if (bd[d].empty()) continue;
        const int a = static_cast<int>(ctx->sched.size() / 4);
        for (int v : bd[d]) put(v);
        ctx->pre_lv.emplace_back(a, static_cast<int>(ctx->sched.size() / 4) - a);
    }
    // work-queue traversal of the vector-ALU and MFMA kernels (tables for
    // every branch)
    const int n_rec = static_cast<int>(ctx->sched.size() / 4);
    ctx->queue = ctx->sched_mode == PHG_SCHEDULE_QUEUE && ctx->S != 4 &&
                 phg::queue_supported(ctx->S, ctx->R, fp32) &&
                 table_slots_for(N, ctx->S, ctx->R, ctx->prec, ctx->table_budget) == 0 &&
                 static_cast<int64_t>(n_rec) * ctx->tiles * phg::kLanes * ctx->R < (int64_t{1} << 31);
    if (!ctx->queue) return;
    // a pre-order record waits on its parent's (which wrote its vector)
    ctx->qdep.assign(static_cast<size_t>(2) * n_rec, -1);
    for (const auto& lv : ctx->pre_lv)
        for (int r = lv.first; r < lv.first + lv.second; ++r) {
            const int k = ctx->sched[4 * r];
            if (k != root) ctx->qdep[2 * r] = ctx->parent[k] - N;
        }
    // items: post-order levels deepest first, then pre-order levels from the
    // root's; within a level tile-major for the vector-ALU kernels (small
    // tables), record-major for the MFMA kernels (a record's large P(t)
    // tables then stay in L2 for its tiles, as in the level launches)
    const bool by_record = phg::uses_gl_kernels(ctx->S, ctx->R, fp32);
    ctx->qitems.clear();
    ctx->qitems.reserve(static_cast<size_t>(2) * n_rec * ctx->tiles);
    for (int pass = 0; pass < 2; ++pass) {
        for (const auto& lv : pass == 0 ? ctx->post_lv : ctx->pre_lv) {
            const int n_in = lv.second * ctx->tiles;
            for (int x = 0; x < n_in; ++x) {
                const int r = lv.first + (by_record ? x / ctx->tiles : x % lv.second);
                const int t = by_record ? x % ctx->tiles : x / lv.second;
                ctx->qitems.push_back(r);
                ctx->qitems.push_back(t);
            }
        }
        if (pass == 0) ctx->q_post = static_cast<int>(ctx->qitems.size() / 2);
    }
    ctx->q_blocks = N - 1;
}

// Devices already checked to be gfx950 (bit per ordinal < 64).
std::atomic<uint64_t> g_verified{0};

phg_status ensure_device(phg_context* ctx) {
    if (ctx->dev_init) {
        PHG_HIP(ctx, hipSetDevice(ctx->device));
        return PHG_OK;
    }
    const uint64_t bit = ctx->device < 64 ? (uint64_t{1} << ctx->device) : 0;
    if (!(bit && (g_verified.load() & bit))) {
        int count = 0;
        hipError_t e = hipGetDeviceCount(&count);
        if (e != hipSuccess || count == 0)
            return ctx->fail(PHG_ERR_DEVICE, "no HIP device available (%s)", hipGetErrorString(e));
        if (ctx->device >= count)
            return ctx->fail(PHG_ERR_DEVICE, "device %d out of range (%d devices)", ctx->device, count);
        PHG_HIP(ctx, hipSetDevice(ctx->device));
        hipDeviceProp_t prop;
        PHG_HIP(ctx, hipGetDeviceProperties(&prop, ctx->device));
        if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
            return ctx->fail(PHG_ERR_DEVICE, "device %d is %s; this library is built for gfx950 only",
                             ctx->device, prop.gcnArchName);
        g_verified.fetch_or(bit);
    }
    PHG_HIP(ctx, hipSetDevice(ctx->device));
    if (!kernels_support(ctx->S, ctx->R))
        return ctx->fail(PHG_ERR_ARG, "no kernel for S=%d, R=%d in this build", ctx->S, ctx->R);

    ctx->table_slots = table_slots_for(ctx->N, ctx->S, ctx->R, ctx->prec, ctx->table_budget);
    ctx->plan = make_plan(ctx->N, ctx->C, ctx->S, ctx->R, ctx->prec, ctx->table_slots);
    if (ctx->bound_ws) {
        if (ctx->bound_ws_bytes < ctx->plan.total)
            return ctx->fail(PHG_ERR_OOM, "bound workspace has %zu bytes, %zu needed",
                             ctx->bound_ws_bytes, ctx->plan.total);
        ctx->arena = ctx->bound_ws;
        ctx->own_arena = false;
    } else {
        void* p = nullptr;
        const hipError_t e = hipMalloc(&p, ctx->plan.total);
        if (e != hipSuccess)
            return ctx->fail(PHG_ERR_OOM, "hipMalloc(%zu) failed: %s", ctx->plan.total,
                             hipGetErrorString(e));
        ctx->arena = static_cast<char*>(p);
        ctx->own_arena = true;
    }
    if (!ctx->stream) {
        PHG_HIP(ctx, hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking));
        ctx->own_stream = true;
    }
    const Plan& pl = ctx->plan;
    char* a = ctx->arena;
    ReqDesc& d = ctx->rd;
    d = ReqDesc{};
    d.N = ctx->N;
    d.C = ctx->C;
    d.Cpad = ctx->Cpad;
    d.S = ctx->S;
    d.S4 = ctx->S4;
    d.R = ctx->R;
    d.tiles = ctx->tiles;
    d.fp32 = ctx->prec == PHG_FP32_SCALED ? 1 : 0;
    d.blocked = ctx->blocked ? 1 : 0;
    d.eig_cat = ctx->eig_cat ? 1 : 0;
    d.level_tables = ctx->table_slots > 0 ? 1 : 0;
    d.sched = reinterpret_cast<const NodeTriple*>(a + pl.sched);
    d.kids = reinterpret_cast<const int32_t*>(a + pl.ch_kids);
    d.codes = reinterpret_cast<const uint8_t*>(a + pl.codes);
    d.part = a + pl.part;
    d.expo = reinterpret_cast<int32_t*>(a + pl.expo);
    d.eloc = reinterpret_cast<int32_t*>(a + pl.eloc);
    d.P64 = reinterpret_cast<double*>(a + pl.P64);
    d.dP64 = reinterpret_cast<double*>(a + pl.dP64);
    d.P32 = reinterpret_cast<float*>(a + pl.P32);
    d.dP32 = reinterpret_cast<float*>(a + pl.dP32);
    d.PB32 = reinterpret_cast<float*>(a + pl.PB32);
    d.PB64 = reinterpret_cast<double*>(a + pl.PB64);
    d.dPB32 = reinterpret_cast<float*>(a + pl.dPB32);
    d.dPB64 = reinterpret_cast<double*>(a + pl.dPB64);
    d.vsum = reinterpret_cast<const double*>(a + pl.vsum);
    d.TT64 = reinterpret_cast<double*>(a + pl.TT64);
    d.dTT64 = reinterpret_cast<double*>(a + pl.dTT64);
    d.TT32 = reinterpret_cast<float*>(a + pl.TT32);
    d.dTT32 = reinterpret_cast<float*>(a + pl.dTT32);
    d.b = reinterpret_cast<const double*>(a + pl.b);
    d.V = reinterpret_cast<const double*>(a + pl.V);
    d.Vinv = reinterpret_cast<const double*>(a + pl.Vinv);
    d.lam = reinterpret_cast<const double*>(a + pl.lam);
    d.rates = reinterpret_cast<const double*>(a + pl.rates);
    d.cweights = reinterpret_cast<const double*>(a + pl.cw);
    d.pi = reinterpret_cast<const double*>(a + pl.pi);
    d.pw = reinterpret_cast<const double*>(a + pl.pw);
    d.sll = reinterpret_cast<double*>(a + pl.sll);
    d.lpart = reinterpret_cast<double*>(a + pl.lpart);
    d.gpart = reinterpret_cast<double*>(a + pl.gpart);
    PHG_HIP(ctx, hipMemcpyAsync(a + pl.desc, &ctx->rd, sizeof(ReqDesc), hipMemcpyHostToDevice,
                                ctx->stream));
    ctx->dev_init = true;
    ctx->dirty = ctx->have | kPw;  // upload everything on first use
    return PHG_OK;
}

// General tip partial vectors in the partials layout of the level kernel
// family that (S, R) runs on, one slot per tip with such a vector, every
// category (the vector does not depend on it); padding patterns are
// all-ones like code S, padding states zero.
template <typename T>
void pack_tip_vectors(const phg_context* ctx, std::vector<T>& out, std::vector<int32_t>& tslot) {
    const int N = ctx->N, C = ctx->C, S = ctx->S, R = ctx->R, Cpad = ctx->Cpad, tiles = ctx->tiles;
    const bool fp32 = ctx->prec == PHG_FP32_SCALED;
    const size_t G = ctx->tip_vectors.size();
    tslot.assign(N, -1);
    auto value = [&](const std::vector<double>& v, int c, int s) { return c < C ? v[static_cast<size_t>(c) * S + s] : 1.0; };
    if (uses_s4_kernels(S, R)) {
        // [slot][tile][R][64 lanes][4 states]
        const size_t per = static_cast<size_t>(tiles) * R * kLanes * 4;
        out.assign(G * per, T(0));
        int gslot = 0;
        for (const auto& kv : ctx->tip_vectors) {
            tslot[kv.first] = gslot;
            for (int c = 0; c < Cpad; ++c)
                for (int r = 0; r < R; ++r)
                    for (int st = 0; st < 4; ++st)
                        out[((static_cast<size_t>(gslot) * tiles + c / kLanes) * R + r) * kLanes * 4 +
                            (c % kLanes) * 4 + st] = static_cast<T>(value(kv.second, c, st));
            ++gslot;
        }
    } else if (uses_vs_kernels(S, R, fp32)) {
        // [slot][tile][R][SP][64]
        const int SP = vs_padded_states(S);
        const size_t per = static_cast<size_t>(tiles) * R * SP * kLanes;
        out.assign(G * per, T(0));
        int gslot = 0;
        for (const auto& kv : ctx->tip_vectors) {
            tslot[kv.first] = gslot;
            for (int c = 0; c < Cpad; ++c)
                for (int r = 0; r < R; ++r)
                    for (int st = 0; st < S; ++st)
                        out[(((static_cast<size_t>(gslot) * tiles + c / kLanes) * R + r) * SP + st) * kLanes +
                            c % kLanes] = static_cast<T>(value(kv.second, c, st));
            ++gslot;
        }
    } else if (uses_gl_kernels(S, R, fp32)) {
        // [slot][tile][R][TP][row], state t at column gl_col(t)
        const int TP = Cpad / tiles, row = gl_row(S), kbp = gl_kbp(S);
        const size_t per = static_cast<size_t>(tiles) * R * TP * row;
        out.assign(G * per, T(0));
        int gslot = 0;
        for (const auto& kv : ctx->tip_vectors) {
            tslot[kv.first] = gslot;
            for (int c = 0; c < Cpad; ++c)
                for (int r = 0; r < R; ++r)
                    for (int st = 0; st < S; ++st)
                        out[(((static_cast<size_t>(gslot) * tiles + c / TP) * R + r) * TP + c % TP) * row +
                            gl_col(st, kbp)] = static_cast<T>(value(kv.second, c, st));
            ++gslot;
        }
    } else {
        // [slot][tile][R][S][TP]
        const int TP = gs_tile_patterns(fp32);
        const size_t per = static_cast<size_t>(tiles) * R * S * TP;
        out.assign(G * per, T(0));
        int gslot = 0;
        for (const auto& kv : ctx->tip_vectors) {
            tslot[kv.first] = gslot;
            for (int c = 0; c < Cpad; ++c)
                for (int r = 0; r < R; ++r)
                    for (int st = 0; st < S; ++st)
                        out[(((static_cast<size_t>(gslot) * tiles + c / TP) * R + r) * S + st) * TP + c % TP] =
                            static_cast<T>(value(kv.second, c, st));
            ++gslot;
        }
    }
}

void free_tip_vectors(phg_context* ctx) {
    if (ctx->d_tipvec) (void)hipFree(ctx->d_tipvec);
    if (ctx->d_tslot) (void)hipFree(ctx->d_tslot);
    ctx->d_tipvec = nullptr;
    ctx->d_tslot = nullptr;
    ctx->d_tipvec_bytes = 0;
    ctx->rd.tslot = nullptr;
    ctx->rd.tipvec = nullptr;
}

phg_status upload_tip_vectors(phg_context* ctx) {
    if (ctx->tip_vectors.empty()) {
        free_tip_vectors(ctx);
        return PHG_OK;
    }
    std::vector<int32_t> tslot;
    std::vector<float> v32;
    std::vector<double> v64;
    const bool fp32 = ctx->prec == PHG_FP32_SCALED;
    if (fp32)
        pack_tip_vectors<float>(ctx, v32, tslot);
    else
        pack_tip_vectors<double>(ctx, v64, tslot);
    const void* src = fp32 ? static_cast<const void*>(v32.data()) : static_cast<const void*>(v64.data());
    const size_t bytes = fp32 ? v32.size() * sizeof(float) : v64.size() * sizeof(double);
    if (bytes != ctx->d_tipvec_bytes || !ctx->d_tslot) {
        free_tip_vectors(ctx);
        PHG_HIP(ctx, hipMalloc(&ctx->d_tipvec, bytes));
        ctx->d_tipvec_bytes = bytes;
        void* ts = nullptr;
        PHG_HIP(ctx, hipMalloc(&ts, static_cast<size_t>(ctx->N) * sizeof(int32_t)));
        ctx->d_tslot = static_cast<int32_t*>(ts);
    }
    PHG_HIP(ctx, hipMemcpyAsync(ctx->d_tipvec, src, bytes, hipMemcpyHostToDevice, ctx->stream));
    PHG_HIP(ctx, hipMemcpyAsync(ctx->d_tslot, tslot.data(), tslot.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                                ctx->stream));
    // the sources are pageable locals: finish the copies before they go
    PHG_HIP(ctx, hipStreamSynchronize(ctx->stream));
    ctx->rd.tslot = ctx->d_tslot;
    ctx->rd.tipvec = ctx->d_tipvec;
    return PHG_OK;
}

phg_status upload(phg_context* ctx) {
    const Plan& pl = ctx->plan;
    char* a = ctx->arena;
    hipStream_t st = ctx->stream;
    const unsigned dirty = ctx->dirty;
    // a new schedule or descriptor changes the launch sequence
    if (dirty & (kTopo | kTipVec | kDesc)) ctx_drop_graphs(ctx);
    auto put = [&](size_t off, const void* src, size_t bytes) {
        return hipMemcpyAsync(a + off, src, bytes, hipMemcpyHostToDevice, st);
    };
    if (dirty & kTipVec) PHG_TRY(upload_tip_vectors(ctx));
    std::vector<uint32_t> zeros;
    if ((dirty & kTopo) && ctx->queue) {
        // completion marks and counters start at zero (epoch 0: the first
        // evaluation's marks are 1); the marks of another topology would not
        // match its records
        const size_t marks = static_cast<size_t>(2) * ctx->q_blocks * ctx->tiles;
        zeros.assign(std::max<size_t>(marks, kQueueWords), 0u);
        PHG_HIP(ctx, put(pl.qitems, ctx->qitems.data(), ctx->qitems.size() * sizeof(int32_t)));
        PHG_HIP(ctx, put(pl.qdep, ctx->qdep.data(), ctx->qdep.size() * sizeof(int32_t)));
        PHG_HIP(ctx, put(pl.qdone, zeros.data(), marks * sizeof(uint32_t)));
        PHG_HIP(ctx, put(pl.qctr, zeros.data(), kQueueWords * sizeof(uint32_t)));
    }
    if (dirty & kTopo) {
        PHG_HIP(ctx, put(pl.sched, ctx->sched.data(), ctx->sched.size() * sizeof(int32_t)));
        PHG_HIP(ctx, put(pl.ch_parent, ctx->parent.data(), ctx->parent.size() * sizeof(int32_t)));
        PHG_HIP(ctx, put(pl.ch_kids, ctx->kids.data(), ctx->kids.size() * sizeof(int32_t)));
    }
    if (dirty & (kTopo | kDesc | kTipVec)) {
        ctx->rd.blocked = ctx->blocked ? 1 : 0;
        ctx->rd.qctr = ctx->queue ? reinterpret_cast<uint32_t*>(a + pl.qctr) : nullptr;
        ctx->rd.eig_cat = ctx->eig_cat ? 1 : 0;
        PHG_HIP(ctx, put(pl.desc, &ctx->rd, sizeof(ReqDesc)));
    }
    if (dirty & kB) PHG_HIP(ctx, put(pl.b, ctx->b.data(), ctx->b.size() * 8));
    if (dirty & kEig) {
        // row sums of Vinv, per model: P 1 = V diag(e) (Vinv 1)
        const size_t S = ctx->S, models = ctx->Vinv.size() / (S * S);
        ctx->vsum.assign(models * S, 0.0);
        for (size_t m = 0; m < models; ++m)
            for (size_t k = 0; k < S; ++k) {
                double acc = 0.0;
                for (size_t t = 0; t < S; ++t) acc += ctx->Vinv[(m * S + k) * S + t];
                ctx->vsum[m * S + k] = acc;
            }
        PHG_HIP(ctx, put(pl.vsum, ctx->vsum.data(), ctx->vsum.size() * 8));
        PHG_HIP(ctx, put(pl.V, ctx->V.data(), ctx->V.size() * 8));
        PHG_HIP(ctx, put(pl.Vinv, ctx->Vinv.data(), ctx->Vinv.size() * 8));
        PHG_HIP(ctx, put(pl.lam, ctx->lam.data(), ctx->lam.size() * 8));
    }
    if (dirty & kPi) PHG_HIP(ctx, put(pl.pi, ctx->pi.data(), ctx->pi.size() * 8));
    if (dirty & kCat) {
        PHG_HIP(ctx, put(pl.rates, ctx->rates.data(), ctx->rates.size() * 8));
        PHG_HIP(ctx, put(pl.cw, ctx->cw.data(), ctx->cw.size() * 8));
    }
    if (dirty & kTips) PHG_HIP(ctx, put(pl.codes, ctx->codes.data(), ctx->codes.size()));
    if (dirty & kPw) PHG_HIP(ctx, put(pl.pw, ctx->pw.data(), ctx->pw.size() * 8));
    if ((dirty & kTime) && !ctx->heights.empty()) {
        PHG_HIP(ctx, put(pl.heights, ctx->heights.data(), ctx->heights.size() * 8));
        PHG_HIP(ctx, put(pl.trates, ctx->trates.data(), ctx->trates.size() * 8));
    }
    if ((dirty & kSets) && ctx->n_sets > 0) {
        PHG_HIP(ctx, put(pl.set_ptr, ctx->set_ptr.data(), ctx->set_ptr.size() * sizeof(int32_t)));
        PHG_HIP(ctx, put(pl.set_idx, ctx->set_idx.data(), ctx->set_idx.size() * sizeof(int32_t)));
    }
    // pageable sources: make sure the copies have consumed them before the
    // host mirrors can change again
    if (dirty) PHG_HIP(ctx, hipStreamSynchronize(st));
    ctx->dirty = 0;
    return PHG_OK;
}

// Record the next profiling event of the current evaluation (no-op when off).
phg_status prof_mark(phg_context* ctx) {
    if (!ctx->prof_on) return PHG_OK;
    if (ctx->prof_used == ctx->prof_pool.size()) {
        hipEvent_t ev;
        PHG_HIP(ctx, hipEventCreate(&ev));
        ctx->prof_pool.push_back(ev);
    }
    PHG_HIP(ctx, hipEventRecord(ctx->prof_pool[ctx->prof_used++], ctx->stream));
    return PHG_OK;
}

SegTable one_segment(const ReqDesc& d, int units, int sched_off, int n_nodes, int flags, double* out_logl,
                     double* out_grad) {
    SegTable t{};
    t.n = 1;
    t.unit_begin[0] = 0;
    t.unit_begin[1] = units;
    t.seg[0] = Segment{0, sched_off, n_nodes, flags, reinterpret_cast<const int32_t*>(d.sched), out_logl, out_grad};
    return t;
}

}  // namespace

namespace phg {

int tuned_value(int S, int R, bool fp32, int param) {
    std::call_once(g_tune_once, tune_load_file);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(TuneKey{S, R, fp32 ? 1 : 0, param});
    if (it == g_tune.end()) it = g_tune.find(TuneKey{S, 0, fp32 ? 1 : 0, param});
    return it == g_tune.end() ? 0 : it->second;
}

// The wait bound of a work item in ticks of the device's constant clock:
// kQueueWaitMs, or the tuned microseconds.
uint64_t queue_wait_ticks(int device, int S, int R, bool fp32) {
    static std::atomic<int> khz[64];
    const int dev = device >= 0 && device < 64 ? device : 0;
    int rate = khz[dev].load();
    if (rate <= 0) {
        if (hipDeviceGetAttribute(&rate, hipDeviceAttributeWallClockRate, device) != hipSuccess || rate <= 0)
            rate = 100000;                                   // 100 MHz
        khz[dev].store(rate);
    }
    const int us = tuned_value(S, R, fp32, PHG_TUNE_QUEUE_WAIT_US);
    return us > 0 ? std::max<uint64_t>(1, static_cast<uint64_t>(rate) * us / 1000)
                  : static_cast<uint64_t>(rate) * kQueueWaitMs;
}

int queue_launches(int S, int R, bool fp32) {
    const int v = tuned_value(S, R, fp32, PHG_TUNE_QUEUE_LAUNCHES);
    return v > 0 ? v : kQueueLaunchesDefault;
}

// One level's launches: the level kernel over its records [a, a + n), or,
// with per-chunk P(t) tables, chunks of at most table_slots / 2 nodes, each
// a P(t) launch building its children's tables and then the level kernel.
phg_status enqueue_level(phg_context* ctx, KernelClass k, int a, int n, int flags) {
    hipStream_t st = ctx->stream;
    const ReqDesc& d = ctx->rd;
    const ReqDesc* descs = ctx_desc_dev(ctx);
    const int chunk = ctx->table_slots > 0 ? ctx->table_slots / 2 : n;
    for (int c0 = 0; c0 < n; c0 += chunk) {
        const int m = std::min(chunk, n - c0);
        if (ctx->table_slots > 0)
            PHG_HIP(ctx, launch_class(kPmat, d, descs, one_segment(d, 2 * m * d.R, a + c0, m, 2, nullptr, nullptr),
                                      st));
        PHG_HIP(ctx, launch_class(k, d, descs, one_segment(d, units_for(k, d, m), a + c0, m, flags, nullptr, nullptr),
                                  st));
    }
    return PHG_OK;
}

phg_status ctx_enqueue_eval(phg_context* ctx, double* d_logl, double* d_grad) {
    hipStream_t st = ctx->stream;
    const ReqDesc& d = ctx->rd;
    const ReqDesc* descs = ctx_desc_dev(ctx);
    PHG_TRY(prof_mark(ctx));
    if (ctx->table_slots == 0)
        PHG_HIP(ctx, launch_class(kPmat, d, descs, one_segment(d, units_for(kPmat, d, 0), 0, 0, 0, nullptr, nullptr),
                                  st));
    PHG_TRY(prof_mark(ctx));
    if (ctx->queue) {
        // work-queue traversal: both passes in one launch, or one launch per
        // pass (always while profiling, so the classes keep their times)
        char* a = ctx->arena;
        const Plan& pl = ctx->plan;
        QueueArgs q{};
        q.items = reinterpret_cast<const int32_t*>(a + pl.qitems);
        q.dep = reinterpret_cast<const int32_t*>(a + pl.qdep);
        q.done = reinterpret_cast<uint32_t*>(a + pl.qdone);
        q.ctr = reinterpret_cast<uint32_t*>(a + pl.qctr);
        q.n_blocks = ctx->q_blocks;
        q.root_rec = ctx->pre_lv.front().first;
        q.wait_ticks = queue_wait_ticks(ctx->device, d.S, d.R, d.fp32 != 0);
        const int n_items = static_cast<int>(ctx->qitems.size() / 2);
        const bool one_launch =
            d_grad && !ctx->prof_on && d.S == 4 && queue_launches(d.S, d.R, d.fp32 != 0) == 1;
        q.t0 = 0;
        q.t1 = one_launch ? n_items : ctx->q_post;
        PHG_HIP(ctx, launch_queue(d, descs, q, one_launch ? 3 : 1, st));
        PHG_TRY(prof_mark(ctx));
        if (d_grad && !one_launch) {
            q.t0 = ctx->q_post;
            q.t1 = n_items;
            PHG_HIP(ctx, launch_queue(d, descs, q, 2, st));
        }
    } else {
        const int H = static_cast<int>(ctx->post_lv.size());
        for (int h = 0; h < H; ++h)
            PHG_TRY(enqueue_level(ctx, kPost, ctx->post_lv[h].first, ctx->post_lv[h].second, h == H - 1 ? 1 : 0));
        PHG_TRY(prof_mark(ctx));
        if (d_grad) {
            for (const auto& lv : ctx->pre_lv) PHG_TRY(enqueue_level(ctx, kPre, lv.first, lv.second, 0));
        }
    }
    PHG_TRY(prof_mark(ctx));
    // without d_grad: log-likelihood only (no pre-order pass; one final unit)
    PHG_HIP(ctx, launch_class(kFinal, d, descs,
                              d_grad ? one_segment(d, units_for(kFinal, d, 0), 0, 0, 0, d_logl, d_grad)
                                     : one_segment(d, 1, 0, 0, 1, d_logl, nullptr),
                              st));
    PHG_TRY(prof_mark(ctx));
    return PHG_OK;
}

void ctx_drop_graphs(phg_context* ctx) {
    for (hipGraphExec_t& g : ctx->graph_exec) {
        if (g) (void)hipGraphExecDestroy(g);
        g = nullptr;
    }
}

void ctx_drop_device(phg_context* ctx) {
    if (!ctx->dev_init) return;
    ctx_drop_graphs(ctx);
    free_tip_vectors(ctx);
    if (ctx->own_arena && ctx->arena) (void)hipFree(ctx->arena);
    if (ctx->host_out) (void)hipHostFree(ctx->host_out);
    ctx->host_out = nullptr;
    ctx->arena = nullptr;
    ctx->own_arena = false;
    ctx->bound_ws = nullptr;
    ctx->bound_ws_bytes = 0;
    ctx->dev_init = false;
    ctx->dirty = ctx->have;
}

phg_status ctx_host_out(phg_context* ctx) {
    if (ctx->host_out) return PHG_OK;
    void* ho = nullptr;
    PHG_HIP(ctx, hipHostMalloc(&ho, out_doubles(ctx->N) * sizeof(double), hipHostMallocDefault));
    ctx->host_out = static_cast<double*>(ho);
    return PHG_OK;
}

ReqDesc* ctx_desc_dev(phg_context* ctx) { return reinterpret_cast<ReqDesc*>(ctx->arena + ctx->plan.desc); }
double* ctx_out_dev(phg_context* ctx) { return reinterpret_cast<double*>(ctx->arena + ctx->plan.out); }

phg_status ctx_ready(phg_context* ctx) {
    if ((ctx->have & kRequired) != kRequired) {
        std::string miss;
        if (!(ctx->have & kTopo)) miss += " topology";
        if (!(ctx->have & kB)) miss += " branch_lengths";
        if (!(ctx->have & kEig)) miss += " eigen";
        if (!(ctx->have & kPi)) miss += " root_frequencies";
        if (!(ctx->have & kCat)) miss += " categories";
        if (!(ctx->have & kTips)) miss += " tip_states";
        return ctx->fail(PHG_ERR_STATE, "inputs not set:%s", miss.c_str());
    }
    phg_status s = ensure_device(ctx);
    if (s != PHG_OK) return s;
    // a context in the shared static array uploads everything again when
    // another context used the array since its last evaluation
    if (ctx->static_ws && scratch_claim(ctx)) ctx->dirty |= ctx->have | kPw | kTopo | kDesc;
    return upload(ctx);
}

double fp32_saturation(const phg_context* ctx) {
    const int N = ctx->N, n = 2 * N - 1, root = n - 1, S = ctx->S, R = ctx->R;
    // fastest category's slowest decay: max_r gamma_r * mu_r, mu_r the
    // smallest |lambda| of category r once its zero eigenvalue is dropped
    double rate = 0.0;
    for (int r = 0; r < R; ++r) {
        const double* lam = ctx->lam.data() + (ctx->eig_cat ? static_cast<size_t>(r) * S : 0);
        int i0 = 0;
        double big = 0.0;
        for (int s = 0; s < S; ++s) {
            big = std::max(big, std::fabs(lam[s]));
            if (std::fabs(lam[s]) < std::fabs(lam[i0])) i0 = s;
        }
        const bool zero = std::fabs(lam[i0]) <= 1e-9 * big;
        double mu = std::numeric_limits<double>::infinity();
        for (int s = 0; s < S; ++s)
            if (!(zero && s == i0)) mu = std::min(mu, std::fabs(lam[s]));
        if (std::isfinite(mu)) rate = std::max(rate, ctx->rates[r] * mu);
    }
    auto L = [&](int v) { return v == root ? std::numeric_limits<double>::infinity() : ctx->b[v] * rate; };
    double stat = 0.0;
    for (int k = N; k < n; ++k) {
        const double lk = L(k);
        for (int j = 0; j < 2; ++j) stat = std::max(stat, std::min(lk, L(ctx->kids[2 * (k - N) + j])));
    }
    return stat;
}

phg_context* eval_target(phg_context* ctx, phg_status* st) {
    *st = PHG_OK;
    // a bound workspace means the caller owns every byte: never route then
    const bool route = ctx->prec == PHG_FP32_SCALED && ctx->fp32_guard > 0.0 && !ctx->bound_ws &&
                       (ctx->have & kRequired) == kRequired && fp32_saturation(ctx) > ctx->fp32_guard;
    if (!route) {
        ctx->last_prec = ctx->prec;
        return ctx;
    }
    phg_context* t = ctx->twin;
    if (!t) {
        *st = phg_create(ctx->N, ctx->C, ctx->S, ctx->R, PHG_FP64, ctx->device, &t);
        if (*st != PHG_OK) {
            ctx->fail(*st, "creating the FP64 twin failed: %s", phg_last_error(nullptr));
            return nullptr;
        }
        ctx->twin = t;
        t->table_budget = ctx->table_budget;
        ctx->sdirty = ~0u;
        if (ctx->stream && !ctx->own_stream) t->stream = ctx->stream;   // caller's stream
    }
    const unsigned sd = ctx->sdirty;
    if (sd & (kTopo | kTipVec)) {
        t->parent = ctx->parent;
        t->tip_vectors = ctx->tip_vectors;
        t->sched_mode = ctx->sched_mode;
        if (ctx->have & kTopo) build_schedule(t);
        t->dirty |= kTopo | kTipVec;
    }
    if (sd & kEig) {
        t->V = ctx->V;
        t->Vinv = ctx->Vinv;
        t->lam = ctx->lam;
        t->eig_cat = ctx->eig_cat;
        t->rd.eig_cat = ctx->rd.eig_cat;
        t->dirty |= kEig | kDesc;
    }
    if (sd & kTips) {
        t->codes = ctx->codes;
        t->dirty |= kTips;
    }
    if (sd & kPi) t->pi = ctx->pi;
    if (sd & kCat) {
        t->rates = ctx->rates;
        t->cw = ctx->cw;
    }
    if (sd & kPw) t->pw = ctx->pw;
    t->dirty |= sd & (kPi | kCat | kPw);
    // small per-evaluation inputs: copied every time
    t->b = ctx->b;
    t->heights = ctx->heights;
    t->trates = ctx->trates;
    t->set_ptr = ctx->set_ptr;
    t->set_idx = ctx->set_idx;
    t->n_sets = ctx->n_sets;
    t->dirty |= kB | kTime | kSets;
    t->have = ctx->have;
    t->prof_on = ctx->prof_on;
    t->graph_on = ctx->graph_on;
    ctx->sdirty = 0;
    ctx->last_prec = PHG_FP64;
    return t;
}

phg_status from_twin(phg_context* ctx, phg_context* t, phg_status s) {
    if (s != PHG_OK && t != ctx) ctx->err = t->err;
    return s;
}

// Kernel launches of one gradient evaluation per profiling class; with
// per-chunk P(t) tables the P(t) launches run inside the level classes.
void launches_per_class(phg_context* ctx, int* out) {
    const int slots = ctx->dev_init ? ctx->table_slots
                                    : table_slots_for(ctx->N, ctx->S, ctx->R, ctx->prec, ctx->table_budget);
    auto count = [&](const std::vector<std::pair<int, int>>& lv) {
        int c = 0;
        for (const auto& l : lv) c += slots > 0 ? 2 * ((l.second + slots / 2 - 1) / (slots / 2)) : 1;
        return c;
    };
    out[PHG_PROF_PMAT] = slots > 0 ? 0 : 1;
    // the work-queue traversal: one launch per pass (profiled evaluations)
    out[PHG_PROF_POST] = ctx->queue ? 1 : count(ctx->post_lv);
    out[PHG_PROF_PRE] = ctx->queue ? 1 : count(ctx->pre_lv);
    out[PHG_PROF_FINAL] = 1;
}

}  // namespace phg

extern "C" {

phg_status phg_create(int n_tips, int n_patterns, int n_states, int n_categories,
                      phg_precision prec, int device, phg_context** out) {
    if (!out) {
        g_create_error = "out is NULL";
        return PHG_ERR_ARG;
    }
    *out = nullptr;
    std::string why;
    phg_status s = check_sizes(n_tips, n_patterns, n_states, n_categories, prec, &why);
    if (s != PHG_OK) {
        g_create_error = why;
        return s;
    }
    if (device < 0) {
        g_create_error = "device must be >= 0";
        return PHG_ERR_ARG;
    }
    phg_context* ctx = new (std::nothrow) phg_context();
    if (!ctx) {
        g_create_error = "host allocation failed";
        return PHG_ERR_OOM;
    }
    ctx->N = n_tips;
    ctx->C = n_patterns;
    ctx->S = n_states;
    ctx->R = n_categories;
    ctx->prec = prec;
    ctx->device = device;
    ctx->Cpad = (n_patterns + phg::kLanes - 1) / phg::kLanes * phg::kLanes;
    ctx->tiles = ctx->Cpad / phg::tile_patterns(n_states, n_categories, prec == PHG_FP32_SCALED);
    ctx->S4 = (n_states + 3) / 4;
    static std::atomic<uint64_t> next_uid{1};
    ctx->uid = next_uid.fetch_add(1);
    ctx->pw.assign(ctx->Cpad, 0.0);
    std::fill(ctx->pw.begin(), ctx->pw.begin() + n_patterns, 1.0);
    ctx->codes.assign(static_cast<size_t>(n_tips) * ctx->Cpad * code_bytes(n_states), 0);
    for (size_t i = 0; i < static_cast<size_t>(n_tips) * ctx->Cpad; ++i) put_code(ctx, i, n_states);
    ctx->have = kPw;
    g_create_error.clear();
    *out = ctx;
    return PHG_OK;
}

phg_status phg_destroy(phg_context* ctx) {
    if (!ctx) return PHG_OK;
    phg_destroy(ctx->twin);
    if (ctx->dev_init) {
        (void)hipSetDevice(ctx->device);
        if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
        ctx_drop_graphs(ctx);
        for (hipEvent_t ev : ctx->prof_pool) (void)hipEventDestroy(ev);
        free_tip_vectors(ctx);
        if (ctx->own_arena && ctx->arena) (void)hipFree(ctx->arena);
        if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
        if (ctx->host_out) (void)hipHostFree(ctx->host_out);
    }
    delete ctx;
    return PHG_OK;
}

const char* phg_last_error(const phg_context* ctx) {
    return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

phg_status phg_set_topology(phg_context* ctx, const int32_t* parent) {
    if (!ctx) return PHG_ERR_ARG;
    if (!parent) return ctx->fail(PHG_ERR_ARG, "parent is NULL");
    const int N = ctx->N, n = 2 * N - 1, root = n - 1;
    if (parent[root] != -1) return ctx->fail(PHG_ERR_ARG, "parent[root=%d] must be -1", root);
    std::vector<int> nkids(n, 0);
    for (int v = 0; v < root; ++v) {
        const int p = parent[v];
        if (p < N || p > root)
            return ctx->fail(PHG_ERR_ARG, "parent[%d]=%d is not an internal node or the root", v, p);
        nkids[p]++;
    }
    for (int v = N; v < n; ++v)
        if (nkids[v] != 2)
            return ctx->fail(PHG_ERR_ARG, "node %d has %d children (need exactly 2)", v, nkids[v]);
    // acyclic: every node must reach the root within n steps
    std::vector<char> ok(n, 0);
    ok[root] = 1;
    for (int v = 0; v < root; ++v) {
        int x = v, steps = 0;
        std::vector<int> path;
        while (!ok[x]) {
            path.push_back(x);
            x = parent[x];
            if (++steps > n) return ctx->fail(PHG_ERR_ARG, "topology has a cycle through node %d", v);
        }
        for (int y : path) ok[y] = 1;
    }
    ctx->parent.assign(parent, parent + n);
    build_schedule(ctx);
    ctx->have |= kTopo;
    ctx->dirty |= kTopo;
    ctx->sdirty |= kTopo;
    ctx->have &= ~kTime;     // heights must be set again for a new topology
    return PHG_OK;
}

phg_status phg_set_branch_lengths(phg_context* ctx, const double* b) {
    if (!ctx) return PHG_ERR_ARG;
    if (!b) return ctx->fail(PHG_ERR_ARG, "b is NULL");
    const size_t E = 2 * static_cast<size_t>(ctx->N) - 2;
    for (size_t x = 0; x < E; ++x)
        if (!std::isfinite(b[x]) || b[x] < 0.0)
            return ctx->fail(PHG_ERR_ARG, "branch length b[%zu]=%g must be finite and >= 0", x, b[x]);
    ctx->b.assign(b, b + E);
    ctx->have |= kB;
    ctx->dirty |= kB;
    ctx->sdirty |= kB;
    ctx->have &= ~kTime;     // lengths no longer come from a time tree
    return PHG_OK;
}

namespace {
phg_status set_eig(phg_context* ctx, const double* V, const double* Vinv, const double* lambda, size_t models) {
    if (!ctx) return PHG_ERR_ARG;
    if (!V || !Vinv || !lambda) return ctx->fail(PHG_ERR_ARG, "NULL eigensystem array");
    const size_t S = ctx->S;
    if (!finite_all(V, models * S * S) || !finite_all(Vinv, models * S * S) || !finite_all(lambda, models * S))
        return ctx->fail(PHG_ERR_ARG, "eigensystem has non-finite entries");
    ctx->V.assign(V, V + models * S * S);
    ctx->Vinv.assign(Vinv, Vinv + models * S * S);
    ctx->lam.assign(lambda, lambda + models * S);
    ctx->eig_cat = models > 1;
    ctx->rd.eig_cat = ctx->eig_cat ? 1 : 0;
    ctx->have |= kEig;
    ctx->dirty |= kEig | kDesc;
    ctx->sdirty |= kEig | kDesc;
    return PHG_OK;
}
}  // namespace

phg_status phg_set_eigen(phg_context* ctx, const double* V, const double* Vinv, const double* lambda) {
    return set_eig(ctx, V, Vinv, lambda, 1);
}

phg_status phg_set_category_eigen(phg_context* ctx, const double* V, const double* Vinv, const double* lambda) {
    if (!ctx) return PHG_ERR_ARG;
    return set_eig(ctx, V, Vinv, lambda, static_cast<size_t>(ctx->R));
}

phg_status phg_set_root_frequencies(phg_context* ctx, const double* pi) {
    if (!ctx) return PHG_ERR_ARG;
    if (!pi) return ctx->fail(PHG_ERR_ARG, "pi is NULL");
    for (int s = 0; s < ctx->S; ++s)
        if (!std::isfinite(pi[s]) || pi[s] < 0.0)
            return ctx->fail(PHG_ERR_ARG, "pi[%d]=%g must be finite and >= 0", s, pi[s]);
    ctx->pi.assign(pi, pi + ctx->S);
    ctx->have |= kPi;
    ctx->dirty |= kPi;
    ctx->sdirty |= kPi;
    return PHG_OK;
}

phg_status phg_set_categories(phg_context* ctx, const double* rates, const double* weights) {
    if (!ctx) return PHG_ERR_ARG;
    if (!rates || !weights) return ctx->fail(PHG_ERR_ARG, "NULL category array");
    for (int r = 0; r < ctx->R; ++r) {
        if (!std::isfinite(rates[r]) || rates[r] < 0.0)
            return ctx->fail(PHG_ERR_ARG, "rates[%d]=%g must be finite and >= 0", r, rates[r]);
        if (!std::isfinite(weights[r]) || weights[r] < 0.0)
            return ctx->fail(PHG_ERR_ARG, "weights[%d]=%g must be finite and >= 0", r, weights[r]);
    }
    ctx->rates.assign(rates, rates + ctx->R);
    ctx->cw.assign(weights, weights + ctx->R);
    ctx->have |= kCat;
    ctx->dirty |= kCat;
    ctx->sdirty |= kCat;
    return PHG_OK;
}

phg_status phg_set_tip_states(phg_context* ctx, const int32_t* codes) {
    if (!ctx) return PHG_ERR_ARG;
    if (!codes) return ctx->fail(PHG_ERR_ARG, "codes is NULL");
    const int N = ctx->N, C = ctx->C, S = ctx->S, Cpad = ctx->Cpad;
    // validate and convert tips [t0, t1): branch-free loops (vectorised),
    // spread over threads for large alignments
    auto rows = [&](int t0, int t1, bool* ok) {
        uint32_t bad = 0;
        for (int t = t0; t < t1; ++t) {
            const int32_t* src = codes + static_cast<size_t>(t) * C;
            for (int c = 0; c < C; ++c) bad |= static_cast<uint32_t>(src[c]) > static_cast<uint32_t>(S);
        }
        *ok = bad == 0;
        if (bad) return;
        for (int t = t0; t < t1; ++t) {
            const int32_t* src = codes + static_cast<size_t>(t) * C;
            if (code_bytes(S) == 1) {
                uint8_t* dst = ctx->codes.data() + static_cast<size_t>(t) * Cpad;
                for (int c = 0; c < C; ++c) dst[c] = static_cast<uint8_t>(src[c]);
            } else {
                for (int c = 0; c < C; ++c) put_code(ctx, static_cast<size_t>(t) * Cpad + c, src[c]);
            }
        }
    };
    const size_t total = static_cast<size_t>(N) * C;
    const int nt = total >= (size_t{1} << 22) ? std::min(8, N) : 1;
    std::vector<char> ok(nt, 0);
    {
        std::vector<std::thread> th;
        for (int k = 1; k < nt; ++k)
            th.emplace_back(rows, N * k / nt, N * (k + 1) / nt, reinterpret_cast<bool*>(&ok[k]));
        rows(0, N / nt, reinterpret_cast<bool*>(&ok[0]));
        for (auto& x : th) x.join();
    }
    for (int k = 0; k < nt; ++k) {
        if (ok[k]) continue;
        for (size_t i = 0; i < total; ++i)        // report the first bad entry
            if (codes[i] < 0 || codes[i] > S)
                return ctx->fail(PHG_ERR_ARG, "tip code %d at tip %zu pattern %zu outside [0, %d]", codes[i],
                                 i / C, i % C, S);
    }
    ctx->have |= kTips;
    ctx->dirty |= kTips;
    ctx->sdirty |= kTips;
    return PHG_OK;
}

phg_status phg_set_tip_partials(phg_context* ctx, int tip, const double* partials) {
    if (!ctx) return PHG_ERR_ARG;
    if (tip < 0 || tip >= ctx->N) return ctx->fail(PHG_ERR_ARG, "tip %d outside [0, %d)", tip, ctx->N);
    if (partials && (ctx->sched_mode == PHG_SCHEDULE_BLOCKS || (ctx->sched_mode == PHG_SCHEDULE_QUEUE && ctx->S == 4)))
        return ctx->fail(PHG_ERR_ARG, "general tip partials need the level schedule (schedule is BLOCKS)");
    const size_t n = static_cast<size_t>(ctx->C) * ctx->S;
    if (partials) {
        for (size_t i = 0; i < n; ++i)
            if (!std::isfinite(partials[i]) || partials[i] < 0.0)
                return ctx->fail(PHG_ERR_ARG, "tip %d partial [%zu][%zu]=%g must be finite and >= 0", tip,
                                 i / ctx->S, i % ctx->S, partials[i]);
        ctx->tip_vectors[tip].assign(partials, partials + n);
    } else {
        ctx->tip_vectors.erase(tip);
    }
    // the schedule depends on whether any tip has a general vector (blocked
    // schedule) and on which tips have one (folded nodes)
    if (ctx->have & kTopo) {
        build_schedule(ctx);
        ctx->dirty |= kTopo;
        ctx->sdirty |= kTopo;
    }
    ctx->have |= kTipVec;
    ctx->dirty |= kTipVec;
    ctx->sdirty |= kTipVec;
    return PHG_OK;
}

phg_status phg_set_pattern_weights(phg_context* ctx, const double* w) {
    if (!ctx) return PHG_ERR_ARG;
    if (!w) return ctx->fail(PHG_ERR_ARG, "w is NULL");
    for (int c = 0; c < ctx->C; ++c)
        if (!std::isfinite(w[c]) || w[c] < 0.0)
            return ctx->fail(PHG_ERR_ARG, "pattern weight w[%d]=%g must be finite and >= 0", c, w[c]);
    std::copy(w, w + ctx->C, ctx->pw.begin());
    ctx->have |= kPw;
    ctx->dirty |= kPw;
    ctx->sdirty |= kPw;
    return PHG_OK;
}

phg_status phg_set_schedule(phg_context* ctx, phg_schedule mode) {
    if (!ctx) return PHG_ERR_ARG;
    if (mode != PHG_SCHEDULE_AUTO && mode != PHG_SCHEDULE_LEVELS && mode != PHG_SCHEDULE_BLOCKS &&
        mode != PHG_SCHEDULE_QUEUE)
        return ctx->fail(PHG_ERR_ARG, "unknown schedule %d", static_cast<int>(mode));
    if (mode == PHG_SCHEDULE_BLOCKS &&
        !phg::blocked_supported(ctx->S, ctx->R, ctx->prec == PHG_FP32_SCALED))
        return ctx->fail(PHG_ERR_ARG, "the blocked schedule needs 4 states and R <= 8");
    if (mode == PHG_SCHEDULE_QUEUE && !phg::queue_supported(ctx->S, ctx->R, ctx->prec == PHG_FP32_SCALED))
        return ctx->fail(PHG_ERR_ARG, "the work-queue traversal needs 4 states with FP32 and R in {1, 2, 4, 8}, "
                                      "or the vector-ALU kernels' shapes");
    if ((mode == PHG_SCHEDULE_BLOCKS || (mode == PHG_SCHEDULE_QUEUE && ctx->S == 4)) && !ctx->tip_vectors.empty())
        return ctx->fail(PHG_ERR_ARG, "the blocked schedule does not take general tip partials");
    ctx->sched_mode = mode;
    if (ctx->have & kTopo) {
        build_schedule(ctx);
        ctx->dirty |= kTopo;
        ctx->sdirty |= kTopo;
    }
    return PHG_OK;
}

phg_status phg_prepare(phg_context* ctx) {
    if (!ctx) return PHG_ERR_ARG;
    phg_status s;
    phg_context* t = eval_target(ctx, &s);
    if (!t) return s;
    return from_twin(ctx, t, ctx_ready(t));
}

namespace {
// One synchronous evaluation on t (the context itself or its FP64 twin);
// grad == nullptr asks for the log-likelihood only.
// The evaluation's launches on t's stream: a replay of the captured graph
// (captured here on first use) or, with graphs off or while profiling, the
// launches themselves.  The graph holds kernel launches only.
phg_status enqueue_graphed(phg_context* t, double* dout, bool with_grad) {
    if (!t->graph_on || t->prof_on) return ctx_enqueue_eval(t, dout, with_grad ? dout + 1 : nullptr);
    hipGraphExec_t& ge = t->graph_exec[with_grad ? 0 : 1];
    if (!ge) {
        PHG_HIP(t, hipStreamBeginCapture(t->stream, hipStreamCaptureModeThreadLocal));
        const phg_status s = ctx_enqueue_eval(t, dout, with_grad ? dout + 1 : nullptr);
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(t->stream, &graph);
        if (s != PHG_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return s;
        }
        if (e != hipSuccess) return t->fail(PHG_ERR_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
        const hipError_t ei = hipGraphInstantiate(&ge, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess) {
            ge = nullptr;
            return t->fail(PHG_ERR_DEVICE, "graph instantiation failed: %s", hipGetErrorString(ei));
        }
        t->graph_captures++;
    } else {
        t->graph_replays++;
    }
    PHG_HIP(t, hipGraphLaunch(ge, t->stream));
    return PHG_OK;
}

phg_status eval_sync(phg_context* t, double* logl, double* grad) {
    phg_status s = ctx_ready(t);
    if (s != PHG_OK) return s;
    PHG_TRY(ctx_host_out(t));
    double* dout = ctx_out_dev(t);
    s = enqueue_graphed(t, dout, grad != nullptr);
    if (s != PHG_OK) return s;
    const size_t E = 2 * static_cast<size_t>(t->N) - 2;
    PHG_HIP(t, hipMemcpyAsync(t->host_out, dout, (grad ? E + 1 : 1) * sizeof(double), hipMemcpyDeviceToHost,
                              t->stream));
    PHG_HIP(t, hipStreamSynchronize(t->stream));
    const double ll = t->host_out[0];
    if (!(ll > -std::numeric_limits<double>::infinity()) || !std::isfinite(ll)) {
        if (logl) *logl = -std::numeric_limits<double>::infinity();
        if (grad)
            for (size_t x = 0; x < E; ++x) grad[x] = std::numeric_limits<double>::quiet_NaN();
        return t->fail(PHG_ERR_NUMERIC, "a weighted site likelihood is zero or not finite");
    }
    if (logl) *logl = ll;
    if (grad) std::memcpy(grad, t->host_out + 1, E * sizeof(double));
    return PHG_OK;
}
}  // namespace

phg_status phg_gradient(phg_context* ctx, double* logl, double* grad) {
    if (!ctx) return PHG_ERR_ARG;
    if (!grad) return ctx->fail(PHG_ERR_ARG, "grad is NULL");
    phg_status s;
    phg_context* t = eval_target(ctx, &s);
    if (!t) return s;
    return from_twin(ctx, t, eval_sync(t, logl, grad));
}

phg_status phg_log_likelihood(phg_context* ctx, double* logl) {
    if (!ctx) return PHG_ERR_ARG;
    if (!logl) return ctx->fail(PHG_ERR_ARG, "logl is NULL");
    phg_status s;
    phg_context* t = eval_target(ctx, &s);
    if (!t) return s;
    return from_twin(ctx, t, eval_sync(t, logl, nullptr));
}

phg_status phg_workspace_size(int n_tips, int n_patterns, int n_states, int n_categories,
                              phg_precision prec, size_t* bytes) {
    std::string why;
    if (!bytes) return PHG_ERR_ARG;
    phg_status s = check_sizes(n_tips, n_patterns, n_states, n_categories, prec, &why);
    if (s != PHG_OK) {
        g_create_error = why;
        return s;
    }
    *bytes = make_plan(n_tips, n_patterns, n_states, n_categories, prec,
                       table_slots_for(n_tips, n_states, n_categories, prec, kDefaultTableBudget))
                 .total;
    return PHG_OK;
}

phg_status phg_kernel_family_of(int n_states, int n_categories, phg_precision prec, int* family) {
    if (!family || (prec != PHG_FP64 && prec != PHG_FP32_SCALED) || !phg::kernels_support(n_states, n_categories))
        return PHG_ERR_ARG;
    const bool fp32 = prec == PHG_FP32_SCALED;
    if (phg::uses_s4_kernels(n_states, n_categories))
        *family = PHG_KERNELS_FOUR_STATE;
    else if (phg::uses_vs_kernels(n_states, n_categories, fp32))
        *family = PHG_KERNELS_VECTOR_ALU;
    else if (phg::uses_gl_kernels(n_states, n_categories, fp32))
        *family = PHG_KERNELS_MFMA;
    else
        *family = PHG_KERNELS_SMALL_MFMA;
    return PHG_OK;
}

phg_status phg_bind_workspace(phg_context* ctx, void* device_ptr, size_t bytes) {
    if (!ctx) return PHG_ERR_ARG;
    if (ctx->dev_init) return ctx->fail(PHG_ERR_STATE, "workspace must be bound before first use");
    if (!device_ptr) return ctx->fail(PHG_ERR_ARG, "device_ptr is NULL");
    if (reinterpret_cast<uintptr_t>(device_ptr) % kAlign != 0)
        return ctx->fail(PHG_ERR_ARG, "workspace must be %zu-byte aligned", kAlign);
    ctx->bound_ws = static_cast<char*>(device_ptr);
    ctx->bound_ws_bytes = bytes;
    return PHG_OK;
}

phg_status phg_bind_stream(phg_context* ctx, void* hip_stream) {
    if (!ctx) return PHG_ERR_ARG;
    if (ctx->twin) PHG_TRY(phg_bind_stream(ctx->twin, hip_stream));
    if (ctx->dev_init && ctx->own_stream && ctx->stream) {
        (void)hipSetDevice(ctx->device);
        (void)hipStreamSynchronize(ctx->stream);
        (void)hipStreamDestroy(ctx->stream);
    }
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    ctx->own_stream = false;
    if (!hip_stream && ctx->dev_init) {
        PHG_HIP(ctx, hipSetDevice(ctx->device));
        PHG_HIP(ctx, hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking));
        ctx->own_stream = true;
    }
    return PHG_OK;
}

phg_status phg_gradient_async(phg_context* ctx, double* d_logl, double* d_grad) {
    if (!ctx) return PHG_ERR_ARG;
    if (!d_logl || !d_grad) return ctx->fail(PHG_ERR_ARG, "NULL device output pointer");
    phg_status s;
    phg_context* t = eval_target(ctx, &s);
    if (!t) return s;
    s = ctx_ready(t);
    if (s == PHG_OK) s = ctx_enqueue_eval(t, d_logl, d_grad);
    return from_twin(ctx, t, s);
}

phg_status phg_set_tuning(int n_states, int n_categories, phg_precision prec, int param, int value) {
    if (n_states < 2 || n_states > 255 || n_categories < 0 || n_categories > 64 ||
        (prec != PHG_FP64 && prec != PHG_FP32_SCALED) || param < 0 || param >= PHG_TUNE_PARAMS) {
        g_create_error = "phg_set_tuning: bad state count, category count, precision or parameter";
        return PHG_ERR_ARG;
    }
    const bool fp32 = prec == PHG_FP32_SCALED;
    if (!tune_value_ok(n_states, n_categories, fp32, param, value)) {
        g_create_error = "phg_set_tuning: value " + std::to_string(value) + " is not built for these sizes";
        return PHG_ERR_ARG;
    }
    std::call_once(g_tune_once, tune_load_file);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const TuneKey key{n_states, n_categories, fp32 ? 1 : 0, param};
    if (value == 0)
        g_tune.erase(key);
    else
        g_tune[key] = value;
    return PHG_OK;
}

phg_status phg_get_tuning(int n_states, int n_categories, phg_precision prec, int param, int* value) {
    if (!value || param < 0 || param >= PHG_TUNE_PARAMS) return PHG_ERR_ARG;
    *value = tuned_value(n_states, n_categories, prec == PHG_FP32_SCALED, param);
    return PHG_OK;
}

phg_status phg_set_table_budget(phg_context* ctx, size_t bytes) {
    if (!ctx) return PHG_ERR_ARG;
    if (ctx->dev_init) return ctx->fail(PHG_ERR_STATE, "the table budget must be set before first use");
    ctx->table_budget = bytes;
    if (ctx->twin) ctx->twin->table_budget = bytes;
    if (ctx->have & kTopo) {   // folded nodes need tables for every branch
        build_schedule(ctx);
        ctx->dirty |= kTopo;
        ctx->sdirty |= kTopo;
    }
    return PHG_OK;
}

phg_status phg_table_slots(phg_context* ctx, int* slots) {
    if (!ctx || !slots) return PHG_ERR_ARG;
    *slots = ctx->dev_init ? ctx->table_slots
                           : table_slots_for(ctx->N, ctx->S, ctx->R, ctx->prec, ctx->table_budget);
    return PHG_OK;
}

phg_status phg_set_graphs(phg_context* ctx, int on) {
    if (!ctx) return PHG_ERR_ARG;
    ctx->graph_on = on != 0;
    if (ctx->twin) ctx->twin->graph_on = ctx->graph_on;
    return PHG_OK;
}

phg_status phg_graph_stats(phg_context* ctx, uint64_t* captures, uint64_t* replays) {
    if (!ctx) return PHG_ERR_ARG;
    const phg_context* t = ctx->twin;
    if (captures) *captures = ctx->graph_captures + (t ? t->graph_captures : 0);
    if (replays) *replays = ctx->graph_replays + (t ? t->graph_replays : 0);
    return PHG_OK;
}

phg_status phg_set_fp32_guard(phg_context* ctx, double threshold) {
    if (!ctx) return PHG_ERR_ARG;
    if (!(threshold >= 0.0)) return ctx->fail(PHG_ERR_ARG, "guard threshold %g must be >= 0", threshold);
    ctx->fp32_guard = threshold;
    return PHG_OK;
}

phg_status phg_fp32_saturation(phg_context* ctx, double* saturation) {
    if (!ctx || !saturation) return PHG_ERR_ARG;
    const unsigned need = kTopo | kB | kEig | kCat;
    if ((ctx->have & need) != need)
        return ctx->fail(PHG_ERR_STATE, "topology, branch lengths, eigensystem and categories must be set");
    *saturation = fp32_saturation(ctx);
    return PHG_OK;
}

phg_status phg_last_precision(phg_context* ctx, int* prec) {
    if (!ctx || !prec) return PHG_ERR_ARG;
    *prec = ctx->last_prec;
    return PHG_OK;
}

phg_status phg_get_schedule(phg_context* ctx, int* schedule) {
    if (!ctx || !schedule) return PHG_ERR_ARG;
    if (!(ctx->have & kTopo)) return ctx->fail(PHG_ERR_STATE, "topology not set");
    *schedule = ctx->queue ? PHG_SCHEDULE_QUEUE : ctx->blocked ? PHG_SCHEDULE_BLOCKS : PHG_SCHEDULE_LEVELS;
    return PHG_OK;
}

phg_status phg_schedule_info(phg_context* ctx, int* n_post_levels, int* n_pre_levels,
                             int* n_launches) {
    if (!ctx) return PHG_ERR_ARG;
    if (!(ctx->have & kTopo)) return ctx->fail(PHG_ERR_STATE, "topology not set");
    const int H = static_cast<int>(ctx->post_lv.size());
    const int D = static_cast<int>(ctx->pre_lv.size());
    if (n_post_levels) *n_post_levels = H;
    if (n_pre_levels) *n_pre_levels = D;
    if (n_launches) {
        int cls[PHG_PROF_CLASSES];
        launches_per_class(ctx, cls);
        // the work-queue traversal may run both passes in one launch
        const bool one =
            ctx->queue && ctx->S == 4 && queue_launches(ctx->S, ctx->R, ctx->prec == PHG_FP32_SCALED) == 1;
        *n_launches = cls[0] + cls[1] + (one ? 0 : cls[2]) + cls[3];
    }
    return PHG_OK;
}

phg_status phg_profile_enable(phg_context* ctx, int on) {
    if (!ctx) return PHG_ERR_ARG;
    ctx->prof_on = on != 0;
    return PHG_OK;
}

phg_status phg_profile_read(phg_context* ctx, double* ms, int* n_evals, int* launches) {
    if (!ctx) return PHG_ERR_ARG;
    const size_t n = ctx->prof_used / kProfEvents;
    double tot[PHG_PROF_CLASSES] = {0, 0, 0, 0};
    if (n > 0) {
        PHG_HIP(ctx, hipSetDevice(ctx->device));
        PHG_HIP(ctx, hipEventSynchronize(ctx->prof_pool[ctx->prof_used - 1]));
        for (size_t e = 0; e < n; ++e)
            for (int k = 0; k < PHG_PROF_CLASSES; ++k) {
                float t = 0.f;
                PHG_HIP(ctx, hipEventElapsedTime(&t, ctx->prof_pool[e * kProfEvents + k],
                                                 ctx->prof_pool[e * kProfEvents + k + 1]));
                tot[k] += t;
            }
    }
    // evaluations the precision guard routed to the FP64 twin
    int n_twin = 0;
    if (ctx->twin && ctx->twin->prof_used > 0) {
        double tw[PHG_PROF_CLASSES];
        PHG_TRY(from_twin(ctx, ctx->twin, phg_profile_read(ctx->twin, tw, &n_twin, nullptr)));
        for (int k = 0; k < PHG_PROF_CLASSES; ++k) tot[k] += tw[k];
    }
    if (ms)
        for (int k = 0; k < PHG_PROF_CLASSES; ++k) ms[k] = tot[k];
    if (n_evals) *n_evals = static_cast<int>(n) + n_twin;
    if (launches) launches_per_class(ctx, launches);
    ctx->prof_used = 0;
    return PHG_OK;
}

}  // extern "C"
