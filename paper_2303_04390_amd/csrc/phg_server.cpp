// Serving engine behind the phg_server_* calls: registered trees, a request
// queue, memory-based admission into one device arena, and a scheduler
// thread that advances every in-flight request by one stage per step with
// requests at the same kind of stage sharing kernel launches (continuous,
// iteration-level batching).
//
// Stages of one request (tree with H post-order and D pre-order levels):
//   0        P(t), dP/dt for all branches and categories
//   1..H     post-order level h-1 (the root level last)
//   H+1..H+D pre-order + gradient level
//   H+D+1    final sums, then the results are copied to pinned host memory
//            and an event marks completion.
// Everything runs on one compute stream in issue order; tree uploads go on a
// separate copy stream and finish before the tree's first kernel is issued.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "phg_context.h"

using namespace phg;

namespace {

constexpr int kMaxStepsAhead = 4;   // scheduler steps queued on the GPU at once

// First-fit allocator over the server's device arena (offsets, 256-byte units).
class ArenaAlloc {
   public:
    void reset(size_t total) {
        free_.clear();
        free_[0] = total;
        used_ = peak_ = 0;
    }
    bool alloc(size_t bytes, size_t* off) {
        bytes = align(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rem = it->second - bytes, start = it->first + bytes;
            free_.erase(it);
            if (rem) free_[start] = rem;
            used_ += bytes;
            peak_ = std::max(peak_, used_);
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = align(bytes);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t peak() const { return peak_; }

   private:
    static size_t align(size_t x) { return (x + 255) / 256 * 256; }
    std::map<size_t, size_t> free_;
    size_t used_ = 0, peak_ = 0;
};

struct Tree {
    uint64_t id = 0;
    phg_context* ctx = nullptr;
    size_t bytes = 0, off = 0;
    bool resident = false;
    bool busy = false;       // an evaluation is in flight
    bool released = false;
    int pending = 0;         // requests queued or in flight
    uint64_t last_use = 0;
    int H = 0, D = 0;
};

enum class RState { kQueued, kActive, kCompleting, kDone };

struct Request {
    uint64_t id = 0, tree = 0;
    std::vector<double> b;
    RState state = RState::kQueued;
    int slot = -1;
    int stage = 0;
    double logl = 0.0;
    std::vector<double> grad;
    phg_status status = PHG_OK;
    uint64_t t_submit = 0, t_done = 0;   // steady clock, ns
};

uint64_t now_ns() {
    return static_cast<uint64_t>(std::chrono::duration_cast<std::chrono::nanoseconds>(
                                     std::chrono::steady_clock::now().time_since_epoch())
                                     .count());
}

struct Slot {
    Request* req = nullptr;
    double* pinned_b = nullptr;
    size_t cap_b = 0;
    double* pinned_out = nullptr;
    size_t cap_out = 0;
    ReqDesc* pinned_desc = nullptr;
    hipEvent_t done = nullptr;
};

}  // namespace

struct phg_server {
    int device = 0;
    size_t budget = 0;
    int max_slots = 0;
    std::string err;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread worker;
    bool stop = false;
    bool failed = false;

    hipStream_t stream = nullptr, copy_stream = nullptr;
    char* arena = nullptr;
    ArenaAlloc alloc;
    ReqDesc* d_descs = nullptr;
    std::vector<Slot> slots;
    std::unordered_map<uint64_t, std::unique_ptr<Tree>> trees;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
    std::deque<Request*> queue;
    uint64_t next_tree = 1, next_req = 1, clock = 0;
    uint64_t n_done = 0, n_steps = 0, n_launches = 0, n_evictions = 0;
    int n_active = 0;
    uint64_t t_created = 0;                  // steady clock, ns
    std::atomic<uint64_t> busy_ns{0};        // device time of finished steps

    phg_status fail(phg_status s, const std::string& m) {
        err = m;
        return s;
    }
};

namespace {

thread_local std::string g_server_error;

// --- helpers that run on the scheduler thread with the lock held ----------

void fail_all(phg_server* s, const std::string& why) {
    s->failed = true;
    s->err = why;
    for (auto& kv : s->reqs) {
        Request* r = kv.second.get();
        if (r->state != RState::kDone) {
            r->state = RState::kDone;
            r->status = PHG_ERR_DEVICE;
        }
    }
    s->queue.clear();
    s->cv_done.notify_all();
}

bool ensure_pinned(double** p, size_t* cap, size_t n) {
    if (*cap >= n) return true;
    if (*p) (void)hipHostFree(*p);
    *p = nullptr;
    *cap = 0;
    void* q = nullptr;
    if (hipHostMalloc(&q, n * sizeof(double), hipHostMallocDefault) != hipSuccess) return false;
    *p = static_cast<double*>(q);
    *cap = n;
    return true;
}

void evict(phg_server* s, Tree* t) {
    ctx_drop_device(t->ctx);
    s->alloc.release(t->off, t->bytes);
    t->resident = false;
    s->n_evictions++;
}

// Make a tree resident: carve its workspace out of the arena (evicting idle
// trees least-recently-used first if needed) and upload its inputs on the copy
// stream.  Returns false if it cannot fit now.
bool make_resident(phg_server* s, Tree* t, phg_status* st) {
    size_t off = 0;
    while (!s->alloc.alloc(t->bytes, &off)) {
        Tree* victim = nullptr;
        for (auto& kv : s->trees) {
            Tree* u = kv.second.get();
            if (u == t || !u->resident || u->busy) continue;
            if (u->pending > 0 && !u->released) continue;   // keep trees with queued work
            if (!victim || u->last_use < victim->last_use) victim = u;
        }
        if (!victim) return false;
        evict(s, victim);
    }
    t->off = off;
    phg_status r = phg_bind_workspace(t->ctx, s->arena + off, t->bytes);
    if (r == PHG_OK) r = ctx_ready(t->ctx);   // allocates nothing: uses the bound workspace
    if (r != PHG_OK) {
        *st = r;
        s->alloc.release(off, t->bytes);
        ctx_drop_device(t->ctx);
        return false;
    }
    t->resident = true;
    return true;
}

// Put request r into a free slot: stage its branch lengths and descriptor.
bool activate(phg_server* s, Request* r, int slot_ix) {
    Tree* t = s->trees[r->tree].get();
    Slot& sl = s->slots[slot_ix];
    const size_t E = r->b.size();
    if (!ensure_pinned(&sl.pinned_b, &sl.cap_b, E) || !ensure_pinned(&sl.pinned_out, &sl.cap_out, E + 1))
        return false;
    std::memcpy(sl.pinned_b, r->b.data(), E * sizeof(double));
    *sl.pinned_desc = t->ctx->rd;
    if (hipMemcpyAsync(t->ctx->arena + t->ctx->plan.b, sl.pinned_b, E * sizeof(double),
                       hipMemcpyHostToDevice, s->stream) != hipSuccess)
        return false;
    if (hipMemcpyAsync(s->d_descs + slot_ix, sl.pinned_desc, sizeof(ReqDesc), hipMemcpyHostToDevice,
                       s->stream) != hipSuccess)
        return false;
    sl.req = r;
    r->slot = slot_ix;
    r->stage = 0;
    r->state = RState::kActive;
    t->busy = true;
    s->n_active++;
    return true;
}

void admit(phg_server* s) {
    for (auto it = s->queue.begin(); it != s->queue.end();) {
        Request* r = *it;
        int free_slot = -1;
        for (int i = 0; i < s->max_slots; ++i)
            if (!s->slots[i].req) {
                free_slot = i;
                break;
            }
        if (free_slot < 0) return;
        Tree* t = s->trees[r->tree].get();
        if (t->busy) {
            ++it;
            continue;
        }
        if (!t->resident) {
            phg_status st = PHG_OK;
            if (!make_resident(s, t, &st)) {
                if (st != PHG_OK) {   // upload failed: this request fails, others go on
                    r->state = RState::kDone;
                    r->status = st;
                    t->pending--;
                    it = s->queue.erase(it);
                    s->cv_done.notify_all();
                    continue;
                }
                ++it;                 // does not fit now; later requests may
                continue;
            }
        }
        if (!activate(s, r, free_slot)) {
            fail_all(s, "staging a request on the device failed");
            return;
        }
        it = s->queue.erase(it);
    }
}

struct GroupKey {
    int cls, a, b, c;
    bool operator<(const GroupKey& o) const {
        return std::tie(cls, a, b, c) < std::tie(o.cls, o.a, o.b, o.c);
    }
};
struct Item {
    int slot, units;
    Segment seg;
    const ReqDesc* shape;
};

// Requests whose level launches can share one kernel: the 4-state kernels
// per category count (and schedule), the vector-ALU kernels per category
// count and padded state count, the MFMA kernels per 16-state block count
// and tile size; always per precision.
GroupKey level_key(KernelClass k, const ReqDesc& d) {
    if (uses_s4_kernels(d.S, d.R)) return GroupKey{k, 1 + 2 * d.blocked, d.fp32, d.R};
    if (uses_vs_kernels(d.S, d.R, d.fp32 != 0)) return GroupKey{k, 4, d.fp32, vs_padded_states(d.S) + 256 * d.R};
    return GroupKey{k, 0, d.fp32, (d.S + 15) / 16 + 256 * (d.Cpad / d.tiles)};
}

// Build and issue one step for every active request; returns false on error.
bool launch_step(phg_server* s) {
    std::map<GroupKey, std::vector<Item>> groups;
    std::vector<Request*> finishing;
    for (int i = 0; i < s->max_slots; ++i) {
        Request* r = s->slots[i].req;
        if (!r || r->state != RState::kActive) continue;
        Tree* t = s->trees[r->tree].get();
        phg_context* c = t->ctx;
        const ReqDesc& d = c->rd;
        const int st = r->stage;
        Item it{i, 0, Segment{i, 0, 0, 0, reinterpret_cast<const int32_t*>(d.sched), nullptr, nullptr}, &d};
        GroupKey key{};
        if (st == 0) {
            // one P(t) kernel per launch: the 4-state one, the generic one
            // (S <= 16), the operand-order one of the MFMA kernels (typed by
            // precision, launched over a grid of output tiles) or the padded
            // one of the vector-ALU kernels (typed by precision and padding)
            const bool f32 = d.fp32 != 0;
            const int kind = d.S == 4 ? 0 : uses_gl_kernels(d.S, d.R, f32) ? 1 : uses_vs_kernels(d.S, d.R, f32) ? 3 : 2;
            key = GroupKey{kPmat, kind, kind == 1 || kind == 3 ? d.fp32 : 0,
                           kind == 1 ? (gl_mat_rows(d.S) + 63) / 64 : (kind == 3 ? vs_padded_states(d.S) : 0)};
            it.units = units_for(kPmat, d, 0);
        } else if (st <= t->H) {
            const int l = st - 1, a = c->post_lv[l].first, n = c->post_lv[l].second;
            it.seg.sched_off = a;
            it.seg.n_nodes = n;
            it.seg.flags = (l == t->H - 1) ? 1 : 0;
            it.units = units_for(kPost, d, n);
            key = level_key(kPost, d);
        } else if (st <= t->H + t->D) {
            const int l = st - t->H - 1, a = c->pre_lv[l].first, n = c->pre_lv[l].second;
            it.seg.sched_off = a;
            it.seg.n_nodes = n;
            it.units = units_for(kPre, d, n);
            key = level_key(kPre, d);
        } else {
            double* out = ctx_out_dev(c);
            it.seg.out_logl = out;
            it.seg.out_grad = out + 1;
            it.units = units_for(kFinal, d, 0);
            key = GroupKey{kFinal, 0, 0, 0};
            finishing.push_back(r);
        }
        groups[key].push_back(it);
    }
    for (auto& kv : groups) {
        const KernelClass k = static_cast<KernelClass>(kv.first.cls);
        const std::vector<Item>& items = kv.second;
        for (size_t b0 = 0; b0 < items.size(); b0 += kMaxSegs) {
            SegTable t{};
            t.n = 0;
            t.unit_begin[0] = 0;
            for (size_t j = b0; j < items.size() && j < b0 + kMaxSegs; ++j) {
                t.seg[t.n] = items[j].seg;
                t.unit_begin[t.n + 1] = t.unit_begin[t.n] + items[j].units;
                t.n++;
            }
            if (launch_class(k, *items[b0].shape, s->d_descs, t, s->stream) != hipSuccess) return false;
            s->n_launches++;
        }
    }
    for (int i = 0; i < s->max_slots; ++i) {
        Request* r = s->slots[i].req;
        if (r && r->state == RState::kActive) r->stage++;
    }
    for (Request* r : finishing) {
        Slot& sl = s->slots[r->slot];
        phg_context* c = s->trees[r->tree]->ctx;
        const size_t E = r->b.size();
        if (hipMemcpyAsync(sl.pinned_out, ctx_out_dev(c), (E + 1) * sizeof(double), hipMemcpyDeviceToHost,
                           s->stream) != hipSuccess)
            return false;
        if (hipEventRecord(sl.done, s->stream) != hipSuccess) return false;
        r->state = RState::kCompleting;
    }
    s->n_steps++;
    return true;
}

// Collect requests whose results reached host memory.
bool poll_completions(phg_server* s) {
    bool any = false;
    for (int i = 0; i < s->max_slots; ++i) {
        Slot& sl = s->slots[i];
        Request* r = sl.req;
        if (!r || r->state != RState::kCompleting) continue;
        const hipError_t q = hipEventQuery(sl.done);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) {
            fail_all(s, std::string("device error: ") + hipGetErrorString(q));
            return false;
        }
        const size_t E = r->b.size();
        r->logl = sl.pinned_out[0];
        r->grad.assign(sl.pinned_out + 1, sl.pinned_out + 1 + E);
        if (!std::isfinite(r->logl)) {
            r->status = PHG_ERR_NUMERIC;
            r->logl = -std::numeric_limits<double>::infinity();
            std::fill(r->grad.begin(), r->grad.end(), std::numeric_limits<double>::quiet_NaN());
        }
        r->state = RState::kDone;
        r->t_done = now_ns();
        r->b.clear();
        r->b.shrink_to_fit();
        Tree* t = s->trees[r->tree].get();
        t->busy = false;
        t->pending--;
        t->last_use = ++s->clock;
        sl.req = nullptr;
        s->n_active--;
        s->n_done++;
        any = true;
        if (t->released && t->pending == 0) {
            if (t->resident) evict(s, t);
            phg_destroy(t->ctx);
            s->trees.erase(t->id);
        }
    }
    if (any) s->cv_done.notify_all();
    return true;
}

void scheduler(phg_server* s) {
    if (hipSetDevice(s->device) != hipSuccess) {
        std::lock_guard<std::mutex> lk(s->mu);
        fail_all(s, "hipSetDevice failed on the scheduler thread");
        return;
    }
    // each step in flight: events before its first launch and after its last
    std::deque<std::pair<hipEvent_t, hipEvent_t>> ahead;
    std::vector<hipEvent_t> pool;
    auto take_event = [&](hipEvent_t* ev) {
        if (!pool.empty()) {
            *ev = pool.back();
            pool.pop_back();
            return true;
        }
        return hipEventCreate(ev) == hipSuccess;
    };
    for (;;) {
        std::unique_lock<std::mutex> lk(s->mu);
        if (s->failed) break;
        if (!poll_completions(s)) break;
        if (!s->stop) admit(s);
        if (s->failed) break;
        bool active = false, completing = false;
        for (int i = 0; i < s->max_slots; ++i) {
            const Request* r = s->slots[i].req;
            if (!r) continue;
            active |= r->state == RState::kActive;
            completing |= r->state == RState::kCompleting;
        }
        if (!active) {
            if (s->stop && !completing) break;
            if (completing) {
                lk.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(20));
            } else {
                s->cv_work.wait_for(lk, std::chrono::milliseconds(2));
            }
            continue;
        }
        hipEvent_t ev0 = nullptr, ev1 = nullptr;
        if (!take_event(&ev0) || !take_event(&ev1)) {
            fail_all(s, "hipEventCreate failed");
            break;
        }
        if (hipEventRecord(ev0, s->stream) != hipSuccess) {
            fail_all(s, "hipEventRecord failed");
            break;
        }
        if (!launch_step(s)) {
            fail_all(s, "kernel launch failed");
            break;
        }
        if (hipEventRecord(ev1, s->stream) != hipSuccess) {
            fail_all(s, "hipEventRecord failed");
            break;
        }
        ahead.emplace_back(ev0, ev1);
        lk.unlock();
        // retire finished steps (and wait while too many are queued)
        while (!ahead.empty()) {
            const bool must = static_cast<int>(ahead.size()) > kMaxStepsAhead;
            const hipError_t q = must ? hipEventSynchronize(ahead.front().second) : hipEventQuery(ahead.front().second);
            if (q == hipErrorNotReady) break;
            if (q != hipSuccess) {
                std::lock_guard<std::mutex> lk2(s->mu);
                fail_all(s, std::string("device error: ") + hipGetErrorString(q));
                break;
            }
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, ahead.front().first, ahead.front().second) == hipSuccess)
                s->busy_ns += static_cast<uint64_t>(static_cast<double>(ms) * 1e6);
            pool.push_back(ahead.front().first);
            pool.push_back(ahead.front().second);
            ahead.pop_front();
        }
    }
    (void)hipStreamSynchronize(s->stream);
    for (auto& e : ahead) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, e.first, e.second) == hipSuccess)
            s->busy_ns += static_cast<uint64_t>(static_cast<double>(ms) * 1e6);
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
}

}  // namespace

extern "C" {

phg_status phg_server_create(int device, size_t mem_budget_bytes, int max_slots, phg_server** out) {
    if (!out) return PHG_ERR_ARG;
    *out = nullptr;
    if (max_slots < 1 || max_slots > kMaxSegs) {
        g_server_error = "max_slots must be in [1, 48]";
        return PHG_ERR_ARG;
    }
    if (device < 0 || mem_budget_bytes < (1u << 20)) {
        g_server_error = "device must be >= 0 and mem_budget_bytes >= 1 MiB";
        return PHG_ERR_ARG;
    }
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= device) {
        g_server_error = "no such HIP device";
        return PHG_ERR_DEVICE;
    }
    hipDeviceProp_t prop;
    if (hipSetDevice(device) != hipSuccess || hipGetDeviceProperties(&prop, device) != hipSuccess ||
        std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        g_server_error = "device is not gfx950";
        return PHG_ERR_DEVICE;
    }
    std::unique_ptr<phg_server> s(new (std::nothrow) phg_server());
    if (!s) return PHG_ERR_OOM;
    s->device = device;
    s->budget = mem_budget_bytes;
    s->max_slots = max_slots;
    s->t_created = now_ns();
    void* p = nullptr;
    if (hipMalloc(&p, mem_budget_bytes) != hipSuccess) {
        g_server_error = "could not reserve the memory budget";
        return PHG_ERR_OOM;
    }
    s->arena = static_cast<char*>(p);
    s->alloc.reset(mem_budget_bytes);
    if (hipMalloc(&p, sizeof(ReqDesc) * max_slots) != hipSuccess) {
        (void)hipFree(s->arena);
        g_server_error = "descriptor table allocation failed";
        return PHG_ERR_OOM;
    }
    s->d_descs = static_cast<ReqDesc*>(p);
    if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking) != hipSuccess) {
        g_server_error = "stream creation failed";
        return PHG_ERR_DEVICE;
    }
    s->slots.resize(max_slots);
    for (Slot& sl : s->slots) {
        void* q = nullptr;
        if (hipHostMalloc(&q, sizeof(ReqDesc), hipHostMallocDefault) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) {
            g_server_error = "slot setup failed";
            return PHG_ERR_DEVICE;
        }
        sl.pinned_desc = static_cast<ReqDesc*>(q);
    }
    phg_server* raw = s.release();
    raw->worker = std::thread(scheduler, raw);
    *out = raw;
    return PHG_OK;
}

phg_status phg_server_destroy(phg_server* s) {
    if (!s) return PHG_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        // queued requests never start
        for (Request* r : s->queue) {
            r->state = RState::kDone;
            r->status = PHG_ERR_STATE;
        }
        s->queue.clear();
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    (void)hipSetDevice(s->device);
    for (auto& kv : s->trees) phg_destroy(kv.second->ctx);
    for (Slot& sl : s->slots) {
        if (sl.pinned_b) (void)hipHostFree(sl.pinned_b);
        if (sl.pinned_out) (void)hipHostFree(sl.pinned_out);
        if (sl.pinned_desc) (void)hipHostFree(sl.pinned_desc);
        if (sl.done) (void)hipEventDestroy(sl.done);
    }
    if (s->d_descs) (void)hipFree(s->d_descs);
    if (s->arena) (void)hipFree(s->arena);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    if (s->copy_stream) (void)hipStreamDestroy(s->copy_stream);
    delete s;
    return PHG_OK;
}

const char* phg_server_last_error(const phg_server* s) {
    return s ? s->err.c_str() : g_server_error.c_str();
}

phg_status phg_server_register_tree(phg_server* s, const phg_tree_desc* d, uint64_t* tree_id) {
    if (!s || !d || !tree_id) return PHG_ERR_ARG;
    phg_context* ctx = nullptr;
    phg_status st = phg_create(d->n_tips, d->n_patterns, d->n_states, d->n_categories, d->prec,
                               s->device, &ctx);
    if (st != PHG_OK) {
        std::lock_guard<std::mutex> lk(s->mu);
        return s->fail(st, phg_last_error(nullptr));
    }
    const size_t E = 2 * static_cast<size_t>(d->n_tips) - 2;
    std::vector<double> b0(E, 0.0);
    ctx->table_budget = static_cast<size_t>(-1);   // one P(t) stage per request: every branch's tables
    if (st == PHG_OK) st = phg_set_topology(ctx, d->parent);
    if (st == PHG_OK)
        st = d->per_category_eigen ? phg_set_category_eigen(ctx, d->V, d->Vinv, d->lambda)
                                   : phg_set_eigen(ctx, d->V, d->Vinv, d->lambda);
    if (st == PHG_OK && d->n_tip_vectors < 0) st = PHG_ERR_ARG;
    if (st == PHG_OK && d->n_tip_vectors > 0 && (!d->tip_vector_tips || !d->tip_vectors)) st = PHG_ERR_ARG;
    for (int v = 0; st == PHG_OK && v < d->n_tip_vectors; ++v)
        st = phg_set_tip_partials(ctx, d->tip_vector_tips[v],
                                  d->tip_vectors + static_cast<size_t>(v) * d->n_patterns * d->n_states);
    if (st == PHG_OK) st = phg_set_root_frequencies(ctx, d->pi);
    if (st == PHG_OK) st = phg_set_categories(ctx, d->rates, d->weights);
    if (st == PHG_OK) st = phg_set_tip_states(ctx, d->codes);
    if (st == PHG_OK && d->pattern_weights) st = phg_set_pattern_weights(ctx, d->pattern_weights);
    if (st == PHG_OK) st = phg_set_branch_lengths(ctx, b0.data());
    std::lock_guard<std::mutex> lk(s->mu);
    if (st == PHG_OK) st = phg_bind_stream(ctx, s->copy_stream);
    if (st != PHG_OK) {
        s->err = phg_last_error(ctx);
        phg_destroy(ctx);
        return st;
    }
    auto t = std::make_unique<Tree>();
    t->ctx = ctx;
    // served trees keep every branch's P(t) tables (one P(t) stage per request)
    t->bytes = make_plan(d->n_tips, d->n_patterns, d->n_states, d->n_categories, d->prec, 0).total;
    if (t->bytes > s->budget) {
        phg_destroy(ctx);
        return s->fail(PHG_ERR_OOM, "tree workspace exceeds the server memory budget");
    }
    t->H = static_cast<int>(ctx->post_lv.size());
    t->D = static_cast<int>(ctx->pre_lv.size());
    t->id = s->next_tree++;
    *tree_id = t->id;
    s->trees[t->id] = std::move(t);
    return PHG_OK;
}

phg_status phg_server_submit(phg_server* s, uint64_t tree_id, const double* b, uint64_t* req_id) {
    if (!s || !b || !req_id) return PHG_ERR_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->failed) return PHG_ERR_DEVICE;
    if (s->stop) return s->fail(PHG_ERR_STATE, "server is shutting down");
    auto it = s->trees.find(tree_id);
    if (it == s->trees.end() || it->second->released)
        return s->fail(PHG_ERR_ARG, "unknown or released tree id");
    Tree* t = it->second.get();
    const size_t E = 2 * static_cast<size_t>(t->ctx->N) - 2;
    for (size_t x = 0; x < E; ++x)
        if (!std::isfinite(b[x]) || b[x] < 0.0)
            return s->fail(PHG_ERR_ARG, "branch lengths must be finite and >= 0");
    auto r = std::make_unique<Request>();
    r->id = s->next_req++;
    r->tree = tree_id;
    r->b.assign(b, b + E);
    r->t_submit = now_ns();
    *req_id = r->id;
    t->pending++;
    s->queue.push_back(r.get());
    s->reqs[r->id] = std::move(r);
    lk.unlock();
    s->cv_work.notify_one();
    return PHG_OK;
}

static phg_status take_result(phg_server* s, Request* r, double* logl, double* grad) {
    if (logl) *logl = r->logl;
    if (grad && !r->grad.empty()) std::memcpy(grad, r->grad.data(), r->grad.size() * sizeof(double));
    const phg_status st = r->status;
    if (st == PHG_ERR_NUMERIC) s->err = "a weighted site likelihood is zero or not finite";
    s->reqs.erase(r->id);
    return st;
}

phg_status phg_server_poll(phg_server* s, uint64_t req_id, double* logl, double* grad, int* done) {
    if (!s || !done) return PHG_ERR_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(req_id);
    if (it == s->reqs.end()) return s->fail(PHG_ERR_ARG, "unknown request id");
    Request* r = it->second.get();
    if (r->state != RState::kDone) {
        *done = 0;
        return s->failed ? PHG_ERR_DEVICE : PHG_OK;
    }
    *done = 1;
    return take_result(s, r, logl, grad);
}

phg_status phg_server_poll_timed(phg_server* s, uint64_t req_id, double* logl, double* grad, int* done,
                                 uint64_t* t_submit_ns, uint64_t* t_done_ns) {
    if (!s || !done) return PHG_ERR_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(req_id);
    if (it == s->reqs.end()) return s->fail(PHG_ERR_ARG, "unknown request id");
    Request* r = it->second.get();
    if (r->state != RState::kDone) {
        *done = 0;
        return s->failed ? PHG_ERR_DEVICE : PHG_OK;
    }
    *done = 1;
    if (t_submit_ns) *t_submit_ns = r->t_submit;
    if (t_done_ns) *t_done_ns = r->t_done;
    return take_result(s, r, logl, grad);
}

phg_status phg_server_wait(phg_server* s, uint64_t req_id, double* logl, double* grad) {
    if (!s) return PHG_ERR_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(req_id);
    if (it == s->reqs.end()) return s->fail(PHG_ERR_ARG, "unknown request id");
    Request* r = it->second.get();
    s->cv_done.wait(lk, [&] { return r->state == RState::kDone; });
    return take_result(s, r, logl, grad);
}

phg_status phg_server_release_tree(phg_server* s, uint64_t tree_id) {
    if (!s) return PHG_ERR_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->trees.find(tree_id);
    if (it == s->trees.end() || it->second->released) return s->fail(PHG_ERR_ARG, "unknown tree id");
    Tree* t = it->second.get();
    t->released = true;
    if (t->pending == 0 && !t->busy) {
        if (t->resident) evict(s, t);
        phg_destroy(t->ctx);
        s->trees.erase(it);
    }
    return PHG_OK;
}

phg_status phg_server_busy(phg_server* s, uint64_t* busy_ns, uint64_t* wall_ns) {
    if (!s) return PHG_ERR_ARG;
    if (busy_ns) *busy_ns = s->busy_ns.load();
    if (wall_ns) *wall_ns = now_ns() - s->t_created;
    return PHG_OK;
}

phg_status phg_server_stats(phg_server* s, uint64_t stats[8]) {
    if (!s || !stats) return PHG_ERR_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    uint64_t resident = 0;
    for (auto& kv : s->trees) resident += kv.second->resident ? 1 : 0;
    stats[0] = s->n_done;
    stats[1] = s->n_steps;
    stats[2] = s->n_launches;
    stats[3] = resident;
    stats[4] = s->n_evictions;
    stats[5] = s->alloc.peak();
    stats[6] = s->queue.size();
    stats[7] = static_cast<uint64_t>(s->n_active);
    return PHG_OK;
}

}  // extern "C"
