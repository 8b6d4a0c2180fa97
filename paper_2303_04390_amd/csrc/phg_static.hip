// phg_gradient_async_noalloc: phg_gradient_async with the context's whole
// workspace (partials, exponents, P(t) tables, per-tile partial sums,
// descriptor and schedule) placed in one library-owned static device array
// per GPU instead of memory the library allocates or the caller binds.  For
// callers that cannot allocate device memory.
//
// In host code `scratch` names a host-side stand-in, not the device array:
// its device address is taken once per device with hipGetSymbolAddress and
// only that address is used (descriptor pointers, uploads).  Every context
// that evaluates here on one GPU shares the array; the last context to use
// it is recorded, and a context whose data another one may have overwritten
// uploads all its inputs again.  Calls that overlap in time on one GPU race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "phg_context.h"

namespace {

static __device__ __align__(256) char scratch[PHG_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};           // device address of scratch, per device
uint64_t g_owner[kMaxDevices] = {};      // uid of the last context evaluated there

}  // namespace

namespace phg {

// Device address of this GPU's scratch array (looked up once per device,
// with that device current).
phg_status scratch_address(phg_context* ctx, void** out) {
    if (ctx->device >= kMaxDevices) return ctx->fail(PHG_ERR_DEVICE, "device %d: no scratch slot", ctx->device);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[ctx->device]) {
        PHG_HIP(ctx, hipSetDevice(ctx->device));
        void* p = nullptr;
        PHG_HIP(ctx, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return ctx->fail(PHG_ERR_DEVICE, "hipGetSymbolAddress returned NULL");
        g_ptr[ctx->device] = p;
    }
    *out = g_ptr[ctx->device];
    return PHG_OK;
}

// Record ctx as the scratch array's user; true if another context used it
// since ctx last did (ctx's device data must then be uploaded again).
bool scratch_claim(const phg_context* ctx) {
    std::lock_guard<std::mutex> lk(g_mu);
    const bool changed = g_owner[ctx->device] != ctx->uid;
    g_owner[ctx->device] = ctx->uid;
    return changed;
}

}  // namespace phg

using namespace phg;

extern "C" phg_status phg_gradient_async_noalloc(phg_context* ctx, double* d_logl, double* d_grad) {
    if (!ctx) return PHG_ERR_ARG;
    if (!d_logl || !d_grad) return ctx->fail(PHG_ERR_ARG, "NULL device output pointer");
    if (!ctx->tip_vectors.empty())
        return ctx->fail(PHG_ERR_ARG, "general tip partials need memory of their own; not available here");
    const size_t need =
        make_plan(ctx->N, ctx->C, ctx->S, ctx->R, ctx->prec,
                  table_slots_for(ctx->N, ctx->S, ctx->R, ctx->prec, ctx->table_budget))
            .total;
    if (need > PHG_NOALLOC_SCRATCH_BYTES)
        return ctx->fail(PHG_ERR_OOM, "workspace of %zu bytes exceeds the %zu-byte static scratch array", need,
                         static_cast<size_t>(PHG_NOALLOC_SCRATCH_BYTES));
    if (!ctx->stream || ctx->own_stream)
        return ctx->fail(PHG_ERR_STATE, "bind a stream first (phg_bind_stream): creating one would allocate");
    if (ctx->dev_init && !ctx->static_ws)
        return ctx->fail(PHG_ERR_STATE, "context already evaluates in other device memory");
    if ((ctx->have & kRequired) != kRequired) return ctx_ready(ctx);   // the usual PHG_ERR_STATE report
    if (!ctx->dev_init) {
        void* p = nullptr;
        PHG_TRY(scratch_address(ctx, &p));
        ctx->bound_ws = static_cast<char*>(p);
        ctx->bound_ws_bytes = PHG_NOALLOC_SCRATCH_BYTES;
        ctx->static_ws = true;
    }
    // no profiling events here: creating one allocates
    const bool prof = ctx->prof_on;
    ctx->prof_on = false;
    phg_status s = ctx_ready(ctx);   // re-uploads everything if another context used the array
    if (s == PHG_OK) s = ctx_enqueue_eval(ctx, d_logl, d_grad);
    ctx->prof_on = prof;
    ctx->last_prec = ctx->prec;
    return s;
}
