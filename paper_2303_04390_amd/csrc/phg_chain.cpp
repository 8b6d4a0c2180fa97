// Host side of the parameter chain rules (include/phg.h, "parameter chain
// rules"): time-tree inputs (node heights, branch rate scalars), branch sets,
// and the evaluations that finish with the chain-rule kernels of
// phg_chain.hip on the context's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <limits>
#include <vector>

#include "phg_context.h"

using namespace phg;

namespace {

ChainArgs chain_args(phg_context* ctx) {
    const Plan& pl = ctx->plan;
    char* a = ctx->arena;
    double* out = ctx_out_dev(ctx);
    const size_t E = 2 * static_cast<size_t>(ctx->N) - 2;
    ChainArgs c{};
    c.N = ctx->N;
    c.n_sets = ctx->n_sets;
    c.parent = reinterpret_cast<const int32_t*>(a + pl.ch_parent);
    c.kids = reinterpret_cast<const int32_t*>(a + pl.ch_kids);
    c.heights = reinterpret_cast<const double*>(a + pl.heights);
    c.rates = reinterpret_cast<const double*>(a + pl.trates);
    c.grad = out + 1;
    c.d_heights = out + 1 + E;
    c.d_rates = out + 1 + E + (E + 1);
    c.set_ptr = reinterpret_cast<const int32_t*>(a + pl.set_ptr);
    c.set_idx = reinterpret_cast<const int32_t*>(a + pl.set_idx);
    c.d_sets = out + 1 + E + (E + 1) + E;
    return c;
}

// One evaluation followed by the chain kernels on t (the context or its FP64
// twin); the whole output region is copied back into t's pinned mirror.
// Numeric failure as phg_gradient.
phg_status eval_chain_on(phg_context* t, bool time_tree) {
    PHG_TRY(ctx_ready(t));
    PHG_TRY(ctx_host_out(t));
    double* dout = ctx_out_dev(t);
    PHG_TRY(ctx_enqueue_eval(t, dout, dout + 1));
    PHG_HIP(t, launch_chain(chain_args(t), time_tree, t->stream));
    PHG_HIP(t, hipMemcpyAsync(t->host_out, dout, out_doubles(t->N) * sizeof(double),
                              hipMemcpyDeviceToHost, t->stream));
    PHG_HIP(t, hipStreamSynchronize(t->stream));
    const double ll = t->host_out[0];
    if (!std::isfinite(ll))
        return t->fail(PHG_ERR_NUMERIC, "a weighted site likelihood is zero or not finite");
    return PHG_OK;
}

// *host receives the pinned mirror that holds the results.
phg_status eval_with_chain(phg_context* ctx, bool time_tree, const double** host) {
    phg_status s;
    phg_context* t = eval_target(ctx, &s);
    if (!t) return s;
    s = from_twin(ctx, t, eval_chain_on(t, time_tree));
    *host = t->host_out;
    return s;
}

void fill_nan(double* p, size_t n) {
    if (p)
        for (size_t i = 0; i < n; ++i) p[i] = std::numeric_limits<double>::quiet_NaN();
}

}  // namespace

extern "C" {

phg_status phg_set_time_tree(phg_context* ctx, const double* heights, const double* rates) {
    if (!ctx) return PHG_ERR_ARG;
    if (!heights || !rates) return ctx->fail(PHG_ERR_ARG, "heights or rates is NULL");
    if (!(ctx->have & kTopo)) return ctx->fail(PHG_ERR_STATE, "topology not set");
    const int N = ctx->N, n = 2 * N - 1;
    for (int v = 0; v < n; ++v)
        if (!std::isfinite(heights[v])) return ctx->fail(PHG_ERR_ARG, "heights[%d] is not finite", v);
    std::vector<double> b(n - 1);
    for (int i = 0; i < n - 1; ++i) {
        if (!std::isfinite(rates[i]) || rates[i] < 0.0)
            return ctx->fail(PHG_ERR_ARG, "rates[%d]=%g must be finite and >= 0", i, rates[i]);
        const int k = ctx->parent[i];
        if (heights[k] < heights[i])
            return ctx->fail(PHG_ERR_ARG, "node %d (height %g) is above its parent %d (height %g)", i,
                             heights[i], k, heights[k]);
        b[i] = (heights[k] - heights[i]) * rates[i];
        if (!std::isfinite(b[i])) return ctx->fail(PHG_ERR_ARG, "branch length of node %d overflows", i);
    }
    ctx->b = std::move(b);
    ctx->heights.assign(heights, heights + n);
    ctx->trates.assign(rates, rates + n - 1);
    ctx->have |= kB | kTime;
    ctx->dirty |= kB | kTime;
    ctx->sdirty |= kB | kTime;
    return PHG_OK;
}

phg_status phg_set_branch_sets(phg_context* ctx, const int32_t* set_of, int n_sets) {
    if (!ctx) return PHG_ERR_ARG;
    const int E = 2 * ctx->N - 2;
    if (n_sets == 0) {
        ctx->n_sets = 0;
        ctx->set_ptr.clear();
        ctx->set_idx.clear();
        ctx->have &= ~kSets;
        return PHG_OK;
    }
    if (n_sets < 0 || n_sets > E) return ctx->fail(PHG_ERR_ARG, "n_sets=%d must be in [0, %d]", n_sets, E);
    if (!set_of) return ctx->fail(PHG_ERR_ARG, "set_of is NULL");
    std::vector<int32_t> ptr(n_sets + 1, 0);
    for (int i = 0; i < E; ++i) {
        if (set_of[i] < -1 || set_of[i] >= n_sets)
            return ctx->fail(PHG_ERR_ARG, "set_of[%d]=%d must be in [-1, %d)", i, set_of[i], n_sets);
        if (set_of[i] >= 0) ptr[set_of[i] + 1]++;
    }
    for (int j = 0; j < n_sets; ++j) ptr[j + 1] += ptr[j];
    std::vector<int32_t> idx(ptr[n_sets] > 0 ? ptr[n_sets] : 1, 0), fill(ptr.begin(), ptr.end() - 1);
    for (int i = 0; i < E; ++i)      // increasing branch index within each set
        if (set_of[i] >= 0) idx[fill[set_of[i]]++] = i;
    ctx->set_ptr = std::move(ptr);
    ctx->set_idx = std::move(idx);
    ctx->n_sets = n_sets;
    ctx->have |= kSets;
    ctx->dirty |= kSets;
    ctx->sdirty |= kSets;
    return PHG_OK;
}

phg_status phg_time_tree_gradient(phg_context* ctx, double* logl, double* d_heights, double* d_rates,
                                  double* d_sets) {
    if (!ctx) return PHG_ERR_ARG;
    if (!(ctx->have & kTime)) return ctx->fail(PHG_ERR_STATE, "no time tree set (phg_set_time_tree)");
    if (d_sets && !(ctx->have & kSets)) return ctx->fail(PHG_ERR_STATE, "d_sets given but no branch sets set");
    const int n_sets = d_sets ? ctx->n_sets : 0;
    const int saved = ctx->n_sets;
    ctx->n_sets = n_sets;     // skip the set kernel when its result is not wanted
    const double* h = nullptr;
    const phg_status s = eval_with_chain(ctx, true, &h);
    ctx->n_sets = saved;
    const size_t E = 2 * static_cast<size_t>(ctx->N) - 2;
    if (s != PHG_OK) {
        if (s == PHG_ERR_NUMERIC) {
            if (logl) *logl = -std::numeric_limits<double>::infinity();
            fill_nan(d_heights, E + 1);
            fill_nan(d_rates, E);
            fill_nan(d_sets, static_cast<size_t>(n_sets));
        }
        return s;
    }
    if (logl) *logl = h[0];
    if (d_heights) std::memcpy(d_heights, h + 1 + E, (E + 1) * sizeof(double));
    if (d_rates) std::memcpy(d_rates, h + 1 + E + (E + 1), E * sizeof(double));
    if (d_sets) std::memcpy(d_sets, h + 1 + E + (E + 1) + E, n_sets * sizeof(double));
    return PHG_OK;
}

phg_status phg_gradient_branch_sets(phg_context* ctx, double* logl, double* d_sets) {
    if (!ctx) return PHG_ERR_ARG;
    if (!d_sets) return ctx->fail(PHG_ERR_ARG, "d_sets is NULL");
    if (!(ctx->have & kSets)) return ctx->fail(PHG_ERR_STATE, "no branch sets set (phg_set_branch_sets)");
    const double* h = nullptr;
    const phg_status s = eval_with_chain(ctx, false, &h);
    const size_t E = 2 * static_cast<size_t>(ctx->N) - 2;
    if (s != PHG_OK) {
        if (s == PHG_ERR_NUMERIC) {
            if (logl) *logl = -std::numeric_limits<double>::infinity();
            fill_nan(d_sets, static_cast<size_t>(ctx->n_sets));
        }
        return s;
    }
    if (logl) *logl = h[0];
    std::memcpy(d_sets, h + 1 + E + (E + 1) + E, ctx->n_sets * sizeof(double));
    return PHG_OK;
}

}  // extern "C"
