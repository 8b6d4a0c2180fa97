// Parameter chain rules on the device, applied to a finished branch gradient
// g_i = d logL / d b_i (indexed by child node):
//
//   time tree (Methods, problem statement: a branch length is the parent-child
//   node-height difference times a branch rate scalar, b_i = (h_pa(i) - h_i) rho_i)
//     d logL / d rho_i = (h_pa(i) - h_i) g_i
//     d logL / d h_k   = sum over children c of k of rho_c g_c  -  rho_k g_k (k not the root)
//   branch sets (gradient-kernel section: a further reduction of the branch
//   derivatives over a chosen set of branches, e.g. for a strict clock)
//     out_j = sum over branches i of set j of v_i, in increasing i.
//
// Both are O(N) and deterministic: one thread per node, then one workgroup
// per set with a fixed-order tree reduction.
#include <hip/hip_runtime.h>

#include "phg_internal.h"

namespace phg {
namespace {

constexpr int kChainBlock = 256;

__global__ __launch_bounds__(kChainBlock) void chain_kernel(const ChainArgs a) {
    const int v = blockIdx.x * kChainBlock + threadIdx.x;
    const int n = 2 * a.N - 1;
    if (v >= n) return;
    const int E = n - 1;
    double dh = 0.0;
    if (v >= a.N) {
        const int c0 = a.kids[2 * (v - a.N)], c1 = a.kids[2 * (v - a.N) + 1];
        dh = a.rates[c0] * a.grad[c0] + a.rates[c1] * a.grad[c1];
    }
    if (v < E) {
        const double g = a.grad[v];
        a.d_rates[v] = (a.heights[a.parent[v]] - a.heights[v]) * g;
        dh -= a.rates[v] * g;
    }
    a.d_heights[v] = dh;
}

__global__ __launch_bounds__(kChainBlock) void set_sum_kernel(const ChainArgs a, const double* __restrict__ vals) {
    __shared__ double red[kChainBlock];
    const int j = blockIdx.x;
    const int lo = a.set_ptr[j], hi = a.set_ptr[j + 1];
    double acc = 0.0;
    for (int t = lo + static_cast<int>(threadIdx.x); t < hi; t += kChainBlock) acc += vals[a.set_idx[t]];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = kChainBlock / 2; h > 0; h >>= 1) {
        if (static_cast<int>(threadIdx.x) < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) a.d_sets[j] = red[0];
}

}  // namespace

hipError_t launch_chain(const ChainArgs& a, bool time_tree, hipStream_t st) {
    if (time_tree) {
        const int n = 2 * a.N - 1;
        hipLaunchKernelGGL(chain_kernel, dim3((n + kChainBlock - 1) / kChainBlock), dim3(kChainBlock), 0, st, a);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (a.n_sets > 0) {
        hipLaunchKernelGGL(set_sum_kernel, dim3(a.n_sets), dim3(kChainBlock), 0, st, a,
                           time_tree ? static_cast<const double*>(a.d_rates) : a.grad);
        return hipGetLastError();
    }
    return hipSuccess;
}

}  // namespace phg
