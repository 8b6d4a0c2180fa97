// Internal declarations shared by the host runtime (phg_host.cpp) and the
// gfx950 kernels (phg_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace phg {

constexpr int kLanes = 64;          // one wavefront = one tile of 64 site patterns

// One parent with its two children, by node id.  Post-order levels list the
// internal nodes of equal height; pre-order levels the internal nodes of
// equal depth.  Children are stored in ascending id order.
struct NodeTriple {
    int32_t k, i, j, pad;
};

// Device-side view of one problem: sizes plus pointers into the workspace.
// Layouts (T = float or double, per precision):
//   codes  uint8  [N][Cpad]                 tip states, S = all-ones, pad = S
//   part   T      [N-1][tiles][R][S4][64][4] post-order partial of each
//                                            internal node (slot = id - N);
//                                            overwritten in place by the
//                                            pre-order partial during the
//                                            pre-order pass
//   expo   int32  [N-1][Cpad]               cumulative power-of-two exponent
//                                            of the subtree below each node
//   P,dP   double [E][R][S][S] (and float copies when T = float)
//   sll    double [Cpad]                    per-pattern log site likelihood
//   lpart  double [tiles]                   per-tile weighted log-likelihood sums
//   gpart  double [E][tiles]                per-tile weighted gradient sums
struct DeviceProblem {
    int N, C, Cpad, S, S4, R, tiles;
    const uint8_t* codes;
    void* part;
    int32_t* expo;
    double* P64;
    double* dP64;
    float* P32;
    float* dP32;
    const double* b;
    const double* V;
    const double* Vinv;
    const double* lam;
    const double* rates;
    const double* cweights;
    const double* pi;
    const double* pw;
    double* sll;
    double* lpart;
    double* gpart;
};

// Kernel launchers (phg_kernels.hip).  All enqueue on `stream` and return the
// launch status.  fp32 selects float partials.
hipError_t launch_pmat(const DeviceProblem& d, bool fp32, hipStream_t stream);
hipError_t launch_post_level(const DeviceProblem& d, bool fp32, const NodeTriple* level,
                             int n_nodes, bool is_root, hipStream_t stream);
hipError_t launch_pre_level(const DeviceProblem& d, bool fp32, const NodeTriple* level,
                            int n_nodes, hipStream_t stream);
hipError_t launch_finalize(const DeviceProblem& d, double* out_logl, double* out_grad,
                           hipStream_t stream);
bool kernels_support(int S, int R);

}  // namespace phg
