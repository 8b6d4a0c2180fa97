// gfx950 kernels for the tree log-likelihood and all branch-length derivatives.
//
// Method (Gangavarapu et al., arXiv:2303.04390, Methods):
//   pmat      P^(r)(b_x) = V diag(exp(gamma_r b_x lam)) Vinv and its
//             b-derivative dP = gamma_r V diag(lam exp(gamma_r b_x lam)) Vinv,
//             for every branch x and category r at once (equation for P).
//   post      p_k = (P_i p_i) o (P_j p_j)                       (pruning equation)
//             with one power-of-two exponent per (node, pattern) shared by
//             all categories; the root level turns the root partial into the
//             log site likelihood (sequence-likelihood equation).
//   pre       for a parent k with children i, j (both at once):
//               m_x = P_x p_x, dm_x = dP_x p_x, u_i = q_k o m_j, u_j = q_k o m_i,
//               q_x = P_x^T u_x                                   (eq:preorder)
//             and the per-pattern derivative ratio of eq:gradient,
//               sum_r w_r u_x.dm_x / sum_r w_r u_x.m_x,
//             which equals sum_r w_r gamma_r p_x^T Q^T q_x / sum_r w_r p_x^T q_x
//             because dP_x = gamma_r P_x Q; weighted by W_c and reduced over
//             the 64 patterns of the wavefront in float64.
//   finalize  fixed-order float64 sums over pattern tiles
//             (eq:gradientSumAcrossColumns) and over patterns for log P(Y).
//
// Work unit: one wavefront = (one node, one tile of 64 consecutive patterns);
// lane = pattern.  For S = 4 each lane keeps the R x 4 values of its pattern
// in registers and loops over categories; P and dP of a branch are the same
// for every lane, so they come through scalar loads.  Partials are stored
// [slot][tile][r][lane][4], so each category of a unit is one contiguous
// 1 KiB (float) wave access.
#include "phg_internal.h"

#include <math.h>

namespace phg {
namespace {

constexpr int kWavesPerBlock = 4;
constexpr int kBlock = kWavesPerBlock * kLanes;

template <typename T>
struct alignas(4 * sizeof(T)) Quad {
    T v[4];
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kLanes);
    return v;
}

__device__ __forceinline__ float exact_ldexp(float x, int e) { return ldexpf(x, e); }
__device__ __forceinline__ double exact_ldexp(double x, int e) { return ldexp(x, e); }
__device__ __forceinline__ int exponent_of(float x) {
    int e = 0;
    if (x > 0.0f) (void)frexpf(x, &e);
    return e;
}
__device__ __forceinline__ int exponent_of(double x) {
    int e = 0;
    if (x > 0.0) (void)frexp(x, &e);
    return e;
}

// Child partial of category r for this lane's pattern.  tip_code < 0 means an
// internal child read from its slot; otherwise the one-hot (or all-ones for
// code 4) tip vector is formed on the fly.
template <typename T, int R>
__device__ __forceinline__ void child_vec(const T* __restrict__ part, int slot, int tile, int tiles,
                                          int r, int lane, int tip_code, T out[4]) {
    if (tip_code < 0) {
        const Quad<T>* src = reinterpret_cast<const Quad<T>*>(part) +
                             ((static_cast<size_t>(slot) * tiles + tile) * R + r) * kLanes + lane;
        const Quad<T> q = *src;
#pragma unroll
        for (int t = 0; t < 4; ++t) out[t] = q.v[t];
    } else {
#pragma unroll
        for (int t = 0; t < 4; ++t) out[t] = (tip_code == t || tip_code >= 4) ? T(1) : T(0);
    }
}

template <typename T, int R>
__device__ __forceinline__ void store_vec(T* __restrict__ part, int slot, int tile, int tiles,
                                          int r, int lane, const T v[4]) {
    Quad<T> q;
#pragma unroll
    for (int t = 0; t < 4; ++t) q.v[t] = v[t];
    reinterpret_cast<Quad<T>*>(part)[((static_cast<size_t>(slot) * tiles + tile) * R + r) * kLanes +
                                     lane] = q;
}

// m = M v for a 4x4 row-major matrix (m_s = sum_t M_st v_t).
template <typename T>
__device__ __forceinline__ void matvec4(const T* __restrict__ M, const T v[4], T m[4]) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
        m[s] = M[4 * s + 0] * v[0] + M[4 * s + 1] * v[1] + M[4 * s + 2] * v[2] + M[4 * s + 3] * v[3];
}

// m = M^T v (m_t = sum_s M_st v_s).
template <typename T>
__device__ __forceinline__ void matvec4_t(const T* __restrict__ M, const T v[4], T m[4]) {
#pragma unroll
    for (int t = 0; t < 4; ++t)
        m[t] = M[t] * v[0] + M[4 + t] * v[1] + M[8 + t] * v[2] + M[12 + t] * v[3];
}

// ---------------------------------------------------------------- post-order

template <typename T, int R>
__global__ __launch_bounds__(kBlock) void post_s4_kernel(
    const NodeTriple* __restrict__ level, int n_units, int tiles, int N, int Cpad,
    const uint8_t* __restrict__ codes, T* __restrict__ part, int32_t* __restrict__ expo,
    const T* __restrict__ P, const double* __restrict__ cw, const double* __restrict__ pi,
    const double* __restrict__ pw, double* __restrict__ sll, double* __restrict__ lpart,
    int is_root) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & (kLanes - 1);
    const int unit = blockIdx.x * kWavesPerBlock + wave;
    if (unit >= n_units) return;
    const int node_ix = unit / tiles;
    const int tile = unit - node_ix * tiles;
    const NodeTriple nt = level[node_ix];
    const int c = tile * kLanes + lane;

    const bool tip_i = nt.i < N, tip_j = nt.j < N;
    const int code_i = tip_i ? codes[static_cast<size_t>(nt.i) * Cpad + c] : -1;
    const int code_j = tip_j ? codes[static_cast<size_t>(nt.j) * Cpad + c] : -1;
    const int ei = tip_i ? 0 : expo[static_cast<size_t>(nt.i - N) * Cpad + c];
    const int ej = tip_j ? 0 : expo[static_cast<size_t>(nt.j - N) * Cpad + c];

    T x[R][4];
    T mx = T(0);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        T vi[4], vj[4], mi[4], mj[4];
        child_vec<T, R>(part, nt.i - N, tile, tiles, r, lane, code_i, vi);
        child_vec<T, R>(part, nt.j - N, tile, tiles, r, lane, code_j, vj);
        matvec4(P + (static_cast<size_t>(nt.i) * R + r) * 16, vi, mi);
        matvec4(P + (static_cast<size_t>(nt.j) * R + r) * 16, vj, mj);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            x[r][s] = mi[s] * mj[s];
            mx = fmax(mx, x[r][s]);
        }
    }
    // one exponent per (node, pattern), shared across categories; exact
    const int e = exponent_of(mx);
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int s = 0; s < 4; ++s) x[r][s] = exact_ldexp(x[r][s], -e);
    const int ek = e + ei + ej;

    if (!is_root) {
#pragma unroll
        for (int r = 0; r < R; ++r) store_vec<T, R>(part, nt.k - N, tile, tiles, r, lane, x[r]);
        expo[static_cast<size_t>(nt.k - N) * Cpad + c] = ek;
    } else {
        double site = 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            double acc = 0.0;
#pragma unroll
            for (int s = 0; s < 4; ++s) acc += pi[s] * static_cast<double>(x[r][s]);
            site += cw[r] * acc;
        }
        // ln of a zero (or round-off negative) site likelihood is -inf
        const double ll = (site > 0.0 ? log(site) : -INFINITY) + static_cast<double>(ek) * 0.69314718055994530942;
        sll[c] = ll;
        const double W = pw[c];
        const double tsum = wave_sum(W != 0.0 ? W * ll : 0.0);
        if (lane == 0) lpart[tile] = tsum;
    }
}

// ---------------------------------------------------------------- pre-order + gradient

template <typename T, int R>
__global__ __launch_bounds__(kBlock) void pre_s4_kernel(
    const NodeTriple* __restrict__ level, int n_units, int tiles, int N, int Cpad,
    const uint8_t* __restrict__ codes, T* __restrict__ part, const T* __restrict__ P,
    const T* __restrict__ dP, const double* __restrict__ cw, const double* __restrict__ pi,
    const double* __restrict__ pw, double* __restrict__ gpart) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & (kLanes - 1);
    const int unit = blockIdx.x * kWavesPerBlock + wave;
    if (unit >= n_units) return;
    const int node_ix = unit / tiles;
    const int tile = unit - node_ix * tiles;
    const NodeTriple nt = level[node_ix];
    const int c = tile * kLanes + lane;
    const bool is_root = nt.k == 2 * N - 2;

    const bool tip_i = nt.i < N, tip_j = nt.j < N;
    const int code_i = tip_i ? codes[static_cast<size_t>(nt.i) * Cpad + c] : -1;
    const int code_j = tip_j ? codes[static_cast<size_t>(nt.j) * Cpad + c] : -1;

    T qi[R][4], qj[R][4];
    T num_i = T(0), num_j = T(0), den = T(0);
    T mxi = T(0), mxj = T(0);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        T q[4];
        if (is_root) {
#pragma unroll
            for (int s = 0; s < 4; ++s) q[s] = static_cast<T>(pi[s]);
        } else {
            child_vec<T, R>(part, nt.k - N, tile, tiles, r, lane, -1, q);
        }
        T vi[4], vj[4], mi[4], mj[4], dmi[4], dmj[4], ui[4], uj[4];
        child_vec<T, R>(part, nt.i - N, tile, tiles, r, lane, code_i, vi);
        child_vec<T, R>(part, nt.j - N, tile, tiles, r, lane, code_j, vj);
        const T* Pi = P + (static_cast<size_t>(nt.i) * R + r) * 16;
        const T* Pj = P + (static_cast<size_t>(nt.j) * R + r) * 16;
        matvec4(Pi, vi, mi);
        matvec4(Pj, vj, mj);
        matvec4(dP + (static_cast<size_t>(nt.i) * R + r) * 16, vi, dmi);
        matvec4(dP + (static_cast<size_t>(nt.j) * R + r) * 16, vj, dmj);
        T a = T(0), bj = T(0), dd = T(0);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            ui[s] = q[s] * mj[s];
            uj[s] = q[s] * mi[s];
            a += ui[s] * dmi[s];
            bj += uj[s] * dmj[s];
            dd += ui[s] * mi[s];
        }
        const T wr = static_cast<T>(cw[r]);
        num_i += wr * a;
        num_j += wr * bj;
        den += wr * dd;
        if (!tip_i) {
            matvec4_t(Pi, ui, qi[r]);
#pragma unroll
            for (int s = 0; s < 4; ++s) mxi = fmax(mxi, qi[r][s]);
        }
        if (!tip_j) {
            matvec4_t(Pj, uj, qj[r]);
#pragma unroll
            for (int s = 0; s < 4; ++s) mxj = fmax(mxj, qj[r][s]);
        }
    }
    // pre-order partials: renormalise by a power of two shared across
    // categories (the gradient ratio is invariant to it), overwrite p in place
    if (!tip_i) {
        const int e = exponent_of(mxi);
#pragma unroll
        for (int r = 0; r < R; ++r) {
#pragma unroll
            for (int s = 0; s < 4; ++s) qi[r][s] = exact_ldexp(qi[r][s], -e);
            store_vec<T, R>(part, nt.i - N, tile, tiles, r, lane, qi[r]);
        }
    }
    if (!tip_j) {
        const int e = exponent_of(mxj);
#pragma unroll
        for (int r = 0; r < R; ++r) {
#pragma unroll
            for (int s = 0; s < 4; ++s) qj[r][s] = exact_ldexp(qj[r][s], -e);
            store_vec<T, R>(part, nt.j - N, tile, tiles, r, lane, qj[r]);
        }
    }
    const double W = pw[c];
    const double dden = static_cast<double>(den);
    const double gi = (W != 0.0) ? W * (static_cast<double>(num_i) / dden) : 0.0;
    const double gj = (W != 0.0) ? W * (static_cast<double>(num_j) / dden) : 0.0;
    const double si = wave_sum(gi);
    const double sj = wave_sum(gj);
    if (lane == 0) {
        gpart[static_cast<size_t>(nt.i) * tiles + tile] = si;
        gpart[static_cast<size_t>(nt.j) * tiles + tile] = sj;
    }
}

// ---------------------------------------------------------------- P(t), dP/dt

template <bool kF32>
__global__ __launch_bounds__(256) void pmat_kernel(int E, int R, int S, const double* __restrict__ b,
                                                   const double* __restrict__ V,
                                                   const double* __restrict__ Vinv,
                                                   const double* __restrict__ lam,
                                                   const double* __restrict__ rates,
                                                   double* __restrict__ P64, double* __restrict__ dP64,
                                                   float* __restrict__ P32, float* __restrict__ dP32) {
    __shared__ double ex[64], dex[64];
    const int pair = blockIdx.x;
    const int x = pair / R;
    const int r = pair - x * R;
    const double g = rates[r];
    const double t = g * b[x];
    for (int k = threadIdx.x; k < S; k += blockDim.x) {
        const double e = exp(lam[k] * t);
        ex[k] = e;
        dex[k] = g * lam[k] * e;
    }
    __syncthreads();
    const size_t base = static_cast<size_t>(pair) * S * S;
    for (int e = threadIdx.x; e < S * S; e += blockDim.x) {
        const int s = e / S;
        const int u = e - s * S;
        double acc = 0.0, dacc = 0.0;
        for (int k = 0; k < S; ++k) {
            const double v = V[s * S + k] * Vinv[k * S + u];
            acc += v * ex[k];
            dacc += v * dex[k];
        }
        P64[base + e] = acc;
        dP64[base + e] = dacc;
        if (kF32) {
            P32[base + e] = static_cast<float>(acc);
            dP32[base + e] = static_cast<float>(dacc);
        }
    }
}

// ---------------------------------------------------------------- final sums

// Block x < E sums branch x's per-tile gradient partials; block E sums the
// per-tile weighted log-likelihood partials.  Fixed order: deterministic.
__global__ __launch_bounds__(256) void finalize_kernel(const double* __restrict__ gpart, int tiles,
                                                       int E, const double* __restrict__ lpart,
                                                       double* __restrict__ out_logl,
                                                       double* __restrict__ out_grad) {
    __shared__ double red[256];
    const int blk = blockIdx.x;
    const double* src = blk < E ? gpart + static_cast<size_t>(blk) * tiles : lpart;
    double acc = 0.0;
    for (int t = threadIdx.x; t < tiles; t += 256) acc += src[t];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (blk < E)
            out_grad[blk] = red[0];
        else
            *out_logl = red[0];
    }
}

template <typename T>
const T* ptab(const DeviceProblem& d);
template <>
const float* ptab<float>(const DeviceProblem& d) { return d.P32; }
template <>
const double* ptab<double>(const DeviceProblem& d) { return d.P64; }
template <typename T>
const T* dptab(const DeviceProblem& d);
template <>
const float* dptab<float>(const DeviceProblem& d) { return d.dP32; }
template <>
const double* dptab<double>(const DeviceProblem& d) { return d.dP64; }

template <typename T, int R>
hipError_t post_r(const DeviceProblem& d, const NodeTriple* level, int n_nodes, bool is_root,
                  hipStream_t st) {
    const int n_units = n_nodes * d.tiles;
    const int blocks = (n_units + kWavesPerBlock - 1) / kWavesPerBlock;
    hipLaunchKernelGGL((post_s4_kernel<T, R>), dim3(blocks), dim3(kBlock), 0, st, level, n_units,
                       d.tiles, d.N, d.Cpad, d.codes, static_cast<T*>(d.part), d.expo, ptab<T>(d),
                       d.cweights, d.pi, d.pw, d.sll, d.lpart, is_root ? 1 : 0);
    return hipGetLastError();
}

template <typename T, int R>
hipError_t pre_r(const DeviceProblem& d, const NodeTriple* level, int n_nodes, hipStream_t st) {
    const int n_units = n_nodes * d.tiles;
    const int blocks = (n_units + kWavesPerBlock - 1) / kWavesPerBlock;
    hipLaunchKernelGGL((pre_s4_kernel<T, R>), dim3(blocks), dim3(kBlock), 0, st, level, n_units,
                       d.tiles, d.N, d.Cpad, d.codes, static_cast<T*>(d.part), ptab<T>(d),
                       dptab<T>(d), d.cweights, d.pi, d.pw, d.gpart);
    return hipGetLastError();
}

#define PHG_DISPATCH_R(FN, T, ...)                  \
    switch (d.R) {                                  \
        case 1: return FN<T, 1>(d, __VA_ARGS__);    \
        case 2: return FN<T, 2>(d, __VA_ARGS__);    \
        case 3: return FN<T, 3>(d, __VA_ARGS__);    \
        case 4: return FN<T, 4>(d, __VA_ARGS__);    \
        case 5: return FN<T, 5>(d, __VA_ARGS__);    \
        case 6: return FN<T, 6>(d, __VA_ARGS__);    \
        case 7: return FN<T, 7>(d, __VA_ARGS__);    \
        case 8: return FN<T, 8>(d, __VA_ARGS__);    \
        default: return hipErrorInvalidValue;       \
    }

}  // namespace

bool kernels_support(int S, int R) { return S == 4 && R >= 1 && R <= 8; }

hipError_t launch_pmat(const DeviceProblem& d, bool fp32, hipStream_t st) {
    const int E = 2 * d.N - 2;
    if (fp32)
        hipLaunchKernelGGL((pmat_kernel<true>), dim3(E * d.R), dim3(256), 0, st, E, d.R, d.S, d.b, d.V,
                           d.Vinv, d.lam, d.rates, d.P64, d.dP64, d.P32, d.dP32);
    else
        hipLaunchKernelGGL((pmat_kernel<false>), dim3(E * d.R), dim3(256), 0, st, E, d.R, d.S, d.b,
                           d.V, d.Vinv, d.lam, d.rates, d.P64, d.dP64, d.P32, d.dP32);
    return hipGetLastError();
}

hipError_t launch_post_level(const DeviceProblem& d, bool fp32, const NodeTriple* level, int n_nodes,
                             bool is_root, hipStream_t st) {
    if (fp32) {
        PHG_DISPATCH_R(post_r, float, level, n_nodes, is_root, st);
    } else {
        PHG_DISPATCH_R(post_r, double, level, n_nodes, is_root, st);
    }
}

hipError_t launch_pre_level(const DeviceProblem& d, bool fp32, const NodeTriple* level, int n_nodes,
                            hipStream_t st) {
    if (fp32) {
        PHG_DISPATCH_R(pre_r, float, level, n_nodes, st);
    } else {
        PHG_DISPATCH_R(pre_r, double, level, n_nodes, st);
    }
}

hipError_t launch_finalize(const DeviceProblem& d, double* out_logl, double* out_grad,
                           hipStream_t st) {
    const int E = 2 * d.N - 2;
    hipLaunchKernelGGL(finalize_kernel, dim3(E + 1), dim3(256), 0, st, d.gpart, d.tiles, E, d.lpart,
                       out_logl, out_grad);
    return hipGetLastError();
}

}  // namespace phg
