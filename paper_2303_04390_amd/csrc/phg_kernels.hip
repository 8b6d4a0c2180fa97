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
//             (eq:gradientSumAcrossColumns) and over tiles for log P(Y).
//
// Every launch carries a segment table: each segment is one request's slice
// (a level of its tree, or its whole pmat / finalize stage), so one launch
// can advance several requests of different trees at once.  Per-request
// pointers and sizes come from a device-resident descriptor table.
//
// Work unit of the level kernels: one wavefront = (one node, one tile of 64
// consecutive patterns); lane = pattern.  For S = 4 each lane keeps the R x 4
// values of its pattern in registers and loops over categories; P and dP of a
// branch are the same for every lane, so they come through scalar loads.
// Partials are stored [slot][tile][r][lane][4], so each category of a unit is
// one contiguous 1 KiB (float) wave access.
#include "phg_internal.h"

#include <math.h>

namespace phg {
namespace {

constexpr int kWavesPerBlock = 4;
constexpr int kBlock = kWavesPerBlock * kLanes;

// Pointers read from a request descriptor are generic (flat) pointers; the
// unit bodies take them in the global address space so that loads are global
// loads and wave-uniform ones (P, dP, pi, weights) become scalar loads.
#define GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ GLOBAL T* g(T* p) {
    return (GLOBAL T*)p;
}

// Four consecutive values of one lane as a native vector (one 16 B / 32 B access).
template <typename T>
struct Vec4T;
template <>
struct Vec4T<float> {
    typedef float type __attribute__((ext_vector_type(4)));
};
template <>
struct Vec4T<double> {
    typedef double type __attribute__((ext_vector_type(4)));
};
template <typename T>
using Vec4 = typename Vec4T<T>::type;
typedef int Int4 __attribute__((ext_vector_type(4)));

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

template <typename T>
__device__ __forceinline__ T* part_of(const ReqDesc& d) {
    return static_cast<T*>(d.part);
}
template <typename T>
__device__ __forceinline__ const T* ptab(const ReqDesc& d);
template <>
__device__ __forceinline__ const float* ptab<float>(const ReqDesc& d) { return d.P32; }
template <>
__device__ __forceinline__ const double* ptab<double>(const ReqDesc& d) { return d.P64; }
template <typename T>
__device__ __forceinline__ const T* dptab(const ReqDesc& d);
template <>
__device__ __forceinline__ const float* dptab<float>(const ReqDesc& d) { return d.dP32; }
template <>
__device__ __forceinline__ const double* dptab<double>(const ReqDesc& d) { return d.dP64; }

// Segment of a (wave-uniform) unit index: linear scan of the table.
__device__ __forceinline__ int find_segment(const SegTable& t, int unit) {
    int s = 0;
    while (s + 1 < t.n && unit >= t.unit_begin[s + 1]) ++s;
    return s;
}

// Child partial of category r for this lane's pattern.  tip_code < 0 means an
// internal child read from its slot; otherwise the one-hot (or all-ones for
// code 4) tip vector is formed on the fly.
template <typename T, int R>
__device__ __forceinline__ void child_vec(const GLOBAL T* __restrict__ part, int slot, int tile, int tiles,
                                          int r, int lane, int tip_code, T out[4]) {
    if (tip_code < 0) {
        const GLOBAL Vec4<T>* src = reinterpret_cast<const GLOBAL Vec4<T>*>(part) +
                                    ((static_cast<size_t>(slot) * tiles + tile) * R + r) * kLanes + lane;
        const Vec4<T> q = *src;
        out[0] = q.x;
        out[1] = q.y;
        out[2] = q.z;
        out[3] = q.w;
    } else {
#pragma unroll
        for (int t = 0; t < 4; ++t) out[t] = (tip_code == t || tip_code >= 4) ? T(1) : T(0);
    }
}

template <typename T, int R>
__device__ __forceinline__ void store_vec(GLOBAL T* __restrict__ part, int slot, int tile, int tiles,
                                          int r, int lane, const T v[4]) {
    Vec4<T> q;
    q.x = v[0];
    q.y = v[1];
    q.z = v[2];
    q.w = v[3];
    reinterpret_cast<GLOBAL Vec4<T>*>(part)[((static_cast<size_t>(slot) * tiles + tile) * R + r) * kLanes +
                                            lane] = q;
}

// m = M v for a 4x4 row-major matrix (m_s = sum_t M_st v_t).
template <typename T>
__device__ __forceinline__ void matvec4(const GLOBAL T* __restrict__ M, const T v[4], T m[4]) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
        m[s] = M[4 * s + 0] * v[0] + M[4 * s + 1] * v[1] + M[4 * s + 2] * v[2] + M[4 * s + 3] * v[3];
}

// m = M^T v (m_t = sum_s M_st v_s).
template <typename T>
__device__ __forceinline__ void matvec4_t(const GLOBAL T* __restrict__ M, const T v[4], T m[4]) {
#pragma unroll
    for (int t = 0; t < 4; ++t)
        m[t] = M[t] * v[0] + M[4 + t] * v[1] + M[8 + t] * v[2] + M[12 + t] * v[3];
}

// ---------------------------------------------------------------- post-order

// Body of one post-order unit.  Pointer parameters are __restrict__ so that,
// once inlined, the compiler knows the stores to part/expo cannot alias the
// matrices and keeps the wave-uniform P loads on the scalar unit.
template <typename T, int R>
__device__ __forceinline__ void post_unit(const NodeTriple nt, const int tile, const int tiles,
                                          const int N, const int Cpad, const int lane, const int flags,
                                          const GLOBAL uint8_t* __restrict__ codes,
                                          GLOBAL T* __restrict__ part, GLOBAL int32_t* __restrict__ expo,
                                          const GLOBAL T* __restrict__ P,
                                          const GLOBAL double* __restrict__ cw,
                                          const GLOBAL double* __restrict__ pi,
                                          const GLOBAL double* __restrict__ pw,
                                          GLOBAL double* __restrict__ sll,
                                          GLOBAL double* __restrict__ lpart) {
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

    if (!(flags & 1)) {
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
        const double ll =
            (site > 0.0 ? log(site) : -INFINITY) + static_cast<double>(ek) * 0.69314718055994530942;
        sll[c] = ll;
        const double W = pw[c];
        const double tsum = wave_sum(W != 0.0 ? W * ll : 0.0);
        if (lane == 0) lpart[tile] = tsum;
    }
}

template <typename T, int R>
__global__ __launch_bounds__(kBlock) void post_s4_kernel(const ReqDesc* __restrict__ descs,
                                                         const SegTable segs) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & (kLanes - 1);
    const int unit = blockIdx.x * kWavesPerBlock + wave;
    if (unit >= segs.unit_begin[segs.n]) return;
    const int sidx = find_segment(segs, unit);
    const Segment sg = segs.seg[sidx];
    const ReqDesc& d = descs[sg.desc];
    const int tiles = d.tiles;
    const int local = unit - segs.unit_begin[sidx];
    const int node_ix = local / tiles;
    const int tile = local - node_ix * tiles;
    const Int4 t4 = reinterpret_cast<const GLOBAL Int4*>(g(d.sched))[sg.sched_off + node_ix];
    const NodeTriple nt{t4.x, t4.y, t4.z, 0};
    post_unit<T, R>(nt, tile, tiles, d.N, d.Cpad, lane, sg.flags, g(d.codes), g(part_of<T>(d)),
                    g(d.expo), g(ptab<T>(d)), g(d.cweights), g(d.pi), g(d.pw), g(d.sll), g(d.lpart));
}

// ---------------------------------------------------------------- pre-order + gradient

// Body of one pre-order + gradient unit (restrict parameters: see post_unit).
template <typename T, int R>
__device__ __forceinline__ void pre_unit(const NodeTriple nt, const int tile, const int tiles,
                                         const int N, const int Cpad, const int lane,
                                         const GLOBAL uint8_t* __restrict__ codes,
                                         GLOBAL T* __restrict__ part, const GLOBAL T* __restrict__ P,
                                         const GLOBAL T* __restrict__ dP,
                                         const GLOBAL double* __restrict__ cw,
                                         const GLOBAL double* __restrict__ pi,
                                         const GLOBAL double* __restrict__ pw,
                                         GLOBAL double* __restrict__ gpart) {
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
        const GLOBAL T* Pi = P + (static_cast<size_t>(nt.i) * R + r) * 16;
        const GLOBAL T* Pj = P + (static_cast<size_t>(nt.j) * R + r) * 16;
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


template <typename T, int R>
__global__ __launch_bounds__(kBlock) void pre_s4_kernel(const ReqDesc* __restrict__ descs,
                                                        const SegTable segs) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & (kLanes - 1);
    const int unit = blockIdx.x * kWavesPerBlock + wave;
    if (unit >= segs.unit_begin[segs.n]) return;
    const int sidx = find_segment(segs, unit);
    const Segment sg = segs.seg[sidx];
    const ReqDesc& d = descs[sg.desc];
    const int tiles = d.tiles;
    const int local = unit - segs.unit_begin[sidx];
    const int node_ix = local / tiles;
    const int tile = local - node_ix * tiles;
    const Int4 t4 = reinterpret_cast<const GLOBAL Int4*>(g(d.sched))[sg.sched_off + node_ix];
    const NodeTriple nt{t4.x, t4.y, t4.z, 0};
    pre_unit<T, R>(nt, tile, tiles, d.N, d.Cpad, lane, g(d.codes), g(part_of<T>(d)), g(ptab<T>(d)),
                   g(dptab<T>(d)), g(d.cweights), g(d.pi), g(d.pw), g(d.gpart));
}

// ---------------------------------------------------------------- P(t), dP/dt

// Small S (<= 8): one thread per (branch, category) pair builds the whole
// S x S pair of matrices.  Units are pairs; a block covers 256 of them.
template <int S>
__global__ __launch_bounds__(256) void pmat_small_kernel(const ReqDesc* __restrict__ descs,
                                                         const SegTable segs) {
    const int unit = blockIdx.x * 256 + threadIdx.x;
    if (unit >= segs.unit_begin[segs.n]) return;
    int sidx = 0;
    while (sidx + 1 < segs.n && unit >= segs.unit_begin[sidx + 1]) ++sidx;
    const ReqDesc& d = descs[segs.seg[sidx].desc];
    const int pair = unit - segs.unit_begin[sidx];
    const int R = d.R;
    const int x = pair / R;
    const int r = pair - x * R;
    const double g = d.rates[r];
    const double t = g * d.b[x];
    double ex[S], dex[S];
#pragma unroll
    for (int k = 0; k < S; ++k) {
        const double e = exp(d.lam[k] * t);
        ex[k] = e;
        dex[k] = g * d.lam[k] * e;
    }
    const size_t base = static_cast<size_t>(pair) * S * S;
#pragma unroll
    for (int s = 0; s < S; ++s) {
#pragma unroll
        for (int u = 0; u < S; ++u) {
            double acc = 0.0, dacc = 0.0;
#pragma unroll
            for (int k = 0; k < S; ++k) {
                const double v = d.V[s * S + k] * d.Vinv[k * S + u];
                acc += v * ex[k];
                dacc += v * dex[k];
            }
            d.P64[base + s * S + u] = acc;
            d.dP64[base + s * S + u] = dacc;
            if (d.fp32) {
                d.P32[base + s * S + u] = static_cast<float>(acc);
                d.dP32[base + s * S + u] = static_cast<float>(dacc);
            }
        }
    }
}

// Any S <= 64: one block per (branch, category) pair.
__global__ __launch_bounds__(256) void pmat_block_kernel(const ReqDesc* __restrict__ descs,
                                                         const SegTable segs) {
    __shared__ double ex[64], dex[64];
    const int unit = blockIdx.x;
    if (unit >= segs.unit_begin[segs.n]) return;
    const int sidx = find_segment(segs, unit);
    const ReqDesc& d = descs[segs.seg[sidx].desc];
    const int pair = unit - segs.unit_begin[sidx];
    const int R = d.R, S = d.S;
    const int x = pair / R;
    const int r = pair - x * R;
    const double g = d.rates[r];
    const double t = g * d.b[x];
    for (int k = threadIdx.x; k < S; k += blockDim.x) {
        const double e = exp(d.lam[k] * t);
        ex[k] = e;
        dex[k] = g * d.lam[k] * e;
    }
    __syncthreads();
    const size_t base = static_cast<size_t>(pair) * S * S;
    for (int e = threadIdx.x; e < S * S; e += blockDim.x) {
        const int s = e / S;
        const int u = e - s * S;
        double acc = 0.0, dacc = 0.0;
        for (int k = 0; k < S; ++k) {
            const double v = d.V[s * S + k] * d.Vinv[k * S + u];
            acc += v * ex[k];
            dacc += v * dex[k];
        }
        d.P64[base + e] = acc;
        d.dP64[base + e] = dacc;
        if (d.fp32) {
            d.P32[base + e] = static_cast<float>(acc);
            d.dP32[base + e] = static_cast<float>(dacc);
        }
    }
}

// ---------------------------------------------------------------- final sums

// Unit x < E sums branch x's per-tile gradient partials; unit E sums the
// per-tile weighted log-likelihood partials.  Fixed order: deterministic.
__global__ __launch_bounds__(256) void finalize_kernel(const ReqDesc* __restrict__ descs,
                                                       const SegTable segs) {
    __shared__ double red[256];
    const int unit = blockIdx.x;
    if (unit >= segs.unit_begin[segs.n]) return;
    const int sidx = find_segment(segs, unit);
    const Segment& sg = segs.seg[sidx];
    const ReqDesc& d = descs[sg.desc];
    const int blk = unit - segs.unit_begin[sidx];
    const int E = 2 * d.N - 2, tiles = d.tiles;
    const double* src = blk < E ? d.gpart + static_cast<size_t>(blk) * tiles : d.lpart;
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
            sg.out_grad[blk] = red[0];
        else
            *sg.out_logl = red[0];
    }
}

template <typename T, int R>
hipError_t level_r(KernelClass k, const ReqDesc* descs, const SegTable& t, hipStream_t st) {
    const int n_units = t.unit_begin[t.n];
    const int blocks = (n_units + kWavesPerBlock - 1) / kWavesPerBlock;
    if (k == kPost)
        hipLaunchKernelGGL((post_s4_kernel<T, R>), dim3(blocks), dim3(kBlock), 0, st, descs, t);
    else
        hipLaunchKernelGGL((pre_s4_kernel<T, R>), dim3(blocks), dim3(kBlock), 0, st, descs, t);
    return hipGetLastError();
}

template <typename T>
hipError_t level_t(KernelClass k, int R, const ReqDesc* descs, const SegTable& t, hipStream_t st) {
    switch (R) {
        case 1: return level_r<T, 1>(k, descs, t, st);
        case 2: return level_r<T, 2>(k, descs, t, st);
        case 3: return level_r<T, 3>(k, descs, t, st);
        case 4: return level_r<T, 4>(k, descs, t, st);
        case 5: return level_r<T, 5>(k, descs, t, st);
        case 6: return level_r<T, 6>(k, descs, t, st);
        case 7: return level_r<T, 7>(k, descs, t, st);
        case 8: return level_r<T, 8>(k, descs, t, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

bool kernels_support(int S, int R) { return S >= 2 && S <= 64 && R >= 1 && R <= 16; }

int tile_patterns(int S, int R, bool fp32) {
    return uses_s4_kernels(S, R) ? kLanes : gs_tile_patterns(fp32);
}

int units_for(KernelClass k, const ReqDesc& d, int n_nodes) {
    switch (k) {
        case kPmat: return (2 * d.N - 2) * d.R;
        case kPost:
        case kPre: return n_nodes * d.tiles;
        case kFinal: return 2 * d.N - 1;
    }
    return 0;
}

hipError_t launch_class(KernelClass k, const ReqDesc& shape, const ReqDesc* descs, const SegTable& t,
                        hipStream_t st) {
    const int n_units = t.unit_begin[t.n];
    if (t.n <= 0 || n_units <= 0) return hipSuccess;
    switch (k) {
        case kPmat:
            if (shape.S == 4) {
                hipLaunchKernelGGL((pmat_small_kernel<4>), dim3((n_units + 255) / 256), dim3(256), 0, st,
                                   descs, t);
            } else {
                hipLaunchKernelGGL(pmat_block_kernel, dim3(n_units), dim3(256), 0, st, descs, t);
            }
            return hipGetLastError();
        case kPost:
        case kPre:
            if (!uses_s4_kernels(shape.S, shape.R)) return launch_level_gs(k, shape, descs, t, st);
            if (shape.fp32) return level_t<float>(k, shape.R, descs, t, st);
            return level_t<double>(k, shape.R, descs, t, st);
        case kFinal:
            hipLaunchKernelGGL(finalize_kernel, dim3(n_units), dim3(256), 0, st, descs, t);
            return hipGetLastError();
    }
    return hipErrorInvalidValue;
}

}  // namespace phg
