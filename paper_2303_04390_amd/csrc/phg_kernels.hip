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

template <typename T>
__device__ __forceinline__ const T* ttab(const ReqDesc& d);
template <>
__device__ __forceinline__ const float* ttab<float>(const ReqDesc& d) { return d.TT32; }
template <>
__device__ __forceinline__ const double* ttab<double>(const ReqDesc& d) { return d.TT64; }
template <typename T>
__device__ __forceinline__ const T* dttab(const ReqDesc& d);
template <>
__device__ __forceinline__ const float* dttab<float>(const ReqDesc& d) { return d.dTT32; }
template <>
__device__ __forceinline__ const double* dttab<double>(const ReqDesc& d) { return d.dTT64; }

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

// ---------------------------------------------------------------- blocked schedule (4 states)
//
// A block (BlockRec) is a block root with its internal children and
// grandchildren, laid out as a heap of positions 1..15.  Only block roots'
// partials live in HBM: the post-order unit computes the in-block partials in
// registers (positions 7..1) and stores the block root's; the pre-order unit
// recomputes the in-block partials from the frontier, then walks positions
// 1..7 top-down keeping in-block pre-order partials in registers and writing
// only the frontier block roots' q.  Heap positions are compile-time
// constants after unrolling, so every in-block vector is a register.
//
// One workgroup = one (block, 64-pattern tile) unit with one wavefront per
// rate category (lane = pattern), so a wave holds 4 values per vector and
// only its own category's P and dP (scalar registers).  What couples the
// categories -- the shared power-of-two exponent of each node's partial and
// the category sums in the gradient ratio -- goes through LDS with one barrier
// per node (every wave follows the same block shape, so the barrier is
// uniform).  Tip children use the tip tables: P e_y and dP e_y are one load.

template <typename T, int R>
struct Xch {
    T v[2][5][R][kLanes];     // double-buffered exchange: [buf][field][category][lane]
};

// m = P_x v for the child at heap position CP in category r: a tip-table load
// for a tip, else P times the in-block partial (CP < 8) or the frontier
// block root's stored partial (CP >= 8).
template <typename T, int R>
__device__ __forceinline__ void blk_m(const int cp, const int cn, const int N, const int r, const int tile,
                                      const int tiles, const int lane, const int code,
                                      const GLOBAL T* __restrict__ part, const GLOBAL T* __restrict__ M,
                                      const GLOBAL T* __restrict__ TT, const T (&preg)[8][4], T m[4]) {
    if (cn < N) {
        const Vec4<T> t = reinterpret_cast<const GLOBAL Vec4<T>*>(TT)[(static_cast<size_t>(cn) * R + r) * 5 + code];
        m[0] = t.x;
        m[1] = t.y;
        m[2] = t.z;
        m[3] = t.w;
        return;
    }
    T v[4];
    if (cp < 8) {
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = preg[cp][u];
    } else {
        child_vec<T, R>(part, cn - N, tile, tiles, r, lane, -1, v);
    }
    matvec4(M + (static_cast<size_t>(cn) * R + r) * 16, v, m);
}

// In-block post-order over heap positions 7..LO in this wave's category.
// Returns the sum of exponents taken (in-block nodes and frontier roots).
template <typename T, int R, int LO>
__device__ __forceinline__ int blkc_postorder(const int (&nd)[16], const int r, const int tile, const int tiles,
                                              const int N, const int Cpad, const int lane,
                                              const GLOBAL uint8_t* __restrict__ codes,
                                              const GLOBAL T* __restrict__ part,
                                              const GLOBAL int32_t* __restrict__ expo,
                                              const GLOBAL T* __restrict__ P, const GLOBAL T* __restrict__ TT,
                                              T (&p)[8][4], Xch<T, R>& xch, int& buf) {
    const int c = tile * kLanes + lane;
    int esum = 0;
#pragma unroll
    for (int pos = 7; pos >= LO; --pos) {
        const int k = nd[pos];
        if (k < N) continue;                       // absent or a tip (uniform over the workgroup)
        const int c0 = nd[2 * pos], c1 = nd[2 * pos + 1];
        const int code0 = c0 < N ? codes[static_cast<size_t>(c0) * Cpad + c] : 0;
        const int code1 = c1 < N ? codes[static_cast<size_t>(c1) * Cpad + c] : 0;
        if (2 * pos >= 8) {
            if (c0 >= N) esum += expo[static_cast<size_t>(c0 - N) * Cpad + c];
            if (c1 >= N) esum += expo[static_cast<size_t>(c1 - N) * Cpad + c];
        }
        T m0[4], m1[4];
        blk_m<T, R>(2 * pos, c0, N, r, tile, tiles, lane, code0, part, P, TT, p, m0);
        blk_m<T, R>(2 * pos + 1, c1, N, r, tile, tiles, lane, code1, part, P, TT, p, m1);
        T lmx = T(0);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            p[pos][u] = m0[u] * m1[u];
            lmx = fmax(lmx, p[pos][u]);
        }
        xch.v[buf][0][r][lane] = lmx;
        __syncthreads();
        T mx = xch.v[buf][0][0][lane];
#pragma unroll
        for (int rr = 1; rr < R; ++rr) mx = fmax(mx, xch.v[buf][0][rr][lane]);
        buf ^= 1;
        const int e = exponent_of(mx);
#pragma unroll
        for (int u = 0; u < 4; ++u) p[pos][u] = exact_ldexp(p[pos][u], -e);
        esum += e;
    }
    return esum;
}

template <typename T, int R>
__global__ __launch_bounds__(kLanes * R) void post_blk_kernel(const ReqDesc* __restrict__ descs,
                                                              const SegTable segs) {
    __shared__ Xch<T, R> xch;
    __shared__ double sx[R][kLanes];
    const int r = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & (kLanes - 1);
    const int unit = blockIdx.x;
    if (unit >= segs.unit_begin[segs.n]) return;
    const int sidx = find_segment(segs, unit);
    const Segment sg = segs.seg[sidx];
    const ReqDesc& d = descs[sg.desc];
    const int tiles = d.tiles, N = d.N, Cpad = d.Cpad;
    const int local = unit - segs.unit_begin[sidx];
    const int bix = local / tiles;
    const int tile = local - bix * tiles;
    const GLOBAL int32_t* heap =
        reinterpret_cast<const GLOBAL int32_t*>(g(d.sched)) + static_cast<size_t>(sg.sched_off + bix) * 16;
    int nd[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) nd[i] = heap[i];
    GLOBAL T* part = g(part_of<T>(d));
    GLOBAL int32_t* expo = g(d.expo);
    const GLOBAL T* P = g(ptab<T>(d));
    const GLOBAL T* TT = g(ttab<T>(d));
    const int c = tile * kLanes + lane;
    T p[8][4];
    int buf = 0;
    const int ek = blkc_postorder<T, R, 1>(nd, r, tile, tiles, N, Cpad, lane, g(d.codes), part, expo, P, TT,
                                           p, xch, buf);
    if (!(sg.flags & 1)) {
        store_vec<T, R>(part, nd[1] - N, tile, tiles, r, lane, p[1]);
        if (r == 0) expo[static_cast<size_t>(nd[1] - N) * Cpad + c] = ek;
    } else {
        const GLOBAL double* pi = g(d.pi);
        double acc = 0.0;
#pragma unroll
        for (int u = 0; u < 4; ++u) acc += pi[u] * static_cast<double>(p[1][u]);
        sx[r][lane] = g(d.cweights)[r] * acc;
        __syncthreads();
        if (r == 0) {
            double site = 0.0;
#pragma unroll
            for (int rr = 0; rr < R; ++rr) site += sx[rr][lane];
            const double ll =
                (site > 0.0 ? log(site) : -INFINITY) + static_cast<double>(ek) * 0.69314718055994530942;
            g(d.sll)[c] = ll;
            const double W = g(d.pw)[c];
            const double tsum = wave_sum(W != 0.0 ? W * ll : 0.0);
            if (lane == 0) g(d.lpart)[tile] = tsum;
        }
    }
}

template <typename T, int R>
__global__ __launch_bounds__(kLanes * R) void pre_blk_kernel(const ReqDesc* __restrict__ descs,
                                                             const SegTable segs) {
    __shared__ Xch<T, R> xch;
    const int r = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & (kLanes - 1);
    const int unit = blockIdx.x;
    if (unit >= segs.unit_begin[segs.n]) return;
    const int sidx = find_segment(segs, unit);
    const Segment sg = segs.seg[sidx];
    const ReqDesc& d = descs[sg.desc];
    const int tiles = d.tiles, N = d.N, Cpad = d.Cpad;
    const int local = unit - segs.unit_begin[sidx];
    const int bix = local / tiles;
    const int tile = local - bix * tiles;
    const GLOBAL int32_t* heap =
        reinterpret_cast<const GLOBAL int32_t*>(g(d.sched)) + static_cast<size_t>(sg.sched_off + bix) * 16;
    int nd[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) nd[i] = heap[i];
    GLOBAL T* part = g(part_of<T>(d));
    const GLOBAL uint8_t* codes = g(d.codes);
    const GLOBAL T* P = g(ptab<T>(d));
    const GLOBAL T* dP = g(dptab<T>(d));
    const GLOBAL T* TT = g(ttab<T>(d));
    const GLOBAL T* dTT = g(dttab<T>(d));
    GLOBAL double* gpart = g(d.gpart);
    const int c = tile * kLanes + lane;
    T p[8][4];
    int buf = 0;
    (void)blkc_postorder<T, R, 2>(nd, r, tile, tiles, N, Cpad, lane, codes, part, g(d.expo), P, TT, p, xch, buf);
    T q[8][4];
    if (nd[1] == 2 * N - 2) {
        const GLOBAL double* pi = g(d.pi);
#pragma unroll
        for (int u = 0; u < 4; ++u) q[1][u] = static_cast<T>(pi[u]);
    } else {
        child_vec<T, R>(part, nd[1] - N, tile, tiles, r, lane, -1, q[1]);
    }
    const double W = g(d.pw)[c];
    const T wr = static_cast<T>(g(d.cweights)[r]);
#pragma unroll
    for (int pos = 1; pos <= 7; ++pos) {
        const int k = nd[pos];
        if (k < N) continue;
        const int c0 = nd[2 * pos], c1 = nd[2 * pos + 1];
        const bool in0 = c0 >= N, in1 = c1 >= N;
        const int code0 = in0 ? 0 : codes[static_cast<size_t>(c0) * Cpad + c];
        const int code1 = in1 ? 0 : codes[static_cast<size_t>(c1) * Cpad + c];
        T m0[4], m1[4], dm0[4], dm1[4], v0[4], v1[4];
        if (in0) {
            if (2 * pos < 8) {
#pragma unroll
                for (int u = 0; u < 4; ++u) v0[u] = p[2 * pos][u];
            } else {
                child_vec<T, R>(part, c0 - N, tile, tiles, r, lane, -1, v0);
            }
            matvec4(P + (static_cast<size_t>(c0) * R + r) * 16, v0, m0);
            matvec4(dP + (static_cast<size_t>(c0) * R + r) * 16, v0, dm0);
        } else {
            const size_t ti = (static_cast<size_t>(c0) * R + r) * 5 + code0;
            const Vec4<T> a = reinterpret_cast<const GLOBAL Vec4<T>*>(TT)[ti];
            const Vec4<T> b = reinterpret_cast<const GLOBAL Vec4<T>*>(dTT)[ti];
            m0[0] = a.x; m0[1] = a.y; m0[2] = a.z; m0[3] = a.w;
            dm0[0] = b.x; dm0[1] = b.y; dm0[2] = b.z; dm0[3] = b.w;
        }
        if (in1) {
            if (2 * pos + 1 < 8) {
#pragma unroll
                for (int u = 0; u < 4; ++u) v1[u] = p[2 * pos + 1][u];
            } else {
                child_vec<T, R>(part, c1 - N, tile, tiles, r, lane, -1, v1);
            }
            matvec4(P + (static_cast<size_t>(c1) * R + r) * 16, v1, m1);
            matvec4(dP + (static_cast<size_t>(c1) * R + r) * 16, v1, dm1);
        } else {
            const size_t ti = (static_cast<size_t>(c1) * R + r) * 5 + code1;
            const Vec4<T> a = reinterpret_cast<const GLOBAL Vec4<T>*>(TT)[ti];
            const Vec4<T> b = reinterpret_cast<const GLOBAL Vec4<T>*>(dTT)[ti];
            m1[0] = a.x; m1[1] = a.y; m1[2] = a.z; m1[3] = a.w;
            dm1[0] = b.x; dm1[1] = b.y; dm1[2] = b.z; dm1[3] = b.w;
        }
        T u0[4], u1[4], a0 = T(0), a1 = T(0), dd = T(0);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            u0[u] = q[pos][u] * m1[u];
            u1[u] = q[pos][u] * m0[u];
            a0 += u0[u] * dm0[u];
            a1 += u1[u] * dm1[u];
            dd += u0[u] * m0[u];
        }
        T q0[4], q1[4], mx0 = T(0), mx1 = T(0);
        if (in0) {
            matvec4_t(P + (static_cast<size_t>(c0) * R + r) * 16, u0, q0);
#pragma unroll
            for (int u = 0; u < 4; ++u) mx0 = fmax(mx0, q0[u]);
        }
        if (in1) {
            matvec4_t(P + (static_cast<size_t>(c1) * R + r) * 16, u1, q1);
#pragma unroll
            for (int u = 0; u < 4; ++u) mx1 = fmax(mx1, q1[u]);
        }
        xch.v[buf][0][r][lane] = wr * a0;
        xch.v[buf][1][r][lane] = wr * a1;
        xch.v[buf][2][r][lane] = wr * dd;
        xch.v[buf][3][r][lane] = mx0;
        xch.v[buf][4][r][lane] = mx1;
        __syncthreads();
        T num0 = T(0), num1 = T(0), den = T(0), MX0 = T(0), MX1 = T(0);
#pragma unroll
        for (int rr = 0; rr < R; ++rr) {
            num0 += xch.v[buf][0][rr][lane];
            num1 += xch.v[buf][1][rr][lane];
            den += xch.v[buf][2][rr][lane];
            MX0 = fmax(MX0, xch.v[buf][3][rr][lane]);
            MX1 = fmax(MX1, xch.v[buf][4][rr][lane]);
        }
        buf ^= 1;
        if (in0) {
            const int e = exponent_of(MX0);
#pragma unroll
            for (int u = 0; u < 4; ++u) q0[u] = exact_ldexp(q0[u], -e);
            if (2 * pos < 8) {
#pragma unroll
                for (int u = 0; u < 4; ++u) q[2 * pos][u] = q0[u];
            } else {
                store_vec<T, R>(part, c0 - N, tile, tiles, r, lane, q0);
            }
        }
        if (in1) {
            const int e = exponent_of(MX1);
#pragma unroll
            for (int u = 0; u < 4; ++u) q1[u] = exact_ldexp(q1[u], -e);
            if (2 * pos + 1 < 8) {
#pragma unroll
                for (int u = 0; u < 4; ++u) q[2 * pos + 1][u] = q1[u];
            } else {
                store_vec<T, R>(part, c1 - N, tile, tiles, r, lane, q1);
            }
        }
        // gradient contributions: wave 0 takes child 0, wave 1 (or 0 if R == 1) child 1
        const double dden = static_cast<double>(den);
        if (r == 0) {
            const double g0 = (W != 0.0) ? W * (static_cast<double>(num0) / dden) : 0.0;
            const double s0 = wave_sum(g0);
            if (lane == 0) gpart[static_cast<size_t>(c0) * tiles + tile] = s0;
        }
        if (r == (R > 1 ? 1 : 0)) {
            const double g1 = (W != 0.0) ? W * (static_cast<double>(num1) / dden) : 0.0;
            const double s1 = wave_sum(g1);
            if (lane == 0) gpart[static_cast<size_t>(c1) * tiles + tile] = s1;
        }
    }
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
    double Pm[S][S], dPm[S][S];
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
            Pm[s][u] = acc;
            dPm[s][u] = dacc;
            d.P64[base + s * S + u] = acc;
            d.dP64[base + s * S + u] = dacc;
            if (d.fp32) {
                d.P32[base + s * S + u] = static_cast<float>(acc);
                d.dP32[base + s * S + u] = static_cast<float>(dacc);
            }
        }
    }
    if (S == 4) {
        // tip tables: entry y < 4 is column y (P e_y), entry 4 the row sums (P 1)
        const size_t tb = static_cast<size_t>(pair) * 20;
#pragma unroll
        for (int y = 0; y <= S; ++y)
#pragma unroll
            for (int s = 0; s < S; ++s) {
                double v = 0.0, dv = 0.0;
                if (y < S) {
                    v = Pm[s][y];
                    dv = dPm[s][y];
                } else {
#pragma unroll
                    for (int u = 0; u < S; ++u) {
                        v += Pm[s][u];
                        dv += dPm[s][u];
                    }
                }
                d.TT64[tb + 4 * y + s] = v;
                d.dTT64[tb + 4 * y + s] = dv;
                if (d.fp32) {
                    d.TT32[tb + 4 * y + s] = static_cast<float>(v);
                    d.dTT32[tb + 4 * y + s] = static_cast<float>(dv);
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
hipError_t level_r(KernelClass k, bool blocked, const ReqDesc* descs, const SegTable& t, hipStream_t st) {
    const int n_units = t.unit_begin[t.n];
    const int blocks = (n_units + kWavesPerBlock - 1) / kWavesPerBlock;
    if (blocked) {
        if (k == kPost)
            hipLaunchKernelGGL((post_blk_kernel<T, R>), dim3(n_units), dim3(kLanes * R), 0, st, descs, t);
        else
            hipLaunchKernelGGL((pre_blk_kernel<T, R>), dim3(n_units), dim3(kLanes * R), 0, st, descs, t);
    } else if (k == kPost) {
        hipLaunchKernelGGL((post_s4_kernel<T, R>), dim3(blocks), dim3(kBlock), 0, st, descs, t);
    } else {
        hipLaunchKernelGGL((pre_s4_kernel<T, R>), dim3(blocks), dim3(kBlock), 0, st, descs, t);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t level_t(KernelClass k, int R, bool blocked, const ReqDesc* descs, const SegTable& t,
                   hipStream_t st) {
    switch (R) {
        case 1: return level_r<T, 1>(k, blocked, descs, t, st);
        case 2: return level_r<T, 2>(k, blocked, descs, t, st);
        case 3: return level_r<T, 3>(k, blocked, descs, t, st);
        case 4: return level_r<T, 4>(k, blocked, descs, t, st);
        case 5: return level_r<T, 5>(k, blocked, descs, t, st);
        case 6: return level_r<T, 6>(k, blocked, descs, t, st);
        case 7: return level_r<T, 7>(k, blocked, descs, t, st);
        case 8: return level_r<T, 8>(k, blocked, descs, t, st);
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
            if (shape.fp32) return level_t<float>(k, shape.R, shape.blocked != 0, descs, t, st);
            return level_t<double>(k, shape.R, shape.blocked != 0, descs, t, st);
        case kFinal:
            hipLaunchKernelGGL(finalize_kernel, dim3(n_units), dim3(256), 0, st, descs, t);
            return hipGetLastError();
    }
    return hipErrorInvalidValue;
}

}  // namespace phg
