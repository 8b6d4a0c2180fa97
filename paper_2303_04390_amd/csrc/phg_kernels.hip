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
#include "phg_queue_device.h"

#include <math.h>

#include <algorithm>
#include <type_traits>

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

// Compile-time loop: f(IntC<i>{}) for i = B .. E-1, so the index can size
// and select register arrays.
template <int I>
struct IntC {
    static constexpr int value = I;
};
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (B < E) {
        f(IntC<B>{});
        static_for<B + 1, E>(f);
    }
}

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
                                          GLOBAL double* __restrict__ lpart,
                                          const GLOBAL int32_t* __restrict__ tslot,
                                          const GLOBAL T* __restrict__ tipvec) {
    const int c = tile * kLanes + lane;
    const bool tip_i = nt.i < N, tip_j = nt.j < N;
    // a tip reads its code, or its general partial vector (slot >= 0)
    const int vsi = (tip_i && tslot) ? tslot[nt.i] : -1;
    const int vsj = (tip_j && tslot) ? tslot[nt.j] : -1;
    const int code_i = tip_i && vsi < 0 ? codes[static_cast<size_t>(nt.i) * Cpad + c] : -1;
    const int code_j = tip_j && vsj < 0 ? codes[static_cast<size_t>(nt.j) * Cpad + c] : -1;
    const GLOBAL T* src_i = tip_i ? tipvec : part;
    const GLOBAL T* src_j = tip_j ? tipvec : part;
    const int slot_i = tip_i ? vsi : nt.i - N;
    const int slot_j = tip_j ? vsj : nt.j - N;
    const int ei = tip_i ? 0 : expo[static_cast<size_t>(nt.i - N) * Cpad + c];
    const int ej = tip_j ? 0 : expo[static_cast<size_t>(nt.j - N) * Cpad + c];

    T x[R][4];
    T mx = T(0);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        T vi[4], vj[4], mi[4], mj[4];
        child_vec<T, R>(src_i, slot_i, tile, tiles, r, lane, code_i, vi);
        child_vec<T, R>(src_j, slot_j, tile, tiles, r, lane, code_j, vj);
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
                    g(d.expo), g(ptab<T>(d)), g(d.cweights), g(d.pi), g(d.pw), g(d.sll), g(d.lpart),
                    g(d.tslot), g(static_cast<const T*>(d.tipvec)));
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
                                         GLOBAL double* __restrict__ gpart,
                                         const GLOBAL int32_t* __restrict__ tslot,
                                         const GLOBAL T* __restrict__ tipvec) {
    const int c = tile * kLanes + lane;
    const bool is_root = nt.k == 2 * N - 2;
    const bool tip_i = nt.i < N, tip_j = nt.j < N;
    const int vsi = (tip_i && tslot) ? tslot[nt.i] : -1;
    const int vsj = (tip_j && tslot) ? tslot[nt.j] : -1;
    const int code_i = tip_i && vsi < 0 ? codes[static_cast<size_t>(nt.i) * Cpad + c] : -1;
    const int code_j = tip_j && vsj < 0 ? codes[static_cast<size_t>(nt.j) * Cpad + c] : -1;
    const GLOBAL T* src_i = tip_i ? tipvec : part;
    const GLOBAL T* src_j = tip_j ? tipvec : part;
    const int slot_i = tip_i ? vsi : nt.i - N;
    const int slot_j = tip_j ? vsj : nt.j - N;

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
        child_vec<T, R>(src_i, slot_i, tile, tiles, r, lane, code_i, vi);
        child_vec<T, R>(src_j, slot_j, tile, tiles, r, lane, code_j, vj);
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
                   g(dptab<T>(d)), g(d.cweights), g(d.pi), g(d.pw), g(d.gpart), g(d.tslot),
                   g(static_cast<const T*>(d.tipvec)));
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

// FP64 asks for 4 waves per SIMD: 133-139 registers otherwise (3 waves);
// at 128 it spills 20-52 bytes per lane and still runs faster (1000-taxon
// HKY+G4 evaluation 1.074 -> 1.008 ms, results bit for bit the same).
template <typename T, int R>
__global__ __launch_bounds__(kLanes * R, sizeof(T) == 8 ? 4 : 1) void pre_blk_kernel(const ReqDesc* __restrict__ descs,
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
    constexpr int kSlots = (14 + R - 1) / R;
    T gn[kSlots], gd[kSlots];
    int gc[kSlots];
#pragma unroll
    for (int i = 0; i < kSlots; ++i) {
        gn[i] = gd[i] = T(0);
        gc[i] = -1;
    }
    static_for<1, 8>([&](auto P_) {
        constexpr int pos = decltype(P_)::value;
        const int k = nd[pos];
        if (k < N) return;
        const int c0 = nd[2 * pos], c1 = nd[2 * pos + 1];
        const bool in0 = c0 >= N, in1 = c1 >= N;
        const int code0 = in0 ? 0 : codes[static_cast<size_t>(c0) * Cpad + c];
        const int code1 = in1 ? 0 : codes[static_cast<size_t>(c1) * Cpad + c];
        T m0[4], m1[4], dm0[4], dm1[4], v0[4], v1[4];
        if (in0) {
            if constexpr (2 * pos < 8) {
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
            if constexpr (2 * pos + 1 < 8) {
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
            if constexpr (2 * pos < 8) {
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
            if constexpr (2 * pos + 1 < 8) {
#pragma unroll
                for (int u = 0; u < 4; ++u) q[2 * pos + 1][u] = q1[u];
            } else {
                store_vec<T, R>(part, c1 - N, tile, tiles, r, lane, q1);
            }
        }
        // gradient ratio terms, kept for the reduction after the loop: child
        // slot j = 2 (pos - 1) + side belongs to wave j mod R
        {
            constexpr int j0 = 2 * (pos - 1), j1 = j0 + 1;
            if (j0 % R == r) {
                gn[j0 / R] = num0;
                gd[j0 / R] = den;
                gc[j0 / R] = c0;
            }
            if (j1 % R == r) {
                gn[j1 / R] = num1;
                gd[j1 / R] = den;
                gc[j1 / R] = c1;
            }
        }
    });
    // per-tile sums of W_c * num / den, all of a wave's slots in lockstep so the
    // cross-lane reductions overlap
    double gs[kSlots];
#pragma unroll
    for (int i = 0; i < kSlots; ++i)
        gs[i] = (gc[i] >= 0 && W != 0.0) ? W * (static_cast<double>(gn[i]) / static_cast<double>(gd[i])) : 0.0;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
        for (int i = 0; i < kSlots; ++i) gs[i] += __shfl_xor(gs[i], off, kLanes);
    }
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < kSlots; ++i)
            if (gc[i] >= 0) gpart[static_cast<size_t>(gc[i]) * tiles + tile] = gs[i];
    }
}

// ------------------------------------------- blocked schedule, categories in lanes
//
// FP32 variant of the blocked kernels for R in {1, 2, 4, 8}: a wave holds
// 64 / R patterns x R categories (lane = r * (64 / R) + pattern), so the
// shared per-(node, pattern) rescale maximum over categories is a cross-lane
// operation inside the wave.  The 4x4 products P v, dP v and P^T u run on the
// matrix cores as four rank-1 steps of v_mfma_f32_4x4x1f32: each group of four
// lanes is one 4 x 4 block whose columns are its four patterns, lane (i mod 4)
// supplies row i of the matrix, and the result lands with the states in the
// four accumulator registers of the pattern's own lane.
//
// Latency: a prologue stages the matrices of the block's (up to 14) child
// branches in LDS, each row padded to 8 floats with its row sum in column 4
// (P 1, the vector of a fully ambiguous tip), and packs the block's tip codes
// of the lane's pattern into two registers.  After one barrier every matrix
// row, column or tip vector is an LDS read; the only global loads left in the
// per-node chain are stored partials of frontier block roots.

typedef float F4 __attribute__((ext_vector_type(4)));

// LDS image of one branch-category matrix: rows of 6 floats (8-byte
// aligned), columns 0..3 the matrix, column 4 the row sum.
constexpr int kRow = 6;
constexpr int kMat = 4 * kRow;

template <int R, int NM>
struct BmfMats {
    float m[14][R][NM][kMat];     // [child position - 2][category][P, dP][row][col]
};

// Per-lane constants of the categories-in-lanes layout.
struct BmfLane {
    int r;             // category
    int pat;           // pattern within the 64-pattern tile
    uint32_t part;     // byte offset of (r, pat) inside one (slot, tile) chunk of R * 64 float4
    int i;             // row / column this lane supplies to a 4x4 MFMA block
};

template <int R>
__device__ __forceinline__ BmfLane bmf_lane(int w, int lane) {
    constexpr int PW = kLanes / R;
    BmfLane L;
    L.r = lane / PW;
    L.pat = w * PW + lane % PW;
    L.part = static_cast<uint32_t>(L.r * kLanes + L.pat) * 16u;
    L.i = lane & 3;
    return L;
}

// Uniform base of the (slot, tile) chunk of the partials, as bytes.
template <int R>
__device__ __forceinline__ GLOBAL char* chunk(GLOBAL F4* part, unsigned slot, unsigned tile, unsigned tiles) {
    return reinterpret_cast<GLOBAL char*>(part) +
           (static_cast<size_t>(slot) * tiles + tile) * (static_cast<size_t>(R) * kLanes * 16);
}

// Loads and stores of the partials and exponents that one work item writes
// and another reads.  kCoh = false: ordinary accesses (level launches, where
// the launch boundary orders producer and consumer).  kCoh = true (the
// work-queue kernel, where both run inside one launch): device-coherent
// (queue::ld / queue::st).  The partial of (slot, tile) for the lane
// (r, pattern), at byte offset `off` of the chunk, and the exponent of
// (slot, pattern c = tile * 64 + pat).
template <int R, bool kCoh>
__device__ __forceinline__ F4 ld_part(GLOBAL F4* part, unsigned slot, unsigned tile, unsigned tiles, uint32_t off) {
    const GLOBAL F4* base = reinterpret_cast<const GLOBAL F4*>(chunk<R>(part, slot, tile, tiles));
    if constexpr (kCoh) return queue::ld(base, off / 16, R * kLanes);
    return base[off / 16];
}
template <int R, bool kCoh>
__device__ __forceinline__ void st_part(GLOBAL F4* part, unsigned slot, unsigned tile, unsigned tiles, uint32_t off,
                                        F4 v) {
    GLOBAL F4* base = reinterpret_cast<GLOBAL F4*>(chunk<R>(part, slot, tile, tiles));
    if constexpr (kCoh)
        queue::st(base, off / 16, R * kLanes, v);
    else
        base[off / 16] = v;
}
template <bool kCoh>
__device__ __forceinline__ int ld_expo(const GLOBAL int32_t* expo, unsigned slot, int Cpad, unsigned tile, int pat) {
    const GLOBAL int32_t* base = expo + static_cast<size_t>(slot) * Cpad + static_cast<size_t>(tile) * kLanes;
    if constexpr (kCoh) return queue::ld(base, pat, kLanes);
    return base[pat];
}
template <bool kCoh>
__device__ __forceinline__ void st_expo(GLOBAL int32_t* expo, unsigned slot, int Cpad, unsigned tile, int pat, int v) {
    GLOBAL int32_t* base = expo + static_cast<size_t>(slot) * Cpad + static_cast<size_t>(tile) * kLanes;
    if constexpr (kCoh)
        queue::st(base, pat, kLanes, v);
    else
        base[pat] = v;
}

__device__ __forceinline__ void f4_to(const F4 q, float out[4]) {
    out[0] = q.x;
    out[1] = q.y;
    out[2] = q.z;
    out[3] = q.w;
}
__device__ __forceinline__ F4 to_f4(const float v[4]) {
    F4 q;
    q.x = v[0];
    q.y = v[1];
    q.z = v[2];
    q.w = v[3];
    return q;
}

// v with lane J replaced by the wave-uniform value X (v_writelane_b32; X is
// moved to a scalar register first).
__device__ __forceinline__ int write_lane(int v, int x, const int j) {
    const int xs = __builtin_amdgcn_readfirstlane(x);
    asm volatile("v_writelane_b32 %0, %1, %2" : "+v"(v) : "s"(xs), "i"(j));
    return v;
}

// Stage the matrices (NM = 1: P; NM = 2: P and dP) of every child branch of
// the block in LDS, with row sums.  All threads of the workgroup take part,
// every row load of a thread in flight at once; the caller synchronises.
template <int R, int NM>
__device__ __forceinline__ void stage_mats(BmfMats<R, NM>& S, const int (&nd)[16],
                                           const GLOBAL float* __restrict__ P, const GLOBAL float* __restrict__ dP) {
    // lanes 0..15 of every wave hold the heap record (from the wave-uniform
    // copy, no memory access); a thread's child index comes from there by a
    // cross-lane permute
    int ndv = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) ndv = write_lane(ndv, nd[j], j);
    constexpr int kItems = 14 * R * NM * 4;          // one matrix row each
    constexpr int kThreads = kLanes * R;
    constexpr int kIters = (kItems + kThreads - 1) / kThreads;
    F4 row[kIters];
#pragma unroll
    for (int k = 0; k < kIters; ++k) {
        const int it = min(static_cast<int>(threadIdx.x) + k * kThreads, kItems - 1);
        const int u = it & 3;
        const int mm = (it >> 2) % NM;
        const int r = (it / (4 * NM)) % R;
        const int ch = it / (4 * NM * R);
        const int cn = max(__builtin_amdgcn_ds_bpermute((ch + 2) << 2, ndv), 0);   // absent: branch 0, never read
        row[k] = *reinterpret_cast<const GLOBAL F4*>((mm == 0 ? P : dP) + (static_cast<size_t>(cn) * R + r) * 16 +
                                                     u * 4);
    }
#pragma unroll
    for (int k = 0; k < kIters; ++k) {
        const int it = static_cast<int>(threadIdx.x) + k * kThreads;
        if (it >= kItems) continue;
        const int u = it & 3;
        const int mm = (it >> 2) % NM;
        const int r = (it / (4 * NM)) % R;
        const int ch = it / (4 * NM * R);
        float* dst = &S.m[ch][r][mm][u * kRow];
        dst[0] = row[k].x;
        dst[1] = row[k].y;
        dst[2] = row[k].z;
        dst[3] = row[k].w;
        dst[4] = ((row[k].x + row[k].y) + row[k].z) + row[k].w;
    }
}

// Tip codes of the block's child positions 2..15 for the tile's 64 patterns,
// staged in LDS: row j = position j + 2, one byte per pattern.  Each row is 64
// contiguous bytes of the code matrix, read as 16 dwords, so one wave
// instruction fetches four rows (a non-tip row reads tip 0's codes, unused).
// All threads take part; the caller synchronises.
template <int R>
__device__ __forceinline__ void stage_codes(uint32_t (&CL)[14][16], const int (&nd)[16], const int N,
                                            const int Cpad, const int c0, const GLOBAL uint8_t* __restrict__ codes) {
    int ndv = 0;                                        // lanes 0..15: the heap record
#pragma unroll
    for (int j = 0; j < 16; ++j) ndv = write_lane(ndv, nd[j], j);
    constexpr int kRowsPerPass = 4 * R;
#pragma unroll
    for (int j0 = 0; j0 < 14; j0 += kRowsPerPass) {
        const int j = j0 + static_cast<int>(threadIdx.x >> 4);
        const int cn = __builtin_amdgcn_ds_bpermute((min(j, 13) + 2) << 2, ndv);
        const size_t row = (cn >= 0 && cn < N) ? static_cast<size_t>(cn) : 0;
        const uint32_t wv =
            *reinterpret_cast<const GLOBAL uint32_t*>(codes + row * Cpad + c0 + 4 * (threadIdx.x & 15));
        if (j < 14) CL[j][threadIdx.x & 15] = wv;
    }
}
__device__ __forceinline__ int code_at(const uint32_t (&CL)[14][16], int cp, int pat) {
    return reinterpret_cast<const uint8_t*>(&CL[cp - 2][0])[pat];
}

// Column CODE of a staged matrix (P e_code, or the row sums for code 4).
__device__ __forceinline__ void lds_column(const float* M, int code, float m[4]) {
#pragma unroll
    for (int u = 0; u < 4; ++u) m[u] = M[u * kRow + code];
}

// m = M v (kTransposed = false) or M^T v (true) on the matrix cores for this
// lane's pattern; M is the staged matrix of the lane's category.
template <bool kTransposed>
__device__ __forceinline__ void mfma_mv(const float* M, const BmfLane& L, const float v[4], float m[4]) {
    float a[4];
    if (kTransposed) {
#pragma unroll
        for (int k = 0; k < 4; ++k) a[k] = M[k * kRow + L.i];
    } else {
        typedef float F2 __attribute__((ext_vector_type(2)));
        const F2 lo = *reinterpret_cast<const F2*>(M + L.i * kRow);
        const F2 hi = *reinterpret_cast<const F2*>(M + L.i * kRow + 2);
        a[0] = lo.x;
        a[1] = lo.y;
        a[2] = hi.x;
        a[3] = hi.y;
    }
    F4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int k = 0; k < 4; ++k) acc = __builtin_amdgcn_mfma_f32_4x4x1f32(a[k], v[k], acc, 0, 0, 0);
    f4_to(acc, m);
}

// Maximum over the R lanes of one pattern (lane xor 32, 16, 8 partners) of
// values >= 0 given as their bit patterns: for IEEE floats >= 0 the signed
// integer order is the float order, and any negative rounding residue (a
// negative bit pattern) loses to a non-negative one.  Every lane of the
// pattern ends with the same value.
template <int R>
__device__ __forceinline__ int max_over_categories(int v) {
    if constexpr (R >= 8) v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x128, 0xF, 0xF, false));  // row_ror:8
    if constexpr (R >= 4) {
        const auto s = __builtin_amdgcn_permlane16_swap(static_cast<unsigned>(v), static_cast<unsigned>(v),
                                                        false, false);
        v = max(static_cast<int>(s[0]), static_cast<int>(s[1]));
    }
    if constexpr (R >= 2) {
        const auto s = __builtin_amdgcn_permlane32_swap(static_cast<unsigned>(v), static_cast<unsigned>(v),
                                                        false, false);
        v = max(static_cast<int>(s[0]), static_cast<int>(s[1]));
    }
    return v;
}

// Sum over the R lanes of one pattern; pairs are combined commutatively, so
// every lane of the pattern ends with the bitwise-same result.
template <int R>
__device__ __forceinline__ float sum_over_categories(float v) {
    if constexpr (R >= 8)
        v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x128, 0xF, 0xF, false));
    if constexpr (R >= 4) {
        const auto s = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
        v = __uint_as_float(s[0]) + __uint_as_float(s[1]);
    }
    if constexpr (R >= 2) {
        const auto s = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
        v = __uint_as_float(s[0]) + __uint_as_float(s[1]);
    }
    return v;
}

// Exponent e of the per-pattern maximum of the four values over all R
// categories, and the values scaled by 2^-e (exact).
template <int R>
__device__ __forceinline__ int rescale_shared(float x[4]) {
    int b = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) b = max(b, __float_as_int(x[u]));
    const int e = exponent_of(__int_as_float(max_over_categories<R>(b)));
#pragma unroll
    for (int u = 0; u < 4; ++u) x[u] = exact_ldexp(x[u], -e);
    return e;
}

// The stored partials (and, with kExpo, exponents) of the block's frontier
// block roots, heap positions 8..15, for this lane's (category, pattern), all
// loads issued together: one memory round trip for the block's inputs, each
// read once.  Tips and absent positions give zeros.  The post-order kernel
// always does this (it stays at 8 waves per SIMD); in the pre-order kernel the
// registers stay live through the pre-order phase and cost occupancy, so it
// pays only in launches too narrow to fill the chip (near the root), where
// latency, not occupancy, bounds them.
template <int R, bool kExpo, bool kCoh>
__device__ __forceinline__ void load_frontier(const int (&nd)[16], const BmfLane& L, const int tile,
                                              const int tiles, const int N, const int Cpad,
                                              GLOBAL F4* __restrict__ part, const GLOBAL int32_t* __restrict__ expo,
                                              float (&fr)[8][4], int (&fe)[8]) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int cn = nd[8 + j];
        F4 v = {0.0f, 0.0f, 0.0f, 0.0f};
        int e = 0;
        if (cn >= N) {
            v = ld_part<R, kCoh>(part, cn - N, tile, tiles, L.part);
            if (kExpo) e = ld_expo<kCoh>(expo, cn - N, Cpad, tile, L.pat);
        }
        f4_to(v, fr[j]);
        fe[j] = e;
    }
}

// In-block post-order over heap positions 7..LO for this lane's (category,
// pattern).  With kExpo, returns the sum of exponents taken (in-block nodes and
// frontier block roots); otherwise exponents are not read.  Frontier inputs
// come from load_frontier (kPre) or are loaded per position.
template <int R, int NM, int LO, bool kExpo, bool kPre, bool kCoh>
__device__ __forceinline__ int bmf_postorder(const int (&nd)[16], const BmfLane& L, const BmfMats<R, NM>& S,
                                             const uint32_t (&CL)[14][16], const int tile, const int tiles,
                                             const int N, const int Cpad, GLOBAL F4* __restrict__ part,
                                             const GLOBAL int32_t* __restrict__ expo, const float (&fr)[8][4],
                                             const int (&fe)[8], float (&p)[8][4]) {
    int esum = 0;
    static_for<0, 8 - LO>([&](auto I_) {
        constexpr int pos = 7 - decltype(I_)::value;
        const int k = nd[pos];
        if (k < N) return;
        float m[2][4], v[2][4];
        if constexpr (pos >= 4 && kPre) {
#pragma unroll
            for (int s = 0; s < 2; ++s) {
#pragma unroll
                for (int u = 0; u < 4; ++u) v[s][u] = fr[2 * pos + s - 8][u];
                if (kExpo) esum += fe[2 * pos + s - 8];     // zero for a tip
            }
        } else if constexpr (pos >= 4) {
            // frontier children: both stored partials (and exponents) are
            // loaded before either is used; a tip child reads slot 0, unused
            int ex[2];
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const int cn = nd[2 * pos + s];
                const int slot = cn >= N ? cn - N : 0;
                f4_to(ld_part<R, kCoh>(part, slot, tile, tiles, L.part), v[s]);
                ex[s] = kExpo ? ld_expo<kCoh>(expo, slot, Cpad, tile, L.pat) : 0;
            }
#pragma unroll
            for (int s = 0; s < 2; ++s)
                if (kExpo && nd[2 * pos + s] >= N) esum += ex[s];
        } else {
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int u = 0; u < 4; ++u) v[s][u] = p[pos < 4 ? 2 * pos + s : 0][u];
        }
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int cp = 2 * pos + s;
            const float* M = S.m[cp - 2][L.r][0];
            if (nd[cp] < N)
                lds_column(M, code_at(CL, cp, L.pat), m[s]);
            else
                mfma_mv<false>(M, L, v[s], m[s]);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) p[pos][u] = m[0][u] * m[1][u];
        esum += rescale_shared<R>(p[pos]);
    });
    return esum;
}

// Common prologue: unit -> (segment, block, tile), the block's heap record.
struct BmfUnit {
    const ReqDesc* d;
    Segment sg;
    int tile, tiles, N, Cpad;
    const GLOBAL int32_t* heap;
};
__device__ __forceinline__ bool bmf_unit(const ReqDesc* __restrict__ descs, const SegTable& segs, BmfUnit& U) {
    const int unit = blockIdx.x;
    if (unit >= segs.unit_begin[segs.n]) return false;
    const int sidx = find_segment(segs, unit);
    U.sg = segs.seg[sidx];
    U.d = &descs[U.sg.desc];
    // tiles from the segment's unit count (kernel argument), not the descriptor
    U.tiles = (segs.unit_begin[sidx + 1] - segs.unit_begin[sidx]) / U.sg.n_nodes;
    U.N = U.d->N;
    U.Cpad = U.d->Cpad;
    const int local = unit - segs.unit_begin[sidx];
    const int bix = local / U.tiles;
    U.tile = local - bix * U.tiles;
    // from the segment (kernel argument), so this load does not wait for the descriptor
    U.heap = reinterpret_cast<const GLOBAL int32_t*>(g(U.sg.sched)) + static_cast<size_t>(U.sg.sched_off + bix) * 16;
    return true;
}

template <int R>
__global__ __launch_bounds__(kLanes * R) __attribute__((amdgpu_waves_per_eu(4))) void post_bmf_kernel(
    const ReqDesc* __restrict__ descs, const SegTable segs) {
    constexpr int PW = kLanes / R;
    __shared__ BmfMats<R, 1> S;
    __shared__ uint32_t CL[14][16];                     // tip codes of the block, [position - 2][pattern]
    __shared__ double sw[R];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & (kLanes - 1);
    const BmfLane L = bmf_lane<R>(w, lane);
    BmfUnit U;
    if (!bmf_unit(descs, segs, U)) return;
    const ReqDesc& d = *U.d;
    const int N = U.N, tile = U.tile;
    int nd[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) nd[i] = U.heap[i];
    const int c = tile * kLanes + L.pat;
    GLOBAL F4* part = reinterpret_cast<GLOBAL F4*>(g(part_of<float>(d)));
    GLOBAL int32_t* expo = g(d.expo);
    float fr[8][4];
    int fe[8];
    load_frontier<R, true, false>(nd, L, tile, U.tiles, N, U.Cpad, part, expo, fr, fe);
    stage_codes<R>(CL, nd, N, U.Cpad, tile * kLanes, g(d.codes));
    stage_mats<R, 1>(S, nd, g(d.P32), nullptr);
    __syncthreads();
    float p[8][4];
    const int ek =
        bmf_postorder<R, 1, 1, true, true, false>(nd, L, S, CL, tile, U.tiles, N, U.Cpad, part, expo, fr, fe, p);
    if (!(U.sg.flags & 1)) {
        *reinterpret_cast<GLOBAL F4*>(chunk<R>(part, nd[1] - N, tile, U.tiles) + L.part) = to_f4(p[1]);
        if (L.r == 0) expo[static_cast<size_t>(nd[1] - N) * U.Cpad + c] = ek;
        return;
    }
    // the tree root: log site likelihood and this tile's weighted sum
    const GLOBAL double* pi = g(d.pi);
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u) acc += pi[u] * static_cast<double>(p[1][u]);
    double site = g(d.cweights)[L.r] * acc;
#pragma unroll
    for (int off = kLanes / 2; off >= PW; off >>= 1) site += __shfl_xor(site, off, kLanes);
    double contrib = 0.0;
    if (L.r == 0) {
        const double ll = (site > 0.0 ? log(site) : -INFINITY) + static_cast<double>(ek) * 0.69314718055994530942;
        g(d.sll)[c] = ll;
        const double W = g(d.pw)[c];
        contrib = W != 0.0 ? W * ll : 0.0;
    }
    const double ws = wave_sum(contrib);
    if (lane == 0) sw[w] = ws;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
#pragma unroll
        for (int i = 0; i < R; ++i) t += sw[i];
        g(d.lpart)[tile] = t;
    }
}

template <int R, bool kPre>
__global__ __launch_bounds__(kLanes * R) __attribute__((amdgpu_waves_per_eu(4))) void pre_bmf_kernel(
    const ReqDesc* __restrict__ descs, const SegTable segs) {
    __shared__ BmfMats<R, 2> S;
    __shared__ uint32_t CL[14][16];                     // tip codes of the block, [position - 2][pattern]
    // per child slot j = 2 (pos - 1) + side: sum_r w_r u . dm; per position:
    // sum_r w_r u . m (the same for both children); lane = pattern of the tile
    __shared__ float gnum[14][kLanes];
    __shared__ float gden[7][kLanes];
    __shared__ double wl[kLanes];                       // pattern weights of the tile
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & (kLanes - 1);
    const BmfLane L = bmf_lane<R>(w, lane);
    BmfUnit U;
    if (!bmf_unit(descs, segs, U)) return;
    const ReqDesc& d = *U.d;
    const int N = U.N, tile = U.tile, tiles = U.tiles;
    int nd[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) nd[i] = U.heap[i];
    const int c = tile * kLanes + L.pat;
    GLOBAL F4* part = reinterpret_cast<GLOBAL F4*>(g(part_of<float>(d)));
    float fr[8][4];
    int fe[8];
    if constexpr (kPre) load_frontier<R, false, false>(nd, L, tile, tiles, N, U.Cpad, part, nullptr, fr, fe);
    stage_codes<R>(CL, nd, N, U.Cpad, tile * kLanes, g(d.codes));
    float q[8][4];
    if (nd[1] == 2 * N - 2) {
        const GLOBAL double* pi = g(d.pi);
#pragma unroll
        for (int u = 0; u < 4; ++u) q[1][u] = static_cast<float>(pi[u]);
    } else {
        f4_to(*reinterpret_cast<const GLOBAL F4*>(chunk<R>(part, nd[1] - N, tile, tiles) + L.part), q[1]);
    }
    if (L.r == 0) wl[L.pat] = g(d.pw)[c];
    stage_mats<R, 2>(S, nd, g(d.P32), g(d.dP32));
    __syncthreads();
    float p[8][4];
    (void)bmf_postorder<R, 2, 2, false, kPre, false>(nd, L, S, CL, tile, tiles, N, U.Cpad, part, nullptr, fr, fe, p);
    const float wr = static_cast<float>(g(d.cweights)[L.r]);
    static_for<1, 8>([&](auto P_) {
        constexpr int pos = decltype(P_)::value;
        const int k = nd[pos];
        if (k < N) return;
        float m[2][4], dm[2][4], v[2][4];
        bool in[2];
        if constexpr (pos >= 4 && kPre) {
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int u = 0; u < 4; ++u) v[s][u] = fr[2 * pos + s - 8][u];
        } else if constexpr (pos >= 4) {
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const int cn = nd[2 * pos + s];
                f4_to(*reinterpret_cast<const GLOBAL F4*>(chunk<R>(part, cn >= N ? cn - N : 0, tile, tiles) +
                                                          L.part),
                      v[s]);
            }
        } else {
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int u = 0; u < 4; ++u) v[s][u] = p[pos < 4 ? 2 * pos + s : 0][u];
        }
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int cp = 2 * pos + s;
            const float* M = S.m[cp - 2][L.r][0];
            const float* dM = S.m[cp - 2][L.r][1];
            in[s] = nd[cp] >= N;
            if (!in[s]) {
                const int code = code_at(CL, cp, L.pat);
                lds_column(M, code, m[s]);
                lds_column(dM, code, dm[s]);
            } else {
                mfma_mv<false>(M, L, v[s], m[s]);
                mfma_mv<false>(dM, L, v[s], dm[s]);
            }
        }
        float uu[2][4], a0 = 0.0f, a1 = 0.0f, dd = 0.0f;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            uu[0][u] = q[pos][u] * m[1][u];
            uu[1][u] = q[pos][u] * m[0][u];
            a0 += uu[0][u] * dm[0][u];
            a1 += uu[1][u] * dm[1][u];
            dd += uu[0][u] * m[0][u];
        }
        const float num0 = sum_over_categories<R>(wr * a0);
        const float num1 = sum_over_categories<R>(wr * a1);
        const float den = sum_over_categories<R>(wr * dd);
        if (L.r == 0) {
            gnum[2 * pos - 2][L.pat] = num0;
            gnum[2 * pos - 1][L.pat] = num1;
            gden[pos - 1][L.pat] = den;
        }
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            if (!in[s]) continue;
            const int cp = 2 * pos + s;
            const int cn = nd[cp];
            float qn[4];
            mfma_mv<true>(S.m[cp - 2][L.r][0], L, uu[s], qn);
            (void)rescale_shared<R>(qn);
            if (cp < 8) {
#pragma unroll
                for (int u = 0; u < 4; ++u) q[cp < 8 ? cp : 0][u] = qn[u];
            } else {
                *reinterpret_cast<GLOBAL F4*>(chunk<R>(part, cn - N, tile, tiles) + L.part) = to_f4(qn);
            }
        }
    });
    __syncthreads();
    // per-tile sums of W_c num / den for the (up to) 14 child branches: sixteen
    // threads per branch, four patterns each, then a sixteen-lane reduction;
    // fixed order, so results are deterministic
    constexpr int kThreads = kLanes * R;
    GLOBAL double* gpart = g(d.gpart);
    int ndv = 0;                                        // lanes 0..15: the heap record
#pragma unroll
    for (int j = 0; j < 16; ++j) ndv = write_lane(ndv, nd[j], j);
#pragma unroll
    for (int t0 = 0; t0 < 14 * 16; t0 += kThreads) {
        const int t = t0 + static_cast<int>(threadIdx.x);
        const int j = min(t >> 4, 13);
        const int sub = t & 15;
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int pp = sub * 4 + i;
            const double W = wl[pp];
            if (W != 0.0) acc += W * (static_cast<double>(gnum[j][pp]) / static_cast<double>(gden[j >> 1][pp]));
        }
#pragma unroll
        for (int off = 8; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 16);
        const int parent_node = __builtin_amdgcn_ds_bpermute(((j >> 1) + 1) << 2, ndv);
        const int child = __builtin_amdgcn_ds_bpermute((j + 2) << 2, ndv);
        if (sub == 0 && t < 14 * 16 && parent_node >= N) gpart[static_cast<size_t>(child) * tiles + tile] = acc;
    }
}

// Item bodies of the work-queue traversal (below): the post_bmf_kernel and
// pre_bmf_kernel arithmetic for one (block, tile), with device-coherent
// accesses to the partials and exponents that cross items, and the matrices
// and codes staged before the dependency wait.  LDS of the two bodies:
template <int R>
struct PostBmfLds {
    BmfMats<R, 1> S;
    uint32_t CL[14][16];                     // tip codes of the block, [position - 2][pattern]
    double sw[R];
};
template <int R>
struct PreBmfLds {
    BmfMats<R, 2> S;
    uint32_t CL[14][16];                     // tip codes of the block, [position - 2][pattern]
    // per child slot j = 2 (pos - 1) + side: sum_r w_r u . dm; per position:
    // sum_r w_r u . m (the same for both children); lane = pattern of the tile
    float gnum[14][kLanes];
    float gden[7][kLanes];
    double wl[kLanes];                       // pattern weights of the tile
};

// Post-order of one (block, tile) with the block's heap record at `heap`;
// root: the block holds the tree root.  `wait` returns (after a barrier) once
// the frontier block roots' partials of this tile are complete.
template <int R, class Wait>
__device__ __forceinline__ void post_bmf_body(const ReqDesc& d, const GLOBAL int32_t* __restrict__ heap,
                                              const int tile, const int tiles, const bool root,
                                              PostBmfLds<R>& sm, const int w, const int lane, Wait&& wait) {
    constexpr int PW = kLanes / R;
    const BmfLane L = bmf_lane<R>(w, lane);
    const int N = d.N, Cpad = d.Cpad;
    int nd[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) nd[i] = heap[i];
    const int c = tile * kLanes + L.pat;
    GLOBAL F4* part = reinterpret_cast<GLOBAL F4*>(g(part_of<float>(d)));
    GLOBAL int32_t* expo = g(d.expo);
    stage_codes<R>(sm.CL, nd, N, Cpad, tile * kLanes, g(d.codes));
    stage_mats<R, 1>(sm.S, nd, g(d.P32), nullptr);
    wait();
    float fr[8][4];
    int fe[8];
    load_frontier<R, true, true>(nd, L, tile, tiles, N, Cpad, part, expo, fr, fe);
    float p[8][4];
    const int ek =
        bmf_postorder<R, 1, 1, true, true, true>(nd, L, sm.S, sm.CL, tile, tiles, N, Cpad, part, expo, fr, fe, p);
    if (!root) {
        st_part<R, true>(part, nd[1] - N, tile, tiles, L.part, to_f4(p[1]));
        if (L.r == 0) st_expo<true>(expo, nd[1] - N, Cpad, tile, L.pat, ek);
        return;
    }
    // the tree root: log site likelihood and this tile's weighted sum
    const GLOBAL double* pi = g(d.pi);
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u) acc += pi[u] * static_cast<double>(p[1][u]);
    double site = g(d.cweights)[L.r] * acc;
#pragma unroll
    for (int off = kLanes / 2; off >= PW; off >>= 1) site += __shfl_xor(site, off, kLanes);
    double contrib = 0.0;
    if (L.r == 0) {
        const double ll = (site > 0.0 ? log(site) : -INFINITY) + static_cast<double>(ek) * 0.69314718055994530942;
        g(d.sll)[c] = ll;
        const double W = g(d.pw)[c];
        contrib = W != 0.0 ? W * ll : 0.0;
    }
    const double ws = wave_sum(contrib);
    if (lane == 0) sm.sw[w] = ws;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
#pragma unroll
        for (int i = 0; i < R; ++i) t += sm.sw[i];
        g(d.lpart)[tile] = t;
    }
}

// Pre-order and gradient sums of one (block, tile).  `wait` returns (after a
// barrier) once the pre-order vector of the block root (written by the
// parent block's item) is complete.
template <int R, class Wait>
__device__ __forceinline__ void pre_bmf_body(const ReqDesc& d, const GLOBAL int32_t* __restrict__ heap,
                                             const int tile, const int tiles, PreBmfLds<R>& sm, const int w,
                                             const int lane, Wait&& wait) {
    const BmfLane L = bmf_lane<R>(w, lane);
    const int N = d.N, Cpad = d.Cpad;
    int nd[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) nd[i] = heap[i];
    const int c = tile * kLanes + L.pat;
    GLOBAL F4* part = reinterpret_cast<GLOBAL F4*>(g(part_of<float>(d)));
    float fr[8][4];                                     // unused: frontier partials are loaded per position
    int fe[8];
    stage_codes<R>(sm.CL, nd, N, Cpad, tile * kLanes, g(d.codes));
    if (L.r == 0) sm.wl[L.pat] = g(d.pw)[c];
    stage_mats<R, 2>(sm.S, nd, g(d.P32), g(d.dP32));
    wait();
    float q[8][4];
    if (nd[1] == 2 * N - 2) {
        const GLOBAL double* pi = g(d.pi);
#pragma unroll
        for (int u = 0; u < 4; ++u) q[1][u] = static_cast<float>(pi[u]);
    } else {
        f4_to(ld_part<R, true>(part, nd[1] - N, tile, tiles, L.part), q[1]);
    }
    float p[8][4];
    (void)bmf_postorder<R, 2, 2, false, false, true>(nd, L, sm.S, sm.CL, tile, tiles, N, Cpad, part, nullptr, fr,
                                                     fe, p);
    const float wr = static_cast<float>(g(d.cweights)[L.r]);
    static_for<1, 8>([&](auto P_) {
        constexpr int pos = decltype(P_)::value;
        const int k = nd[pos];
        if (k < N) return;
        float m[2][4], dm[2][4], v[2][4];
        bool in[2];
        if constexpr (pos >= 4) {
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const int cn = nd[2 * pos + s];
                f4_to(ld_part<R, true>(part, cn >= N ? cn - N : 0, tile, tiles, L.part), v[s]);
            }
        } else {
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int u = 0; u < 4; ++u) v[s][u] = p[pos < 4 ? 2 * pos + s : 0][u];
        }
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int cp = 2 * pos + s;
            const float* M = sm.S.m[cp - 2][L.r][0];
            const float* dM = sm.S.m[cp - 2][L.r][1];
            in[s] = nd[cp] >= N;
            if (!in[s]) {
                const int code = code_at(sm.CL, cp, L.pat);
                lds_column(M, code, m[s]);
                lds_column(dM, code, dm[s]);
            } else {
                mfma_mv<false>(M, L, v[s], m[s]);
                mfma_mv<false>(dM, L, v[s], dm[s]);
            }
        }
        float uu[2][4], a0 = 0.0f, a1 = 0.0f, dd = 0.0f;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            uu[0][u] = q[pos][u] * m[1][u];
            uu[1][u] = q[pos][u] * m[0][u];
            a0 += uu[0][u] * dm[0][u];
            a1 += uu[1][u] * dm[1][u];
            dd += uu[0][u] * m[0][u];
        }
        const float num0 = sum_over_categories<R>(wr * a0);
        const float num1 = sum_over_categories<R>(wr * a1);
        const float den = sum_over_categories<R>(wr * dd);
        if (L.r == 0) {
            sm.gnum[2 * pos - 2][L.pat] = num0;
            sm.gnum[2 * pos - 1][L.pat] = num1;
            sm.gden[pos - 1][L.pat] = den;
        }
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            if (!in[s]) continue;
            const int cp = 2 * pos + s;
            const int cn = nd[cp];
            float qn[4];
            mfma_mv<true>(sm.S.m[cp - 2][L.r][0], L, uu[s], qn);
            (void)rescale_shared<R>(qn);
            if (cp < 8) {
#pragma unroll
                for (int u = 0; u < 4; ++u) q[cp < 8 ? cp : 0][u] = qn[u];
            } else {
                st_part<R, true>(part, cn - N, tile, tiles, L.part, to_f4(qn));
            }
        }
    });
    __syncthreads();
    // per-tile sums of W_c num / den for the (up to) 14 child branches: sixteen
    // threads per branch, four patterns each, then a sixteen-lane reduction;
    // fixed order, so results are deterministic
    constexpr int kThreads = kLanes * R;
    GLOBAL double* gpart = g(d.gpart);
    int ndv = 0;                                        // lanes 0..15: the heap record
#pragma unroll
    for (int j = 0; j < 16; ++j) ndv = write_lane(ndv, nd[j], j);
#pragma unroll
    for (int t0 = 0; t0 < 14 * 16; t0 += kThreads) {
        const int t = t0 + static_cast<int>(threadIdx.x);
        const int j = min(t >> 4, 13);
        const int sub = t & 15;
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int pp = sub * 4 + i;
            const double W = sm.wl[pp];
            if (W != 0.0)
                acc += W * (static_cast<double>(sm.gnum[j][pp]) / static_cast<double>(sm.gden[j >> 1][pp]));
        }
#pragma unroll
        for (int off = 8; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 16);
        const int parent_node = __builtin_amdgcn_ds_bpermute(((j >> 1) + 1) << 2, ndv);
        const int child = __builtin_amdgcn_ds_bpermute((j + 2) << 2, ndv);
        if (sub == 0 && t < 14 * 16 && parent_node >= N) gpart[static_cast<size_t>(child) * tiles + tile] = acc;
    }
}

// ------------------------------------------- work-queue traversal (blocked, FP32)
//
// One launch per pass (or one for both) in place of one launch per block
// level.  Work items are (block, tile) pairs, numbered so that every item's
// inputs come from items with smaller numbers: post-order levels deepest
// first, then pre-order levels from the root's down; within a level
// tile-major, so one tile's items finish close together and the next level's
// items of that tile are ready when they are reached.  Tiles are independent,
// so one tile's items near the root run while other tiles are still in wide
// levels: no launch boundary and no level-wide barrier.
//
// Workgroup i takes item t0 + i and waits only on items with smaller numbers.
// Forward progress rests on the dispatcher starting a launch's workgroups in
// increasing order on each XCD: then the unfinished item with the smallest
// number is running or next to start on its XCD (every earlier workgroup of
// that XCD has finished), and its inputs are complete.  (A device-wide ticket
// counter would not need that order, but one atomic per workgroup on one
// address serialises: it made the traversal ~2.8x slower than the level
// launches.)  An item is complete when its completion mark, per (pass, block,
// tile), equals the evaluation's epoch, which the evaluation's P(t) launch
// advances; marks of earlier evaluations hold other values, so nothing is
// cleared between evaluations and the launches replay in a graph.  Every wait
// is bounded: past `wait_ticks` of the device's constant clock the item sets
// the fault word and goes on, its results invalid (the final sums then turn
// to NaN), and once the word is set every other wait ends at its next poll,
// so every workgroup exits.
//
// Partials and exponents that cross items use device-coherent accesses
// (kCoh); an item's mark is stored after its stores have completed at device
// scope (vmcnt(0) in every wave, then a barrier).

// kPasses: 1 post-order items only, 2 pre-order items only, 3 both.  Eight
// waves per SIMD: the pre-order body then fits 64 VGPRs without spilling
// (66 at four; measured 3% faster on the 1000-taxon workload).
template <int R, int kPasses>
__global__ __launch_bounds__(kLanes * R) __attribute__((amdgpu_waves_per_eu(8))) void queue_bmf_kernel(
    const ReqDesc* __restrict__ descs, const QueueArgs q) {
    union Lds {
        PostBmfLds<R> post;
        PreBmfLds<R> pre;
    };
    __shared__ Lds sm;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & (kLanes - 1);
    const ReqDesc& d = descs[0];
    const int tiles = d.tiles;
    const int B = q.n_blocks;
    const int n_marks = 2 * B * tiles;
    const uint32_t target = queue::epoch(q);
    const int t = q.t0 + static_cast<int>(blockIdx.x);
    if (t >= q.t1) return;
    const int code = g(q.items)[2 * static_cast<size_t>(t)];
    const int tile = g(q.items)[2 * static_cast<size_t>(t) + 1];
    const int pass = kPasses == 3 ? code >> 30 : kPasses - 1;
    const int rec = code & 0x3FFFFFFF;
    const GLOBAL int32_t* heap = reinterpret_cast<const GLOBAL int32_t*>(g(d.sched)) + static_cast<size_t>(rec) * 16;
    // wave 0 polls the marks this item needs: post-order, lane j < 8 the
    // block rooted at frontier position 8 + j; pre-order, lane 0 the parent
    // block's pre-order mark (the root block: its own post-order mark, which
    // implies every post-order item of the tile)
    auto wait = [&]() {
        if (w == 0) {
            int m = -1;
            const GLOBAL int32_t* dep = g(q.dep) + static_cast<size_t>(rec) * 16;
            if (pass == 0) {
                if (lane < 8) {
                    const int cb = dep[lane];
                    if (cb >= 0) m = cb * tiles + tile;
                }
            } else if (lane == 0) {
                const int pb = dep[8];
                m = pb >= 0 ? (B + pb) * tiles + tile : rec * tiles + tile;
            }
            queue::wait_marks(q, m, target, n_marks, lane);
        }
        __syncthreads();
    };
    if constexpr (kPasses == 1) {
        post_bmf_body<R>(d, heap, tile, tiles, rec == q.root_rec, sm.post, w, lane, wait);
    } else if constexpr (kPasses == 2) {
        pre_bmf_body<R>(d, heap, tile, tiles, sm.pre, w, lane, wait);
    } else {
        if (pass == 0)
            post_bmf_body<R>(d, heap, tile, tiles, rec == q.root_rec, sm.post, w, lane, wait);
        else
            pre_bmf_body<R>(d, heap, tile, tiles, sm.pre, w, lane, wait);
    }
    queue::stores_complete();
    __syncthreads();
    if (threadIdx.x == 0) queue::set_mark(q, (pass * B + rec) * tiles + tile, target, n_marks);
}

// S = 4: one thread per row s of one (branch, category) pair, so a pair's
// four rows come from four neighbouring lanes (contiguous stores) and even a
// small tree spreads over many workgroups.  Row s of P and dP:
//   P[s][u] = sum_k V[s][k] Vinv[k][u] exp(gamma b lam_k),
//   dP[s][u] = sum_k V[s][k] Vinv[k][u] gamma lam_k exp(gamma b lam_k).
// Also the tip tables: entry y < 4 is column y of P (P e_y), entry 4 the row
// sums (P 1, a fully ambiguous tip); component s comes from row s.
constexpr int kPmatBlock = 64;
__global__ __launch_bounds__(kPmatBlock) void pmat4_kernel(const ReqDesc* __restrict__ descs,
                                                           const SegTable segs) {
    constexpr int S = 4;
    const int gid = blockIdx.x * kPmatBlock + threadIdx.x;
    const int unit = gid >> 2;
    const int s = gid & 3;
    // a new evaluation of a work-queue context
    if (gid == 0 && descs[segs.seg[0].desc].qctr) queue::new_evaluation(descs[segs.seg[0].desc].qctr);
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
    // per-category models: category r's eigensystem
    const double* lam = d.lam + (d.eig_cat ? r * S : 0);
    const double* V = d.V + (d.eig_cat ? r * S * S : 0);
    const double* Vinv = d.Vinv + (d.eig_cat ? r * S * S : 0);
    double ex[S], dex[S];
#pragma unroll
    for (int k = 0; k < S; ++k) {
        const double e = exp(lam[k] * t);
        ex[k] = e;
        dex[k] = g * lam[k] * e;
    }
    const size_t base = static_cast<size_t>(pair) * S * S + s * S;
    double Pr[S], dPr[S], rs = 0.0, drs = 0.0;
#pragma unroll
    for (int u = 0; u < S; ++u) {
        double acc = 0.0, dacc = 0.0;
#pragma unroll
        for (int k = 0; k < S; ++k) {
            const double v = V[s * S + k] * Vinv[k * S + u];
            acc += v * ex[k];
            dacc += v * dex[k];
        }
        Pr[u] = acc;
        dPr[u] = dacc;
        rs += acc;
        drs += dacc;
    }
    const size_t tb = static_cast<size_t>(pair) * 20 + s;
#pragma unroll
    for (int u = 0; u < S; ++u) {
        d.P64[base + u] = Pr[u];
        d.dP64[base + u] = dPr[u];
        d.TT64[tb + 4 * u] = Pr[u];
        d.dTT64[tb + 4 * u] = dPr[u];
    }
    d.TT64[tb + 16] = rs;
    d.dTT64[tb + 16] = drs;
    if (d.fp32) {
#pragma unroll
        for (int u = 0; u < S; ++u) {
            d.P32[base + u] = static_cast<float>(Pr[u]);
            d.dP32[base + u] = static_cast<float>(dPr[u]);
            d.TT32[tb + 4 * u] = static_cast<float>(Pr[u]);
            d.dTT32[tb + 4 * u] = static_cast<float>(dPr[u]);
        }
        d.TT32[tb + 16] = static_cast<float>(rs);
        d.dTT32[tb + 16] = static_cast<float>(drs);
    }
}

// Any S: one block per (branch, category) pair.
__global__ __launch_bounds__(256) void pmat_block_kernel(const ReqDesc* __restrict__ descs,
                                                         const SegTable segs) {
    __shared__ double ex[256], dex[256];
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
    // per-category models: category r's eigensystem
    const double* lam = d.lam + (d.eig_cat ? r * S : 0);
    const double* V = d.V + (d.eig_cat ? static_cast<size_t>(r) * S * S : 0);
    const double* Vinv = d.Vinv + (d.eig_cat ? static_cast<size_t>(r) * S * S : 0);
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
    const int E = 2 * d.N - 2, tiles = d.tiles;
    // flags 1: log-likelihood only (one unit; the gradient partials are not
    // formed by a log-likelihood-only evaluation)
    const int blk = (sg.flags & 1) ? E : unit - segs.unit_begin[sidx];
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
        // a work-queue traversal whose dependency wait gave up: invalid sums
        const bool fault =
            d.qctr && __hip_atomic_load(&d.qctr[kQueueFault], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
        const double v = fault ? __builtin_nan("") : red[0];
        if (blk < E)
            sg.out_grad[blk] = v;
        else
            *sg.out_logl = v;
    }
}

template <typename T, int R>
hipError_t level_r(KernelClass k, bool blocked, const ReqDesc* descs, const SegTable& t, hipStream_t st) {
    const int n_units = t.unit_begin[t.n];
    const int blocks = (n_units + kWavesPerBlock - 1) / kWavesPerBlock;
    if constexpr (std::is_same<T, float>::value && (R & (R - 1)) == 0) {
        if (blocked) {
            // pre-order launches whose workgroups all fit on the chip at once
            // with the frontier held in registers (5 waves per SIMD, 4 SIMDs,
            // 256 CUs) are latency-bound: take the variant with one load round
            // trip (the post-order kernel holds it at full occupancy always)
            const int tuned = tuned_value(4, R, true, PHG_TUNE_NARROW_UNITS);
            const bool narrow = n_units <= (tuned > 0 ? tuned : 256 * 4 * 5 / R);
            if (k == kPost) {
                hipLaunchKernelGGL((post_bmf_kernel<R>), dim3(n_units), dim3(kLanes * R), 0, st, descs, t);
            } else {
                if (narrow)
                    hipLaunchKernelGGL((pre_bmf_kernel<R, true>), dim3(n_units), dim3(kLanes * R), 0, st, descs, t);
                else
                    hipLaunchKernelGGL((pre_bmf_kernel<R, false>), dim3(n_units), dim3(kLanes * R), 0, st, descs, t);
            }
            return hipGetLastError();
        }
    }
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

// More than 8 categories (any S) run on the MFMA kernels, which take the
// categories of a (node, tile) one at a time, so R is bounded only by this
// check.
bool kernels_support(int S, int R) { return S >= 2 && S <= 256 && R >= 1 && R <= 64; }

int tile_patterns(int S, int R, bool fp32) {
    if (uses_gl_kernels(S, R, fp32)) return 16 * gl_row_blocks(S, R, fp32);
    return (uses_s4_kernels(S, R) || uses_vs_kernels(S, R, fp32)) ? kLanes : gs_tile_patterns(fp32);
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
                hipLaunchKernelGGL(pmat4_kernel, dim3((4 * n_units + kPmatBlock - 1) / kPmatBlock),
                                   dim3(kPmatBlock), 0, st, descs, t);
            } else if (uses_vs_kernels(shape.S, shape.R, shape.fp32 != 0)) {
                return launch_vs(kPmat, shape, descs, t, st);
            } else if (uses_gl_kernels(shape.S, shape.R, shape.fp32 != 0)) {
                return launch_pmat_gl(shape, descs, t, st);
            } else {
                hipLaunchKernelGGL(pmat_block_kernel, dim3(n_units), dim3(256), 0, st, descs, t);
            }
            return hipGetLastError();
        case kPost:
        case kPre:
            if (uses_vs_kernels(shape.S, shape.R, shape.fp32 != 0)) return launch_vs(k, shape, descs, t, st);
            if (uses_gl_kernels(shape.S, shape.R, shape.fp32 != 0)) return launch_level_gl(k, shape, descs, t, st);
            if (!uses_s4_kernels(shape.S, shape.R)) return launch_level_gs(k, shape, descs, t, st);
            if (shape.fp32) return level_t<float>(k, shape.R, shape.blocked != 0, descs, t, st);
            return level_t<double>(k, shape.R, shape.blocked != 0, descs, t, st);
        case kFinal:
            hipLaunchKernelGGL(finalize_kernel, dim3(n_units), dim3(256), 0, st, descs, t);
            return hipGetLastError();
    }
    return hipErrorInvalidValue;
}

namespace {
template <int R>
hipError_t queue_r(const ReqDesc* descs, const QueueArgs& q, int passes, hipStream_t st) {
    const dim3 grid(q.t1 - q.t0), block(kLanes * R);
    if (passes == 1)
        hipLaunchKernelGGL((queue_bmf_kernel<R, 1>), grid, block, 0, st, descs, q);
    else if (passes == 2)
        hipLaunchKernelGGL((queue_bmf_kernel<R, 2>), grid, block, 0, st, descs, q);
    else
        hipLaunchKernelGGL((queue_bmf_kernel<R, 3>), grid, block, 0, st, descs, q);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_queue(const ReqDesc& shape, const ReqDesc* descs, const QueueArgs& q, int passes,
                        hipStream_t st) {
    if (q.t1 <= q.t0) return hipSuccess;
    if (!queue_supported(shape.S, shape.R, shape.fp32 != 0) || passes < 1 || passes > 3) return hipErrorInvalidValue;
    if (shape.S != 4) {
        if (passes == 3) return hipErrorInvalidValue;
        if (uses_vs_kernels(shape.S, shape.R, shape.fp32 != 0)) return launch_vs_queue(shape, descs, q, passes, st);
        return launch_gl_queue(shape, descs, q, passes, st);
    }
    switch (shape.R) {
        case 1: return queue_r<1>(descs, q, passes, st);
        case 2: return queue_r<2>(descs, q, passes, st);
        case 4: return queue_r<4>(descs, q, passes, st);
        case 8: return queue_r<8>(descs, q, passes, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace phg
