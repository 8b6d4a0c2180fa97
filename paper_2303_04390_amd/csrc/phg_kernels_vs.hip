// gfx950 level kernels for 17..32 states (amino acids) on the vector ALUs.
//
// Same method as the other kernels (Methods: pruning equation, eq:preorder,
// eq:gradient).  One workgroup takes one (node, 64-pattern tile); wave r of
// the workgroup holds category r and lane l pattern l of the tile, with the
// node's vectors for that (category, pattern) in registers (SP values, the
// state count padded to a multiple of 4 with zeros).  Every lane of a wave
// uses the same matrix, so an S x S product is SP^2 fused multiply-adds per
// lane whose matrix operand is wave-uniform.  Each wave first copies the
// P(t) tables of its category for the node's internal children into its own
// LDS region -- all loads in flight at once, so the workgroup waits for
// memory once -- and then reads matrix rows as LDS broadcasts (a row read
// straight from memory before each row's multiply-adds would wait for
// memory once per row).  Per-pattern quantities shared by the categories
// (the rescaling maximum, the gradient's numerator and denominator sums) go
// through LDS once per node.
//
// Layouts (all zero-padded, so no load is masked):
//   partials  [slot][tile][r][SP states][64 patterns]   (state-major: a
//             state of a wave is 64 contiguous values)
//   forward   P, dP  [branch][r][SP rows s][SP cols t] = P[s][t]
//   backward  P, dP  [branch][r][SP + 1 rows][SP]: row t < S holds column t
//             (P[.][t]), rows S..SP-1 zeros, row SP the row sums P 1.
// A tip given by code y takes row y of the backward tables as its P e_y and
// dP e_y (row SP for the ambiguous code S); P^T u accumulates the rows of
// the forward table, P^T u = sum_s u_s P[s][.].
//
// An internal node whose two children are tips given by codes is folded
// (when every branch has its tables): it has no launch of its own.  Its
// parent forms its partial (P_a e_ya) o (P_b e_yb) from two table rows --
// such nodes are never rescaled, so this is bit for bit the vector that
// would have been stored, at less cost than writing and reading it -- and
// turns its pre-order vector into the gradient sums of the two tip branches
// by the operations its own pre-order launch would use.
//
// Scaling as in the 4-state kernels: one power-of-two exponent per (node,
// pattern) shared by all categories; stored post-order partials are
// normalised and the exponents cumulative per subtree; pre-order vectors are
// normalised and their exponents dropped (the gradient ratio does not depend
// on them).
#include "phg_internal.h"
#include "phg_queue_device.h"

#include <math.h>

#include <type_traits>
#include <utility>

namespace phg {
namespace {

#define GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ GLOBAL T* g(T* p) {
    return (GLOBAL T*)p;
}

constexpr int kVL = 64;   // patterns per tile (one per lane)

template <typename T>
__device__ __forceinline__ T* fwdP(const ReqDesc& d);
template <>
__device__ __forceinline__ float* fwdP<float>(const ReqDesc& d) { return d.P32; }
template <>
__device__ __forceinline__ double* fwdP<double>(const ReqDesc& d) { return d.P64; }
template <typename T>
__device__ __forceinline__ T* fwddP(const ReqDesc& d);
template <>
__device__ __forceinline__ float* fwddP<float>(const ReqDesc& d) { return d.dP32; }
template <>
__device__ __forceinline__ double* fwddP<double>(const ReqDesc& d) { return d.dP64; }
template <typename T>
__device__ __forceinline__ T* bwdP(const ReqDesc& d);
template <>
__device__ __forceinline__ float* bwdP<float>(const ReqDesc& d) { return d.PB32; }
template <>
__device__ __forceinline__ double* bwdP<double>(const ReqDesc& d) { return d.PB64; }
template <typename T>
__device__ __forceinline__ T* bwddP(const ReqDesc& d);
template <>
__device__ __forceinline__ float* bwddP<float>(const ReqDesc& d) { return d.dPB32; }
template <>
__device__ __forceinline__ double* bwddP<double>(const ReqDesc& d) { return d.dPB64; }

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
__device__ __forceinline__ float exact_ldexp(float x, int e) { return ldexpf(x, e); }
__device__ __forceinline__ double exact_ldexp(double x, int e) { return ldexp(x, e); }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ int seg_index(const SegTable& t, int unit) {
    int s = 0;
    while (s + 1 < t.n && unit >= t.unit_begin[s + 1]) ++s;
    return s;
}

// A stored vector of this lane's (category, pattern): SP values.
template <typename T, int SP>
__device__ __forceinline__ void vs_load(const GLOBAL T* __restrict__ base, int lane, T (&v)[SP]) {
#pragma unroll
    for (int s = 0; s < SP; ++s) v[s] = base[s * kVL + lane];
}
template <typename T, int SP>
__device__ __forceinline__ void vs_store(GLOBAL T* __restrict__ base, int lane, const T (&v)[SP]) {
#pragma unroll
    for (int s = 0; s < SP; ++s) base[s * kVL + lane] = v[s];
}

// The same with device-coherent accesses (kCoh: vectors that another item of
// a work-queue launch writes or reads).
template <typename T, int SP, bool kCoh>
__device__ __forceinline__ void vs_load_k(const GLOBAL T* __restrict__ base, int lane, T (&v)[SP]) {
    if constexpr (kCoh) {
#pragma unroll
        for (int s = 0; s < SP; ++s) v[s] = queue::ld(base, s * kVL + lane, SP * kVL);
    } else {
        vs_load<T, SP>(base, lane, v);
    }
}
template <typename T, int SP, bool kCoh>
__device__ __forceinline__ void vs_store_k(GLOBAL T* __restrict__ base, int lane, const T (&v)[SP]) {
    if constexpr (kCoh) {
#pragma unroll
        for (int s = 0; s < SP; ++s) queue::st(base, s * kVL + lane, SP * kVL, v[s]);
    } else {
        vs_store<T, SP>(base, lane, v);
    }
}
// Cumulative exponent of internal node x at this lane's pattern c.
template <bool kCoh>
__device__ __forceinline__ int vs_expo(const ReqDesc& d, int x, int tile, int lane) {
    const GLOBAL int32_t* base =
        g(d.expo) + static_cast<size_t>(x - d.N) * d.Cpad + static_cast<size_t>(tile) * kVL;
    if constexpr (kCoh) return queue::ld(base, lane, kVL);
    return base[lane];
}
template <bool kCoh>
__device__ __forceinline__ void vs_set_expo(const ReqDesc& d, int x, int tile, int lane, int e) {
    GLOBAL int32_t* base = g(d.expo) + static_cast<size_t>(x - d.N) * d.Cpad + static_cast<size_t>(tile) * kVL;
    if constexpr (kCoh)
        queue::st(base, lane, kVL, e);
    else
        base[lane] = e;
}

// Row s of a wave-uniform SP x SP matrix (in LDS) times this lane's vector v.
template <typename T, int SP>
__device__ __forceinline__ T vs_row(const T* __restrict__ M, int s, const T (&v)[SP]) {
    T a = T(0);
#pragma unroll
    for (int t = 0; t < SP; ++t) a = fma(M[s * SP + t], v[t], a);
    return a;
}
// Keeps a matrix row's LDS reads beside its multiply-adds, so the registers
// in use stay those of about one row.
__device__ __forceinline__ void row_fence() { __builtin_amdgcn_sched_barrier(0); }

// Copying a wave's SP x SP tables into LDS: 16-byte pieces, all loads of a
// stage issued before the first store.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
template <typename T, int SP>
struct Stage {
    static constexpr int kPieces = SP * SP * static_cast<int>(sizeof(T)) / 16;
    static constexpr int kIters = (kPieces + kVL - 1) / kVL;
    u32x4 r[kIters];
    __device__ __forceinline__ void load(const GLOBAL T* src, int lane) {
        const GLOBAL u32x4* s4 = reinterpret_cast<const GLOBAL u32x4*>(src);
#pragma unroll
        for (int it = 0; it < kIters; ++it)
            if (it * kVL + lane < kPieces) r[it] = s4[it * kVL + lane];
    }
    __device__ __forceinline__ void store(T* dst, int lane) const {
        u32x4* d4 = reinterpret_cast<u32x4*>(dst);
#pragma unroll
        for (int it = 0; it < kIters; ++it)
            if (it * kVL + lane < kPieces) d4[it * kVL + lane] = r[it];
    }
};

// Child x's input for this (category, tile): its stored partial (internal),
// a general tip vector, or null (a tip given by its code).
template <typename T, int SP>
__device__ __forceinline__ const GLOBAL T* vs_src(const ReqDesc& d, int x, int tile, int r) {
    const size_t per = static_cast<size_t>(SP) * kVL;
    if (x >= d.N)
        return g(static_cast<const T*>(d.part)) + ((static_cast<size_t>(x - d.N) * d.tiles + tile) * d.R + r) * per;
    const int gx = d.tslot ? g(d.tslot)[x] : -1;
    return gx >= 0 ? g(static_cast<const T*>(d.tipvec)) + ((static_cast<size_t>(gx) * d.tiles + tile) * d.R + r) * per
                   : nullptr;
}

// Row of a tip's backward table for code y: y itself for a state, row SP
// (the row sums) for the ambiguous code S.
template <int SP>
__device__ __forceinline__ int tip_row(int y, int S) {
    return (y < S ? y : SP) * SP;
}

struct VsUnit {
    const ReqDesc* d;
    Segment sg;
    int i, j, k, tile;
    int ti, tj;   // P(t) tables of the children: by branch, or by slot in per-chunk tables
    bool fi, fj;  // child i / j is a folded node
    bool root;    // k is the tree root
    int rec;      // work-queue launches: the record's index in the schedule
};
__device__ __forceinline__ bool vs_unit(const ReqDesc* __restrict__ descs, const SegTable& segs, VsUnit& U) {
    const int unit = blockIdx.x;
    if (unit >= segs.unit_begin[segs.n]) return false;
    const int sidx = seg_index(segs, unit);
    U.sg = segs.seg[sidx];
    U.d = &descs[U.sg.desc];
    const int tiles = U.d->tiles;
    const int local = unit - segs.unit_begin[sidx];
    const int node_ix = local / tiles;
    U.tile = local - node_ix * tiles;
    const GLOBAL int32_t* rec = g(U.sg.sched) + static_cast<size_t>(U.sg.sched_off + node_ix) * 4;
    U.k = rec[0];
    U.i = rec[1];
    U.j = rec[2];
    U.ti = U.d->level_tables ? 2 * node_ix : U.i;
    U.tj = U.d->level_tables ? 2 * node_ix + 1 : U.j;
    U.fi = (rec[3] & 1) != 0;
    U.fj = (rec[3] & 2) != 0;
    U.root = (U.sg.flags & 1) != 0;
    return true;
}
// Work-queue launches (the context's descriptor is descs[0]): workgroup i
// takes item t0 + i, a (record, tile) pair of this launch's pass.
__device__ __forceinline__ bool vs_unit(const ReqDesc* __restrict__ descs, const QueueArgs& q, VsUnit& U) {
    const int t = q.t0 + static_cast<int>(blockIdx.x);
    if (t >= q.t1) return false;
    U.d = &descs[0];
    U.sg = Segment{};
    U.rec = g(q.items)[2 * static_cast<size_t>(t)];
    U.tile = g(q.items)[2 * static_cast<size_t>(t) + 1];
    const GLOBAL int32_t* rec = reinterpret_cast<const GLOBAL int32_t*>(g(U.d->sched)) + static_cast<size_t>(U.rec) * 4;
    U.k = rec[0];
    U.i = rec[1];
    U.j = rec[2];
    U.ti = U.i;
    U.tj = U.j;
    U.fi = (rec[3] & 1) != 0;
    U.fj = (rec[3] & 2) != 0;
    U.root = U.k == 2 * U.d->N - 2;
    return true;
}

// Completion marks of the work-queue launches, per node slot and tile:
// post-order [0, I tiles), pre-order [I tiles, 2 I tiles), I = q.n_blocks.
// A post-order item waits on its stored children's marks, a pre-order item
// on its parent's (which wrote its pre-order vector); wave 0 polls, then the
// workgroup synchronises.
__device__ __forceinline__ void vs_wait_post(const QueueArgs& q, const VsUnit& U, int r, int lane, uint32_t target) {
    if (r == 0) {
        const ReqDesc& d = *U.d;
        int m = -1;
        if (lane == 0 && U.i >= d.N && !U.fi) m = (U.i - d.N) * d.tiles + U.tile;
        if (lane == 1 && U.j >= d.N && !U.fj) m = (U.j - d.N) * d.tiles + U.tile;
        queue::wait_marks(q, m, target, 2u * q.n_blocks * d.tiles, lane);
    }
    __syncthreads();
}
__device__ __forceinline__ void vs_wait_pre(const QueueArgs& q, const VsUnit& U, int r, int lane, uint32_t target) {
    if (r == 0) {
        const ReqDesc& d = *U.d;
        const int p = g(q.dep)[2 * static_cast<size_t>(U.rec)];     // the parent's slot, -1 at the root
        const int m = lane == 0 && p >= 0 ? (q.n_blocks + p) * d.tiles + U.tile : -1;
        queue::wait_marks(q, m, target, 2u * q.n_blocks * d.tiles, lane);
    }
    __syncthreads();
}
// End of an item: every wave's stores complete, then its mark.
__device__ __forceinline__ void vs_done(const QueueArgs& q, const VsUnit& U, bool pre, uint32_t target) {
    const ReqDesc& d = *U.d;
    queue::stores_complete();
    __syncthreads();
    if (threadIdx.x == 0)
        queue::set_mark(q, ((pre ? q.n_blocks : 0) + U.k - d.N) * d.tiles + U.tile, target,
                        2u * q.n_blocks * d.tiles);
}

// A folded child x (internal, both children a, b tips given by codes): its
// partial (P_a e_ya) o (P_b e_yb) is not stored; consumers form it from two
// rows of the backward tables (folding needs tables for every branch).  A
// node whose children are both tips given by codes is never rescaled
// (exponent 0), so this is bit for bit the vector a post-order launch of x
// would have stored.
template <typename T, int SP>
__device__ __forceinline__ void vs_folded(const ReqDesc& d, int x, int r, int c, T (&v)[SP]) {
    const GLOBAL int32_t* kk = g(d.kids) + 2 * static_cast<size_t>(x - d.N);
    const int a = kk[0], b = kk[1];
    const size_t bmat = static_cast<size_t>(SP + 1) * SP;
    const GLOBAL T* Ba = g(bwdP<T>(d)) + (static_cast<size_t>(a) * d.R + r) * bmat +
                         tip_row<SP>(g(d.codes)[static_cast<size_t>(a) * d.Cpad + c], d.S);
    const GLOBAL T* Bb = g(bwdP<T>(d)) + (static_cast<size_t>(b) * d.R + r) * bmat +
                         tip_row<SP>(g(d.codes)[static_cast<size_t>(b) * d.Cpad + c], d.S);
#pragma unroll
    for (int s = 0; s < SP; ++s) v[s] = Ba[s] * Bb[s];
}
// Child x's input vector: folded (formed from its tips) or loaded.
template <typename T, int SP, bool kCoh = false>
__device__ __forceinline__ void vs_input(const ReqDesc& d, bool folded, const GLOBAL T* src, int x, int r, int c,
                                         int lane, T (&v)[SP]) {
    if (folded)
        vs_folded<T, SP>(d, x, r, c, v);
    else
        vs_load_k<T, SP, kCoh>(src, lane, v);
}

// The gradient sums of a folded node x's two tip branches a < b, formed from
// x's rescaled pre-order vector q by the same operations as a pre-order
// launch of x would use: with m, dm the tips' table rows, u_a = q o m_b and
// u_b = q o m_a, na = u_a . dm_a, nb = u_b . dm_b, den = u_a . m_a.
// Consumes q.
template <typename T, int SP>
__device__ __forceinline__ void folded_grad_sums(const ReqDesc& d, int x, int r, int c, T (&q)[SP], T& na, T& nb,
                                                 T& den) {
    const GLOBAL int32_t* kk = g(d.kids) + 2 * static_cast<size_t>(x - d.N);
    const int a = kk[0], b = kk[1];
    const size_t bmat = static_cast<size_t>(SP + 1) * SP;
    const size_t oa = (static_cast<size_t>(a) * d.R + r) * bmat +
                      tip_row<SP>(g(d.codes)[static_cast<size_t>(a) * d.Cpad + c], d.S);
    const size_t ob = (static_cast<size_t>(b) * d.R + r) * bmat +
                      tip_row<SP>(g(d.codes)[static_cast<size_t>(b) * d.Cpad + c], d.S);
    const GLOBAL T* P = g(bwdP<T>(d));
    const GLOBAL T* dP = g(bwddP<T>(d));
    T ua[SP], dmb[SP];
#pragma unroll
    for (int s = 0; s < SP; ++s) {
        ua[s] = q[s] * P[ob + s];
        dmb[s] = dP[ob + s];
    }
    na = T(0);
    nb = T(0);
    den = T(0);
#pragma unroll
    for (int s = 0; s < SP; ++s) {
        const T m = P[oa + s], dm = dP[oa + s];
        na = fma(ua[s], dm, na);
        den = fma(ua[s], m, den);
        q[s] *= m;
        nb = fma(q[s], dmb[s], nb);
    }
}

// Per-tile gradient sums of branches bi, bj from the categories' weighted
// numerators and denominator in LDS (wave 0).
template <typename T, int R>
__device__ __forceinline__ void write_grad(const ReqDesc& d, const T (&xn_i)[R][kVL], const T (&xn_j)[R][kVL],
                                           const T (&xden)[R][kVL], int lane, int c, int tile, int bi, int bj) {
    T Ni = xn_i[0][lane], Nj = xn_j[0][lane], Dn = xden[0][lane];
#pragma unroll
    for (int rr = 1; rr < R; ++rr) {
        Ni += xn_i[rr][lane];
        Nj += xn_j[rr][lane];
        Dn += xden[rr][lane];
    }
    const double W = g(d.pw)[c];
    const double di = (W != 0.0) ? W * (static_cast<double>(Ni) / static_cast<double>(Dn)) : 0.0;
    const double dj = (W != 0.0) ? W * (static_cast<double>(Nj) / static_cast<double>(Dn)) : 0.0;
    const double si = wave_sum(di), sj = wave_sum(dj);
    if (lane == 0) {
        g(d.gpart)[static_cast<size_t>(bi) * d.tiles + tile] = si;
        g(d.gpart)[static_cast<size_t>(bj) * d.tiles + tile] = sj;
    }
}

// ---------------------------------------------------------------- post-order

// p_k = (P_i p_i) o (P_j p_j) per category, rescaled by the largest entry
// over the node's categories; at the root the site likelihood instead.
template <typename T, int SP, int R, bool kQ, typename Arg>
__device__ __forceinline__ void post_vs_body(const ReqDesc* __restrict__ descs, const Arg& arg) {
    __shared__ __align__(16) T tab[R][2][SP * SP];   // P_i, P_j of each category
    __shared__ T xmax[R][kVL];
    __shared__ double xsite[R][kVL];
    const int r = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & (kVL - 1);
    VsUnit U;
    if (!vs_unit(descs, arg, U)) return;
    const ReqDesc& d = *U.d;
    const int N = d.N, S = d.S, Cpad = d.Cpad, tile = U.tile;
    const int c = tile * kVL + lane;
    const size_t mat = static_cast<size_t>(SP) * SP, bmat = static_cast<size_t>(SP + 1) * SP;
    // children that take a product: internal (stored or folded) or general tip vectors
    const GLOBAL T* src_i = vs_src<T, SP>(d, U.i, tile, r);
    const GLOBAL T* src_j = vs_src<T, SP>(d, U.j, tile, r);
    {   // this category's tables of those children
        Stage<T, SP> si, sj;
        if (src_i) si.load(g(fwdP<T>(d)) + (static_cast<size_t>(U.ti) * R + r) * mat, lane);
        if (src_j) sj.load(g(fwdP<T>(d)) + (static_cast<size_t>(U.tj) * R + r) * mat, lane);
        if (src_i) si.store(tab[r][0], lane);
        if (src_j) sj.store(tab[r][1], lane);
    }
    // the children's cumulative exponents (a folded child's is 0)
    uint32_t target = 0;
    if constexpr (kQ) {
        target = queue::epoch(arg);
        vs_wait_post(arg, U, r, lane, target);
    }
    int ec = 0;
    if constexpr (kQ) {
        if (U.i >= N && !U.fi) ec += vs_expo<true>(d, U.i, tile, lane);
        if (U.j >= N && !U.fj) ec += vs_expo<true>(d, U.j, tile, lane);
    } else {
        if (U.i >= N && !U.fi) ec += g(d.expo)[static_cast<size_t>(U.i - N) * Cpad + c];
        if (U.j >= N && !U.fj) ec += g(d.expo)[static_cast<size_t>(U.j - N) * Cpad + c];
    }
    __syncthreads();
    T p[SP];
    if (src_i) {   // p = P_i p_i
        T v[SP];
        vs_input<T, SP, kQ>(d, U.fi, src_i, U.i, r, c, lane, v);
#pragma unroll
        for (int s = 0; s < SP; ++s) {
            p[s] = vs_row<T, SP>(tab[r][0], s, v);
            row_fence();
        }
    } else {
        const GLOBAL T* B = g(bwdP<T>(d)) + (static_cast<size_t>(U.ti) * R + r) * bmat +
                            tip_row<SP>(g(d.codes)[static_cast<size_t>(U.i) * Cpad + c], S);
#pragma unroll
        for (int s = 0; s < SP; ++s) p[s] = B[s];
    }
    if (src_j) {   // p *= P_j p_j
        T v[SP];
        vs_input<T, SP, kQ>(d, U.fj, src_j, U.j, r, c, lane, v);
#pragma unroll
        for (int s = 0; s < SP; ++s) {
            p[s] *= vs_row<T, SP>(tab[r][1], s, v);
            row_fence();
        }
    } else {
        const GLOBAL T* B = g(bwdP<T>(d)) + (static_cast<size_t>(U.tj) * R + r) * bmat +
                            tip_row<SP>(g(d.codes)[static_cast<size_t>(U.j) * Cpad + c], S);
#pragma unroll
        for (int s = 0; s < SP; ++s) p[s] *= B[s];
    }
    if (!U.root) {
        // rescale, unless both children are tips given by codes (a product of
        // two table entries needs none, and folded nodes rely on exponent 0)
        int e = 0;
        if (src_i || src_j) {
            T lmx = T(0);
#pragma unroll
            for (int s = 0; s < SP; ++s) lmx = fmax(lmx, p[s]);
            xmax[r][lane] = lmx;
            __syncthreads();
            T mx = xmax[0][lane];
#pragma unroll
            for (int rr = 1; rr < R; ++rr) mx = fmax(mx, xmax[rr][lane]);
            e = exponent_of(mx);
#pragma unroll
            for (int s = 0; s < SP; ++s) p[s] = exact_ldexp(p[s], -e);
        }
        vs_store_k<T, SP, kQ>(g(static_cast<T*>(d.part)) +
                            ((static_cast<size_t>(U.k - N) * d.tiles + tile) * R + r) * SP * kVL,
                        lane, p);
        if constexpr (kQ) {
            if (r == 0) vs_set_expo<true>(d, U.k, tile, lane, e + ec);
        } else {
            if (r == 0) g(d.expo)[static_cast<size_t>(U.k - N) * Cpad + c] = e + ec;
        }
    } else {
        // root: site likelihood sum_r w_r pi . p_r, categories summed in a fixed order
        double acc = 0.0;
#pragma unroll
        for (int s = 0; s < SP; ++s)
            if (s < S) acc += g(d.pi)[s] * static_cast<double>(p[s]);
        xsite[r][lane] = g(d.cweights)[r] * acc;
        __syncthreads();
        if (r == 0) {
            double site = 0.0;
#pragma unroll
            for (int rr = 0; rr < R; ++rr) site += xsite[rr][lane];
            const double ll = (site > 0.0 ? log(site) : -INFINITY) + static_cast<double>(ec) * 0.69314718055994530942;
            g(d.sll)[c] = ll;
            const double W = g(d.pw)[c];
            const double tsum = wave_sum(W != 0.0 ? W * ll : 0.0);
            if (lane == 0) g(d.lpart)[tile] = tsum;
        }
    }
    if constexpr (kQ) vs_done(arg, U, false, target);
}

template <typename T, int SP, int R>
__global__ __launch_bounds__(kVL * R) void post_vs_kernel(const ReqDesc* __restrict__ descs, const SegTable segs) {
    post_vs_body<T, SP, R, false>(descs, segs);
}
// The same over a work-queue launch's items.
template <typename T, int SP, int R>
__global__ __launch_bounds__(kVL * R) void post_vs_queue_kernel(const ReqDesc* __restrict__ descs, const QueueArgs q) {
    post_vs_body<T, SP, R, true>(descs, q);
}

// ---------------------------------------------------------------- pre-order + gradient

// With q the parent's pre-order vector (pi at the root), m_x = P_x p_x and
// dm_x = dP_x p_x:  u_i = q o m_j, u_j = q o m_i; the children's pre-order
// vectors P_i^T u_i, P_j^T u_j (rescaled as in the post-order pass) replace
// their partials; the per-pattern gradient of branch i is
// sum_r w_r u_i . dm_i over sum_r w_r u_i . m_i (likewise j).  Child i is
// taken row by row, so at most four vectors per lane are live.
template <typename T, int SP, int R, bool kQ, typename Arg>
__device__ __forceinline__ void pre_vs_body(const ReqDesc* __restrict__ descs, const Arg& arg) {
    __shared__ __align__(16) T tab[R][4][SP * SP];   // P_i, dP_i, P_j, dP_j of each category
    __shared__ T xch[5][R][kVL];
    __shared__ T xg[6][R][kVL];                      // folded children's gradient sums
    const int r = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & (kVL - 1);
    VsUnit U;
    if (!vs_unit(descs, arg, U)) return;
    const ReqDesc& d = *U.d;
    const int N = d.N, S = d.S, Cpad = d.Cpad, tile = U.tile, tiles = d.tiles;
    const int c = tile * kVL + lane;
    const size_t mat = static_cast<size_t>(SP) * SP, bmat = static_cast<size_t>(SP + 1) * SP;
    const size_t per = static_cast<size_t>(SP) * kVL;
    GLOBAL T* part = g(static_cast<T*>(d.part));
    const bool in_i = U.i >= N, in_j = U.j >= N;
    const GLOBAL T* src_i = vs_src<T, SP>(d, U.i, tile, r);
    const GLOBAL T* src_j = vs_src<T, SP>(d, U.j, tile, r);
    {   // this category's tables of the children that take a product
        const size_t oi = (static_cast<size_t>(U.ti) * R + r) * mat, oj = (static_cast<size_t>(U.tj) * R + r) * mat;
        Stage<T, SP> a, da, b, db;
        if (src_i) {
            a.load(g(fwdP<T>(d)) + oi, lane);
            da.load(g(fwddP<T>(d)) + oi, lane);
        }
        if (src_j) {
            b.load(g(fwdP<T>(d)) + oj, lane);
            db.load(g(fwddP<T>(d)) + oj, lane);
        }
        if (src_i) {
            a.store(tab[r][0], lane);
            da.store(tab[r][1], lane);
        }
        if (src_j) {
            b.store(tab[r][2], lane);
            db.store(tab[r][3], lane);
        }
    }
    uint32_t target = 0;
    if constexpr (kQ) {
        target = queue::epoch(arg);
        vs_wait_pre(arg, U, r, lane, target);
    }
    T q[SP];
    if (U.k == 2 * N - 2) {
#pragma unroll
        for (int s = 0; s < SP; ++s) q[s] = s < S ? static_cast<T>(g(d.pi)[s]) : T(0);
    } else {
        vs_load_k<T, SP, kQ>(part + ((static_cast<size_t>(U.k - N) * tiles + tile) * R + r) * per, lane, q);
    }
    __syncthreads();
    // child j: u_i = q o m_j and dm_j
    T ui[SP], dmj[SP];
    if (src_j) {
        T v[SP];
        vs_input<T, SP>(d, U.fj, src_j, U.j, r, c, lane, v);
#pragma unroll
        for (int s = 0; s < SP; ++s) {
            ui[s] = q[s] * vs_row<T, SP>(tab[r][2], s, v);
            dmj[s] = vs_row<T, SP>(tab[r][3], s, v);
            row_fence();
        }
    } else {
        const size_t bo = (static_cast<size_t>(U.tj) * R + r) * bmat +
                          tip_row<SP>(g(d.codes)[static_cast<size_t>(U.j) * Cpad + c], S);
        const GLOBAL T* B = g(bwdP<T>(d)) + bo;
        const GLOBAL T* B2 = g(bwddP<T>(d)) + bo;
#pragma unroll
        for (int s = 0; s < SP; ++s) {
            ui[s] = q[s] * B[s];
            dmj[s] = B2[s];
        }
    }
    // child i, one state at a time: the sums, and q becomes u_j = q o m_i
    T ni = T(0), nj = T(0), den = T(0);
    if (src_i) {
        T v[SP];
        vs_input<T, SP>(d, U.fi, src_i, U.i, r, c, lane, v);
#pragma unroll
        for (int s = 0; s < SP; ++s) {
            const T m = vs_row<T, SP>(tab[r][0], s, v), dm = vs_row<T, SP>(tab[r][1], s, v);
            ni = fma(ui[s], dm, ni);
            den = fma(ui[s], m, den);
            q[s] *= m;
            nj = fma(q[s], dmj[s], nj);
            row_fence();
        }
    } else {
        const size_t bo = (static_cast<size_t>(U.ti) * R + r) * bmat +
                          tip_row<SP>(g(d.codes)[static_cast<size_t>(U.i) * Cpad + c], S);
        const GLOBAL T* B = g(bwdP<T>(d)) + bo;
        const GLOBAL T* B2 = g(bwddP<T>(d)) + bo;
#pragma unroll
        for (int s = 0; s < SP; ++s) {
            const T m = B[s], dm = B2[s];
            ni = fma(ui[s], dm, ni);
            den = fma(ui[s], m, den);
            q[s] *= m;
            nj = fma(q[s], dmj[s], nj);
        }
    }
    // pre-order vectors of internal children: P^T u = sum_s u_s P[s][.]
    T qi[SP], qj[SP];
    T mxi = T(0), mxj = T(0);
    if (in_i) {
#pragma unroll
        for (int t = 0; t < SP; ++t) qi[t] = T(0);
#pragma unroll
        for (int s = 0; s < SP; ++s) {
            const T us = ui[s];
#pragma unroll
            for (int t = 0; t < SP; ++t) qi[t] = fma(tab[r][0][s * SP + t], us, qi[t]);
            row_fence();
        }
#pragma unroll
        for (int t = 0; t < SP; ++t) mxi = fmax(mxi, qi[t]);
    }
    if (in_j) {
#pragma unroll
        for (int t = 0; t < SP; ++t) qj[t] = T(0);
#pragma unroll
        for (int s = 0; s < SP; ++s) {
            const T us = q[s];
#pragma unroll
            for (int t = 0; t < SP; ++t) qj[t] = fma(tab[r][2][s * SP + t], us, qj[t]);
            row_fence();
        }
#pragma unroll
        for (int t = 0; t < SP; ++t) mxj = fmax(mxj, qj[t]);
    }
    const T wr = static_cast<T>(g(d.cweights)[r]);
    xch[0][r][lane] = wr * ni;
    xch[1][r][lane] = wr * nj;
    xch[2][r][lane] = wr * den;
    xch[3][r][lane] = mxi;
    xch[4][r][lane] = mxj;
    __syncthreads();
    T Mi = xch[3][0][lane], Mj = xch[4][0][lane];
#pragma unroll
    for (int rr = 1; rr < R; ++rr) {
        Mi = fmax(Mi, xch[3][rr][lane]);
        Mj = fmax(Mj, xch[4][rr][lane]);
    }
    // a child's rescaled pre-order vector is stored, or, for a folded child,
    // turned into its tip branches' gradient sums at once
    if (in_i) {
        const int e = exponent_of(Mi);
#pragma unroll
        for (int s = 0; s < SP; ++s) qi[s] = exact_ldexp(qi[s], -e);
        if (U.fi) {
            T na, nb, dn;
            folded_grad_sums<T, SP>(d, U.i, r, c, qi, na, nb, dn);
            xg[0][r][lane] = wr * na;
            xg[1][r][lane] = wr * nb;
            xg[2][r][lane] = wr * dn;
        } else {
            vs_store_k<T, SP, kQ>(part + ((static_cast<size_t>(U.i - N) * tiles + tile) * R + r) * per, lane, qi);
        }
    }
    if (in_j) {
        const int e = exponent_of(Mj);
#pragma unroll
        for (int s = 0; s < SP; ++s) qj[s] = exact_ldexp(qj[s], -e);
        if (U.fj) {
            T na, nb, dn;
            folded_grad_sums<T, SP>(d, U.j, r, c, qj, na, nb, dn);
            xg[3][r][lane] = wr * na;
            xg[4][r][lane] = wr * nb;
            xg[5][r][lane] = wr * dn;
        } else {
            vs_store_k<T, SP, kQ>(part + ((static_cast<size_t>(U.j - N) * tiles + tile) * R + r) * per, lane, qj);
        }
    }
    if (U.fi || U.fj) __syncthreads();
    if (r == 0) {
        write_grad<T, R>(d, xch[0], xch[1], xch[2], lane, c, tile, U.i, U.j);
        const GLOBAL int32_t* kk = g(d.kids);
        if (U.fi) write_grad<T, R>(d, xg[0], xg[1], xg[2], lane, c, tile, kk[2 * (U.i - N)], kk[2 * (U.i - N) + 1]);
        if (U.fj) write_grad<T, R>(d, xg[3], xg[4], xg[5], lane, c, tile, kk[2 * (U.j - N)], kk[2 * (U.j - N) + 1]);
    }
    if constexpr (kQ) vs_done(arg, U, true, target);
}

template <typename T, int SP, int R>
__global__ __launch_bounds__(kVL * R) void pre_vs_kernel(const ReqDesc* __restrict__ descs, const SegTable segs) {
    pre_vs_body<T, SP, R, false>(descs, segs);
}
// The same over a work-queue launch's items.
template <typename T, int SP, int R>
__global__ __launch_bounds__(kVL * R) void pre_vs_queue_kernel(const ReqDesc* __restrict__ descs, const QueueArgs q) {
    pre_vs_body<T, SP, R, true>(descs, q);
}

// ---------------------------------------------------------------- FP32, 20 states: matrices in registers

// The FP32 kernels at 17..20 states stage the tables in LDS as the others
// do, then copy the one matrix a pass needs into VGPRs and feed every
// multiply-add its matrix entry as a DPP row_newbcast operand (the value in
// lane n of each 16-lane row, broadcast to the row), so the products read
// no LDS: a 20 x 20 matrix is 25 registers, replicated in the
// four 16-lane rows -- register s (s < 20) holds M[s][0..15] in lanes 0..15,
// register 20 + j holds M[s][16..19] for rows s = 4j..4j+3 in lanes
// 4 (s mod 4) .. 4 (s mod 4) + 3.  The multiply-adds are written as
// v_fmac_f32_dpp in inline assembly (the compiler does not fold a DPP move
// into an accumulating FMA); each block opens with five wait states, which
// covers the DPP read-after-VALU-write and EXEC-write hazards for whatever
// the compiler placed before it.  Products accumulate in the same order as
// the other kernels' (t ascending, first term a plain product), so results
// are bit for bit theirs.
struct MatReg20 {
    float r[25];
    // from a row-major 20 x 20 table staged in LDS (25 reads of 4 bytes per lane)
    __device__ __forceinline__ void load(const float* __restrict__ M, int lane) {
        const int n = lane & 15;
#pragma unroll
        for (int s = 0; s < 20; ++s) r[s] = M[s * 20 + n];
#pragma unroll
        for (int j = 0; j < 5; ++j) r[20 + j] = M[(4 * j + n / 4) * 20 + 16 + (n & 3)];
    }
};

// a = M[s][0..15] . v[0..15]  (mr = register s)
__device__ __forceinline__ float dpp_dot16(float mr, const float (&v)[20]) {
    float a;
    asm(
        "s_nop 4\n\t"
        "v_mul_f32_dpp %0, %1, %2 row_newbcast:0 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %3 row_newbcast:1 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %4 row_newbcast:2 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %5 row_newbcast:3 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %6 row_newbcast:4 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %7 row_newbcast:5 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %8 row_newbcast:6 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %9 row_newbcast:7 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %10 row_newbcast:8 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %11 row_newbcast:9 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %12 row_newbcast:10 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %13 row_newbcast:11 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %14 row_newbcast:12 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %15 row_newbcast:13 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %16 row_newbcast:14 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %17 row_newbcast:15 row_mask:0xf bank_mask:0xf"
        : "=&v"(a)
        : "v"(mr), "v"(v[0]), "v"(v[1]), "v"(v[2]), "v"(v[3]), "v"(v[4]), "v"(v[5]), "v"(v[6]), "v"(v[7]),
          "v"(v[8]), "v"(v[9]), "v"(v[10]), "v"(v[11]), "v"(v[12]), "v"(v[13]), "v"(v[14]), "v"(v[15]));
    return a;
}
// a += M[s][16..19] . v[16..19]  (tr = the tail register, lanes B..B+3)
template <int B>
__device__ __forceinline__ void dpp_dot4(float& a, float tr, const float (&v)[20]) {
    asm(
        "s_nop 4\n\t"
        "v_fmac_f32_dpp %0, %1, %2 row_newbcast:%6 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %3 row_newbcast:%7 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %4 row_newbcast:%8 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %5 row_newbcast:%9 row_mask:0xf bank_mask:0xf"
        : "+v"(a)
        : "v"(tr), "v"(v[16]), "v"(v[17]), "v"(v[18]), "v"(v[19]), "i"(B), "i"(B + 1), "i"(B + 2), "i"(B + 3));
}
// (M v)_s
template <int S>
__device__ __forceinline__ float dpp_row(const MatReg20& M, const float (&v)[20]) {
    float a = dpp_dot16(M.r[S], v);
    dpp_dot4<4 * (S % 4)>(a, M.r[20 + S / 4], v);
    return a;
}
// q[t] += M[s][t] u_s for every t (row s of P^T u)
template <int S>
__device__ __forceinline__ void dpp_acc_row(const MatReg20& M, float us, float (&q)[20]) {
    asm(
        "s_nop 4\n\t"
        "v_fmac_f32_dpp %0, %16, %17 row_newbcast:0 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %1, %16, %17 row_newbcast:1 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %2, %16, %17 row_newbcast:2 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %3, %16, %17 row_newbcast:3 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %4, %16, %17 row_newbcast:4 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %5, %16, %17 row_newbcast:5 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %6, %16, %17 row_newbcast:6 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %7, %16, %17 row_newbcast:7 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %8, %16, %17 row_newbcast:8 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %9, %16, %17 row_newbcast:9 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %10, %16, %17 row_newbcast:10 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %11, %16, %17 row_newbcast:11 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %12, %16, %17 row_newbcast:12 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %13, %16, %17 row_newbcast:13 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %14, %16, %17 row_newbcast:14 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %15, %16, %17 row_newbcast:15 row_mask:0xf bank_mask:0xf"
        : "+v"(q[0]), "+v"(q[1]), "+v"(q[2]), "+v"(q[3]), "+v"(q[4]), "+v"(q[5]), "+v"(q[6]), "+v"(q[7]),
          "+v"(q[8]), "+v"(q[9]), "+v"(q[10]), "+v"(q[11]), "+v"(q[12]), "+v"(q[13]), "+v"(q[14]), "+v"(q[15])
        : "v"(M.r[S]), "v"(us));
    asm(
        "s_nop 4\n\t"
        "v_fmac_f32_dpp %0, %4, %5 row_newbcast:%6 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %1, %4, %5 row_newbcast:%7 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %2, %4, %5 row_newbcast:%8 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %3, %4, %5 row_newbcast:%9 row_mask:0xf bank_mask:0xf"
        : "+v"(q[16]), "+v"(q[17]), "+v"(q[18]), "+v"(q[19])
        : "v"(M.r[20 + S / 4]), "v"(us), "i"(4 * (S % 4)), "i"(4 * (S % 4) + 1), "i"(4 * (S % 4) + 2),
          "i"(4 * (S % 4) + 3));
}

template <typename F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
// f(std::integral_constant<int, i>) for i = 0 .. n-1, in order.
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// Post-order, FP32, 17..20 states (as post_vs_kernel, products on registers).
template <int R, bool kQ, typename Arg>
__device__ __forceinline__ void post_vd_body(const ReqDesc* __restrict__ descs, const Arg& arg) {
    constexpr int SP = 20;
    using T = float;
    __shared__ __align__(16) T tab[R][2][SP * SP];   // P_i, P_j of each category
    __shared__ T xmax[R][kVL];
    __shared__ double xsite[R][kVL];
    const int r = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & (kVL - 1);
    VsUnit U;
    if (!vs_unit(descs, arg, U)) return;
    const ReqDesc& d = *U.d;
    const int N = d.N, S = d.S, Cpad = d.Cpad, tile = U.tile;
    const int c = tile * kVL + lane;
    const size_t mat = static_cast<size_t>(SP) * SP, bmat = static_cast<size_t>(SP + 1) * SP;
    const GLOBAL T* src_i = vs_src<T, SP>(d, U.i, tile, r);
    const GLOBAL T* src_j = vs_src<T, SP>(d, U.j, tile, r);
    {
        Stage<T, SP> si, sj;
        if (src_i) si.load(g(fwdP<T>(d)) + (static_cast<size_t>(U.ti) * R + r) * mat, lane);
        if (src_j) sj.load(g(fwdP<T>(d)) + (static_cast<size_t>(U.tj) * R + r) * mat, lane);
        if (src_i) si.store(tab[r][0], lane);
        if (src_j) sj.store(tab[r][1], lane);
    }
    uint32_t target = 0;
    if constexpr (kQ) {
        target = queue::epoch(arg);
        vs_wait_post(arg, U, r, lane, target);
    }
    int ec = 0;
    if constexpr (kQ) {
        if (U.i >= N && !U.fi) ec += vs_expo<true>(d, U.i, tile, lane);
        if (U.j >= N && !U.fj) ec += vs_expo<true>(d, U.j, tile, lane);
    } else {
        if (U.i >= N && !U.fi) ec += g(d.expo)[static_cast<size_t>(U.i - N) * Cpad + c];
        if (U.j >= N && !U.fj) ec += g(d.expo)[static_cast<size_t>(U.j - N) * Cpad + c];
    }
    __syncthreads();
    T p[SP];
    if (src_i) {   // p = P_i p_i
        T v[SP];
        vs_input<T, SP, kQ>(d, U.fi, src_i, U.i, r, c, lane, v);
        MatReg20 M;
        M.load(tab[r][0], lane);
        static_for<SP>([&](auto s) { p[s] = dpp_row<s>(M, v); });
    } else {
        const GLOBAL T* B = g(bwdP<T>(d)) + (static_cast<size_t>(U.ti) * R + r) * bmat +
                            tip_row<SP>(g(d.codes)[static_cast<size_t>(U.i) * Cpad + c], S);
#pragma unroll
        for (int s = 0; s < SP; ++s) p[s] = B[s];
    }
    if (src_j) {   // p *= P_j p_j
        T v[SP];
        vs_input<T, SP, kQ>(d, U.fj, src_j, U.j, r, c, lane, v);
        MatReg20 M;
        M.load(tab[r][1], lane);
        static_for<SP>([&](auto s) { p[s] *= dpp_row<s>(M, v); });
    } else {
        const GLOBAL T* B = g(bwdP<T>(d)) + (static_cast<size_t>(U.tj) * R + r) * bmat +
                            tip_row<SP>(g(d.codes)[static_cast<size_t>(U.j) * Cpad + c], S);
#pragma unroll
        for (int s = 0; s < SP; ++s) p[s] *= B[s];
    }
    if (!U.root) {
        int e = 0;
        if (src_i || src_j) {
            T lmx = T(0);
#pragma unroll
            for (int s = 0; s < SP; ++s) lmx = fmax(lmx, p[s]);
            xmax[r][lane] = lmx;
            __syncthreads();
            T mx = xmax[0][lane];
#pragma unroll
            for (int rr = 1; rr < R; ++rr) mx = fmax(mx, xmax[rr][lane]);
            e = exponent_of(mx);
#pragma unroll
            for (int s = 0; s < SP; ++s) p[s] = exact_ldexp(p[s], -e);
        }
        vs_store_k<T, SP, kQ>(g(static_cast<T*>(d.part)) +
                            ((static_cast<size_t>(U.k - N) * d.tiles + tile) * R + r) * SP * kVL,
                        lane, p);
        if constexpr (kQ) {
            if (r == 0) vs_set_expo<true>(d, U.k, tile, lane, e + ec);
        } else {
            if (r == 0) g(d.expo)[static_cast<size_t>(U.k - N) * Cpad + c] = e + ec;
        }
    } else {
        double acc = 0.0;
#pragma unroll
        for (int s = 0; s < SP; ++s)
            if (s < S) acc += g(d.pi)[s] * static_cast<double>(p[s]);
        xsite[r][lane] = g(d.cweights)[r] * acc;
        __syncthreads();
        if (r == 0) {
            double site = 0.0;
#pragma unroll
            for (int rr = 0; rr < R; ++rr) site += xsite[rr][lane];
            const double ll = (site > 0.0 ? log(site) : -INFINITY) + static_cast<double>(ec) * 0.69314718055994530942;
            g(d.sll)[c] = ll;
            const double W = g(d.pw)[c];
            const double tsum = wave_sum(W != 0.0 ? W * ll : 0.0);
            if (lane == 0) g(d.lpart)[tile] = tsum;
        }
    }
    if constexpr (kQ) vs_done(arg, U, false, target);
}

template <int R>
__global__ __launch_bounds__(kVL * R) void post_vd_kernel(const ReqDesc* __restrict__ descs, const SegTable segs) {
    post_vd_body<R, false>(descs, segs);
}
// The same over a work-queue launch's items.
template <int R>
__global__ __launch_bounds__(kVL * R) void post_vd_queue_kernel(const ReqDesc* __restrict__ descs, const QueueArgs q) {
    post_vd_body<R, true>(descs, q);
}

// Pre-order and gradient, FP32, 17..20 states (as pre_vs_kernel, products on
// registers, one matrix at a time: each child's P and dP products run as
// two passes, and P^T u accumulates the rows of the forward table).  Every
// sum keeps its order, so results are those of pre_vs_kernel bit for bit.
template <int R, bool kQ, typename Arg>
__device__ __forceinline__ void pre_vd_body(const ReqDesc* __restrict__ descs, const Arg& arg) {
    constexpr int SP = 20;
    using T = float;
    __shared__ __align__(16) T tab[R][4][SP * SP];   // P_i, dP_i, P_j, dP_j of each category
    __shared__ T xch[5][R][kVL];
    __shared__ T xg[6][R][kVL];
    const int r = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & (kVL - 1);
    VsUnit U;
    if (!vs_unit(descs, arg, U)) return;
    const ReqDesc& d = *U.d;
    const int N = d.N, S = d.S, Cpad = d.Cpad, tile = U.tile, tiles = d.tiles;
    const int c = tile * kVL + lane;
    const size_t mat = static_cast<size_t>(SP) * SP, bmat = static_cast<size_t>(SP + 1) * SP;
    const size_t per = static_cast<size_t>(SP) * kVL;
    GLOBAL T* part = g(static_cast<T*>(d.part));
    const bool in_i = U.i >= N, in_j = U.j >= N;
    const GLOBAL T* src_i = vs_src<T, SP>(d, U.i, tile, r);
    const GLOBAL T* src_j = vs_src<T, SP>(d, U.j, tile, r);
    {
        const size_t oi = (static_cast<size_t>(U.ti) * R + r) * mat, oj = (static_cast<size_t>(U.tj) * R + r) * mat;
        Stage<T, SP> a, da, b, db;
        if (src_i) {
            a.load(g(fwdP<T>(d)) + oi, lane);
            da.load(g(fwddP<T>(d)) + oi, lane);
        }
        if (src_j) {
            b.load(g(fwdP<T>(d)) + oj, lane);
            db.load(g(fwddP<T>(d)) + oj, lane);
        }
        if (src_i) {
            a.store(tab[r][0], lane);
            da.store(tab[r][1], lane);
        }
        if (src_j) {
            b.store(tab[r][2], lane);
            db.store(tab[r][3], lane);
        }
    }
    uint32_t target = 0;
    if constexpr (kQ) {
        target = queue::epoch(arg);
        vs_wait_pre(arg, U, r, lane, target);
    }
    T q[SP];
    if (U.k == 2 * N - 2) {
#pragma unroll
        for (int s = 0; s < SP; ++s) q[s] = s < S ? static_cast<T>(g(d.pi)[s]) : T(0);
    } else {
        vs_load_k<T, SP, kQ>(part + ((static_cast<size_t>(U.k - N) * tiles + tile) * R + r) * per, lane, q);
    }
    __syncthreads();
    // child j: u_i = q o m_j, then dm_j
    T ui[SP], dmj[SP];
    if (src_j) {
        T v[SP];
        vs_input<T, SP>(d, U.fj, src_j, U.j, r, c, lane, v);
        {
            MatReg20 M;
            M.load(tab[r][2], lane);
            static_for<SP>([&](auto s) { ui[s] = q[s] * dpp_row<s>(M, v); });
        }
        {
            MatReg20 M;
            M.load(tab[r][3], lane);
            static_for<SP>([&](auto s) { dmj[s] = dpp_row<s>(M, v); });
        }
    } else {
        const size_t bo = (static_cast<size_t>(U.tj) * R + r) * bmat +
                          tip_row<SP>(g(d.codes)[static_cast<size_t>(U.j) * Cpad + c], S);
        const GLOBAL T* B = g(bwdP<T>(d)) + bo;
        const GLOBAL T* B2 = g(bwddP<T>(d)) + bo;
#pragma unroll
        for (int s = 0; s < SP; ++s) {
            ui[s] = q[s] * B[s];
            dmj[s] = B2[s];
        }
    }
    // child i: with m_i the sums den, nj and q becomes u_j = q o m_i; with dm_i, ni
    T ni = T(0), nj = T(0), den = T(0);
    if (src_i) {
        T v[SP];
        vs_input<T, SP>(d, U.fi, src_i, U.i, r, c, lane, v);
        {
            MatReg20 M;
            M.load(tab[r][0], lane);
            static_for<SP>([&](auto s) {
                const T m = dpp_row<s>(M, v);
                den = fma(ui[s], m, den);
                q[s] *= m;
                nj = fma(q[s], dmj[s], nj);
            });
        }
        {
            MatReg20 M;
            M.load(tab[r][1], lane);
            static_for<SP>([&](auto s) { ni = fma(ui[s], dpp_row<s>(M, v), ni); });
        }
    } else {
        const size_t bo = (static_cast<size_t>(U.ti) * R + r) * bmat +
                          tip_row<SP>(g(d.codes)[static_cast<size_t>(U.i) * Cpad + c], S);
        const GLOBAL T* B = g(bwdP<T>(d)) + bo;
        const GLOBAL T* B2 = g(bwddP<T>(d)) + bo;
#pragma unroll
        for (int s = 0; s < SP; ++s) {
            const T m = B[s], dm = B2[s];
            ni = fma(ui[s], dm, ni);
            den = fma(ui[s], m, den);
            q[s] *= m;
            nj = fma(q[s], dmj[s], nj);
        }
    }
    // pre-order vectors of internal children: P^T u = sum_s u_s P[s][.]
    T qi[SP], qj[SP];
    T mxi = T(0), mxj = T(0);
    if (in_i) {
        MatReg20 M;
        M.load(tab[r][0], lane);
#pragma unroll
        for (int t = 0; t < SP; ++t) qi[t] = T(0);
        static_for<SP>([&](auto s) { dpp_acc_row<s>(M, ui[s], qi); });
#pragma unroll
        for (int t = 0; t < SP; ++t) mxi = fmax(mxi, qi[t]);
    }
    if (in_j) {
        MatReg20 M;
        M.load(tab[r][2], lane);
#pragma unroll
        for (int t = 0; t < SP; ++t) qj[t] = T(0);
        static_for<SP>([&](auto s) { dpp_acc_row<s>(M, q[s], qj); });
#pragma unroll
        for (int t = 0; t < SP; ++t) mxj = fmax(mxj, qj[t]);
    }
    const T wr = static_cast<T>(g(d.cweights)[r]);
    xch[0][r][lane] = wr * ni;
    xch[1][r][lane] = wr * nj;
    xch[2][r][lane] = wr * den;
    xch[3][r][lane] = mxi;
    xch[4][r][lane] = mxj;
    __syncthreads();
    T Mi = xch[3][0][lane], Mj = xch[4][0][lane];
#pragma unroll
    for (int rr = 1; rr < R; ++rr) {
        Mi = fmax(Mi, xch[3][rr][lane]);
        Mj = fmax(Mj, xch[4][rr][lane]);
    }
    // a child's rescaled pre-order vector is stored, or, for a folded child,
    // turned into its tip branches' gradient sums at once
    if (in_i) {
        const int e = exponent_of(Mi);
#pragma unroll
        for (int s = 0; s < SP; ++s) qi[s] = exact_ldexp(qi[s], -e);
        if (U.fi) {
            T na, nb, dn;
            folded_grad_sums<T, SP>(d, U.i, r, c, qi, na, nb, dn);
            xg[0][r][lane] = wr * na;
            xg[1][r][lane] = wr * nb;
            xg[2][r][lane] = wr * dn;
        } else {
            vs_store_k<T, SP, kQ>(part + ((static_cast<size_t>(U.i - N) * tiles + tile) * R + r) * per, lane, qi);
        }
    }
    if (in_j) {
        const int e = exponent_of(Mj);
#pragma unroll
        for (int s = 0; s < SP; ++s) qj[s] = exact_ldexp(qj[s], -e);
        if (U.fj) {
            T na, nb, dn;
            folded_grad_sums<T, SP>(d, U.j, r, c, qj, na, nb, dn);
            xg[3][r][lane] = wr * na;
            xg[4][r][lane] = wr * nb;
            xg[5][r][lane] = wr * dn;
        } else {
            vs_store_k<T, SP, kQ>(part + ((static_cast<size_t>(U.j - N) * tiles + tile) * R + r) * per, lane, qj);
        }
    }
    if (U.fi || U.fj) __syncthreads();
    if (r == 0) {
        write_grad<T, R>(d, xch[0], xch[1], xch[2], lane, c, tile, U.i, U.j);
        const GLOBAL int32_t* kk = g(d.kids);
        if (U.fi) write_grad<T, R>(d, xg[0], xg[1], xg[2], lane, c, tile, kk[2 * (U.i - N)], kk[2 * (U.i - N) + 1]);
        if (U.fj) write_grad<T, R>(d, xg[3], xg[4], xg[5], lane, c, tile, kk[2 * (U.j - N)], kk[2 * (U.j - N) + 1]);
    }
    if constexpr (kQ) vs_done(arg, U, true, target);
}

template <int R>
__global__ __launch_bounds__(kVL * R) __attribute__((amdgpu_waves_per_eu(4)))
void pre_vd_kernel(const ReqDesc* __restrict__ descs, const SegTable segs) {
    pre_vd_body<R, false>(descs, segs);
}
// The same over a work-queue launch's items.
template <int R>
__global__ __launch_bounds__(kVL * R) __attribute__((amdgpu_waves_per_eu(4)))
void pre_vd_queue_kernel(const ReqDesc* __restrict__ descs, const QueueArgs q) {
    pre_vd_body<R, true>(descs, q);
}

// ---------------------------------------------------------------- P(t) tables

// One workgroup per (branch, category) pair: P and dP (FP64 sums stored in
// the path's type) as zero-padded forward tables and as backward tables with
// the row sums P 1 = V (e o Vinv 1), dP 1 in row SP.
template <typename T, int SP>
__global__ __launch_bounds__(256) void pmat_vs_kernel(const ReqDesc* __restrict__ descs, const SegTable segs) {
    __shared__ double ex[SP], dex[SP];
    __shared__ double sV[SP * SP], sVi[SP * SP];     // V and V^-1 (S x S used), read once from memory
    const int unit = blockIdx.x;
    // a new evaluation of a work-queue context
    if (unit == 0 && threadIdx.x == 0 && descs[segs.seg[0].desc].qctr)
        queue::new_evaluation(descs[segs.seg[0].desc].qctr);
    if (unit >= segs.unit_begin[segs.n]) return;
    const int sidx = seg_index(segs, unit);
    const Segment& sg = segs.seg[sidx];
    const ReqDesc& d = descs[sg.desc];
    const int pair = unit - segs.unit_begin[sidx];   // table (branch or slot) * R + category
    const int R = d.R, S = d.S;
    const int slot = pair / R;
    const int r = pair - slot * R;
    int x = slot;                                    // the branch: its own table
    if (sg.flags & 2) {                              // per-chunk tables: child (slot & 1) of record slot / 2
        const GLOBAL int32_t* rec = g(sg.sched) + static_cast<size_t>(sg.sched_off + slot / 2) * 4;
        x = (slot & 1) ? rec[2] : rec[1];
    }
    const double gr = d.rates[r];
    const double bt = gr * d.b[x];
    const double* lam = d.lam + (d.eig_cat ? r * S : 0);
    const double* V = d.V + (d.eig_cat ? static_cast<size_t>(r) * S * S : 0);
    const double* Vinv = d.Vinv + (d.eig_cat ? static_cast<size_t>(r) * S * S : 0);
    const double* vs = d.vsum + (d.eig_cat ? r * S : 0);
    for (int k = threadIdx.x; k < S; k += blockDim.x) {
        const double e = exp(lam[k] * bt);
        ex[k] = e;
        dex[k] = gr * lam[k] * e;
    }
    for (int i = threadIdx.x; i < S * S; i += blockDim.x) {
        sV[i] = V[i];
        sVi[i] = Vinv[i];
    }
    __syncthreads();
    GLOBAL T* F = g(fwdP<T>(d)) + static_cast<size_t>(pair) * SP * SP;
    GLOBAL T* dF = g(fwddP<T>(d)) + static_cast<size_t>(pair) * SP * SP;
    GLOBAL T* Bk = g(bwdP<T>(d)) + static_cast<size_t>(pair) * (SP + 1) * SP;
    GLOBAL T* dB = g(bwddP<T>(d)) + static_cast<size_t>(pair) * (SP + 1) * SP;
    for (int e = threadIdx.x; e < SP * SP; e += blockDim.x) {
        const int s = e / SP, t = e - s * SP;
        double acc = 0.0, dacc = 0.0;
        if (s < S && t < S) {
            for (int k = 0; k < S; ++k) {
                const double v = sV[s * S + k] * sVi[k * S + t];
                acc += v * ex[k];
                dacc += v * dex[k];
            }
        }
        F[e] = static_cast<T>(acc);
        dF[e] = static_cast<T>(dacc);
        Bk[t * SP + s] = static_cast<T>(acc);
        dB[t * SP + s] = static_cast<T>(dacc);
    }
    for (int s = threadIdx.x; s < SP; s += blockDim.x) {
        double rs = 0.0, drs = 0.0;
        if (s < S)
            for (int k = 0; k < S; ++k) {
                const double a = sV[s * S + k] * vs[k];
                rs += a * ex[k];
                drs += a * dex[k];
            }
        Bk[SP * SP + s] = static_cast<T>(rs);
        dB[SP * SP + s] = static_cast<T>(drs);
    }
}

template <typename T, int SP>
hipError_t launch_vs_sp(KernelClass k, int R, const ReqDesc* descs, const SegTable& t, hipStream_t st) {
    const int n_units = t.unit_begin[t.n];
    if (k == kPmat) {
        hipLaunchKernelGGL((pmat_vs_kernel<T, SP>), dim3(n_units), dim3(256), 0, st, descs, t);
        return hipGetLastError();
    }
#define PHG_VS_CASE(RV)                                                                                    \
    if constexpr (vs_lds_bytes(SP, RV, sizeof(T)) <= kVsLdsMax)                                            \
    if (R == RV) {                                                                                         \
        if constexpr (sizeof(T) == 4 && SP == 20) {                                                        \
            if (k == kPost)                                                                                \
                hipLaunchKernelGGL((post_vd_kernel<RV>), dim3(n_units), dim3(kVL * RV), 0, st, descs, t);  \
            else                                                                                           \
                hipLaunchKernelGGL((pre_vd_kernel<RV>), dim3(n_units), dim3(kVL * RV), 0, st, descs, t);   \
        } else {                                                                                           \
            if (k == kPost)                                                                                \
                hipLaunchKernelGGL((post_vs_kernel<T, SP, RV>), dim3(n_units), dim3(kVL * RV), 0, st, descs, t); \
            else                                                                                           \
                hipLaunchKernelGGL((pre_vs_kernel<T, SP, RV>), dim3(n_units), dim3(kVL * RV), 0, st, descs, t);  \
        }                                                                                                  \
        return hipGetLastError();                                                                          \
    }
    PHG_VS_CASE(1)
    PHG_VS_CASE(2)
    PHG_VS_CASE(4)
    PHG_VS_CASE(8)
#undef PHG_VS_CASE
    return hipErrorInvalidValue;
}

// Work-queue launches: post-order (pass 1) or pre-order (pass 2) items
// [q.t0, q.t1), one workgroup each.
template <typename T, int SP>
hipError_t launch_vs_queue_sp(int pass, int R, const ReqDesc* descs, const QueueArgs& q, hipStream_t st) {
    const dim3 grid(q.t1 - q.t0);
#define PHG_VSQ_CASE(RV)                                                                                   \
    if constexpr (vs_lds_bytes(SP, RV, sizeof(T)) <= kVsLdsMax)                                            \
    if (R == RV) {                                                                                         \
        if constexpr (sizeof(T) == 4 && SP == 20) {                                                        \
            if (pass == 1)                                                                                 \
                hipLaunchKernelGGL((post_vd_queue_kernel<RV>), grid, dim3(kVL * RV), 0, st, descs, q);    \
            else                                                                                           \
                hipLaunchKernelGGL((pre_vd_queue_kernel<RV>), grid, dim3(kVL * RV), 0, st, descs, q);     \
        } else {                                                                                           \
            if (pass == 1)                                                                                 \
                hipLaunchKernelGGL((post_vs_queue_kernel<T, SP, RV>), grid, dim3(kVL * RV), 0, st, descs, q); \
            else                                                                                           \
                hipLaunchKernelGGL((pre_vs_queue_kernel<T, SP, RV>), grid, dim3(kVL * RV), 0, st, descs, q);  \
        }                                                                                                  \
        return hipGetLastError();                                                                          \
    }
    PHG_VSQ_CASE(1)
    PHG_VSQ_CASE(2)
    PHG_VSQ_CASE(4)
    PHG_VSQ_CASE(8)
#undef PHG_VSQ_CASE
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_vs_queue_t(int pass, int S, int R, const ReqDesc* descs, const QueueArgs& q, hipStream_t st) {
    if (vs_padded_states(S) == 20) return launch_vs_queue_sp<T, 20>(pass, R, descs, q, st);
    if (vs_padded_states(S) == 24) return launch_vs_queue_sp<T, 24>(pass, R, descs, q, st);
    if constexpr (sizeof(T) == 4) return launch_vs_queue_sp<T, 32>(pass, R, descs, q, st);
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_vs_t(KernelClass k, int S, int R, const ReqDesc* descs, const SegTable& t, hipStream_t st) {
    if (vs_padded_states(S) == 20) return launch_vs_sp<T, 20>(k, R, descs, t, st);
    if (vs_padded_states(S) == 24) return launch_vs_sp<T, 24>(k, R, descs, t, st);
    if constexpr (sizeof(T) == 4) return launch_vs_sp<T, 32>(k, R, descs, t, st);
    return hipErrorInvalidValue;   // FP64 takes these kernels up to 24 states
}

}  // namespace

hipError_t launch_vs(KernelClass k, const ReqDesc& shape, const ReqDesc* descs, const SegTable& t,
                     hipStream_t st) {
    if (t.n <= 0 || t.unit_begin[t.n] <= 0) return hipSuccess;
    if (shape.fp32) return launch_vs_t<float>(k, shape.S, shape.R, descs, t, st);
    return launch_vs_t<double>(k, shape.S, shape.R, descs, t, st);
}

hipError_t launch_vs_queue(const ReqDesc& shape, const ReqDesc* descs, const QueueArgs& q, int pass,
                           hipStream_t st) {
    if (q.t1 <= q.t0) return hipSuccess;
    if (pass != 1 && pass != 2) return hipErrorInvalidValue;
    if (shape.fp32) return launch_vs_queue_t<float>(pass, shape.S, shape.R, descs, q, st);
    return launch_vs_queue_t<double>(pass, shape.S, shape.R, descs, q, st);
}

}  // namespace phg
