// gfx950 level kernels for larger state spaces (5..64 states: amino acids,
// codons), built on MFMA 16x16x4 tiles (f32 for the FP32 path, f64 for the
// FP64 path).
//
// Same method as the 4-state kernels (Methods: pruning equation,
// eq:preorder, eq:gradient), arranged as small matrix products:
//   forward   m[c][s]  = sum_t P[s][t] p[c][t]      (P_x p_x, dP_x p_x)
//   backward  q[c][t]  = sum_s u[c][s] P[s][t]     (q_x = P_x^T u_x)
// with c over the patterns of a tile and s, t over states padded to a
// multiple of 16.  MFMA 16x16x4 computes D(16x16) += A(16x4) B(4x16); lane l
// holds A[l%16][l/16] and B[l/16][l%16].  Its 4 output registers hold
// D[4(l/16)+i][l%16] for the f32 instruction and D[4i+l/16][l%16] for the f64
// one (measured on gfx950).  Here A rows are patterns, B is P (forward:
// B[t][s] = P[s][t]; backward: B[s][t] = P[s][t]) and D rows are patterns, so
// an output vector lives in "D layout": lane (g = l/16, n = l%16) holds, for
// state 16cb + n of every row block rb and column block cb, the four patterns
// dpat(rb, g, 0..3) (16rb + 4g + i for float, 16rb + 4i + g for double).
//
// Partials are stored [slot][tile][r][state][TP patterns] (exact state count,
// no padding): a stored partial loads directly as A fragments (lane reads
// pattern 16rb + n of state 4kk + g) and a D-layout vector stores as 16-byte
// runs of 4 patterns.  Computed vectors that feed a backward product (u) go
// through a per-wave LDS buffer to change from D to A layout.
//
// Tip children form their A fragments from the tip codes (one-hot, or all
// ones for the ambiguous code S), so P p for a tip is the same product as
// for an internal child and the ambiguous case is the literal row sum.
//
// Scaling matches the 4-state path: one power-of-two exponent per (node,
// pattern) shared by all categories.  Categories are processed one at a time
// (register budget), so each output is written unscaled in a first pass and
// rescaled in place once the exponent is known (the second pass hits L2).
#include "phg_internal.h"

#include <math.h>

namespace phg {
namespace {

#define GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ GLOBAL T* g(T* p) {
    return (GLOBAL T*)p;
}

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

__device__ __forceinline__ Vec4<float> mfma(float a, float b, Vec4<float> c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ Vec4<double> mfma(double a, double b, Vec4<double> c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
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

// Reductions over the 16 lanes that share a pattern group (same l/16).
template <typename V>
__device__ __forceinline__ V group16_sum(V v) {
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) v += __shfl_xor(v, off, 64);
    return v;
}
template <typename V>
__device__ __forceinline__ V group16_max(V v) {
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
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

__device__ __forceinline__ int find_segment(const SegTable& t, int unit) {
    int s = 0;
    while (s + 1 < t.n && unit >= t.unit_begin[s + 1]) ++s;
    return s;
}

// Pattern (within the tile) of output register i of row block rb for lane
// group g: the MFMA D layout of the f32 and f64 instructions.
template <typename T>
__device__ __forceinline__ int dpat(int rb, int gq, int i) {
    return sizeof(T) == 4 ? 16 * rb + 4 * gq + i : 16 * rb + 4 * i + gq;
}

// A D-layout vector: RB row blocks x NB column blocks, 4 values each.
template <typename T, int RB, int NB>
struct DVec {
    Vec4<T> v[RB][NB];
};

// Where one child's A operand comes from.
template <typename T>
struct Source {
    const GLOBAL T* base;   // stored partial of (slot, tile, r); null for a tip
    int code[4];            // tip codes of patterns 16rb + n (tip children)
};

template <typename T, int RB, int NB>
__device__ __forceinline__ void zero(DVec<T, RB, NB>& x) {
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) x.v[rb][cb] = Vec4<T>{0, 0, 0, 0};
}

// Load / store a stored partial of (slot, tile, r) in D layout.
template <typename T, int RB, int NB, int TP>
__device__ __forceinline__ void load_d(const GLOBAL T* __restrict__ base, int S, int lane,
                                       DVec<T, RB, NB>& x) {
    const int gq = lane >> 4, n = lane & 15;
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) {
        const int s = 16 * cb + n;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            if (s >= S) {
                x.v[rb][cb] = Vec4<T>{0, 0, 0, 0};
            } else if (sizeof(T) == 4) {
                x.v[rb][cb] = *reinterpret_cast<const GLOBAL Vec4<T>*>(base + s * TP + 16 * rb + 4 * gq);
            } else {
#pragma unroll
                for (int i = 0; i < 4; ++i) x.v[rb][cb][i] = base[s * TP + dpat<T>(rb, gq, i)];
            }
        }
    }
}

template <typename T, int RB, int NB, int TP>
__device__ __forceinline__ void store_d(GLOBAL T* __restrict__ base, int S, int lane,
                                        const DVec<T, RB, NB>& x) {
    const int gq = lane >> 4, n = lane & 15;
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) {
        const int s = 16 * cb + n;
        if (s < S) {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                if (sizeof(T) == 4) {
                    *reinterpret_cast<GLOBAL Vec4<T>*>(base + s * TP + 16 * rb + 4 * gq) = x.v[rb][cb];
                } else {
#pragma unroll
                    for (int i = 0; i < 4; ++i) base[s * TP + dpat<T>(rb, gq, i)] = x.v[rb][cb][i];
                }
            }
        }
    }
}

// out[c][s] = sum_t M[s][t] in[c][t] (M row-major S x S), in from `src`.
template <typename T, int RB, int NB, int TP>
__device__ __forceinline__ void forward(const GLOBAL T* __restrict__ M, const Source<T>& src, int S,
                                        int lane, DVec<T, RB, NB>& out) {
    const int gq = lane >> 4, n = lane & 15;
    zero(out);
    constexpr int KB = 4 * NB;  // k-steps of 4 states over the padded width
#pragma unroll 4
    for (int kk = 0; kk < KB; ++kk) {
        const int t = 4 * kk + gq;                 // input state this lane feeds
        T a[RB];
        if (src.base) {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) a[rb] = (t < S) ? src.base[t * TP + 16 * rb + n] : T(0);
        } else {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
                a[rb] = (src.code[rb] == t || (src.code[rb] >= S && t < S)) ? T(1) : T(0);
        }
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) {
            const int s = 16 * cb + n;             // output state of this lane's B column
            const T b = (s < S && t < S) ? M[s * S + t] : T(0);
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) out.v[rb][cb] = mfma(a[rb], b, out.v[rb][cb]);
        }
    }
}

// out[c][t] = sum_s u[c][s] M[s][t]; u is read from the wave's LDS buffer
// laid out [state][LS] (LS = padded row stride).
template <typename T, int RB, int NB, int LS>
__device__ __forceinline__ void backward(const GLOBAL T* __restrict__ M, const T* lds, int S, int lane,
                                         DVec<T, RB, NB>& out) {
    const int gq = lane >> 4, n = lane & 15;
    zero(out);
    constexpr int KB = 4 * NB;
#pragma unroll 4
    for (int kk = 0; kk < KB; ++kk) {
        const int s = 4 * kk + gq;                 // summed state this lane feeds
        T a[RB];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) a[rb] = lds[s * LS + 16 * rb + n];
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) {
            const int t = 16 * cb + n;
            const T b = (s < S && t < S) ? M[s * S + t] : T(0);
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) out.v[rb][cb] = mfma(a[rb], b, out.v[rb][cb]);
        }
    }
}

// Write a D-layout vector into the wave's LDS buffer ([state][LS]).
template <typename T, int RB, int NB, int LS>
__device__ __forceinline__ void to_lds(T* lds, int lane, const DVec<T, RB, NB>& x) {
    const int gq = lane >> 4, n = lane & 15;
#pragma unroll
    for (int cb = 0; cb < NB; ++cb)
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            if (sizeof(T) == 4) {
                *reinterpret_cast<Vec4<T>*>(lds + (16 * cb + n) * LS + 16 * rb + 4 * gq) = x.v[rb][cb];
            } else {
#pragma unroll
                for (int i = 0; i < 4; ++i) lds[(16 * cb + n) * LS + dpat<T>(rb, gq, i)] = x.v[rb][cb][i];
            }
        }
}

// Per-pattern partial dot product over this lane's states: acc[rb][i] += sum_cb x*y.
template <typename T, int RB, int NB>
__device__ __forceinline__ void dot_acc(const DVec<T, RB, NB>& x, const DVec<T, RB, NB>& y,
                                        T acc[RB][4]) {
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < NB; ++cb)
#pragma unroll
            for (int i = 0; i < 4; ++i) acc[rb][i] += x.v[rb][cb][i] * y.v[rb][cb][i];
}

template <typename T, int RB, int NB>
__device__ __forceinline__ void max_acc(const DVec<T, RB, NB>& x, T mx[RB][4]) {
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < NB; ++cb)
#pragma unroll
            for (int i = 0; i < 4; ++i) mx[rb][i] = fmax(mx[rb][i], x.v[rb][cb][i]);
}

// Scale a stored (slot, tile) partial, all categories, by 2^-e per pattern.
template <typename T, int RB, int NB, int TP>
__device__ __forceinline__ void rescale_stored(GLOBAL T* __restrict__ slot_tile, int R, int S, int lane,
                                               const int e[RB][4]) {
    for (int r = 0; r < R; ++r) {
        GLOBAL T* base = slot_tile + static_cast<size_t>(r) * S * TP;
        DVec<T, RB, NB> x;
        load_d<T, RB, NB, TP>(base, S, lane, x);
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int cb = 0; cb < NB; ++cb)
#pragma unroll
                for (int i = 0; i < 4; ++i) x.v[rb][cb][i] = exact_ldexp(x.v[rb][cb][i], -e[rb][i]);
        store_d<T, RB, NB, TP>(base, S, lane, x);
    }
}

// ---------------------------------------------------------------- post-order

template <typename T, int RB, int NB>
__device__ __forceinline__ void post_unit_gs(const NodeTriple nt, const int tile, const int N,
                                             const int Cpad, const int S, const int R, const int lane,
                                             const int flags, const GLOBAL uint8_t* __restrict__ codes,
                                             GLOBAL T* __restrict__ part, GLOBAL int32_t* __restrict__ expo,
                                             const GLOBAL T* __restrict__ P,
                                             const GLOBAL double* __restrict__ cw,
                                             const GLOBAL double* __restrict__ pi,
                                             const GLOBAL double* __restrict__ pw,
                                             GLOBAL double* __restrict__ sll, GLOBAL double* __restrict__ lpart,
                                             const int tiles, const GLOBAL int32_t* __restrict__ tslot,
                                             const GLOBAL T* __restrict__ tipvec) {
    constexpr int TP = 16 * RB;
    const int gq = lane >> 4, n = lane & 15;
    const size_t rstride = static_cast<size_t>(S) * TP;          // one category
    const size_t tstride = rstride * R;                           // one (slot, tile)
    Source<T> si{}, sj{};
    const bool tip_i = nt.i < N, tip_j = nt.j < N;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
        const int c = tile * TP + 16 * rb + n;
        si.code[rb] = tip_i ? codes[static_cast<size_t>(nt.i) * Cpad + c] : 0;
        sj.code[rb] = tip_j ? codes[static_cast<size_t>(nt.j) * Cpad + c] : 0;
    }
    // a tip's input: its code, or its general partial vector (slot >= 0)
    const int vsi = (tip_i && tslot) ? tslot[nt.i] : -1;
    const int vsj = (tip_j && tslot) ? tslot[nt.j] : -1;
    const GLOBAL T* pi_base = !tip_i  ? part + (static_cast<size_t>(nt.i - N) * tiles + tile) * tstride
                              : vsi >= 0 ? tipvec + (static_cast<size_t>(vsi) * tiles + tile) * tstride
                                        : nullptr;
    const GLOBAL T* pj_base = !tip_j  ? part + (static_cast<size_t>(nt.j - N) * tiles + tile) * tstride
                              : vsj >= 0 ? tipvec + (static_cast<size_t>(vsj) * tiles + tile) * tstride
                                        : nullptr;
    GLOBAL T* out_base = part + (static_cast<size_t>(nt.k - N) * tiles + tile) * tstride;
    const bool root = flags & 1;

    T mx[RB][4];
    double site[RB][4];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            mx[rb][i] = T(0);
            site[rb][i] = 0.0;
        }
    for (int r = 0; r < R; ++r) {
        si.base = pi_base ? pi_base + r * rstride : nullptr;
        sj.base = pj_base ? pj_base + r * rstride : nullptr;
        const GLOBAL T* Pi = P + (static_cast<size_t>(nt.i) * R + r) * S * S;
        const GLOBAL T* Pj = P + (static_cast<size_t>(nt.j) * R + r) * S * S;
        DVec<T, RB, NB> mi, mj;
        forward<T, RB, NB, TP>(Pi, si, S, lane, mi);
        forward<T, RB, NB, TP>(Pj, sj, S, lane, mj);
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int cb = 0; cb < NB; ++cb) mi.v[rb][cb] *= mj.v[rb][cb];
        if (!root) {
            max_acc(mi, mx);
            store_d<T, RB, NB, TP>(out_base + r * rstride, S, lane, mi);
        } else {
            const double wr = cw[r];
#pragma unroll
            for (int cb = 0; cb < NB; ++cb) {
                const int s = 16 * cb + n;
                const double ps = (s < S) ? pi[s] : 0.0;
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                    for (int i = 0; i < 4; ++i) site[rb][i] += wr * ps * static_cast<double>(mi.v[rb][cb][i]);
            }
        }
    }
    // cumulative exponents of the children for this lane's patterns 16rb + 4g + i
    int ec[RB][4];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int c = tile * TP + dpat<T>(rb, gq, i);
            ec[rb][i] = (tip_i ? 0 : expo[static_cast<size_t>(nt.i - N) * Cpad + c]) +
                        (tip_j ? 0 : expo[static_cast<size_t>(nt.j - N) * Cpad + c]);
        }
    if (!root) {
        int e[RB][4];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int i = 0; i < 4; ++i) e[rb][i] = exponent_of(group16_max(mx[rb][i]));
        rescale_stored<T, RB, NB, TP>(out_base, R, S, lane, e);
        if (n == 0) {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    expo[static_cast<size_t>(nt.k - N) * Cpad + tile * TP + dpat<T>(rb, gq, i)] =
                        e[rb][i] + ec[rb][i];
        }
    } else {
        double tsum = 0.0;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const double sv = group16_sum(site[rb][i]);
                const int c = tile * TP + dpat<T>(rb, gq, i);
                const double ll = (sv > 0.0 ? log(sv) : -INFINITY) +
                                  static_cast<double>(ec[rb][i]) * 0.69314718055994530942;
                const double W = pw[c];
                if (n == 0) {
                    sll[c] = ll;
                    tsum += (W != 0.0) ? W * ll : 0.0;
                }
            }
        tsum = wave_sum(tsum);
        if (lane == 0) lpart[tile] = tsum;
    }
}

template <typename T, int RB, int NB>
__global__ __launch_bounds__(256) void post_gs_kernel(const ReqDesc* __restrict__ descs,
                                                      const SegTable segs) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int unit = blockIdx.x * 4 + wave;
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
    post_unit_gs<T, RB, NB>(nt, tile, d.N, d.Cpad, d.S, d.R, lane, sg.flags, g(d.codes),
                            g(static_cast<T*>(d.part)), g(d.expo), g(ptab<T>(d)), g(d.cweights), g(d.pi),
                            g(d.pw), g(d.sll), g(d.lpart), tiles, g(d.tslot), g(static_cast<const T*>(d.tipvec)));
}

// ---------------------------------------------------------------- pre-order + gradient

template <typename T, int RB, int NB>
__device__ __forceinline__ void pre_unit_gs(const NodeTriple nt, const int tile, const int N,
                                            const int Cpad, const int S, const int R, const int lane,
                                            const GLOBAL uint8_t* __restrict__ codes,
                                            GLOBAL T* __restrict__ part, const GLOBAL T* __restrict__ P,
                                            const GLOBAL T* __restrict__ dP,
                                            const GLOBAL double* __restrict__ cw,
                                            const GLOBAL double* __restrict__ pi,
                                            const GLOBAL double* __restrict__ pw,
                                            GLOBAL double* __restrict__ gpart, const int tiles, T* lds,
                                            const GLOBAL int32_t* __restrict__ tslot,
                                            const GLOBAL T* __restrict__ tipvec) {
    constexpr int TP = 16 * RB;
    constexpr int LS = TP + 16 * 4 / static_cast<int>(sizeof(T));   // LDS row stride (padded)
    const int gq = lane >> 4, n = lane & 15;
    const size_t rstride = static_cast<size_t>(S) * TP;
    const size_t tstride = rstride * R;
    const bool is_root = nt.k == 2 * N - 2;
    const bool tip_i = nt.i < N, tip_j = nt.j < N;
    Source<T> si{}, sj{};
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
        const int c = tile * TP + 16 * rb + n;
        si.code[rb] = tip_i ? codes[static_cast<size_t>(nt.i) * Cpad + c] : 0;
        sj.code[rb] = tip_j ? codes[static_cast<size_t>(nt.j) * Cpad + c] : 0;
    }
    GLOBAL T* pi_base = tip_i ? nullptr : part + (static_cast<size_t>(nt.i - N) * tiles + tile) * tstride;
    GLOBAL T* pj_base = tip_j ? nullptr : part + (static_cast<size_t>(nt.j - N) * tiles + tile) * tstride;
    const GLOBAL T* qk_base = is_root ? nullptr : part + (static_cast<size_t>(nt.k - N) * tiles + tile) * tstride;
    // inputs: stored partials, or a tip's general partial vector (slot >= 0),
    // or (null) its code; q is written for internal children only
    const int vsi = (tip_i && tslot) ? tslot[nt.i] : -1;
    const int vsj = (tip_j && tslot) ? tslot[nt.j] : -1;
    const GLOBAL T* pi_src = vsi >= 0 ? tipvec + (static_cast<size_t>(vsi) * tiles + tile) * tstride : pi_base;
    const GLOBAL T* pj_src = vsj >= 0 ? tipvec + (static_cast<size_t>(vsj) * tiles + tile) * tstride : pj_base;

    T num_i[RB][4], num_j[RB][4], den[RB][4], mxi[RB][4], mxj[RB][4];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int i = 0; i < 4; ++i) num_i[rb][i] = num_j[rb][i] = den[rb][i] = mxi[rb][i] = mxj[rb][i] = T(0);

    for (int r = 0; r < R; ++r) {
        si.base = pi_src ? pi_src + r * rstride : nullptr;
        sj.base = pj_src ? pj_src + r * rstride : nullptr;
        const size_t moff = (static_cast<size_t>(0) + r) * S * S;
        const GLOBAL T* Pi = P + static_cast<size_t>(nt.i) * R * S * S + moff;
        const GLOBAL T* Pj = P + static_cast<size_t>(nt.j) * R * S * S + moff;
        const GLOBAL T* dPi = dP + static_cast<size_t>(nt.i) * R * S * S + moff;
        const GLOBAL T* dPj = dP + static_cast<size_t>(nt.j) * R * S * S + moff;
        const T wr = static_cast<T>(cw[r]);

        DVec<T, RB, NB> qk, a, b, acc;
        if (is_root) {
#pragma unroll
            for (int cb = 0; cb < NB; ++cb) {
                const int s = 16 * cb + n;
                const T v = (s < S) ? static_cast<T>(pi[s]) : T(0);
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) qk.v[rb][cb] = Vec4<T>{v, v, v, v};
            }
        } else {
            load_d<T, RB, NB, TP>(qk_base + r * rstride, S, lane, qk);
        }
        forward<T, RB, NB, TP>(Pj, sj, S, lane, a);          // a = m_j
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int cb = 0; cb < NB; ++cb) a.v[rb][cb] *= qk.v[rb][cb];   // a = u_i
        forward<T, RB, NB, TP>(Pi, si, S, lane, b);          // b = m_i
        T dd[RB][4] = {};
        dot_acc(a, b, dd);                                    // u_i . m_i
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int cb = 0; cb < NB; ++cb) b.v[rb][cb] *= qk.v[rb][cb];   // b = u_j
        forward<T, RB, NB, TP>(dPi, si, S, lane, acc);       // dm_i
        T ni[RB][4] = {}, nj[RB][4] = {};
        dot_acc(a, acc, ni);
        forward<T, RB, NB, TP>(dPj, sj, S, lane, acc);       // dm_j
        dot_acc(b, acc, nj);
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                num_i[rb][i] += wr * ni[rb][i];
                num_j[rb][i] += wr * nj[rb][i];
                den[rb][i] += wr * dd[rb][i];
            }
        // q_x = P_x^T u_x for internal children, written unscaled over p_x
        if (!tip_i) {
            to_lds<T, RB, NB, LS>(lds, lane, a);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            backward<T, RB, NB, LS>(Pi, lds, S, lane, acc);
            max_acc(acc, mxi);
            store_d<T, RB, NB, TP>(pi_base + r * rstride, S, lane, acc);
            __builtin_amdgcn_wave_barrier();
        }
        if (!tip_j) {
            to_lds<T, RB, NB, LS>(lds, lane, b);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            backward<T, RB, NB, LS>(Pj, lds, S, lane, acc);
            max_acc(acc, mxj);
            store_d<T, RB, NB, TP>(pj_base + r * rstride, S, lane, acc);
            __builtin_amdgcn_wave_barrier();
        }
    }
    if (!tip_i) {
        int e[RB][4];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int i = 0; i < 4; ++i) e[rb][i] = exponent_of(group16_max(mxi[rb][i]));
        rescale_stored<T, RB, NB, TP>(pi_base, R, S, lane, e);
    }
    if (!tip_j) {
        int e[RB][4];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int i = 0; i < 4; ++i) e[rb][i] = exponent_of(group16_max(mxj[rb][i]));
        rescale_stored<T, RB, NB, TP>(pj_base, R, S, lane, e);
    }
    double gi = 0.0, gj = 0.0;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const double Ni = static_cast<double>(group16_sum(num_i[rb][i]));
            const double Nj = static_cast<double>(group16_sum(num_j[rb][i]));
            const double Dn = static_cast<double>(group16_sum(den[rb][i]));
            const int c = tile * TP + dpat<T>(rb, gq, i);
            const double W = pw[c];
            if (n == 0 && W != 0.0) {
                gi += W * (Ni / Dn);
                gj += W * (Nj / Dn);
            }
        }
    gi = wave_sum(gi);
    gj = wave_sum(gj);
    if (lane == 0) {
        gpart[static_cast<size_t>(nt.i) * tiles + tile] = gi;
        gpart[static_cast<size_t>(nt.j) * tiles + tile] = gj;
    }
}

template <typename T, int RB, int NB>
__global__ __launch_bounds__(256) void pre_gs_kernel(const ReqDesc* __restrict__ descs,
                                                     const SegTable segs) {
    constexpr int TP = 16 * RB;
    constexpr int LS = TP + 16 * 4 / static_cast<int>(sizeof(T));
    __shared__ T lds_all[4][16 * NB * LS];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int unit = blockIdx.x * 4 + wave;
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
    pre_unit_gs<T, RB, NB>(nt, tile, d.N, d.Cpad, d.S, d.R, lane, g(d.codes), g(static_cast<T*>(d.part)),
                           g(ptab<T>(d)), g(dptab<T>(d)), g(d.cweights), g(d.pi), g(d.pw), g(d.gpart),
                           tiles, lds_all[wave], g(d.tslot), g(static_cast<const T*>(d.tipvec)));
}

template <typename T, int RB>
hipError_t launch_nb(KernelClass k, int NB, const ReqDesc* descs, const SegTable& t, hipStream_t st) {
    const int n_units = t.unit_begin[t.n];
    const int blocks = (n_units + 3) / 4;
#define PHG_GS_CASE(NBV)                                                                              \
    case NBV:                                                                                         \
        if (k == kPost)                                                                               \
            hipLaunchKernelGGL((post_gs_kernel<T, RB, NBV>), dim3(blocks), dim3(256), 0, st, descs, t); \
        else                                                                                          \
            hipLaunchKernelGGL((pre_gs_kernel<T, RB, NBV>), dim3(blocks), dim3(256), 0, st, descs, t);  \
        return hipGetLastError();
    switch (NB) {
        PHG_GS_CASE(1)
        PHG_GS_CASE(2)
        PHG_GS_CASE(3)
        PHG_GS_CASE(4)
        default: return hipErrorInvalidValue;
    }
#undef PHG_GS_CASE
}

}  // namespace

int gs_tile_patterns(bool fp32) { return fp32 ? 32 : 16; }

hipError_t launch_level_gs(KernelClass k, const ReqDesc& shape, const ReqDesc* descs, const SegTable& t,
                           hipStream_t st) {
    const int NB = (shape.S + 15) / 16;
    if (shape.fp32) return launch_nb<float, 2>(k, NB, descs, t, st);
    return launch_nb<double, 1>(k, NB, descs, t, st);
}

}  // namespace phg
