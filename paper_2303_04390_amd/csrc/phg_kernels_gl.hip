// gfx950 level kernels for 17..255 states (amino acids, codons, Markov-
// modulated and phylogeographic models), on MFMA 16x16x4 tiles (f32 for the
// FP32 path, f64 for the FP64 path).
//
// Same method as the other kernels (Methods: pruning equation, eq:preorder,
// eq:gradient), as small matrix products over a tile of patterns:
//   forward   m[c][s] = sum_t P[s][t] p[c][t]      (P_x p_x, dP_x p_x)
//   backward  q[c][t] = sum_s u[c][s] P[s][t]      (q_x = P_x^T u_x)
// One workgroup of W waves takes one (node, pattern tile); wave w owns the
// output states [w * 16 NBW, (w + 1) * 16 NBW) of every product (NBW column
// blocks of 16; W = ceil(S / 16) waves of one block up to 128 states, four
// waves above), and runs the full sum over input states itself:
// matrices come from HBM/L2; the input vectors of a category (stored partials
// of the children, q of the parent) are staged once per workgroup in LDS by
// 16-byte loads, and the vectors u that feed P^T u are written there by all
// the waves.
//
// MFMA 16x16x4 computes D(16x16) += A(16x4) B(4x16); lane l holds A[l%16][l/16]
// and B[l/16][l%16]; the four output registers hold D[4(l/16)+i][l%16] (f32)
// or D[4i+l/16][l%16] (f64).  A rows are the tile's patterns, B is P, D rows
// are patterns: lane (g = l/16, n = l%16) holds state (column base + 16cb + n)
// of patterns opat(rb, g, 0..3) for every row block rb.
//
// Operand order (gl_col): a stored vector or matrix row holds state t at
// column (t mod 4) KBP + t / 4, so the states lane group g consumes on
// consecutive k-steps (4k + g) are adjacent: G = 2 or 4 k-steps of an operand
// arrive by one 8- or 16-byte load.  Partials are stored
// [slot][tile][r][TP patterns][row], TP = 16 RB; the forward matrices P, dP
// as [row s][column of t] and P a second time as [row t][column of s] for
// the backward product, all zero-padded, so no operand load is masked.
// Scaling: one power-of-two exponent e per (node, pattern), shared by all
// categories and states, as in the other kernels, but applied by the
// consumer: a kernel stores its outputs unscaled, category by category, and
// records e (eloc); whoever reads them scales its MFMA outputs (rows =
// patterns) by 2^-e.  Power-of-two scaling commutes exactly with the
// products, so this equals storing normalised partials, without a second
// pass over the outputs.
#include "phg_internal.h"
#include "phg_queue_device.h"

#include <math.h>

namespace phg {
namespace {

#define GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ GLOBAL T* g(T* p) {
    return (GLOBAL T*)p;
}

template <typename T>
struct V4T;
template <>
struct V4T<float> {
    typedef float type __attribute__((ext_vector_type(4)));
};
template <>
struct V4T<double> {
    typedef double type __attribute__((ext_vector_type(4)));
};
template <typename T>
using V4 = typename V4T<T>::type;
typedef int I4 __attribute__((ext_vector_type(4)));

// A tile is RB row blocks of 16 patterns (TP = 16 RB); a [state][pattern]
// vector in LDS has row stride TP + 1.

__device__ __forceinline__ V4<float> mma(float a, float b, V4<float> c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ V4<double> mma(double a, double b, V4<double> c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ float scale2(float x, int e) { return ldexpf(x, e); }
__device__ __forceinline__ double scale2(double x, int e) { return ldexp(x, e); }
__device__ __forceinline__ int exp_of(float x) {
    int e = 0;
    if (x > 0.0f) (void)frexpf(x, &e);
    return e;
}
__device__ __forceinline__ int exp_of(double x) {
    int e = 0;
    if (x > 0.0) (void)frexp(x, &e);
    return e;
}

// Pattern (within the tile) of output register i of row block rb for lane
// group gq.
template <typename T>
__device__ __forceinline__ int opat(int rb, int gq, int i) {
    return 16 * rb + (sizeof(T) == 4 ? 4 * gq + i : 4 * i + gq);
}

template <typename V>
__device__ __forceinline__ V sum16(V v) {
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) v += __shfl_xor(v, off, 64);
    return v;
}
template <typename V>
__device__ __forceinline__ V max16(V v) {
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Forward tables of P and dP and the backward table of P, in the path's type.
template <typename T>
__device__ __forceinline__ T* tabP(const ReqDesc& d);
template <>
__device__ __forceinline__ float* tabP<float>(const ReqDesc& d) { return d.P32; }
template <>
__device__ __forceinline__ double* tabP<double>(const ReqDesc& d) { return d.P64; }
template <typename T>
__device__ __forceinline__ T* tabdP(const ReqDesc& d);
template <>
__device__ __forceinline__ float* tabdP<float>(const ReqDesc& d) { return d.dP32; }
template <>
__device__ __forceinline__ double* tabdP<double>(const ReqDesc& d) { return d.dP64; }
template <typename T>
__device__ __forceinline__ T* tabPB(const ReqDesc& d);
template <>
__device__ __forceinline__ float* tabPB<float>(const ReqDesc& d) { return d.PB32; }
template <>
__device__ __forceinline__ double* tabPB<double>(const ReqDesc& d) { return d.PB64; }

template <typename T>
__device__ __forceinline__ T* tabdPB(const ReqDesc& d);
template <>
__device__ __forceinline__ float* tabdPB<float>(const ReqDesc& d) { return d.dPB32; }
template <>
__device__ __forceinline__ double* tabdPB<double>(const ReqDesc& d) { return d.dPB64; }

template <typename T, int G>
using VecG = T __attribute__((ext_vector_type(G)));

__device__ __forceinline__ int seg_of(const SegTable& t, int unit) {
    int s = 0;
    while (s + 1 < t.n && unit >= t.unit_begin[s + 1]) ++s;
    return s;
}

// This wave's columns of one vector: RB x NBW blocks of 16 patterns x 16
// states, 4 patterns per lane each.
template <typename T, int RB, int NBW>
struct Cols {
    V4<T> v[RB][NBW];
};

// Where a child's input vector comes from (a tip given by its codes does not
// go through the products: see tip_lookup).
template <typename T, int RB>
struct Input {
    const T* lds;           // staged [TP][la] vector of (child, tile, r) in LDS, or null
    const GLOBAL T* base;   // or the stored [TP][row] block in HBM
};

// k-steps whose operands are loaded together before their MFMAs run (one
// memory round trip per chunk instead of one per step): 8, or 4 for f64
// except with one row block of two column blocks per wave, and for four
// column blocks (registers).  With two f64 row blocks at eight waves the
// smaller chunk ends most of the pre-order spill (192 -> 48 bytes per
// lane) and fits two post-order workgroups per CU (160 -> 128 registers):
// 122 states 131 -> 148 evaluations/s.  With one f64 row block and column
// block it takes the pre-order kernel to 158 registers, 3 waves per SIMD
// without spilling (61 states 227 -> 238).  With two f64 column blocks
// (240 states) it measured slower (61 -> 51).
template <typename T, int RB, int NBW>
constexpr int chunk_of() {
    return ((sizeof(T) == 8 && (RB >= 2 || NBW != 2)) || NBW >= 4) ? 4 : 8;
}

// Operand geometry shared by the products of one kernel.
struct Geo {
    int S;      // states
    int kbp;    // k-steps per lane group in a row (gl_kbp)
    int row;    // row length in HBM (4 kbp)
    int la;     // row stride of a vector staged in LDS: row + 16 bytes (bank spread)
};

// G adjacent operand values (k-steps k .. k+G-1 of this lane) from a row in
// HBM, one 8-, 16- or 32-byte load.
template <typename T, int G>
__device__ __forceinline__ void load_run(const GLOBAL T* __restrict__ p, T (&out)[G]) {
    const VecG<T, G> v = *reinterpret_cast<const GLOBAL VecG<T, G>*>(p);
#pragma unroll
    for (int j = 0; j < G; ++j) out[j] = v[j];
}
// The same from a row staged in LDS, in pieces of at most 16 bytes.
template <typename T, int G>
__device__ __forceinline__ void lds_run(const T* p, T (&out)[G]) {
    constexpr int E = (G * static_cast<int>(sizeof(T)) > 16) ? 16 / static_cast<int>(sizeof(T)) : G;
#pragma unroll
    for (int q = 0; q < G / E; ++q) {
        const VecG<T, E> v = *reinterpret_cast<const VecG<T, E>*>(p + q * E);
#pragma unroll
        for (int j = 0; j < E; ++j) out[q * E + j] = v[j];
    }
}

// Copy a stored [TP][row] block (contiguous in HBM) into an LDS [TP][la]
// buffer in 16-byte pieces.  All threads take part; each issues all of its
// (at most KIT) loads before its first LDS write.  The caller synchronises.
template <typename T, int TP, int KIT, bool kCoh = false>
__device__ __forceinline__ void stage_vec(T* buf, const GLOBAL T* __restrict__ src, const Geo& ge) {
    constexpr int E = 16 / static_cast<int>(sizeof(T));
    const int per_row = ge.row / E;
    const int n = TP * per_row;
    VecG<T, E> v[KIT];
#pragma unroll
    for (int it = 0; it < KIT; ++it) {
        const int t = static_cast<int>(threadIdx.x) + it * static_cast<int>(blockDim.x);
        if (t < n) {
            const int p = t / per_row, c = (t - p * per_row) * E;
            if constexpr (kCoh)   // device-coherent (work-queue launches): piece t of the [TP][row] block
                v[it] = queue::ld(reinterpret_cast<const GLOBAL VecG<T, E>*>(src), static_cast<uint32_t>(t),
                                  static_cast<uint32_t>(n));
            else
                v[it] = *reinterpret_cast<const GLOBAL VecG<T, E>*>(src + p * ge.row + c);
        }
    }
#pragma unroll
    for (int it = 0; it < KIT; ++it) {
        const int t = static_cast<int>(threadIdx.x) + it * static_cast<int>(blockDim.x);
        if (t < n) {
            const int p = t / per_row, c = (t - p * per_row) * E;
            *reinterpret_cast<VecG<T, E>*>(buf + p * ge.la + c) = v[it];
        }
    }
}

// A folded child x's partial -- (P_a e_ya) o (P_b e_yb) for its tip children
// a < b, the product of two rows of the backward P tables (which hold each
// tip's P e_y in the stored operand order; the row-sum row for the
// ambiguous code) -- into an LDS [TP][la] buffer, as stage_vec would copy
// the stored block.  Folding needs tables for every branch.  The caller
// synchronises.
template <typename T, int TP, int KIT>
__device__ __forceinline__ void stage_folded(T* buf, const ReqDesc& d, int x, int r, int tile, size_t bstride,
                                             const Geo& ge) {
    constexpr int E = 16 / static_cast<int>(sizeof(T));
    const int per_row = ge.row / E;
    const int n = TP * per_row;
    const GLOBAL int32_t* kk = g(d.kids) + 2 * static_cast<size_t>(x - d.N);
    const int a = kk[0], b = kk[1];
    const GLOBAL T* PB = g(tabPB<T>(d));
    const GLOBAL T* Ba = PB + (static_cast<size_t>(a) * d.R + r) * bstride;
    const GLOBAL T* Bb = PB + (static_cast<size_t>(b) * d.R + r) * bstride;
    const size_t ca = static_cast<size_t>(a) * d.Cpad + static_cast<size_t>(tile) * TP;
    const size_t cb = static_cast<size_t>(b) * d.Cpad + static_cast<size_t>(tile) * TP;
    const int sum_row = gl_mat_rows(ge.S);
    const bool wide = code_bytes(ge.S) == 2;
    const GLOBAL uint8_t* codes = g(d.codes);
    VecG<T, E> va[KIT], vb[KIT];
#pragma unroll
    for (int it = 0; it < KIT; ++it) {
        const int t = static_cast<int>(threadIdx.x) + it * static_cast<int>(blockDim.x);
        if (t < n) {
            const int p = t / per_row, c = (t - p * per_row) * E;
            const int ya = wide ? reinterpret_cast<const GLOBAL uint16_t*>(codes)[ca + p] : codes[ca + p];
            const int yb = wide ? reinterpret_cast<const GLOBAL uint16_t*>(codes)[cb + p] : codes[cb + p];
            va[it] = *reinterpret_cast<const GLOBAL VecG<T, E>*>(Ba + (ya < ge.S ? ya : sum_row) * ge.row + c);
            vb[it] = *reinterpret_cast<const GLOBAL VecG<T, E>*>(Bb + (yb < ge.S ? yb : sum_row) * ge.row + c);
        }
    }
#pragma unroll
    for (int it = 0; it < KIT; ++it) {
        const int t = static_cast<int>(threadIdx.x) + it * static_cast<int>(blockDim.x);
        if (t < n) {
            const int p = t / per_row, c = (t - p * per_row) * E;
            *reinterpret_cast<VecG<T, E>*>(buf + p * ge.la + c) = va[it] * vb[it];
        }
    }
}

// out1 = M1 v (and, with M2, out2 = M2 v) on this wave's columns:
// out[c][s] = sum_t M[s][t] in[c][t], s = cb0 + 16 cb + n, from forward
// tables; v from LDS (kLds) or HBM.  One operand stream of v feeds both
// products (P p and dP p of one child).
template <typename T, int RB, int NBW, int G, bool kTwo, bool kLds = true>
__device__ __forceinline__ void fwd(const GLOBAL T* __restrict__ M1, const GLOBAL T* __restrict__ M2,
                                    const Input<T, RB>& in, const Geo& ge, int cb0, int lane,
                                    Cols<T, RB, NBW>& out1, Cols<T, RB, NBW>& out2) {
    constexpr int kChunk = chunk_of<T, RB, NBW>();
    const int gq = lane >> 4, n = lane & 15;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < NBW; ++cb) out1.v[rb][cb] = out2.v[rb][cb] = V4<T>{0, 0, 0, 0};
    const int off = gq * ge.kbp;
    const T* ar[RB];
    const GLOBAL T* ag[RB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
        ar[rb] = kLds ? in.lds + (16 * rb + n) * ge.la + off : nullptr;
        ag[rb] = !kLds ? in.base + (16 * rb + n) * ge.row + off : nullptr;
    }
    const GLOBAL T* br1[NBW];
    const GLOBAL T* br2[NBW];
#pragma unroll
    for (int cb = 0; cb < NBW; ++cb) {
        const size_t o = static_cast<size_t>(cb0 + 16 * cb + n) * ge.row + off;
        br1[cb] = M1 + o;
        br2[cb] = kTwo ? M2 + o : M1;
    }
    for (int k0 = 0; k0 < ge.kbp; k0 += kChunk) {
        T a[kChunk][RB], b1[kChunk][NBW], b2[kChunk][NBW];
#pragma unroll
        for (int v = 0; v < kChunk / G; ++v) {
            const int k = k0 + v * G;
            if (k < ge.kbp) {             // uniform; rows are padded to whole runs
#pragma unroll
                for (int cb = 0; cb < NBW; ++cb) {
                    T x[G];
                    load_run<T, G>(br1[cb] + k, x);
#pragma unroll
                    for (int j = 0; j < G; ++j) b1[v * G + j][cb] = x[j];
                    if (kTwo) {
                        load_run<T, G>(br2[cb] + k, x);
#pragma unroll
                        for (int j = 0; j < G; ++j) b2[v * G + j][cb] = x[j];
                    }
                }
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) {
                    T x[G];
                    if (kLds)
                        lds_run<T, G>(ar[rb] + k, x);
                    else
                        load_run<T, G>(ag[rb] + k, x);
#pragma unroll
                    for (int j = 0; j < G; ++j) a[v * G + j][rb] = x[j];
                }
            }
        }
#pragma unroll
        for (int c = 0; c < kChunk; ++c) {
            if (k0 + c >= ge.kbp) break;
#pragma unroll
            for (int cb = 0; cb < NBW; ++cb)
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) {
                    out1.v[rb][cb] = mma(a[c][rb], b1[c][cb], out1.v[rb][cb]);
                    if (kTwo) out2.v[rb][cb] = mma(a[c][rb], b2[c][cb], out2.v[rb][cb]);
                }
        }
    }
}

// out = M^T u on this wave's columns: out[c][t] = sum_s u[c][s] M[s][t], from
// the backward table (row t), u staged in LDS like an input vector.
template <typename T, int RB, int NBW, int G>
__device__ __forceinline__ void bwd(const GLOBAL T* __restrict__ MB, const T* U, const Geo& ge, int cb0,
                                    int lane, Cols<T, RB, NBW>& out) {
    constexpr int kChunk = chunk_of<T, RB, NBW>();
    const int gq = lane >> 4, n = lane & 15;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < NBW; ++cb) out.v[rb][cb] = V4<T>{0, 0, 0, 0};
    const int off = gq * ge.kbp;
    const T* ur[RB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) ur[rb] = U + (16 * rb + n) * ge.la + off;
    const GLOBAL T* br[NBW];
#pragma unroll
    for (int cb = 0; cb < NBW; ++cb) br[cb] = MB + static_cast<size_t>(cb0 + 16 * cb + n) * ge.row + off;
    for (int k0 = 0; k0 < ge.kbp; k0 += kChunk) {
        T a[kChunk][RB], b[kChunk][NBW];
#pragma unroll
        for (int v = 0; v < kChunk / G; ++v) {
            const int k = k0 + v * G;
            if (k < ge.kbp) {
#pragma unroll
                for (int cb = 0; cb < NBW; ++cb) {
                    T x[G];
                    load_run<T, G>(br[cb] + k, x);
#pragma unroll
                    for (int j = 0; j < G; ++j) b[v * G + j][cb] = x[j];
                }
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) {
                    T x[G];
                    lds_run<T, G>(ur[rb] + k, x);
#pragma unroll
                    for (int j = 0; j < G; ++j) a[v * G + j][rb] = x[j];
                }
            }
        }
#pragma unroll
        for (int c = 0; c < kChunk; ++c) {
            if (k0 + c >= ge.kbp) break;
#pragma unroll
            for (int cb = 0; cb < NBW; ++cb)
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) out.v[rb][cb] = mma(a[c][rb], b[c][cb], out.v[rb][cb]);
        }
    }
}

// A stored [TP][row] block in HBM -> this wave's columns, and back (states
// past S are zeros; states past the row do not exist).
template <typename T, int RB, int NBW, bool kCoh = false>
__device__ __forceinline__ void load_cols(const GLOBAL T* __restrict__ base, const Geo& ge, int cb0, int lane,
                                          Cols<T, RB, NBW>& x) {
    const int gq = lane >> 4, n = lane & 15;
#pragma unroll
    for (int cb = 0; cb < NBW; ++cb) {
        const int s = cb0 + 16 * cb + n;
        const int col = gl_col(s, ge.kbp);
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int ix = opat<T>(rb, gq, i) * ge.row + col;
                if constexpr (kCoh)   // device-coherent (work-queue launches)
                    x.v[rb][cb][i] = s < ge.row ? queue::ld(base, ix, 16 * RB * ge.row) : T(0);
                else
                    x.v[rb][cb][i] = s < ge.row ? base[ix] : T(0);
            }
    }
}
template <typename T, int RB, int NBW, bool kCoh = false>
__device__ __forceinline__ void store_cols(GLOBAL T* __restrict__ base, const Geo& ge, int cb0, int lane,
                                           const Cols<T, RB, NBW>& x) {
    const int gq = lane >> 4, n = lane & 15;
#pragma unroll
    for (int cb = 0; cb < NBW; ++cb) {
        const int s = cb0 + 16 * cb + n;
        const int col = gl_col(s, ge.kbp);
        if (s < ge.row) {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int ix = opat<T>(rb, gq, i) * ge.row + col;
                    if constexpr (kCoh)   // device-coherent (work-queue launches)
                        queue::st(base, ix, 16 * RB * ge.row, x.v[rb][cb][i]);
                    else
                        base[ix] = x.v[rb][cb][i];
                }
        }
    }
}
// A tip given by its codes: its vector is e_y (or all ones for code S), so
// M e_y is column y of M, i.e. row y of M's backward table (row y holds
// M[s][y] at column gl_col(s)), and M 1 is the row-sum row that follows the
// table's gl_mat_rows(S) rows.  out1[c][s] = MB1[y_c][s] (and out2 from MB2)
// on this wave's columns: a gather from the L2-resident table instead of
// products on one-hot operands.  Code c0 + p is pattern p of the tile (bytes,
// or 16-bit codes above 255 states).
template <typename T, int RB, int NBW, bool kTwo>
__device__ __forceinline__ void tip_lookup(const GLOBAL T* __restrict__ MB1, const GLOBAL T* __restrict__ MB2,
                                           const GLOBAL uint8_t* __restrict__ codes, size_t c0, const Geo& ge,
                                           int cb0, int lane, Cols<T, RB, NBW>& out1, Cols<T, RB, NBW>& out2) {
    const int gq = lane >> 4, n = lane & 15;
    const int sum_row = gl_mat_rows(ge.S);
    const bool wide = code_bytes(ge.S) == 2;
    int yo[RB][4];      // row offset of each of this lane's patterns
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const size_t c = c0 + opat<T>(rb, gq, i);
            const int y = wide ? reinterpret_cast<const GLOBAL uint16_t*>(codes)[c] : codes[c];
            yo[rb][i] = (y < ge.S ? y : sum_row) * ge.row;
        }
#pragma unroll
    for (int cb = 0; cb < NBW; ++cb) {
        const int s = cb0 + 16 * cb + n;
        const bool in_row = s < ge.row;
        const int col = in_row ? gl_col(s, ge.kbp) : 0;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                out1.v[rb][cb][i] = in_row ? MB1[yo[rb][i] + col] : T(0);
                if (kTwo) out2.v[rb][cb][i] = in_row ? MB2[yo[rb][i] + col] : T(0);
            }
    }
}

// An LDS [TP][la] vector <-> this wave's columns.
template <typename T, int RB, int NBW>
__device__ __forceinline__ void vbuf_to_cols(const T* buf, const Geo& ge, int cb0, int lane, Cols<T, RB, NBW>& x) {
    const int gq = lane >> 4, n = lane & 15;
#pragma unroll
    for (int cb = 0; cb < NBW; ++cb) {
        const int s = cb0 + 16 * cb + n;
        const int col = gl_col(s, ge.kbp);
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int i = 0; i < 4; ++i) x.v[rb][cb][i] = s < ge.row ? buf[opat<T>(rb, gq, i) * ge.la + col] : T(0);
    }
}
template <typename T, int RB, int NBW>
__device__ __forceinline__ void cols_to_vbuf(T* buf, const Geo& ge, int cb0, int lane, const Cols<T, RB, NBW>& x) {
    const int gq = lane >> 4, n = lane & 15;
#pragma unroll
    for (int cb = 0; cb < NBW; ++cb) {
        const int s = cb0 + 16 * cb + n;
        const int col = gl_col(s, ge.kbp);
        if (s < ge.row) {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int i = 0; i < 4; ++i) buf[opat<T>(rb, gq, i) * ge.la + col] = x.v[rb][cb][i];
        }
    }
}

template <typename T, int RB, int NBW>
__device__ __forceinline__ void mul_cols(Cols<T, RB, NBW>& x, const Cols<T, RB, NBW>& y) {
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < NBW; ++cb) x.v[rb][cb] *= y.v[rb][cb];
}

// Per-pattern partial sum over this wave's columns of x * y.
template <typename T, int RB, int NBW>
__device__ __forceinline__ void dot_cols(const Cols<T, RB, NBW>& x, const Cols<T, RB, NBW>& y, T acc[RB][4]) {
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < NBW; ++cb)
#pragma unroll
            for (int i = 0; i < 4; ++i) acc[rb][i] += x.v[rb][cb][i] * y.v[rb][cb][i];
}
template <typename T, int RB, int NBW>
__device__ __forceinline__ void max_cols(const Cols<T, RB, NBW>& x, T mx[RB][4]) {
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < NBW; ++cb)
#pragma unroll
            for (int i = 0; i < 4; ++i) mx[rb][i] = fmax(mx[rb][i], x.v[rb][cb][i]);
}

// Maximum over the workgroup of per-pattern values (each lane's after max16):
// via LDS, fixed order.  red has W * TP slots.
template <typename T, int RB, int W>
__device__ __forceinline__ void wg_max(T mx[RB][4], T* red, int w, int lane) {
    constexpr int TP = 16 * RB;
    const int gq = lane >> 4, n = lane & 15;
    if (n == 0) {
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int i = 0; i < 4; ++i) red[w * TP + opat<T>(rb, gq, i)] = mx[rb][i];
    }
    __syncthreads();
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            T m = red[opat<T>(rb, gq, i)];
#pragma unroll
            for (int ww = 1; ww < W; ++ww) m = fmax(m, red[ww * TP + opat<T>(rb, gq, i)]);
            mx[rb][i] = m;
        }
    __syncthreads();
}

// x *= 2^-e per pattern row, e from LDS (TP exponents of one node).
template <typename T, int RB, int NBW>
__device__ __forceinline__ void scale_rows(Cols<T, RB, NBW>& x, const int* e, int lane) {
    const int gq = lane >> 4;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int ei = e[opat<T>(rb, gq, i)];
#pragma unroll
            for (int cb = 0; cb < NBW; ++cb) x.v[rb][cb][i] = scale2(x.v[rb][cb][i], -ei);
        }
}

// An exponent word another item of a work-queue launch writes or reads
// (kCoh: device-coherent), at a per-lane address.
template <bool kCoh>
__device__ __forceinline__ int ld_int(const GLOBAL int32_t* p) {
    if constexpr (kCoh) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return *p;
}
template <bool kCoh>
__device__ __forceinline__ void st_int(GLOBAL int32_t* p, int v) {
    if constexpr (kCoh)
        __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
        *p = v;
}

// Stage the own exponents (eloc) of up to three nodes for the tile's
// patterns in LDS: row c holds node[c]'s, zeros for a tip or a negative id.
// The caller synchronises.
template <int TP, int NC, bool kCoh = false>
__device__ __forceinline__ void stage_exps(int (&esh)[NC][TP], const int (&node)[NC], const ReqDesc& d, int tile) {
    const int N = d.N;
    for (int t = threadIdx.x; t < NC * TP; t += blockDim.x) {
        const int c = t / TP, p = t - c * TP;
        const int x = node[c];
        esh[c][p] = x >= N ? ld_int<kCoh>(g(d.eloc) + static_cast<size_t>(x - N) * d.Cpad + tile * TP + p) : 0;
    }
}

// Where child x's input vector lives for (tile): an internal child's stored
// partial, a tip's general partial vector (tslot >= 0), or null for a tip
// given by its code.
template <typename T>
__device__ __forceinline__ const GLOBAL T* tip_src(const ReqDesc& d, int x, int tile, int tiles, size_t tstride,
                                                   const GLOBAL T* part) {
    const int N = d.N;
    if (x >= N) return part + (static_cast<size_t>(x - N) * tiles + tile) * tstride;
    const int gx = d.tslot ? g(d.tslot)[x] : -1;
    return gx >= 0 ? g(static_cast<const T*>(d.tipvec)) + (static_cast<size_t>(gx) * tiles + tile) * tstride
                   : nullptr;
}

struct GlUnit {
    const ReqDesc* d;
    Segment sg;
    NodeTriple nt;
    int tile, tiles;
    int node_ix;    // the node's place in its segment
    bool fi, fj;    // child i / j is a folded node (NodeTriple::fold)
    bool root;      // post-order: the record of the tree root
    int rec;        // work-queue launches: the record's index in the schedule
};
__device__ __forceinline__ bool gl_unit(const ReqDesc* __restrict__ descs, const SegTable& segs, GlUnit& U) {
    const int unit = blockIdx.x;
    if (unit >= segs.unit_begin[segs.n]) return false;
    const int sidx = seg_of(segs, unit);
    U.sg = segs.seg[sidx];
    U.d = &descs[U.sg.desc];
    U.tiles = U.d->tiles;
    const int local = unit - segs.unit_begin[sidx];
    const int node_ix = local / U.tiles;
    U.tile = local - node_ix * U.tiles;
    U.node_ix = node_ix;
    const I4 t4 = reinterpret_cast<const GLOBAL I4*>(g(U.sg.sched))[U.sg.sched_off + node_ix];
    U.nt = NodeTriple{t4.x, t4.y, t4.z, 0};
    U.fi = (t4.w & 1) != 0;
    U.fj = (t4.w & 2) != 0;
    U.root = (U.sg.flags & 1) != 0;
    return true;
}
// Work-queue launches (the context's descriptor is descs[0]; tables for
// every branch): workgroup i takes item t0 + i, a (record, tile) pair.
__device__ __forceinline__ bool gl_unit(const ReqDesc* __restrict__ descs, const QueueArgs& q, GlUnit& U) {
    const int t = q.t0 + static_cast<int>(blockIdx.x);
    if (t >= q.t1) return false;
    U.d = &descs[0];
    U.sg = Segment{};
    U.tiles = U.d->tiles;
    U.rec = g(q.items)[2 * static_cast<size_t>(t)];
    U.tile = g(q.items)[2 * static_cast<size_t>(t) + 1];
    U.node_ix = 0;
    const I4 t4 = reinterpret_cast<const GLOBAL I4*>(g(U.d->sched))[U.rec];
    U.nt = NodeTriple{t4.x, t4.y, t4.z, 0};
    U.fi = (t4.w & 1) != 0;
    U.fj = (t4.w & 2) != 0;
    U.root = t4.x == 2 * U.d->N - 2;
    return true;
}
// Marks per (pass, node slot, tile), I = q.n_blocks node slots: a post-order
// item waits on its stored children, a pre-order item on its parent (which
// wrote its pre-order vector and exponent); wave 0 polls, then the workgroup
// synchronises.  At the end every wave's stores complete, then the mark.
__device__ __forceinline__ void gl_wait(const QueueArgs& q, const GlUnit& U, bool pre, int w, int lane,
                                        uint32_t target) {
    if (w == 0) {
        const ReqDesc& d = *U.d;
        const int N = d.N;
        int m = -1;
        if (!pre) {
            if (lane == 0 && U.nt.i >= N && !U.fi) m = (U.nt.i - N) * U.tiles + U.tile;
            if (lane == 1 && U.nt.j >= N && !U.fj) m = (U.nt.j - N) * U.tiles + U.tile;
        } else if (lane == 0) {
            const int par = g(q.dep)[2 * static_cast<size_t>(U.rec)];   // the parent's slot, -1 at the root
            if (par >= 0) m = (q.n_blocks + par) * U.tiles + U.tile;
        }
        queue::wait_marks(q, m, target, 2u * q.n_blocks * U.tiles, lane);
    }
    __syncthreads();
}
__device__ __forceinline__ void gl_done(const QueueArgs& q, const GlUnit& U, bool pre, uint32_t target) {
    queue::stores_complete();
    __syncthreads();
    if (threadIdx.x == 0)
        queue::set_mark(q, ((pre ? q.n_blocks : 0) + U.nt.k - U.d->N) * U.tiles + U.tile, target,
                        2u * q.n_blocks * U.tiles);
}

// ---------------------------------------------------------------- post-order

template <typename T, int RB, int NBW, int W, bool kQ, typename Arg>
__device__ __forceinline__ void post_gl_body(const ReqDesc* __restrict__ descs, const Arg& arg) {
    constexpr int TP = 16 * RB;
    constexpr int G = (NBW == 1 && W <= 2) ? 2 : 4;   // gl_vec: 2 up to 32 states
    constexpr int SP = 16 * NBW * W;                // padded states (>= the row length)
    constexpr int E = 16 / static_cast<int>(sizeof(T));
    constexpr int LA = SP + E;                      // LDS row stride bound
    constexpr int KIT = (TP * NBW + 4 * E - 1) / (4 * E);   // staging pieces per thread
    __shared__ __align__(16) T vb[2][TP * LA];      // staged p_i, p_j of one category
    __shared__ T red[W * TP];
    __shared__ double dred[W * TP];
    __shared__ int esh[2][TP];                      // own exponents of the children
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int gq = lane >> 4, n = lane & 15;
    GlUnit U;
    if (!gl_unit(descs, arg, U)) return;
    const ReqDesc& d = *U.d;
    const int N = d.N, S = d.S, R = d.R, Cpad = d.Cpad, tile = U.tile, tiles = U.tiles;
    const NodeTriple nt = U.nt;
    const int cb0 = w * 16 * NBW;
    const Geo ge{S, gl_kbp(S), gl_row(S), gl_row(S) + E};
    const size_t rstride = static_cast<size_t>(TP) * ge.row;
    const size_t tstride = rstride * R;
    const size_t mstride = static_cast<size_t>(gl_mat_rows(S)) * ge.row;   // one (branch, category) table
    const size_t bstride = static_cast<size_t>(gl_back_rows(S)) * ge.row;   // one backward table
    GLOBAL T* part = g(static_cast<T*>(d.part));
    const GLOBAL T* P = g(tabP<T>(d));
    const GLOBAL T* PB = g(tabPB<T>(d));
    const bool tip_i = nt.i < N, tip_j = nt.j < N;
    // inputs: stored partials, or a tip's general partial vector, or (null) its codes
    const GLOBAL T* pi_base = tip_src<T>(d, nt.i, tile, tiles, tstride, part);
    const GLOBAL T* pj_base = tip_src<T>(d, nt.j, tile, tiles, tstride, part);
    const size_t ci = static_cast<size_t>(nt.i) * Cpad + tile * TP;
    const size_t cj = static_cast<size_t>(nt.j) * Cpad + tile * TP;
    // P(t) tables of the children: by branch, or by slot in per-chunk tables
    const int ti = d.level_tables ? 2 * U.node_ix : nt.i, tj = d.level_tables ? 2 * U.node_ix + 1 : nt.j;
    GLOBAL T* out_base = part + (static_cast<size_t>(nt.k - N) * tiles + tile) * tstride;
    const bool root = U.root;
    uint32_t target = 0;
    if constexpr (kQ) {
        target = queue::epoch(arg);
        gl_wait(arg, U, false, w, lane, target);
    }
    {
        const int kids[2] = {U.fi ? -1 : nt.i, U.fj ? -1 : nt.j};   // a folded child's exponent is 0
        stage_exps<TP, 2, kQ>(esh, kids, d, tile);      // read after the first barrier below
    }
    const Input<T, RB> si{vb[0], nullptr}, sj{vb[1], nullptr};
    T mx[RB][4] = {};
    double site[RB][4] = {};
    for (int r = 0; r < R; ++r) {
        if (U.fi)
            stage_folded<T, TP, KIT>(vb[0], d, nt.i, r, tile, bstride, ge);
        else if (pi_base)
            stage_vec<T, TP, KIT, kQ>(vb[0], pi_base + r * rstride, ge);
        if (U.fj)
            stage_folded<T, TP, KIT>(vb[1], d, nt.j, r, tile, bstride, ge);
        else if (pj_base)
            stage_vec<T, TP, KIT, kQ>(vb[1], pj_base + r * rstride, ge);
        __syncthreads();
        Cols<T, RB, NBW> mi, mj, unused;
        if (pi_base) {
            fwd<T, RB, NBW, G, false>(P + (static_cast<size_t>(ti) * R + r) * mstride, nullptr, si, ge, cb0,
                                      lane, mi, unused);
            if (!tip_i) scale_rows<T, RB, NBW>(mi, esh[0], lane);
        } else {
            tip_lookup<T, RB, NBW, false>(PB + (static_cast<size_t>(ti) * R + r) * bstride, nullptr, g(d.codes), ci,
                                          ge, cb0, lane, mi, unused);
        }
        if (pj_base) {
            fwd<T, RB, NBW, G, false>(P + (static_cast<size_t>(tj) * R + r) * mstride, nullptr, sj, ge, cb0,
                                      lane, mj, unused);
            if (!tip_j) scale_rows<T, RB, NBW>(mj, esh[1], lane);
        } else {
            tip_lookup<T, RB, NBW, false>(PB + (static_cast<size_t>(tj) * R + r) * bstride, nullptr, g(d.codes), cj,
                                          ge, cb0, lane, mj, unused);
        }
        mul_cols<T, RB, NBW>(mi, mj);
        if (!root) {
            max_cols<T, RB, NBW>(mi, mx);
            store_cols<T, RB, NBW, kQ>(out_base + r * rstride, ge, cb0, lane, mi);
        } else {
            const double wr = g(d.cweights)[r];
#pragma unroll
            for (int cb = 0; cb < NBW; ++cb) {
                const int s = cb0 + 16 * cb + n;
                const double ps = s < S ? g(d.pi)[s] : 0.0;
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                    for (int i = 0; i < 4; ++i) site[rb][i] += wr * ps * static_cast<double>(mi.v[rb][cb][i]);
            }
        }
        __syncthreads();      // every wave done with the staged inputs of category r
    }
    int ec[RB][4];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int c = tile * TP + opat<T>(rb, gq, i);
            ec[rb][i] = (tip_i || U.fi ? 0 : ld_int<kQ>(g(d.expo) + static_cast<size_t>(nt.i - N) * Cpad + c)) +
                        (tip_j || U.fj ? 0 : ld_int<kQ>(g(d.expo) + static_cast<size_t>(nt.j - N) * Cpad + c));
        }
    if (!root) {
        // a node whose children are both tips given by codes is never
        // rescaled (folded nodes rely on exponent 0; its entries are products
        // of two table entries)
        const bool tiptip = !pi_base && !pj_base;
        int e[RB][4] = {};
        if (!tiptip) {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int i = 0; i < 4; ++i) mx[rb][i] = max16(mx[rb][i]);
            wg_max<T, RB, W>(mx, red, w, lane);
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int i = 0; i < 4; ++i) e[rb][i] = exp_of(mx[rb][i]);
        }
        if (w == 0 && n == 0) {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const size_t c = static_cast<size_t>(nt.k - N) * Cpad + tile * TP + opat<T>(rb, gq, i);
                    st_int<kQ>(g(d.eloc) + c, e[rb][i]);
                    st_int<kQ>(g(d.expo) + c, e[rb][i] + ec[rb][i]);
                }
        }
    } else {
        // site likelihood: sum over this wave's states, then over waves (fixed order)
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int i = 0; i < 4; ++i) site[rb][i] = sum16(site[rb][i]);
        if (n == 0) {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int i = 0; i < 4; ++i) dred[w * TP + opat<T>(rb, gq, i)] = site[rb][i];
        }
        __syncthreads();
        if (w == 0) {
            double tsum = 0.0;
            if (n == 0) {
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int p = opat<T>(rb, gq, i);
                        double sv = dred[p];
#pragma unroll
                        for (int ww = 1; ww < W; ++ww) sv += dred[ww * TP + p];
                        const int c = tile * TP + p;
                        const double ll = (sv > 0.0 ? log(sv) : -INFINITY) +
                                          static_cast<double>(ec[rb][i]) * 0.69314718055994530942;
                        g(d.sll)[c] = ll;
                        const double Wc = g(d.pw)[c];
                        tsum += (Wc != 0.0) ? Wc * ll : 0.0;
                    }
            }
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) tsum += __shfl_xor(tsum, off, 64);
            if (lane == 0) g(d.lpart)[tile] = tsum;
        }
    }
    if constexpr (kQ) gl_done(arg, U, false, target);
}

// FP32, one row block, four waves: 78 registers, so 6 waves per SIMD fit
// without spilling (1% on the 61-state level launches).
template <typename T, int RB, int NBW, int W>
__global__ __launch_bounds__(64 * W, (RB == 1 && W == 4 && sizeof(T) == 4) ? 6 : 1)
void post_gl_kernel(const ReqDesc* __restrict__ descs, const SegTable segs) {
    post_gl_body<T, RB, NBW, W, false>(descs, segs);
}
// The same over a work-queue launch's items.
template <typename T, int RB, int NBW, int W>
__global__ __launch_bounds__(64 * W, (RB == 1 && W == 4 && sizeof(T) == 4) ? 6 : 1)
void post_gl_queue_kernel(const ReqDesc* __restrict__ descs, const QueueArgs q) {
    post_gl_body<T, RB, NBW, W, true>(descs, q);
}

// ---------------------------------------------------------------- pre-order + gradient

// FP32 with one row block and two or four waves (up to 32 states, and 49..64
// states where one row block is chosen) the kernel fits in 128 registers:
// ask for 4 waves per SIMD (61 states: 3 waves at 136 registers before,
// 2.29 -> 2.17 ms per 128-taxon evaluation).  FP64 with one row block and
// four waves asks for 3 (158 registers with operand chunks of 4).
template <typename T, int RB, int NBW, int W, bool kQ, typename Arg>
__device__ __forceinline__ void pre_gl_body(const ReqDesc* __restrict__ descs, const Arg& arg) {
    constexpr int TP = 16 * RB;
    constexpr int G = (NBW == 1 && W <= 2) ? 2 : 4;   // gl_vec: 2 up to 32 states
    constexpr int SP = 16 * NBW * W;                // padded states (>= the row length)
    constexpr int E = 16 / static_cast<int>(sizeof(T));
    constexpr int LA = SP + E;                      // LDS row stride bound
    constexpr int KIT = (TP * NBW + 4 * E - 1) / (4 * E);   // staging pieces per thread
    // With three or more waves the inputs of a category (p_i, p_j, q_k) are
    // staged in LDS once instead of read by every wave; with two the extra
    // barriers cost more than they save.  u_i, u_j go to vb[0], vb[1].
    constexpr bool kStage = W >= 3;
    __shared__ __align__(16) T vb[kStage ? 3 : 2][TP * LA];
    __shared__ T red[3 * W * TP];
    __shared__ int esh[3][TP];                      // own exponents: p_i, p_j (post-order), q_k
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int gq = lane >> 4, n = lane & 15;
    GlUnit U;
    if (!gl_unit(descs, arg, U)) return;
    const ReqDesc& d = *U.d;
    const int N = d.N, S = d.S, R = d.R, Cpad = d.Cpad, tile = U.tile, tiles = U.tiles;
    const NodeTriple nt = U.nt;
    const int cb0 = w * 16 * NBW;
    const Geo ge{S, gl_kbp(S), gl_row(S), gl_row(S) + E};
    const size_t rstride = static_cast<size_t>(TP) * ge.row;
    const size_t tstride = rstride * R;
    const size_t mstride = static_cast<size_t>(gl_mat_rows(S)) * ge.row;   // one (branch, category) table
    GLOBAL T* part = g(static_cast<T*>(d.part));
    const GLOBAL T* P = g(tabP<T>(d));
    const GLOBAL T* dP = g(tabdP<T>(d));
    const GLOBAL T* PB = g(tabPB<T>(d));
    const GLOBAL T* dPB = g(tabdPB<T>(d));
    const size_t bstride = static_cast<size_t>(gl_back_rows(S)) * ge.row;   // one backward table
    const bool is_root = nt.k == 2 * N - 2;
    const bool tip_i = nt.i < N, tip_j = nt.j < N;
    const size_t ci = static_cast<size_t>(nt.i) * Cpad + tile * TP;
    const size_t cj = static_cast<size_t>(nt.j) * Cpad + tile * TP;
    // P(t) tables of the children: by branch, or by slot in per-chunk tables
    const int ti = d.level_tables ? 2 * U.node_ix : nt.i, tj = d.level_tables ? 2 * U.node_ix + 1 : nt.j;
    Input<T, RB> si{nullptr, nullptr}, sj{nullptr, nullptr};
    GLOBAL T* pi_base = tip_i ? nullptr : part + (static_cast<size_t>(nt.i - N) * tiles + tile) * tstride;
    GLOBAL T* pj_base = tip_j ? nullptr : part + (static_cast<size_t>(nt.j - N) * tiles + tile) * tstride;
    const GLOBAL T* qk_base = is_root ? nullptr : part + (static_cast<size_t>(nt.k - N) * tiles + tile) * tstride;
    // inputs (q is written over p for internal children only)
    const GLOBAL T* pi_src = tip_src<T>(d, nt.i, tile, tiles, tstride, part);
    const GLOBAL T* pj_src = tip_src<T>(d, nt.j, tile, tiles, tstride, part);
    uint32_t target = 0;
    if constexpr (kQ) {
        target = queue::epoch(arg);
        gl_wait(arg, U, true, w, lane, target);
    }
    {
        // a folded child's exponent is 0 (folding happens only where kStage)
        const int nodes[3] = {U.fi ? -1 : nt.i, U.fj ? -1 : nt.j, is_root ? -1 : nt.k};
        stage_exps<TP, 3, kQ>(esh, nodes, d, tile);
    }
    if constexpr (!kStage) __syncthreads();    // exponents in LDS (staging has its own barrier)
    si.lds = kStage && pi_src ? vb[0] : nullptr;
    sj.lds = kStage && pj_src ? vb[1] : nullptr;
    T num_i[RB][4] = {}, num_j[RB][4] = {}, den[RB][4] = {}, mxi[RB][4] = {}, mxj[RB][4] = {};
    for (int r = 0; r < R; ++r) {
        si.base = !kStage && pi_src ? pi_src + r * rstride : nullptr;
        sj.base = !kStage && pj_src ? pj_src + r * rstride : nullptr;
        if constexpr (kStage) {
            if (U.fi)
                stage_folded<T, TP, KIT>(vb[0], d, nt.i, r, tile, bstride, ge);
            else if (pi_src)
                stage_vec<T, TP, KIT>(vb[0], pi_src + r * rstride, ge);
            if (U.fj)
                stage_folded<T, TP, KIT>(vb[1], d, nt.j, r, tile, bstride, ge);
            else if (pj_src)
                stage_vec<T, TP, KIT>(vb[1], pj_src + r * rstride, ge);
            if (!is_root) stage_vec<T, TP, KIT, kQ>(vb[kStage ? 2 : 0], qk_base + r * rstride, ge);
            __syncthreads();  // inputs of category r staged
        }
        const size_t mo_i = (static_cast<size_t>(ti) * R + r) * mstride;
        const size_t mo_j = (static_cast<size_t>(tj) * R + r) * mstride;
        const size_t bo_i = (static_cast<size_t>(ti) * R + r) * bstride;
        const size_t bo_j = (static_cast<size_t>(tj) * R + r) * bstride;
        const T wr = static_cast<T>(g(d.cweights)[r]);
        Cols<T, RB, NBW> qk, a, b, acc, dmj;
        if (is_root) {
#pragma unroll
            for (int cb = 0; cb < NBW; ++cb) {
                const int s = cb0 + 16 * cb + n;
                const T v = s < S ? static_cast<T>(g(d.pi)[s]) : T(0);
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) qk.v[rb][cb] = V4<T>{v, v, v, v};
            }
        } else {
            if constexpr (kStage)
                vbuf_to_cols<T, RB, NBW>(vb[kStage ? 2 : 0], ge, cb0, lane, qk);
            else
                load_cols<T, RB, NBW, kQ>(qk_base + r * rstride, ge, cb0, lane, qk);
            scale_rows<T, RB, NBW>(qk, esh[2], lane);
        }
        if (pj_src) {
            fwd<T, RB, NBW, G, true, kStage>(P + mo_j, dP + mo_j, sj, ge, cb0, lane, a, dmj);   // a = m_j, dm_j
            if (!tip_j) {
                scale_rows<T, RB, NBW>(a, esh[1], lane);
                scale_rows<T, RB, NBW>(dmj, esh[1], lane);
            }
        } else {
            tip_lookup<T, RB, NBW, true>(PB + bo_j, dPB + bo_j, g(d.codes), cj, ge, cb0, lane, a, dmj);
        }
        mul_cols<T, RB, NBW>(a, qk);                                           // a = u_i
        if (pi_src) {
            fwd<T, RB, NBW, G, true, kStage>(P + mo_i, dP + mo_i, si, ge, cb0, lane, b, acc);  // b = m_i, acc = dm_i
            if (!tip_i) {
                scale_rows<T, RB, NBW>(b, esh[0], lane);
                scale_rows<T, RB, NBW>(acc, esh[0], lane);
            }
        } else {
            tip_lookup<T, RB, NBW, true>(PB + bo_i, dPB + bo_i, g(d.codes), ci, ge, cb0, lane, b, acc);
        }
        T dd[RB][4] = {}, ni[RB][4] = {}, nj[RB][4] = {};
        dot_cols<T, RB, NBW>(a, b, dd);                                        // u_i . m_i
        dot_cols<T, RB, NBW>(a, acc, ni);                                      // u_i . dm_i
        mul_cols<T, RB, NBW>(b, qk);                                           // b = u_j
        dot_cols<T, RB, NBW>(b, dmj, nj);                                      // u_j . dm_j
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                num_i[rb][i] += wr * ni[rb][i];
                num_j[rb][i] += wr * nj[rb][i];
                den[rb][i] += wr * dd[rb][i];
            }
        if constexpr (kStage) __syncthreads();   // every wave is done reading the staged p_i, p_j, q_k
        if (!tip_i) cols_to_vbuf<T, RB, NBW>(vb[0], ge, cb0, lane, a);       // u_i over p_i
        if (!tip_j) cols_to_vbuf<T, RB, NBW>(vb[1], ge, cb0, lane, b);       // u_j over p_j
        __syncthreads();      // u complete in LDS
        if (!tip_i) {
            bwd<T, RB, NBW, G>(PB + bo_i, vb[0], ge, cb0, lane, acc);    // q_i = P_i^T u_i, stored over p_i
            max_cols<T, RB, NBW>(acc, mxi);
            store_cols<T, RB, NBW, kQ>(pi_base + r * rstride, ge, cb0, lane, acc);
        }
        if (!tip_j) {
            bwd<T, RB, NBW, G>(PB + bo_j, vb[1], ge, cb0, lane, acc);
            max_cols<T, RB, NBW>(acc, mxj);
            store_cols<T, RB, NBW, kQ>(pj_base + r * rstride, ge, cb0, lane, acc);
        }
        __syncthreads();      // before the next category's staging overwrites u
    }
    if (!tip_i) {
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int i = 0; i < 4; ++i) mxi[rb][i] = max16(mxi[rb][i]);
        wg_max<T, RB, W>(mxi, red, w, lane);
        int e[RB][4];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int i = 0; i < 4; ++i) e[rb][i] = exp_of(mxi[rb][i]);
        if (w == 0 && n == 0) {              // q_i is stored unscaled: record its exponent
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    st_int<kQ>(g(d.eloc) + static_cast<size_t>(nt.i - N) * Cpad + tile * TP + opat<T>(rb, gq, i),
                               e[rb][i]);
        }
    }
    if (!tip_j) {
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int i = 0; i < 4; ++i) mxj[rb][i] = max16(mxj[rb][i]);
        wg_max<T, RB, W>(mxj, red, w, lane);
        int e[RB][4];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int i = 0; i < 4; ++i) e[rb][i] = exp_of(mxj[rb][i]);
        if (w == 0 && n == 0) {              // q_j is stored unscaled: record its exponent
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    st_int<kQ>(g(d.eloc) + static_cast<size_t>(nt.j - N) * Cpad + tile * TP + opat<T>(rb, gq, i),
                               e[rb][i]);
        }
    }
    // per-pattern sums over all states: this wave's part, then the waves in order
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            num_i[rb][i] = sum16(num_i[rb][i]);
            num_j[rb][i] = sum16(num_j[rb][i]);
            den[rb][i] = sum16(den[rb][i]);
        }
    if (n == 0) {
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int p = opat<T>(rb, gq, i);
                red[(0 * W + w) * TP + p] = num_i[rb][i];
                red[(1 * W + w) * TP + p] = num_j[rb][i];
                red[(2 * W + w) * TP + p] = den[rb][i];
            }
    }
    __syncthreads();
    if (w == 0) {
        double gi = 0.0, gj = 0.0;
        if (n == 0) {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int p = opat<T>(rb, gq, i);
                    T Ni = red[p], Nj = red[W * TP + p], Dn = red[2 * W * TP + p];
#pragma unroll
                    for (int ww = 1; ww < W; ++ww) {
                        Ni += red[ww * TP + p];
                        Nj += red[(W + ww) * TP + p];
                        Dn += red[(2 * W + ww) * TP + p];
                    }
                    const double Wc = g(d.pw)[tile * TP + p];
                    if (Wc != 0.0) {
                        gi += Wc * (static_cast<double>(Ni) / static_cast<double>(Dn));
                        gj += Wc * (static_cast<double>(Nj) / static_cast<double>(Dn));
                    }
                }
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            gi += __shfl_xor(gi, off, 64);
            gj += __shfl_xor(gj, off, 64);
        }
        if (lane == 0) {
            g(d.gpart)[static_cast<size_t>(nt.i) * tiles + tile] = gi;
            g(d.gpart)[static_cast<size_t>(nt.j) * tiles + tile] = gj;
        }
    }
    if constexpr (kQ) gl_done(arg, U, true, target);
}

template <typename T, int RB, int NBW, int W>
__global__ __launch_bounds__(64 * W, (RB == 1 && sizeof(T) == 4 && (W == 2 || W == 4)) ? 4 : (RB == 1 && W == 4 && sizeof(T) == 8) ? 3 : 1)
void pre_gl_kernel(const ReqDesc* __restrict__ descs, const SegTable segs) {
    pre_gl_body<T, RB, NBW, W, false>(descs, segs);
}
// The same over a work-queue launch's items.
template <typename T, int RB, int NBW, int W>
__global__ __launch_bounds__(64 * W, (RB == 1 && sizeof(T) == 4 && (W == 2 || W == 4)) ? 4 : (RB == 1 && W == 4 && sizeof(T) == 8) ? 3 : 1)
void pre_gl_queue_kernel(const ReqDesc* __restrict__ descs, const QueueArgs q) {
    pre_gl_body<T, RB, NBW, W, true>(descs, q);
}

// ---------------------------------------------------------------- P(t) tables

// P = V diag(exp(g lam b)) V^-1 and dP = V diag(g lam exp(g lam b)) V^-1 for
// one (branch, category) pair (blockIdx.x) and one 64 x 64 tile of (s, t)
// (blockIdx.y), FP64 sums stored in the path's type, written as the forward
// tables of P and dP and their backward tables, zeros included; the first
// column tile of each row tile also writes the row sums P 1, dP 1 (the
// vector of a fully ambiguous tip) after the backward tables' rows.  V's
// columns and V^-1's rows pass through LDS in chunks of 16 k, V^-1 already
// scaled by exp and its derivative; a thread accumulates a 4 x 4 block.
constexpr int kPmTile = 64, kPmK = 16;

__host__ __device__ inline int pmat_gl_tiles(int S) { return (gl_mat_rows(S) + kPmTile - 1) / kPmTile; }

template <typename T>
__global__ __launch_bounds__(256) void pmat_gl_kernel(const ReqDesc* __restrict__ descs, const SegTable segs) {
    __shared__ double ex[256], dex[256], wsum[256];
    __shared__ __align__(16) double As[kPmK][kPmTile], Be[kPmK][kPmTile], Bd[kPmK][kPmTile];
    const int unit = blockIdx.x;
    // a new evaluation of a work-queue context
    if (unit == 0 && blockIdx.y == 0 && threadIdx.x == 0 && descs[segs.seg[0].desc].qctr)
        queue::new_evaluation(descs[segs.seg[0].desc].qctr);
    if (unit >= segs.unit_begin[segs.n]) return;
    const int sidx = seg_of(segs, unit);
    const Segment& sg = segs.seg[sidx];
    const ReqDesc& d = descs[sg.desc];
    const int pair = unit - segs.unit_begin[sidx];   // table (branch or slot) * R + category
    const int R = d.R, S = d.S;
    const int nt = pmat_gl_tiles(S);
    if (static_cast<int>(blockIdx.y) >= nt * nt) return;  // whole workgroup: smaller S in a shared launch
    const int ts = blockIdx.y / nt, tt = blockIdx.y - ts * nt;
    const int slot = pair / R;
    const int r = pair - slot * R;
    int x = slot;                                    // the branch: its own table
    if (sg.flags & 2) {                              // per-chunk tables: child (slot & 1) of record slot / 2
        const I4 t4 = reinterpret_cast<const GLOBAL I4*>(g(sg.sched))[sg.sched_off + slot / 2];
        x = (slot & 1) ? t4.z : t4.y;
    }
    const double gr = d.rates[r];
    const double bt = gr * d.b[x];
    const double* lam = d.lam + (d.eig_cat ? r * S : 0);
    const double* V = d.V + (d.eig_cat ? static_cast<size_t>(r) * S * S : 0);
    const double* Vinv = d.Vinv + (d.eig_cat ? static_cast<size_t>(r) * S * S : 0);
    const double* vs = d.vsum + (d.eig_cat ? r * S : 0);
    const int tid = threadIdx.x;
    for (int k = tid; k < S; k += blockDim.x) {
        const double e = exp(lam[k] * bt);
        ex[k] = e;
        dex[k] = gr * lam[k] * e;
        wsum[k] = vs[k];
    }
    // the first column tile also forms the row sums P 1 = V (e o Vinv 1) and
    // dP 1 for its 64 rows (thread tid < 64 owns row s_base + tid)
    double rsum = 0.0, drsum = 0.0;
    const int bs = tid / 16, bq = tid % 16;
    const int s_base = ts * kPmTile, t_base = tt * kPmTile;
    const int s0 = s_base + bs * 4, t0 = t_base + bq * 4;
    double acc[4][4] = {}, dacc[4][4] = {};
    for (int k0 = 0; k0 < S; k0 += kPmK) {
        __syncthreads();  // ex ready (first chunk); previous chunk consumed
#pragma unroll
        for (int m = 0; m < kPmK * kPmTile / 256; ++m) {
            const int idx = tid + 256 * m;
            const int kk = idx % kPmK, si = idx / kPmK;  // V: k contiguous in a row
            const int sv = s_base + si, kv = k0 + kk;
            As[kk][si] = (sv < S && kv < S) ? V[static_cast<size_t>(sv) * S + kv] : 0.0;
            const int ti = idx % kPmTile, kb = idx / kPmTile;  // V^-1: t contiguous in a row
            const int tv = t_base + ti, kw = k0 + kb;
            double vb = 0.0, e = 0.0, de = 0.0;
            if (tv < S && kw < S) {
                vb = Vinv[static_cast<size_t>(kw) * S + tv];
                e = ex[kw];
                de = dex[kw];
            }
            Be[kb][ti] = vb * e;
            Bd[kb][ti] = vb * de;
        }
        __syncthreads();
        if (tt == 0 && tid < kPmTile) {
            for (int kk = 0; kk < kPmK && k0 + kk < S; ++kk) {
                const double a = As[kk][tid] * wsum[k0 + kk];
                rsum += a * ex[k0 + kk];
                drsum += a * dex[k0 + kk];
            }
        }
#pragma unroll 4
        for (int kk = 0; kk < kPmK; ++kk) {
            double vs[4], ve[4], vd[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                vs[i] = As[kk][bs * 4 + i];
                ve[i] = Be[kk][bq * 4 + i];
                vd[i] = Bd[kk][bq * 4 + i];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    acc[i][j] += vs[i] * ve[j];
                    dacc[i][j] += vs[i] * vd[j];
                }
        }
    }
    const int rows = gl_mat_rows(S), row = gl_row(S), kbp = gl_kbp(S);
    const size_t base = static_cast<size_t>(pair) * rows * row;
    const size_t bbase = static_cast<size_t>(pair) * gl_back_rows(S) * row;
    GLOBAL T* PF = g(tabP<T>(d)) + base;
    GLOBAL T* dPF = g(tabdP<T>(d)) + base;
    GLOBAL T* PB = g(tabPB<T>(d)) + bbase;
    GLOBAL T* dPB = g(tabdPB<T>(d)) + bbase;
    if (tt == 0 && tid < kPmTile && s_base + tid < row) {   // the row-sum rows (zeros past S)
        PB[static_cast<size_t>(rows) * row + gl_col(s_base + tid, kbp)] = static_cast<T>(rsum);
        dPB[static_cast<size_t>(rows) * row + gl_col(s_base + tid, kbp)] = static_cast<T>(drsum);
    }
    if (s0 >= rows || t0 >= rows) return;  // after the last barrier
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int sr = s0 + i, tc = t0 + j;
            if (tc < row) {
                PF[static_cast<size_t>(sr) * row + gl_col(tc, kbp)] = static_cast<T>(acc[i][j]);
                dPF[static_cast<size_t>(sr) * row + gl_col(tc, kbp)] = static_cast<T>(dacc[i][j]);
            }
            if (sr < row) {
                PB[static_cast<size_t>(tc) * row + gl_col(sr, kbp)] = static_cast<T>(acc[i][j]);
                dPB[static_cast<size_t>(tc) * row + gl_col(sr, kbp)] = static_cast<T>(dacc[i][j]);
            }
        }
}

template <typename T, bool kQ = false, typename Arg>
hipError_t launch_gl_t(KernelClass k, int S, int rb, const ReqDesc* descs, const Arg& t, hipStream_t st) {
    int n_units = 0;
    if constexpr (kQ)
        n_units = t.t1 - t.t0;
    else
        n_units = t.unit_begin[t.n];
    // up to 128 states: one 16-state block per wave, ceil(S / 16) waves (at
    // 65..128 eight waves of one block beat four of two: fewer registers and
    // matrix loads per wave).  Above: FP32 four waves of ceil(S / 64) blocks
    // (two row blocks), FP64 ceil(S / 32) waves of two blocks (one row
    // block).  Rows read, 16 NBW W, stay within the table's rows.
    const bool f32 = sizeof(T) == 4;
    const int nbw = S <= 128 ? 1 : (f32 ? (S + 63) / 64 : 2);
    const int w = S <= 128 ? (S + 15) / 16 : (f32 ? 4 : (S + 31) / 32);
#define PHG_GL_CASE(RBV, NBV, WV)                                                                           \
    if (rb == RBV && nbw == NBV && w == WV) {                                                             \
        if constexpr (kQ) {                                                                                 \
            if (k == kPost)                                                                                 \
                hipLaunchKernelGGL((post_gl_queue_kernel<T, RBV, NBV, WV>), dim3(n_units), dim3(64 * WV), 0, \
                                   st, descs, t);                                                           \
            else                                                                                            \
                hipLaunchKernelGGL((pre_gl_queue_kernel<T, RBV, NBV, WV>), dim3(n_units), dim3(64 * WV), 0,  \
                                   st, descs, t);                                                           \
        } else {                                                                                            \
            if (k == kPost)                                                                                 \
                hipLaunchKernelGGL((post_gl_kernel<T, RBV, NBV, WV>), dim3(n_units), dim3(64 * WV), 0, st,  \
                                   descs, t);                                                               \
            else                                                                                            \
                hipLaunchKernelGGL((pre_gl_kernel<T, RBV, NBV, WV>), dim3(n_units), dim3(64 * WV), 0, st,   \
                                   descs, t);                                                               \
        }                                                                                                   \
        return hipGetLastError();                                                                           \
    }
    if constexpr (sizeof(T) == 4) {
        PHG_GL_CASE(2, 1, 3)
        PHG_GL_CASE(2, 1, 4)
        PHG_GL_CASE(2, 3, 4)
        PHG_GL_CASE(2, 4, 4)
        PHG_GL_CASE(4, 1, 2)
        PHG_GL_CASE(4, 1, 3)
        PHG_GL_CASE(4, 1, 4)
    } else {
        PHG_GL_CASE(1, 2, 5)
        PHG_GL_CASE(1, 2, 6)
        PHG_GL_CASE(1, 2, 7)
        PHG_GL_CASE(1, 2, 8)
    }
    PHG_GL_CASE(2, 1, 5)
    PHG_GL_CASE(2, 1, 6)
    PHG_GL_CASE(2, 1, 7)
    PHG_GL_CASE(2, 1, 8)
    PHG_GL_CASE(1, 1, 2)
    PHG_GL_CASE(1, 1, 3)
    PHG_GL_CASE(1, 1, 4)
    PHG_GL_CASE(2, 1, 2)
#undef PHG_GL_CASE
    return hipErrorInvalidValue;
}

}  // namespace

bool gl_row_blocks_allowed(int S, bool fp32, int rb) {
    // the instantiations of launch_gl_t
    if (S <= 32) return rb == 1 || rb == 2 || (fp32 && rb == 4);
    if (S <= 64) return rb == 1 || (fp32 && (rb == 2 || rb == 4));
    if (S <= 128) return rb == 2;
    return fp32 ? rb == 2 : rb == 1;
}

namespace {

}  // namespace

hipError_t launch_pmat_gl(const ReqDesc& shape, const ReqDesc* descs, const SegTable& t, hipStream_t st) {
    // every request of one launch has shape.S's tile count or fewer
    const int n_units = t.unit_begin[t.n], nt = pmat_gl_tiles(shape.S);
    if (shape.fp32)
        hipLaunchKernelGGL(pmat_gl_kernel<float>, dim3(n_units, nt * nt), dim3(256), 0, st, descs, t);
    else
        hipLaunchKernelGGL(pmat_gl_kernel<double>, dim3(n_units, nt * nt), dim3(256), 0, st, descs, t);
    return hipGetLastError();
}

hipError_t launch_level_gl(KernelClass k, const ReqDesc& shape, const ReqDesc* descs, const SegTable& t,
                           hipStream_t st) {
    const int rb = shape.Cpad / shape.tiles / 16;   // the context's own tile
    if (shape.fp32) return launch_gl_t<float>(k, shape.S, rb, descs, t, st);
    return launch_gl_t<double>(k, shape.S, rb, descs, t, st);
}

hipError_t launch_gl_queue(const ReqDesc& shape, const ReqDesc* descs, const QueueArgs& q, int pass,
                           hipStream_t st) {
    if (q.t1 <= q.t0) return hipSuccess;
    if (pass != 1 && pass != 2) return hipErrorInvalidValue;
    const KernelClass k = pass == 1 ? kPost : kPre;
    const int rb = shape.Cpad / shape.tiles / 16;
    if (shape.fp32) return launch_gl_t<float, true>(k, shape.S, rb, descs, q, st);
    return launch_gl_t<double, true>(k, shape.S, rb, descs, q, st);
}

}  // namespace phg
