// Internal declarations shared by the host runtime (phg_host.cpp, phg_server.cpp)
// and the gfx950 kernels (phg_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

#include "../../include/phg.h"

namespace phg {

constexpr int kLanes = 64;          // one wavefront = one tile of 64 site patterns

// One parent with its two children, by node id.  Post-order levels list the
// internal nodes of equal height; pre-order levels the internal nodes of
// equal depth.  Children are stored in ascending id order.  fold (kernel
// families with folds_tip_pairs): bit 0 / bit 1 set when child i / j is a
// folded node -- an internal node (not the root) whose two children are tips
// given by codes.  Folded nodes have no post-order records: their parent's
// launches form their partial from the two tips' rows of the P(t) tables
// (such nodes are never rescaled, so that is the vector a launch of theirs
// would have stored).  With folds_pre_order they have no pre-order records
// either: the parent's pre-order launch forms the gradient sums of their tip
// branches.
struct NodeTriple {
    int32_t k, i, j, fold;
};

// A block of the tree for the blocked 4-state schedule: a block root at a
// depth that is a multiple of 3 with its internal children and grandchildren,
// as a heap: node[1] is the root, node[2p], node[2p+1] are the children of
// node[p] when node[p] is an internal node at a position p < 8, and -1
// otherwise.  Positions 2..7 that hold internal nodes are inside the block;
// positions 8..15 hold the frontier (tips or the roots of deeper blocks).
struct BlockRec {
    int32_t node[16];   // node[0] unused
};

// Device-resident description of one evaluation request (one tree and
// alignment with its own workspace).  Layouts (T = float or double):
//   codes  uint8  [N][Cpad]                  tip states, S = all-ones, pad = S
//   part   T      4 states: [N-1][tiles][R][64][4] (lane-major quads)
//                 vector-ALU kernels (17..32 states): [N-1][tiles][R][SP][64]
//                   (state rows of the tile's 64 patterns, SP = vs_padded_states)
//                 MFMA kernels (17..256 states): [N-1][tiles][R][TP][gl_row(S)]
//                   (pattern rows in the MFMA operand order gl_col, zero-padded)
//                 otherwise: [N-1][tiles][R][S][TP] (state rows of TP patterns)
//                                             post-order partial of each
//                                             internal node (slot = id - N);
//                                             overwritten in place by the
//                                             pre-order partial
//   expo   int32  [N-1][Cpad]                cumulative power-of-two exponent
//                                             of the subtree below each node
//   eloc   int32  [N-1][Cpad]                MFMA kernels: the node's own
//                                             exponent e; its stored partial
//                                             is 2^e times the normalised one
//                                             (after the pre-order: that of q)
//   P64,dP64 double [E][R][S][S]; P32,dP32 float copies (FP32 path only);
//                 17..255 states: only the table of the path's type T, as
//                 [E][R][gl_mat_rows(S)][gl_row(S)] with row s holding P[s][t]
//                 at column gl_col(t) (forward operand), and PB32 / PB64 the
//                 same with row t holding P[s][t] at gl_col(s) (backward);
//                 vector-ALU kernels: forward [E][R][SP][SP] (row s = P[s][.])
//                 and backward [E][R][SP + 1][SP] (row t = P[.][t], row SP the
//                 row sums), zero-padded, for P and dP alike
//   sll    double [Cpad]                     per-pattern log site likelihood
//   lpart  double [tiles]                    per-tile weighted log-likelihood
//   gpart  double [E][tiles]                 per-tile weighted gradient sums
//   sched  NodeTriple [2(N-1)]               post-order levels then pre-order
//                                             levels of this request's tree
struct ReqDesc {
    int32_t N, C, Cpad, S, S4, R, tiles, fp32;
    int32_t blocked;        // sched holds BlockRec records, else NodeTriple
    int32_t level_tables;   // 17..255 states: P(t) tables per launch chunk (slot 2 n + c for child c of
                            // the chunk's node n), built by a P(t) launch over the same records
    int32_t eig_cat;        // 1: V, Vinv [R][S][S] and lam [R][S], one model per category
    const NodeTriple* sched;
    const int32_t* kids;    // [N-1][2] children of internal node N + k
    const uint8_t* codes;
    void* part;
    int32_t* expo;
    int32_t* eloc;
    double* P64;
    double* dP64;
    float* P32;
    float* dP32;
    float* PB32;
    double* PB64;
    // 17..255 states: backward copy of dP (row t holds dP[s][t] at column
    // gl_col(s)), and for P and dP one more row after the gl_mat_rows(S)
    // rows of each backward table holding the row sums (a fully ambiguous
    // tip's vector); vsum[m][k] = sum_t Vinv_m[k][t] (host-computed)
    float* dPB32;
    double* dPB64;
    const double* vsum;
    // 4 states: tip tables [E][R][5][4]: entry y (0..3) is column y of P (or
    // dP), entry 4 its row sums (the ambiguous code), so P e_y is one load
    double* TT64;
    double* dTT64;
    float* TT32;
    float* dTT32;
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
    // General tip partials (level schedule only): tslot[tip] is -1 for a tip
    // given by codes, else the tip's slot in tipvec, which holds its C x S
    // vector in the partials layout of the kernels (T, every category).
    // Null when no tip has one.
    const int32_t* tslot;
    const void* tipvec;
    // Work-queue traversal: its counter words (phg::kQueueWords), else
    // null.  The P(t) launch of an evaluation advances the epoch and clears
    // the fault word; the final sums turn to NaN if it is set.
    uint32_t* qctr;
};

// A launch processes the work units of up to kMaxSegs segments; a segment is
// one request's slice of that launch (one level, or the whole pmat/finalize
// stage).  Units of segment s are [unit_begin[s], unit_begin[s+1]).
constexpr int kMaxSegs = 48;
struct Segment {
    int32_t desc;        // index into the descriptor table
    int32_t sched_off;   // first NodeTriple of the level in `sched` (levels only)
    int32_t n_nodes;     // nodes in the level (levels only)
    int32_t flags;       // bit 0: this post-order level is the root level; bit 1 (P(t) of the
                         // MFMA kernels): tables of the children of records [sched_off, + n_nodes)
    const int32_t* sched;  // the request's schedule records (device), as in its descriptor
    double* out_logl;    // finalize only: where log P(Y) goes
    double* out_grad;    // finalize only: where the 2N-2 derivatives go
};
struct SegTable {
    int32_t n;
    int32_t unit_begin[kMaxSegs + 1];
    Segment seg[kMaxSegs];
};

enum KernelClass { kPmat = 0, kPost = 1, kPre = 2, kFinal = 3 };

// Work units one segment contributes to a launch of the given class.
int units_for(KernelClass k, const ReqDesc& d, int n_nodes);

// Kernel launchers (phg_kernels.hip).  All requests in one table share S, R
// and precision.  `descs` and `sched` are device pointers.
hipError_t launch_class(KernelClass k, const ReqDesc& shape, const ReqDesc* descs,
                        const SegTable& t, hipStream_t stream);
bool kernels_support(int S, int R);

// Patterns per work-unit tile: 64 for the 4-state kernels (R <= 8); for the
// MFMA kernels of other state counts 32 (float) or 16 (double).
int tile_patterns(int S, int R, bool fp32);
// Whether (S, R) runs on the dedicated 4-state kernels.
inline bool uses_s4_kernels(int S, int R) { return S == 4 && R <= 8; }
// Tree depth spanned by one block of the blocked 4-state schedule.
constexpr int kBlockDepth = 3;
// Whether the blocked schedule has kernels for (S, R, precision) that keep
// every in-block vector in registers.
inline bool blocked_supported(int S, int R, bool /*fp32*/) { return S == 4 && R <= 8; }

// Work-queue traversals: one launch per pass (or, 4 states, one for both)
// instead of one per level, over the blocked schedule (FP32, 4 states, R in
// {1, 2, 4, 8}) or the level schedule of the vector-ALU kernels (with P(t)
// tables for every branch).
inline bool queue_supported(int S, int R, bool fp32);
// Counter words of a context's queue (each on a 64-byte line of its own):
// the epoch and the fault word.
constexpr int kQueueEpoch = 0, kQueueFault = 16, kQueueWords = 32;
// Milliseconds before a dependency wait gives up: far above any legitimate
// wait (an item waits only on items already running).
constexpr int kQueueWaitMs = 2000;
uint64_t queue_wait_ticks(int device, int S, int R, bool fp32);
// Launches per evaluation with the gradient (1: both passes in one, 2: one per
// pass) unless tuned (PHG_TUNE_QUEUE_LAUNCHES).
constexpr int kQueueLaunchesDefault = 2;
int queue_launches(int S, int R, bool fp32);
struct QueueArgs {
    const int32_t* items;   // [n][2]: (block record | pass << 30, tile); pass 0 post-order, 1 pre-order;
                            // numbered so that every item's inputs come from smaller numbers
    const int32_t* dep;     // [B][16]: j < 8 the record of the block rooted at heap position 8 + j
                            // (-1: none); 8 the parent block's record (-1: the root block)
    uint32_t* done;         // [2][B][tiles] completion marks (post-order, pre-order)
    uint32_t* ctr;          // [kQueueWords] counter words: epoch, fault
    int32_t t0, t1;         // this launch's items (workgroup i takes item t0 + i)
    int32_t n_blocks;       // B
    int32_t root_rec;       // record of the block holding the tree root
    uint64_t wait_ticks;    // constant-clock ticks before a wait gives up
};
// Items [q.t0, q.t1) of the context whose descriptor is descs[0], one
// workgroup each; passes: 1 the range holds post-order items only, 2
// pre-order items only, 3 both (4 states only).  Records: block records
// (4 states; dep [B][16]: frontier children's blocks, parent block) or level
// records (vector-ALU kernels; dep [records][2]: the parent's node slot of a
// pre-order record, marks per node slot).
hipError_t launch_queue(const ReqDesc& shape, const ReqDesc* descs, const QueueArgs& q, int passes,
                        hipStream_t stream);

// Default threshold of the FP32 precision guard: an FP32 context evaluates in
// FP64 when some internal node k has a child x' with min(L_k, L_x') above it,
// where L_v = b_v * max_r(gamma_r * mu_r) is branch v's length in units of
// the slowest decay of its fastest category (mu_r = smallest non-zero
// |lambda| of category r's generator; the root branch counts as infinite).
// There, nearly stationary pre-order vectors meet nearly flat sibling
// vectors and a single float32 rounding of the stored partials already moves
// some gradient components by ~1e-4 of themselves (measured in a float32
// emulation of the recursion; 4-state trees first fail near 2.8).
constexpr double kDefaultFp32Guard = 1.5;

// Chain rules on a finished branch gradient (phg_chain.hip).  All pointers
// are device pointers into the context's workspace.
struct ChainArgs {
    int N, n_sets;
    const int32_t* parent;   // [2N-1], parent of the root = -1
    const int32_t* kids;     // [N-1][2] children of internal node N + k
    const double* heights;   // [2N-1]
    const double* rates;     // [2N-2] branch rate scalars
    const double* grad;      // [2N-2] d logL / d b
    double* d_heights;       // [2N-1]
    double* d_rates;         // [2N-2]
    const int32_t* set_ptr;  // [n_sets + 1] CSR offsets into set_idx
    const int32_t* set_idx;  // branches of each set, increasing
    double* d_sets;          // [n_sets]
};
// time_tree: heights / rates chain rule; then, if n_sets > 0, set sums of
// d_rates (time_tree) or of grad.
hipError_t launch_chain(const ChainArgs& a, bool time_tree, hipStream_t stream);

// Vector-ALU level kernels for 17..32 states (FP32; 17..24 in FP64, whose
// registers hold four padded vectors per lane) at 1, 2, 4 or 8 categories
// (phg_kernels_vs.hip): one workgroup per (node, 64-pattern tile), one wave
// per category, one lane per pattern, the matrices wave-uniform and staged
// in LDS.  Their vectors and tables are padded to vs_padded_states(S) states.
__host__ __device__ constexpr inline int vs_padded_states(int S) { return S <= 20 ? 20 : (S <= 24 ? 24 : 32); }
// LDS of a pre-order workgroup: P and dP of both children for each category,
// and eleven per-pattern exchange values per category.  Shapes above
// kVsLdsMax (two workgroups per CU) stay on the MFMA kernels.
__host__ __device__ constexpr inline size_t vs_lds_bytes(int SP, int R, int tsz) {
    return static_cast<size_t>(R) * (4 * SP * SP + 11 * 64) * tsz;
}
constexpr size_t kVsLdsMax = size_t{80} << 10;
inline bool uses_vs_kernels(int S, int R, bool fp32) {
    return S > 16 && S <= (fp32 ? 32 : 24) && R >= 1 && R <= 8 && (R & (R - 1)) == 0 &&
           vs_lds_bytes(vs_padded_states(S), R, fp32 ? 4 : 8) <= kVsLdsMax;
}
hipError_t launch_vs(KernelClass k, const ReqDesc& shape, const ReqDesc* descs, const SegTable& t,
                     hipStream_t stream);

// MFMA level kernels for the other shapes above 16 states (phg_kernels_gl.hip):
// one workgroup per (node, pattern tile), the waves splitting the output states.
inline bool uses_gl_kernels(int S, int R, bool fp32) {
    return S > 16 && !uses_s4_kernels(S, R) && !uses_vs_kernels(S, R, fp32);
}
// Kernel families that fold tip-tip nodes (the node triple's fold bits): the
// vector-ALU kernels, and the MFMA kernels where their pre-order stages its
// inputs in LDS (above 32 states).  The vector-ALU kernels also take a
// folded node's pre-order into its parent's launch; the MFMA kernels keep
// its own pre-order launch.
inline bool folds_tip_pairs(int S, int R, bool fp32) {
    return uses_vs_kernels(S, R, fp32) || (uses_gl_kernels(S, R, fp32) && S > 32);
}
inline bool folds_pre_order(int S, int R, bool fp32) { return uses_vs_kernels(S, R, fp32); }
inline bool queue_supported(int S, int R, bool fp32) {
    return (S == 4 && fp32 && R <= 8 && (R & (R - 1)) == 0) || uses_vs_kernels(S, R, fp32) ||
           uses_gl_kernels(S, R, fp32);
}
hipError_t launch_vs_queue(const ReqDesc& shape, const ReqDesc* descs, const QueueArgs& q, int pass,
                           hipStream_t stream);
hipError_t launch_gl_queue(const ReqDesc& shape, const ReqDesc* descs, const QueueArgs& q, int pass,
                           hipStream_t stream);
// Their operand order: a stored vector (one pattern's partial) or matrix row
// holds state t at column gl_col(t) = (t mod 4) KBP + t / 4, so the states
// 4k + g that MFMA lane group g consumes on k-steps k, k+1, ... are adjacent
// and G of them arrive by one 8- or 16-byte load (G = gl_vec(S)); columns of
// states >= S hold zeros.  Matrices have gl_mat_rows(S) rows (zero-padded to
// the kernels' 16- or 64-state column blocks).
__host__ __device__ constexpr inline int gl_vec(int S) { return S <= 32 ? 2 : 4; }
__host__ __device__ constexpr inline int gl_kbp(int S) {
    return ((S + 3) / 4 + gl_vec(S) - 1) / gl_vec(S) * gl_vec(S);
}
__host__ __device__ constexpr inline int gl_row(int S) { return 4 * gl_kbp(S); }
__host__ __device__ constexpr inline int gl_col(int t, int kbp) { return (t & 3) * kbp + (t >> 2); }
__host__ __device__ constexpr inline int gl_mat_rows(int S) {
    return S <= 64 ? (S + 15) / 16 * 16 : (S + 63) / 64 * 64;
}
// Rows of one (branch, category) backward table: the gl_mat_rows(S) rows of
// states, then the row sums (read for tip code S).
__host__ __device__ constexpr inline int gl_back_rows(int S) { return gl_mat_rows(S) + 1; }
// Bytes per stored tip code: code S marks a fully ambiguous entry, so 256
// states need 16 bits (the MFMA kernels read both widths).
__host__ __device__ constexpr inline int code_bytes(int S) { return S > 255 ? 2 : 1; }
// Row blocks of 16 patterns per tile: two (each matrix operand then feeds two
// MFMAs) for FP32 above 32 states and FP64 at 65..128, one otherwise.
// Measured: above 64 states two win even at one wave per SIMD; four at
// 33..64 states (FP32), two at 33..64 (FP64) and two at 17..32 (FP32) lose.
inline int gl_row_blocks_default(int S, bool fp32) {
    if (S <= 32) return 1;
    if (S > 128) return fp32 ? 2 : 1;
    return (fp32 || S > 64) ? 2 : 1;
}
// Row-block counts the MFMA kernels are built for at (S, precision).
bool gl_row_blocks_allowed(int S, bool fp32, int rb);

// Process-wide tuning table (phg_set_tuning; filled from a tuning file at
// first use): per (state count, category count, precision, parameter) a value,
// 0 meaning the built-in rule.  Read when a context is created (row blocks)
// or a launch is issued (narrow-launch threshold).
int tuned_value(int S, int R, bool fp32, int param);
// Row blocks of 16 patterns per tile of a context created now.
inline int gl_row_blocks(int S, int R, bool fp32) {
    const int t = tuned_value(S, R, fp32, PHG_TUNE_ROW_BLOCKS);
    return t > 0 ? t : gl_row_blocks_default(S, fp32);
}
hipError_t launch_level_gl(KernelClass k, const ReqDesc& shape, const ReqDesc* descs,
                           const SegTable& t, hipStream_t stream);
// P(t) tables of those kernels (forward P, dP and backward P in operand order).
hipError_t launch_pmat_gl(const ReqDesc& shape, const ReqDesc* descs, const SegTable& t, hipStream_t stream);

// MFMA level kernels for other state counts (phg_kernels_gs.hip).
int gs_tile_patterns(bool fp32);
hipError_t launch_level_gs(KernelClass k, const ReqDesc& shape, const ReqDesc* descs,
                           const SegTable& t, hipStream_t stream);

}  // namespace phg
