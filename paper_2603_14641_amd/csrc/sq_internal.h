// Private declarations shared by the kernel files (sq_gates.hip,
// sq_measure.hip, sq_io.hip) and the host
// runtime behind the C ABI (sq_runtime.hip).
//
// Device layout of a tableau of n qubits (column-major, the layout the paper
// uses for gate application in "Tableau Layout and Indexing"):
//   K  = ceil(n / 64) words per half column, L = 2K words per column;
//   word w < K packs destabilizer rows 64w .. 64w+63 (bit b = row 64w+b),
//   word K + w packs stabilizer rows S_{64w} .. S_{64w+63};
//   X[q * Ls + w], Z[q * Ls + w] for qubit column q, with the column stride
//   Ls = L rounded up to 16 words (128 bytes) so every column starts on a
//   cache line; R[w] holds the sign bits of the same 64 rows.
// Bits of rows >= n in the last word of each half are always 0: every gate
// rule and every rowsum maps an all-zero row to itself with sign 0.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sq {

typedef unsigned long long u64;
typedef uint32_t u32;

// Gate-group micro-op codes (4 bits each, packed LSB first into Group::ops;
// 0 ends the list). Slot A is Group::q0, slot B is Group::q1.
enum : u32 {
  UOP_END = 0,
  UOP_H_A = 1, UOP_S_A = 2, UOP_SDG_A = 3, UOP_X_A = 4, UOP_Y_A = 5, UOP_Z_A = 6,
  UOP_H_B = 7, UOP_S_B = 8, UOP_SDG_B = 9, UOP_X_B = 10, UOP_Y_B = 11, UOP_Z_B = 12,
  UOP_CX_AB = 13, UOP_CX_BA = 14, UOP_CZ = 15
};

// Group::q0 carries the slot-A qubit in bits 0..23 and, in bits 24..27,
// which columns the group's ops can change (xa, za, xb, zb): only those are
// stored back.
constexpr u32 GQ_MASK = 0x00FFFFFFu;
constexpr u32 GD_XA = 1u << 24, GD_ZA = 1u << 25, GD_XB = 1u << 26, GD_ZB = 1u << 27;
constexpr u32 G_SINGLE = 0xFFFFFFFFu;  // Group::q1 of a one-qubit group

// A one- or two-qubit group of a gate pass: up to 16 ops on its own qubits.
struct Group {
  u32 q0;
  u32 q1;
  u64 ops;
};
static_assert(sizeof(Group) == 16, "Group must be 16 bytes");

// Wide gate groups (the tableau gate pass): up to WG_MAXQ qubits and
// WG_MAXOPS micro-ops per group. A group is a record of u32 words:
//   word 0: nq (bits 0..3) | nops (bits 4..9) | changed-x flags per slot
//           (bits 16..23) | changed-z flags per slot (bits 24..31);
//   words 1..nq: the qubit (column) of each slot;
//   then the micro-ops, two 16-bit ops per word, low half first.
// A micro-op is type (bits 0..3) | slot a (bits 4..7) | slot b (bits 8..11);
// for CX a is the control and b the target.
constexpr u32 WG_MAXQ = 8, WG_MAXOPS = 32;
constexpr u32 WH_NOPS_SHIFT = 4, WH_DX_SHIFT = 16, WH_DZ_SHIFT = 24;
enum : u32 {
  WOP_H = 1, WOP_S = 2, WOP_SDG = 3, WOP_X = 4, WOP_Y = 5, WOP_Z = 6, WOP_CX = 7, WOP_CZ = 8, WOP_SWAP = 9
};

// Where the sweep over a measured list stands, in device memory. A sweep is
// a fixed sequence of slots queued without host reads: each slot's kernels
// read the list position here and advance it, so the host only reads `i`
// back once after queuing enough slots for the whole list.
//   kb == 1: a slot measures list[i] alone (pivot, gather, rowsum, post);
//   kb >= 2: a slot offers list[i .. i + kb) to the blocked path, which takes
//   its random prefix (k measurements), then measures list[i + k] alone when
//   the block stopped at a deterministic one (`single`).
struct Cursor {
  u32 i;            // next position in the list
  u32 end;          // list length
  u32 kb;           // measurements offered per block (1: every measurement alone)
  u32 single;       // set by the blocked pivot step: this slot's single kernels measure list[i]
  u64 seed, shot;   // coin key
  u64 meas_base;    // measurement index of list[0]
  const u32 *qubits;  // the measured list (device)
  uint8_t *out_bits;  // outcome of list[i] to out_bits[i] (NULL: not written)
  uint8_t *out_rand;  // 1 random / 0 deterministic to out_rand[i] (NULL: not written)
};

constexpr int32_t P_NONE = -2;  // MeasState::p of a slot that measures nothing alone

// Per-measurement device state (one per tableau, reused by every measurement).
struct MeasState {
  int32_t p;      // pivot stabilizer index, -1 if the outcome is deterministic, P_NONE if no measurement
  u32 q;          // the qubit measured alone in this slot
  u32 i;          // its position in the list
  u32 ncols;      // number of non-identity columns of S_p (compacted list length)
  u32 det_acc;    // deterministic case: sum of phase exponents (mod 2^32)
  u32 flags;      // sticky error flags: bit 0 odd rowsum phase, bit 1 bad det product
  u32 rp;         // sign bit of S_p before the update
  u32 coin;       // coin of the current measurement
  u32 mwords;     // nonzero words of the rowsum mask (row words the pass touches)
  u32 awords;     // nonzero destabilizer-half words of column q (deterministic case)
  u32 nx, nz;     // pivot-row columns with x_pj = 1, with z_pj = 1
  u32 nsv;        // sampling: coin columns in which S_p has a 1 (compacted list length)
  u32 det_done;   // deterministic case: k_post's blocks done (bits 0..23) and their phase sum mod 256 (bits 24..31)
  u32 inj;        // CX-injection collapse: bit 0 inverse-phase rotation (else H), bit 1 X injection
  u32 pc;         // row layout: pivot candidate (grid-wide minimum; 0xFFFFFFFF none)
  u32 naff;       // row layout: rows multiplied by the pivot in this measurement
};

// Symbolic-sign context of the sampler's sweep (sq_sample.hip); unused (zero)
// on the plain path. Sign column v < count holds the coefficient of coin v,
// column `count` the constant term, one bit per stabilizer row (K words,
// stride Ks). The position of the current measurement in the list comes from
// MeasState::i (alone) or BlkState::i0 (blocks).
struct SymCtx {
  u64 *sg;
  u32 *svlist;     // coin columns in which S_p has a 1
  uint8_t *kind;   // per measurement: 1 random, 0 deterministic
  u64 *fm;         // per deterministic measurement: coin coefficients (CW words)
  uint8_t *fc;     // ... and the constant term
  u32 Ks, CW, count, pad;
};

// Running totals over all measurements of a tableau, for byte accounting.
struct MeasStats {
  u64 n_random, n_det;
  u64 rowsum_bytes;   // algorithmic bytes of the single-measurement rowsum passes
  u64 det_bytes;      // algorithmic bytes of the deterministic-phase passes
  u64 blocks;         // blocked passes (several random measurements each)
  u64 block_bytes;    // algorithmic bytes of the blocked passes
  u64 inject_bytes;   // algorithmic bytes of the CX-injection passes
};

// Blocked random measurements (sq_block.hip): up to KB per pass.
constexpr u32 KB = 32;
constexpr u32 BLK_PART = 3;  // partial words per (chunk, row word): counter bits 0, 1 and the parity
struct BlkState {
  u32 k;          // random prefix actually processed (the block ends before a deterministic one)
  u32 i0;         // list position of the block's first measurement
  u32 q[KB];      // the qubits of the block's measurements
  u32 p[KB];      // pivot stabilizer index of each
  u32 hitS[KB];   // bit s': pivot s' hit S_{p_s} before it became a pivot
  u32 M[KB];      // bit s2: x of P_s at q_{s2}
  u32 coin[KB];
  u32 dhits[KB];  // bit s2: pivot s2 (> s) hits D_{p_s}
  u32 Qz[KB];     // bit b: z_{P_a} . x_{P_b} (mod 2), row a
  u32 R0[KB];     // bit b: z_{P_a} . x of the original S_{p_b}
  u32 pc0[KB];    // |x & z| of the original S_{p_s}
  u32 pcD[KB];    // |x & z| of the final D_{p_s}
  u32 r0[KB];     // sign of the original S_{p_s}
  u32 lam[KB];    // lam(P_s) = 2 r + |x & z| (mod 4)
  u32 dsign[KB];  // final sign of D_{p_s}
  u32 ncols;      // columns where some pivot is not the identity
  u32 nwords;     // distinct row words (within a half) holding the pivots
  u32 word[KB];   // those words
  u32 wmem[KB];   // bit s: pivot s lies in word[i]
};
struct BlkBuffers {
  u64 *bm;                 // KB * Ls words: hit masks
  u32 *wpart;              // K * 4 * KB: per block of k_blk_rows, its share of the pivot algebra
  u32 *patx, *patz;        // n each: per column, bit s = pivot s has x (z) there
  u64 *part;               // chunks * BLK_PART * Ls partial counters and parities
  BlkState *bs;
  u32 *clist;              // n: the block's supported columns (some pivot not the identity), any order
};

// One circuit of a batched launch (sq_batch.hip): |0...0>, gate passes
// groups[pass_off[p] .. pass_off[p+1]), then `shots` shots of measuring
// qubits[0..count). All pointers are device memory owned by the batch.
struct BatchItem {
  u32 n, Ls, Ks, CW, count, shots, npasses, pad;
  u64 *X, *Z;          // n * Ls words each
  u64 *sg;             // (count + 1) * Ks sign-column words
  u64 *fm;             // count * CW affine-form words
  u64 *coinbuf;        // shots * CW coin words
  u64 *out;            // shots * CW outcome words
  uint8_t *fc, *kind;  // count bytes each
  const Group *groups;
  const u32 *pass_off; // npasses + 1 offsets into groups
  const u32 *qubits;
  u64 seed, shot_begin, meas_base;
  u32 *flags;          // consistency flags of this circuit (OR-ed)
};

struct TabDev {
  u64 *X, *Z, *R;
  u32 n, K, L, Ls;
};

struct LaunchTimer;  // host-side profiling hook (sq_runtime.hip)

// Kernel launchers (sq_gates.hip, sq_measure.hip, sq_sample.hip, sq_batch.hip,
// sq_io.hip). All enqueue on `s` and return the
// launch status.
hipError_t launch_fill_zero(u64 *p, size_t words, hipStream_t s);
hipError_t launch_init_diag(const TabDev &t, hipStream_t s);
hipError_t launch_layer(const TabDev &t, const u32 *words, const u32 *offs, u32 ngroups, u32 block, u32 wpt,
                        u32 gpc, u64 *sign_part, hipStream_t s);
hipError_t launch_sign_reduce(const TabDev &t, const u64 *sign_part, u32 nchunks, hipStream_t s);
// Operator-tableau mode (sq_gates.hip, sq_inject.hip): R holds the image
// signs, word w < K the signs of A_q = image of X_q, word K + w those of B_q.
hipError_t launch_layer_op(const TabDev &t, const u32 *words, const u32 *offs, u32 ngroups, u32 block, u32 gpc,
                           u32 max_groups, u64 *part, u32 *flags, hipStream_t s);
hipError_t launch_inj_pivot(const TabDev &t, Cursor *cur, MeasState *st, u64 *mask, u32 *tw, MeasStats *stats,
                            hipStream_t s);
// Row-contiguous layout (sq_rows.hip).
hipError_t launch_transpose(const TabDev &t, hipStream_t s);
hipError_t launch_row_begin(MeasState *st, hipStream_t s);
hipError_t launch_row_prep(const TabDev &t, Cursor *cur, MeasState *st, u64 *pivx, u64 *pivz, hipStream_t s);
hipError_t launch_row_rowsum(const TabDev &t, MeasState *st, const u64 *pivx, const u64 *pivz, hipStream_t s);
hipError_t launch_row_det(const TabDev &t, MeasState *st, u64 *xsum, u64 *zsum, u32 det_blocks, hipStream_t s);
hipError_t launch_row_finish(const TabDev &t, Cursor *cur, MeasState *st, const u64 *pivx, const u64 *pivz,
                             MeasStats *stats, hipStream_t s);
hipError_t launch_inj_apply(const TabDev &t, const MeasState *st, const u64 *mask, const u32 *tw, uint8_t *pair,
                            MeasStats *stats, hipStream_t s);
hipError_t launch_cursor_init(Cursor *c, u32 end, u32 kb, u64 seed, u64 shot, u64 meas_base, const u32 *qubits,
                              uint8_t *out_bits, uint8_t *out_rand, hipStream_t s);
hipError_t launch_pivot(const TabDev &t, Cursor *cur, MeasState *st, u64 *mask, u32 *alist, u64 *amask,
                        hipStream_t s);
hipError_t launch_gather(const TabDev &t, MeasState *st, u64 *pivx, u64 *pivz, u32 *cols, const SymCtx *sym,
                         hipStream_t s);
hipError_t launch_rowsum(const TabDev &t, const u64 *mask, const u32 *cols, const MeasState *st, u64 *cnt0,
                         u64 *cnt1, u32 block, u32 wpt, u32 cpc, u32 max_chunks, const SymCtx *sym, hipStream_t s);
hipError_t launch_post(const TabDev &t, const Cursor *cur, const u64 *mask, const u64 *pivx, const u64 *pivz,
                       const u64 *cnt0, const u64 *cnt1, const u32 *alist, MeasState *st, MeasStats *stats, u32 cpc,
                       u32 cpw, const SymCtx *sym, hipStream_t s);
// Shot sampling (sq_sample.hip).
hipError_t launch_sample_init(const TabDev &t, u64 *sg, u32 Ks, u32 count, hipStream_t s);
hipError_t launch_coins(u64 *cw, u64 seed, u64 shot_begin, u64 meas_base, u32 shots, u32 count, u32 CW,
                        hipStream_t s);
hipError_t launch_eval(const u64 *cw, const uint8_t *kind, const u64 *fm, const uint8_t *fc, u64 *out, u32 shots,
                       u32 count, u32 CW, hipStream_t s);
hipError_t launch_batch(const BatchItem *items, u32 nitems, u32 *next, u32 block, u32 grid, hipStream_t s);
// waves: PIVOT_AUTO (the C-ABI's SQ_PIVOT_AUTO), or 1..16 for the tiled search
// with that many waves
constexpr u32 PIVOT_AUTO = 255;
// zero_words[0 .. nzero) are cleared by the pivot kernel (the sampler's
// zeroed sign words for the slot's later kernels); nullptr, 0 for none.
hipError_t launch_blk_pivots(const TabDev &t, Cursor *cur, const BlkBuffers &b, u32 waves, u64 *zero_words,
                             u32 nzero, hipStream_t s);
hipError_t launch_blk_prep(const TabDev &t, const BlkBuffers &b, hipStream_t s);
hipError_t launch_blk_pass(const TabDev &t, const BlkBuffers &b, u32 cpc, hipStream_t s);
hipError_t launch_blk_final(const TabDev &t, const BlkBuffers &b, MeasState *st, MeasStats *stats, u32 cpc,
                            const u64 *sg, u32 Ks, u32 count, u32 *svt, hipStream_t s);
hipError_t launch_blk_sv(u64 *sg, u32 Ks, u32 count, const BlkBuffers &b, const u32 *svt, const u64 *cvec, u32 Ls,
                         u32 K, hipStream_t s);
hipError_t launch_frame_init(u64 *Fx, u64 *Fz, u32 n, u32 Lf, u32 Ls, u64 seed, hipStream_t s);
hipError_t launch_frame_measure(const u64 *Fx, u64 *Fz, const u32 *qubits, u32 count, u64 m0, const uint8_t *ref,
                                u64 *rec, u32 n, u32 Lf, u32 Ls, u64 seed, hipStream_t s);
hipError_t launch_frame_transpose(const u64 *rec, u64 *out, u64 M, u32 W, u32 Lf, u32 shots, hipStream_t s);
hipError_t launch_export_rows(const TabDev &t, const u32 *rows, u32 nrows, u32 W, u64 *ox, u64 *oz, uint8_t *orr,
                              hipStream_t s);
hipError_t launch_import(const TabDev &t, const u64 *ix, const u64 *iz, const uint8_t *ir, u32 W, hipStream_t s);

}  // namespace sq
