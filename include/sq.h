/*
 * sq.h -- C ABI of the MI355X stabilizer-tableau library (libsq.so).
 *
 * The library keeps a CHP tableau (Aaronson-Gottesman destabilizer form; the
 * paper's "Tableau Formalism" and "The CHP algorithm" sections) of n qubits
 * resident in GPU memory and evolves it with hand-written HIP kernels for
 * gfx950:
 *   - gate layers (H, S, S^dagger, X, Y, Z, CX, CZ), the column update rules
 *     of the "Tableau Formalism" section (equation update_rules, extended by
 *     conjugation to the other gates), all gates of a layer fused into passes
 *     over the touched columns ("Tableau Evolution under Clifford Gates");
 *   - projective Z measurement: pivot search, the parallel rowsum of every
 *     anticommuting row with the pivot stabilizer (exact mod-4 phase), and
 *     the destabilizer product for deterministic outcomes ("The CHP
 *     algorithm", probabilistic and deterministic cases).
 *
 * Conventions shared by every call:
 *   - All functions return sq_status (0 = SQ_OK, negative = error) unless
 *     documented otherwise; sq_last_error() then describes the failure
 *     (thread-local string, valid until the next call on that thread).
 *   - Validation happens before any device work: a call that fails with
 *     SQ_EINVAL or SQ_ERANGE leaves the tableau unchanged.
 *   - A handle owns its device memory. Host buffers are owned by the caller
 *     and are only read or written during the call, except where a call is
 *     documented as asynchronous.
 *   - All device work of a handle is ordered on the HIP stream given at
 *     creation (NULL = the default stream). Calls that return results in
 *     host memory synchronize that stream before returning.
 *   - A handle must not be used from two threads at once; distinct handles
 *     are independent.
 *
 * Tableau semantics: rows 0..n-1 are the destabilizers D_i, rows n..2n-1 the
 * stabilizers S_i; row g is the Pauli string (-1)^{r_g} P_0 ... P_{n-1} with
 * P_j = I, X, Z, Y for (x_gj, z_gj) = (0,0), (1,0), (0,1), (1,1). A new
 * tableau is |0...0>: D_i = +X_i, S_i = +Z_i.
 *
 * Random outcomes: measurement number m of shot `shot` (counted over every
 * measurement, deterministic ones included, starting at meas_base) draws
 * coin = bit 0 of word 0 of Philox4x64-10(counter = (m, 0, 0, 0),
 * key = (seed, shot)) (Salmon et al., SC'11). A random outcome equals its coin.
 */
#ifndef LIBSQ_SQ_H_
#define LIBSQ_SQ_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SQ_OK = 0,
  SQ_EINVAL = -1,   /* bad argument (NULL pointer, unknown gate type, qubit pair with a == b, ...) */
  SQ_ENOMEM = -2,   /* device or host allocation failed */
  SQ_EDEVICE = -3,  /* a HIP runtime call failed */
  SQ_ERANGE = -5,   /* a qubit index >= n, or a size above a stated limit */
  SQ_ESTATE = -6,   /* a device-side consistency check failed (see sq_error_flags) */
} sq_status;

/* Operation type codes. Gate records and programs use the same codes. */
typedef enum {
  SQ_I = 0, SQ_H = 1, SQ_S = 2, SQ_SDG = 3, SQ_X = 4, SQ_Y = 5, SQ_Z = 6,
  SQ_CX = 7,    /* q0 = control, q1 = target */
  SQ_CZ = 8,
  SQ_CY = 9,    /* controlled-Y, q0 = control, q1 = target */
  SQ_SWAP = 10,
  SQ_ISWAP = 11,
  SQ_MEASURE = 15 /* Z measurement of q0 (programs only) */
} sq_op_type;

/* One operation: 12 bytes, three little-endian uint32. q1 is ignored by
 * single-qubit gates and measurements. */
typedef struct {
  uint32_t type;
  uint32_t q0;
  uint32_t q1;
} sq_op;

typedef struct sq_tableau sq_tableau;   /* opaque; owns its device memory */
typedef struct sq_program sq_program;   /* opaque; a compiled, device-resident circuit */

/* Message of the last failed call on this thread ("" if none). */
const char *sq_last_error(void);
/* Library version string. */
const char *sq_version(void);

/* Device bytes a tableau of n qubits needs (tableau plus working buffers),
 * for admission control and for sq_create_in. 0 if n is 0 or above
 * SQ_MAX_QUBITS. Host only.
 * Defined by: Algorithm alg:parallelSimulation, the allocation step (the
 * extended tableau of 2n rows, X and Z bits plus a sign per row, packed into
 * words of 64 bits), with the column-major layout of "Tableau Layout and
 * Indexing"; plus this library's measurement working buffers. */
#define SQ_MAX_QUBITS 1048576u
size_t sq_bytes_required(uint32_t n);

/* Where the tableau sits inside its device block (host only, no device work):
 * X is n columns of Ls words starting x_offset bytes into the block
 * (X[q * Ls + w], word w < K packs destabilizer rows 64w..64w+63, word K + w
 * stabilizer rows; bit b = row 64w + b), Z likewise at z_offset, and the L
 * sign words at r_offset. bytes = sq_bytes_required(n). Bits of rows >= n are
 * always 0. Errors: SQ_EINVAL (out NULL), SQ_ERANGE (n is 0 or too large).
 * Defined by: "Tableau Layout and Indexing" (column-major words over rows,
 * destabilizer half then stabilizer half of each column). */
typedef struct {
  uint32_t n, K, L, Ls;   /* K = ceil(n/64) words per half column, L = 2K, Ls = column stride in words */
  uint64_t x_offset, z_offset, r_offset, bytes;
} sq_layout_info;
sq_status sq_layout(uint32_t n, sq_layout_info *out);

/* Create a tableau of n qubits (1 <= n <= SQ_MAX_QUBITS) in |0...0> on the
 * current HIP device. hip_stream is a hipStream_t (NULL = default stream);
 * the caller keeps the stream alive for the handle's lifetime. The library
 * allocates the device block (stream-ordered) and frees it in sq_destroy.
 * Errors: SQ_EINVAL (out == NULL, n == 0), SQ_ERANGE (n too large),
 * SQ_ENOMEM, SQ_EDEVICE.
 * Defined by: Algorithm alg:parallelSimulation (allocation and tableau
 * initialisation); the initial extended tableau D_i = +X_i, S_i = +Z_i of
 * equation tableauFormat2 for the all-zero basis state. */
sq_status sq_create(uint32_t n, void *hip_stream, sq_tableau **out);
/* As sq_create, but the tableau lives in a device block the caller owns
 * (for instance a torch tensor's storage): dev_buf, 256-byte aligned, of
 * `bytes` >= sq_bytes_required(n) bytes on the current device. The block must
 * stay allocated until sq_destroy returns; the library never frees it, and the
 * caller must not write it while the handle lives (reading it, e.g. through
 * the offsets of sq_layout, is fine between the handle's synchronizing
 * calls). Calls that need per-call scratch (sq_measure's outcome buffer,
 * sq_sample's workspace, sq_apply_gates' pass records) still allocate it
 * stream-ordered. Errors: SQ_EINVAL (NULL, misaligned), SQ_ERANGE (n, or
 * bytes too small), SQ_EDEVICE.
 * Defined by: as sq_create. */
sq_status sq_create_in(uint32_t n, void *dev_buf, size_t bytes, void *hip_stream, sq_tableau **out);
/* Wait for the handle's work, then free it (and its device block unless it
 * came from sq_create_in). NULL is accepted. */
sq_status sq_destroy(sq_tableau *t);
/* Reset to |0...0> and clear the error flags (asynchronous).
 * Defined by: Algorithm alg:parallelSimulation, tableau initialisation. */
sq_status sq_reset(sq_tableau *t);
/* Block until all device work queued on the handle has finished. */
sq_status sq_sync(sq_tableau *t);

/* How measurements collapse the state, and with it what the sign bits mean.
 *
 * SQ_COLLAPSE_ROWSUM (default): the state tableau above, one sign per
 *   generator row; a random measurement multiplies every other row that
 *   anticommutes with Z_q by the pivot stabilizer (CHP rowsum), a
 *   deterministic one forms the destabilizer-selected product.
 *   Defined by: "The CHP algorithm" (probabilistic and deterministic cases).
 *
 * SQ_COLLAPSE_INJECT: the operator tableau of Algorithm alg:stim. For the
 *   circuit C applied so far, T = C^dagger maps X_q to A_q and Z_q to B_q,
 *   Pauli strings over generator positions k = 0..n-1 with one sign each.
 *   The bit matrices are exactly the state tableau's (row k of the
 *   stabilizer half holds the x part of every B_q and the x part of every
 *   A_q in X and Z, row k of the destabilizer half their z parts: the
 *   paper's XS, ZS, XD, ZD), so gates move the same bits; a gate changes
 *   the images' signs by the phases of image products. Measuring Z_q: the
 *   pivot p is the smallest position with x_q(S_p) = 1; if there is one,
 *   CX gates are injected from p into every later position t with
 *   x_q(S_t) = 1, position p is rotated (H, or the inverse phase gate when
 *   x_q(D_p) = 1 by then) and an X is injected at p when B_q's sign differs
 *   from the coin; the outcome is B_q's sign (the coin when random).
 *   Deterministic outcomes cost a pivot search only. Sign bytes of
 *   sq_export/sq_export_rows/sq_import mean: entry i < n the sign of A_i,
 *   entry n + i the sign of B_i. Outcomes, and the stabilizer group, equal
 *   the rowsum collapse's under the same coins; tableau bits differ.
 *   Defined by: Algorithm alg:stim (ProbabilisticMeasurement, GE,
 *   SwapAntiComm, InjectCX, InjectInvP, InjectHad, InjectX), with the
 *   prefix-XOR unfolding of the injection loop (equations CXSign, zc) and
 *   the target compaction of Algorithm alg:compactPivots.
 *   Not available in this mode: sq_sample, sq_sample_many (SQ_EINVAL).
 *
 * sq_set_collapse resets the tableau to |0...0> (where both readings agree)
 * in the chosen mode; sq_reset keeps the mode. Blocks until the reset is
 * queued; SQ_EINVAL for an unknown mode. */
typedef enum { SQ_COLLAPSE_ROWSUM = 0, SQ_COLLAPSE_INJECT = 1 } sq_collapse;
sq_status sq_set_collapse(sq_tableau *t, uint32_t mode);
uint32_t sq_get_collapse(const sq_tableau *t);  /* 0 for a NULL handle */

/* Memory layout of the tableau's bits (the dual layout of "Tableau Layout
 * and Indexing"; the switch is the tile-wise in-place transpose of
 * Algorithm alg:transpose, each 64 x 64 bit tile transposed in registers
 * and exchanged with its mirror, the same operation both ways).
 *
 * SQ_LAYOUT_COLUMNS (default): column-major, as described at sq_layout
 *   (X[q * Ls + w] packs 64 generator rows of qubit q).
 * SQ_LAYOUT_ROWS: row-contiguous: slot r (the same Ls-word stride) holds
 *   the generator pair r, words w < K the bits of D_r at qubits
 *   64w .. 64w+63, words K + w those of S_r; slots r >= n are zero (X and Z
 *   hold 64K slots in both layouts). Sign words are the same. Measurements
 *   (sq_measure, sq_run measurement segments) then touch whole rows: a
 *   random measurement reads and writes only the rows that anticommute with
 *   Z_q, a deterministic one reads only the stabilizer rows it multiplies
 *   (row-granular bytes), one measurement at a time.
 * Gate application (sq_apply_gates, program gate segments), sampling,
 * export and import switch back to columns first. Only with the rowsum
 * collapse (SQ_EINVAL otherwise). Results are identical in both layouts.
 * Queues the transpose (if the layout changes) on the handle's stream.
 * Defined by: "Tableau Layout and Indexing" (row-major layout for
 * measurement), Algorithm alg:transpose. */
typedef enum { SQ_LAYOUT_COLUMNS = 0, SQ_LAYOUT_ROWS = 1 } sq_layout_kind;
sq_status sq_set_layout(sq_tableau *t, uint32_t layout);
uint32_t sq_get_layout(const sq_tableau *t);  /* 0 for a NULL handle */
uint32_t sq_num_qubits(const sq_tableau *t);

/* Apply gates (host array, program order) to every row. Qubits may repeat:
 * the library groups the sequence into passes of disjoint groups of up to 8
 * qubits and applies each pass in one fused launch. Lists of 2^20 gates or
 * more are grouped in consecutive chunks of 2^19 gates on up to 8 host
 * threads, the chunks' passes following each other. Asynchronous with
 * respect to the device (the host array may be reused on return).
 * Errors: SQ_EINVAL (NULL ops with count > 0, type not a gate, CX/CZ with
 * q0 == q1), SQ_ERANGE (qubit >= n). */
sq_status sq_apply_gates(sq_tableau *t, const sq_op *host_ops, uint64_t count);
/*   Defined by: equation update_rules (H, S = P, CX applied column-wise to
 *   every row, right-hand sides taken before the update), the other gates by
 *   conjugation; fused application of disjoint gates from "Tableau Evolution
 *   under Clifford Gates" (Algorithm alg:buildTableau) and the scheduling of
 *   "Parallel Gate and Measurement Scheduling on CPU". */

/* Measure Z on host_qubits[0..count) in that order (measurement index
 * meas_base + i for the i-th), updating the tableau after each. With
 * tuning.meas_block = k > 1, runs of consecutive random measurements are
 * applied up to k at a time in one pass over the tableau (bit-identical to
 * one at a time). The list is copied to the device and swept by kernels that
 * keep their position in device memory: the host queues one group of
 * launches per k measurements and reads the position back once at the end
 * (again only when deterministic measurements cut blocks short). Writes the
 * outcome bits (0/1) to host_out_bits[0..count) and, if host_out_random is
 * not NULL, 1/0 for random/deterministic outcomes. Blocks until written.
 * Scratch: 6 bytes per measured qubit, allocated stream-ordered and kept by
 * the handle for later calls.
 * Errors: SQ_EINVAL, SQ_ERANGE (qubit >= n), SQ_ENOMEM, SQ_ESTATE (a device
 * check failed, see sq_error_flags; the tableau is then unreliable). */
sq_status sq_measure(sq_tableau *t, const uint32_t *host_qubits, uint32_t count,
                     uint64_t seed, uint64_t shot, uint64_t meas_base,
                     uint8_t *host_out_bits, uint8_t *host_out_random);
/*   Defined by: "Measurements in the Stabilizer Formalism" (equation
 *   eq:meastab: random iff some stabilizer anticommutes with Z_q) and "The CHP
 *   algorithm" (probabilistic case: smallest pivot, every other anticommuting
 *   row times the pivot, D_p <- S_p, S_p <- (-1)^coin Z_q; deterministic case:
 *   the product of the stabilizers the destabilizers select). */

/* sq_measure without device allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same arguments, semantics, ordering
 * and errors as sq_measure, but the measured list and the outcome bytes are
 * staged in a fixed device array compiled into the library (6 bytes per
 * measurement, SQ_NOALLOC_MAX_MEAS measurements: 6 MiB per device, held
 * until the process ends) instead of buffers the handle allocates. Pair it
 * with sq_create_in for a tableau in caller-owned memory. count above
 * SQ_NOALLOC_MAX_MEAS: SQ_ERANGE, nothing done. Calls on one device share
 * the array; the library serializes them (each returns only after its
 * stream has finished with the array). Blocks. */
#define SQ_NOALLOC_MAX_MEAS 1048576u
sq_status sq_measure_noalloc(sq_tableau *t, const uint32_t *host_qubits, uint32_t count, uint64_t seed,
                             uint64_t shot, uint64_t meas_base, uint8_t *out_bits, uint8_t *out_random);

/* Sample `shots` shots of measuring host_qubits[0..count) (in that order) on
 * the current state, without changing the tableau. Shot s (0 <= s < shots)
 * is exactly the outcome string sq_measure would return on a copy of the
 * tableau with shot number shot_begin + s, the same seed and measurement
 * indices meas_base + i (the shots of the paper's sampling workload, drawn
 * with the per-shot CHP semantics). Output: host_out[s * W + i/64] bit i%64,
 * W = ceil(count/64), bits past count zero. Blocks.
 * Work: one measurement sweep on a scratch copy in which stabilizer signs are
 * tracked as affine functions of the coins, then one parity per outcome and
 * shot. Scratch: about sq_bytes_required(n) plus (count+1)*ceil(n/64)*8 and
 * count*W*8 bytes, allocated for the call.
 * Errors: SQ_EINVAL, SQ_ERANGE (qubit >= n), SQ_ENOMEM, SQ_ESTATE. */
sq_status sq_sample(sq_tableau *t, const uint32_t *host_qubits, uint32_t count, uint64_t seed, uint64_t shot_begin,
                    uint32_t shots, uint64_t meas_base, uint64_t *host_out);
/*   Defined by: the many-shot workload of the "Sampling" section, each shot
 *   with the per-shot semantics of "The CHP algorithm". */

/* Several shot sets of the same measured list on the current state, sharing
 * one measurement sweep (which depends on the list, not on the coins): set k
 * gives exactly what sq_sample(t, host_qubits, count, sets[k].seed,
 * sets[k].shot_begin, sets[k].shots, sets[k].meas_base, sets[k].out) gives.
 * The tableau is unchanged. Scratch as sq_sample with the largest set's shot
 * count (sq_sample_bytes). Blocks. Errors as sq_sample.
 * Defined by: as sq_sample. */
typedef struct {
  uint64_t seed, shot_begin, meas_base;
  uint32_t shots, pad;
  uint64_t *out;   /* host, shots * ceil(count/64) words */
} sq_shot_set;
sq_status sq_sample_many(sq_tableau *t, const uint32_t *host_qubits, uint32_t count, const sq_shot_set *sets,
                         uint32_t nsets);
/* Device scratch bytes sq_sample (and sq_sample_many) allocate for a tableau
 * of n qubits, count measured qubits and `shots` shots. Host only; 0 for n
 * out of range. */
size_t sq_sample_bytes(uint32_t n, uint32_t count, uint32_t shots);

/* Batched sampling of many independent circuits (the batched/served
 * workload: circuits of uneven size, each with its own shot count).
 * Item k is, bit for bit, the result of sq_create(n), sq_apply_gates(ops),
 * sq_sample(qubits, count, seed, shot_begin, shots, meas_base, out),
 * sq_destroy. Circuits up to opts->max_batch_n qubits (and at most 16384
 * qubits, fewer than 32768 measurements) run in one persistent launch in
 * which a workgroup takes one circuit at a time, largest first, and runs its
 * gates, measurement sweep and shots without further launches; larger
 * circuits run through the single-tableau kernels, several at once on worker
 * threads with streams of their own, concurrently with that launch. Blocks
 * until every output is written. opts may be NULL (automatic choices).
 * Errors: SQ_EINVAL, SQ_ERANGE, SQ_ENOMEM, SQ_EDEVICE, SQ_ESTATE (a device
 * consistency check of some item failed). */
typedef struct {
  uint32_t n;
  const sq_op *ops;        /* gates only, program order */
  uint64_t nops;
  const uint32_t *qubits;  /* measured list, in order */
  uint32_t count;
  uint32_t shots;
  uint64_t seed;
  uint64_t shot_begin;
  uint64_t meas_base;
  uint64_t *out;           /* host, shots * ceil(count/64) words */
} sq_batch_item;

typedef struct {
  uint32_t block;        /* threads per workgroup of the batched kernel (multiple of 64, <= 512; 0 = automatic) */
  uint32_t grid;         /* workgroups of the persistent launch (0 = automatic) */
  uint32_t max_batch_n;  /* larger circuits take the single-tableau path (0 = automatic: 1024) */
  uint32_t streams;      /* concurrent streams (host worker threads) for those (0 = automatic: 8) */
} sq_batch_opts;

sq_status sq_batch_sample(const sq_batch_item *items, uint32_t nitems, const sq_batch_opts *opts, void *hip_stream);
/*   Defined by: as sq_sample, per item (the batching itself is this
 *   library's; the paper runs one circuit at a time). */

/* Device bytes sq_batch_sample holds for one item of n qubits, nops gates,
 * count measured qubits and `shots` shots while it runs, routed as
 * sq_batch_sample routes it under opts (NULL = automatic): the persistent
 * launch's working set, or for larger items a tableau (sq_bytes_required),
 * sq_sample's workspace and the compiled gate records (counted at their
 * upper bound, 20 bytes per gate). 0 for an item with no measurement or no
 * shot (it takes no device memory) and for n out of range. Host only. For
 * admission control. */
size_t sq_batch_item_bytes(uint32_t n, uint64_t nops, uint32_t count, uint32_t shots, const sq_batch_opts *opts);

/* Compile a circuit of n qubits (gates and SQ_MEASURE records in program
 * order) into a device-resident program on the current device.
 * Errors as sq_apply_gates, plus SQ_ENOMEM. */
sq_status sq_program_create(uint32_t n, const sq_op *host_ops, uint64_t count, sq_program **out);
/*   Defined by: Algorithm alg:parallelSimulation (the circuit scheduled into
 *   gate windows and measurements, copied to the device) and "Parallel Gate
 *   and Measurement Scheduling on CPU". */
sq_status sq_program_destroy(sq_program *p);
uint64_t sq_program_num_measurements(const sq_program *p);
uint64_t sq_program_num_gates(const sq_program *p);
/* Number of fused gate passes the program launches. */
uint64_t sq_program_num_passes(const sq_program *p);

/* Many-shot sampling by Pauli frames (the paper's sampling mode): shots of
 * program p (gates and measurements from |0...0>) without a tableau per shot.
 * host_ref holds one reference outcome (0 or 1) per measurement of p, e.g.
 * the outcomes sq_run gives for some seed and shot. Per shot a frame (x and z
 * bits over the qubits) starts at x = 0 with z drawn at random and is
 * conjugated by every gate; measuring qubit q gives host_ref[i] XOR x_q and
 * draws z_q afresh. Random words: Philox4x64-10, key (seed, 2^63 + w) and
 * counter (e, 0, 0, 0), bit b for shot 64 w + b; event e = q initialises
 * z_q, e = n + i re-draws it after measurement i. The outcomes follow the
 * circuit's distribution (each shot a sample) but are not the per-shot CHP
 * outcomes of sq_sample. Output: host_out[s * W + i/64] bit i%64,
 * W = ceil(M/64), bits past M zero. Runs on hip_stream (NULL = default) in
 * stream-ordered scratch (about 2 n * ceil(shots/64) words of frames plus
 * records); blocks. Errors: SQ_EINVAL (NULL, reference not 0/1, program of
 * another device), SQ_ENOMEM, SQ_EDEVICE. */
sq_status sq_frame_sample(const sq_program *p, const uint8_t *host_ref, uint64_t seed, uint32_t shots,
                          uint64_t *host_out, void *hip_stream);
/*   Defined by: the "Sampling" section, Algorithm alg:sampling (frames
 *   initialised with random Z bits, conjugated by the gates, the x bit
 *   recorded and z re-drawn at each measurement), read with the reference
 *   sample XOR-ed in. */

/* Read an OpenQASM 2.0 circuit (host only, no device work) into operation
 * records for sq_program_create / sq_apply_gates. Accepted: the version line,
 * include lines (ignored), qreg/creg declarations, the gates id, x, y, z, h,
 * s, sdg, cx (and CX), cy, cz, swap, iswap on qubits or whole registers
 * (broadcast over registers of equal size), parameterless gate definitions
 * built from these (expanded at each call; a definition of a known gate name
 * keeps the built-in), measure (qubit or whole register; outcomes come in
 * program order, the classical target is not recorded), barrier (ignored)
 * and // comments. Qubits of several registers are numbered in declaration
 * order. text: len bytes, not necessarily NUL-terminated. Writes up to cap
 * records to host_ops, the number of records to *count and the qubit count
 * to *n (call with cap = 0 to size the buffer).
 * Errors: SQ_EINVAL for anything else (parameters, reset, if, opaque, U,
 * unknown names, bad indices, syntax), with the line in sq_last_error(). */
sq_status sq_qasm_parse(const char *text, size_t len, sq_op *host_ops, uint64_t cap, uint64_t *count, uint32_t *n);
/*   Defined by: the Experiments section (benchmarks given as OpenQASM files
 *   over the gate set X, Y, Z, H, P, P^dagger, CX, CY, CZ, SWAP, iSWAP). */

/* Host-only inspection of how a gate sequence is grouped into passes (no
 * device work; usable without a GPU). A pass holds groups on pairwise
 * disjoint qubit sets, each of at most 8 qubits and 32 micro-ops. Writes, per
 * pass, one word with its group count, then per group: a header word
 * (bits 0..3 qubit count nq, bits 4..9 micro-op count m, bits 16..23 and
 * 24..31 per-slot flags of the x and z columns the group changes), nq words
 * with the qubit of each slot, and m words with one micro-op each: bits 0..3
 * the gate (1 H, 2 S, 3 S^dagger, 4 X, 5 Y, 6 Z, 7 CX, 8 CZ, 9 SWAP), bits
 * 4..7 its (control) slot, bits 8..11 the target slot of CX / other slot of
 * CZ and SWAP. CY and iSWAP appear as their products (S^dagger, CX, S and
 * S, S, CZ, SWAP).
 * *out_len receives the number of words needed; nothing is written past cap.
 * Errors as sq_apply_gates. */
sq_status sq_plan_gates(uint32_t n, const sq_op *host_ops, uint64_t count, uint64_t *out, uint64_t cap,
                        uint64_t *out_len);
/*   Defined by: "Parallel Gate and Measurement Scheduling on CPU" (gates on
 *   disjoint qubits grouped so they can be applied together). */

/* Run a program on a tableau of the same n. All work is queued on the
 * handle's stream; the call returns once the last measurement segment's
 * sweep has been queued and its position read back (one 4-byte read per
 * measurement segment, so the call waits for the work before it), with any
 * gate segment after it queued asynchronously. Outcome i (i-th measurement
 * of the program, index meas_base + i) is written to dev_out_bits[i] and, if
 * not NULL, dev_out_random[i]; both are device buffers of
 * sq_program_num_measurements bytes that must stay valid until the stream
 * reaches that point.
 * From the second run of a program on a tableau, each of its gate segments
 * (the gate passes between two measurement runs) is launched as one HIP graph,
 * captured on that run under the launch geometry then in force (see
 * sq_set_graphs). Errors: SQ_EINVAL (NULL, n mismatch). */
sq_status sq_run(sq_tableau *t, const sq_program *p, uint64_t seed, uint64_t shot, uint64_t meas_base,
                 uint8_t *dev_out_bits, uint8_t *dev_out_random);
/*   Defined by: Algorithm alg:parallelSimulation (the simulation loop over
 *   windows: gate windows applied on the device, measurement windows
 *   dispatched to the measurement procedure), with "The CHP algorithm" for
 *   the measurements. */

/* Graph replay of program gate segments (sq_run). A tableau keeps the
 * instantiated graphs of the last 32 (program, segment, launch geometry)
 * triples it ran, captured on a private stream and launched on its own; a
 * segment run for the first time, or while kernel timing is on, is launched
 * kernel by kernel. on = 0 launches every segment kernel by kernel and frees
 * the graphs (after waiting for the handle's queued work), on = 1 (the
 * default) turns replay back on. Dropping the oldest graph when a 33rd is
 * captured also waits for the handle's queued work. Graphs of a destroyed
 * program are never launched again (programs carry a unique id). */
sq_status sq_set_graphs(sq_tableau *t, int on);
/* Counts since the tableau was created: segments captured as graphs and graph
 * launches. */
sq_status sq_graph_stats(const sq_tableau *t, uint64_t *captures, uint64_t *replays);

/* Copy rows out in canonical row-major form: for the k-th requested global
 * row g (0 <= g < 2n), host_x[k*W + j/64] bit j%64 = x_gj (W = ceil(n/64)),
 * likewise host_z, and host_r[k] = r_g. Blocks. */
sq_status sq_export_rows(sq_tableau *t, const uint32_t *host_rows, uint32_t nrows,
                         uint64_t *host_x, uint64_t *host_z, uint8_t *host_r);
/* All 2n rows (host_x, host_z: 2n*W words; host_r: 2n bytes). Blocks.
 * Defined by (sq_export_rows, sq_export, sq_import): the row form of the
 * extended tableau, equation tableauFormat2. */
sq_status sq_export(sq_tableau *t, uint64_t *host_x, uint64_t *host_z, uint8_t *host_r);
/* Replace the whole tableau from the canonical row-major form (bits at
 * positions >= n in the last word of a row must be 0). Blocks. */
sq_status sq_import(sq_tableau *t, const uint64_t *host_x, const uint64_t *host_z, const uint8_t *host_r);

/* Byte accounting of the measurements run since creation or reset: counts
 * of random and deterministic outcomes, and the algorithmic bytes of their
 * passes. Rowsum: for every row word holding an anticommuting row, read x and
 * z of each non-identity column of the pivot row and write x (where the pivot
 * has x) and z (where it has z). Deterministic: read x and z of every column
 * at each word holding a destabilizer that anticommutes with Z_q. Blocks. */
typedef struct {
  uint64_t n_random;
  uint64_t n_det;
  uint64_t rowsum_bytes;
  uint64_t det_bytes;
  uint64_t blocks;        /* blocked passes (each applying several random measurements) */
  uint64_t block_bytes;   /* algorithmic bytes of the blocked passes */
  uint64_t inject_bytes;  /* CX-injection collapse: per column, read the destabilizer words of x and z at each
                             word holding a target, and read and write the stabilizer word of x (z) there
                             where the pivot has x (z) */
} sq_meas_stats;
sq_status sq_measure_stats(sq_tableau *t, sq_meas_stats *out);
/*   (Accounting of this library; no passage of the paper.) */

/* Algorithmic bytes of all gate passes of a program: per group, read x and z
 * of its one or two columns and write the columns its gates change (the
 * sign column, 2*L words per pass, is not counted). */
uint64_t sq_program_gate_bytes(const sq_program *p);

/* Device-side consistency flags accumulated since creation or reset
 * (bit 0: a rowsum phase exponent was odd; bit 1: a deterministic product was
 * not +-Z_q; bit 2: the blocked pivot step judged a measurement deterministic
 * that the single pivot search found random). Blocks. */
sq_status sq_error_flags(sq_tableau *t, uint32_t *flags);
/*   Defined by: the CHP invariants of "The CHP algorithm" (products of
 *   commuting generators are Hermitian, so phase exponents are even; the
 *   deterministic product equals +-Z_q). */

/* Launch geometry. 0 in a field keeps the current value. Block sizes must be
 * multiples of 64 in [64, 1024]; words per thread 1 or 2. */
typedef struct {
  uint32_t layer_block;        /* threads per workgroup of the gate-pass kernel */
  uint32_t layer_wpt;          /* tableau words per thread in the gate-pass kernel */
  uint32_t layer_groups;       /* gate groups per workgroup (per chunk) */
  uint32_t rowsum_block;       /* threads per workgroup of the rowsum kernel */
  uint32_t rowsum_wpt;         /* words per thread in the rowsum kernel */
  uint32_t rowsum_cols;        /* pivot-row columns per workgroup (per chunk) */
  uint32_t det_cols;           /* columns per workgroup of the deterministic-product phase */
  uint32_t meas_block;         /* sq_measure: random measurements per blocked pass (1 = one at a time, <= 32) */
  uint32_t pivot_waves;        /* blocked pivot search: SQ_PIVOT_AUTO (default: registers when the stabilizer
                                  half has at most 512 words, else tiles over up to 8 waves), or 1..16 =
                                  tiles over that many waves (at most 8) */
} sq_tuning;
#define SQ_PIVOT_AUTO 255u
/* (Launch control of this library; no passage of the paper. Shapes never
 * change results.) */
sq_status sq_get_tuning(const sq_tableau *t, sq_tuning *out);
sq_status sq_set_tuning(sq_tableau *t, const sq_tuning *in);

/* Per-kernel timing with HIP events recorded on the handle's stream around
 * every launch while enabled. Kernel ids: */
enum {
  SQ_K_LAYER = 0,   /* gate pass */
  SQ_K_SIGNS = 1,   /* sign reduction after a gate pass */
  SQ_K_PIVOT = 2,   /* pivot search (one per measurement) */
  SQ_K_GATHER = 3,  /* pivot-row gather */
  SQ_K_ROWSUM = 4,  /* rowsum pass */
  SQ_K_POST = 5,    /* random-case finalisation or deterministic product */
  SQ_K_BPIVOT = 6,  /* blocked measurements: snapshot and sequential pivot step */
  SQ_K_BPREP = 7,   /* blocked measurements: pivot rows and their algebra */
  SQ_K_BPASS = 8,   /* blocked measurements: the streaming pass */
  SQ_K_BFINAL = 9,  /* blocked measurements: signs and pivot rows */
  SQ_K_IPIVOT = 10, /* CX-injection collapse: pivot, target compaction, column q's decisions */
  SQ_K_IAPPLY = 11, /* CX-injection collapse: injections, rotation and X injection on every column */
  SQ_K_TRANSPOSE = 12, /* layout switch: tile transpose of X and Z */
  SQ_K_RPREP = 13,  /* row layout: pivot search and pivot-row copy */
  SQ_K_RROWSUM = 14, /* row layout: rows times the pivot */
  SQ_K_RDET = 15,   /* row layout: deterministic product (block partials and their cross terms) */
  SQ_K_RFINISH = 16, /* row layout: pivot rows, outcome */
  SQ_K_COUNT = 17
};
/* (Profiling of this library; no passage of the paper.) */
sq_status sq_profile_enable(sq_tableau *t, int on);
/* Sum of kernel durations (ms) and launch count for one kernel id since the
 * last sq_profile_reset. Blocks. */
sq_status sq_profile_read(sq_tableau *t, int kernel, double *total_ms, uint64_t *launches);
sq_status sq_profile_reset(sq_tableau *t);

#ifdef __cplusplus
}
#endif
#endif /* LIBSQ_SQ_H_ */
