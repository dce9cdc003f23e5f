// Host runtime behind the C ABI declared in include/sq.h: tableau handles,
// the gate-pass compiler, launch geometry, profiling and error handling.
#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <utility>
#include <vector>

#include "../../include/sq.h"
#include "sq_internal.h"
#include "sq_plan.h"

using namespace sq;

namespace {

thread_local std::string g_err;

sq_status fail(sq_status code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

}  // namespace

// Lets the other host files of the library (the OpenQASM reader) report
// through sq_last_error.
void sq_set_error_message(const char *msg) { g_err = msg ? msg : ""; }

namespace {

#define HIP_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) return fail(SQ_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));   \
  } while (0)

constexpr u32 kMaxChunks = 2048;  // per-launch cap on gate-group and column chunks
constexpr u32 kBlkMaxChunks = 512;  // column chunks of the blocked-measurement pass

inline u32 cdiv(u64 a, u64 b) { return (u32)((a + b - 1) / b); }
inline u32 round_up(u32 a, u32 b) { return (a + b - 1) / b * b; }

bool is_gate(u32 t) { return t <= SQ_ISWAP; }

sq_status validate_ops(u32 n, const sq_op *ops, u64 count, bool allow_measure) {
  if (count && !ops) return fail(SQ_EINVAL, "ops is NULL with count %llu", (unsigned long long)count);
  for (u64 i = 0; i < count; ++i) {
    const sq_op &o = ops[i];
    if (o.type == SQ_MEASURE) {
      if (!allow_measure) return fail(SQ_EINVAL, "op %llu: measurement not allowed here", (unsigned long long)i);
      if (o.q0 >= n) return fail(SQ_ERANGE, "op %llu: qubit %u >= n=%u", (unsigned long long)i, o.q0, n);
      continue;
    }
    if (!is_gate(o.type)) return fail(SQ_EINVAL, "op %llu: unknown type %u", (unsigned long long)i, o.type);
    if (o.q0 >= n) return fail(SQ_ERANGE, "op %llu: qubit %u >= n=%u", (unsigned long long)i, o.q0, n);
    if (is_two_qubit(o.type)) {
      if (o.q1 >= n) return fail(SQ_ERANGE, "op %llu: qubit %u >= n=%u", (unsigned long long)i, o.q1, n);
      if (o.q1 == o.q0) return fail(SQ_EINVAL, "op %llu: two-qubit gate on qubit %u twice", (unsigned long long)i, o.q0);
    }
  }
  return SQ_OK;
}

struct Dims {
  u32 n, K, L, Ls;
};

Dims dims_of(u32 n) {
  Dims d;
  d.n = n;
  d.K = cdiv(n, 64);
  d.L = 2 * d.K;
  d.Ls = round_up(d.L, 16);
  return d;
}

}  // namespace

// ----------------------------------------------------------------------------
struct sq_tableau {
  int device = 0;
  hipStream_t stream = nullptr;
  Dims d{};
  TabDev t{};
  u64 *base = nullptr;      // one device block for every device buffer below
  bool owns_base = true;    // false for sq_create_in: the caller's block
  u64 *mask = nullptr, *pivx = nullptr, *pivz = nullptr, *cnt0 = nullptr, *cnt1 = nullptr, *sign_part = nullptr;
  u32 *cols = nullptr;
  MeasState *st = nullptr;
  MeasStats *stats = nullptr;
  BlkBuffers blk{};
  u32 blk_cpc = 0;
  Cursor *cur = nullptr;      // where the current measurement sweep stands (device)
  u32 *cur_host = nullptr;    // pinned: the sweep's list position, read back once per round of slots
  uint8_t *dev_out = nullptr;  // sq_measure: outcome and random-flag bytes
  size_t dev_out_cap = 0;
  u32 *dev_q = nullptr;        // sq_measure: the measured list on the device
  size_t dev_q_cap = 0;
  u32 *dev_words = nullptr;  // gate-pass records of the last sq_apply_gates call
  size_t dev_words_cap = 0;
  u32 *dev_offs = nullptr;
  size_t dev_offs_cap = 0;
  sq_tuning tun{};
  u32 collapse = SQ_COLLAPSE_ROWSUM;  // what the sign bits mean and how measurements collapse
  bool rows = false;                  // row-contiguous layout (sq_set_layout)
  WideBuilder builder;
  // program gate segments replayed as graphs, most recently used last
  struct SegGraph {
    u64 prog = 0, first = 0, count = 0;
    u32 layer_block = 0, layer_wpt = 0, layer_groups = 0, collapse = 0;
    hipGraphExec_t exec = nullptr;  // null until the segment's second run
  };
  std::vector<SegGraph> graphs;
  hipStream_t cap_stream = nullptr;
  bool use_graphs = true;
  uint64_t graph_captures = 0, graph_replays = 0;
  // profiling
  bool prof = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[SQ_K_COUNT];
  std::vector<hipEvent_t> pool;
  double ms[SQ_K_COUNT] = {};
  uint64_t launches[SQ_K_COUNT] = {};
};

struct sq_program {
  u64 uid = 0;  // unique per program created in this process
  int device = 0;
  u32 n = 0;
  Dims d{};
  u32 *dev_words = nullptr;  // gate-pass records and their offsets, device resident
  u32 *dev_offs = nullptr;
  u32 *dev_meas = nullptr;   // the measured qubits in program order, device resident
  std::vector<PassRange> passes;
  struct Seg {
    int kind;  // 0 gate passes [first, first+count), 1 measurements [first, first+count)
    u64 first, count;
  };
  std::vector<Seg> segs;
  std::vector<u32> meas_qubits;
  u64 ngates = 0;
  u64 gate_bytes = 0;
};

namespace {

// Columns per chunk of the blocked pass: 8192 / (L / 256) chunks, so that
// late in a measurement sweep, when the stabilizer half's row words stop
// being hit and their tiles exit at once, the remaining tiles still have
// enough workgroups (at n = 180,000: 11 tiles of 512 row words x 372
// chunks).
static_assert(SQ_PIVOT_AUTO == PIVOT_AUTO, "pivot_waves sentinel");

u32 blk_cpc_of(const Dims &d) {
  const u32 tiles = cdiv(d.L, 256);
  const u32 want = std::max<u32>(1, 8192 / tiles);
  u32 cpc = std::max<u32>(16, cdiv(d.n, want));
  return std::max<u32>(cpc, cdiv(d.n, kBlkMaxChunks));
}

constexpr int kLayoutSlots = 20;

size_t layout_words(const Dims &d, size_t *off) {
  // offsets (in words) of: X, Z, R, mask, pivx, pivz, cnt0, cnt1, sign_part, cols, st, stats,
  // then the blocked-measurement buffers: bm, wpart, patx, patz, part, bs; then the sweep cursor
  size_t o = 0;
  auto take = [&](size_t words) {
    size_t r = o;
    o += (words + 31) / 32 * 32;  // 256-byte alignment
    return r;
  };
  // X and Z hold 64K column slots (K = ceil(n/64)): the row layout needs a
  // square 64K x 64K bit matrix per half; slots n .. 64K-1 stay zero
  off[0] = take((size_t)64 * d.K * d.Ls);
  off[1] = take((size_t)64 * d.K * d.Ls);
  off[2] = take(d.Ls);
  off[3] = take(d.Ls);
  off[4] = take(d.K);
  off[5] = take(d.K);
  off[6] = take((size_t)kMaxChunks * d.Ls);
  off[7] = take((size_t)kMaxChunks * d.Ls);
  off[8] = take((size_t)kMaxChunks * d.Ls);
  off[9] = take((d.n + 1) / 2);
  off[10] = take(sizeof(MeasState) / 8 + 1);
  off[11] = take(sizeof(MeasStats) / 8 + 1);
  off[12] = take((size_t)KB * d.Ls);
  off[13] = take((size_t)2 * KB * d.K);  // 4 * KB u32 per word
  off[14] = take((d.n + 1) / 2);
  off[15] = take((d.n + 1) / 2);
  off[16] = take((size_t)cdiv(d.n, blk_cpc_of(d)) * BLK_PART * d.Ls);
  off[17] = take(sizeof(BlkState) / 8 + 1);
  off[18] = take(sizeof(Cursor) / 8 + 1);
  off[19] = take((d.n + 1) / 2);  // supported-column list of a measurement block (n u32)
  return o;
}

void default_tuning(const Dims &d, sq_tuning *t) {
  t->layer_block = d.L >= 1024 ? 256 : 64;
  t->layer_wpt = d.L >= 512 ? 2 : 1;
  t->layer_groups = 0;  // automatic
  t->rowsum_block = d.L >= 1024 ? 256 : 64;
  t->rowsum_wpt = d.L >= 512 ? 2 : 1;
  t->rowsum_cols = 0;   // automatic
  t->det_cols = 0;      // automatic
  t->meas_block = KB;
  t->pivot_waves = SQ_PIVOT_AUTO;
}

u32 layer_gpc(const sq_tableau *T, u32 ngroups) {
  const u32 tiles = cdiv(T->d.L, (u64)T->tun.layer_block * T->tun.layer_wpt);
  u32 gpc = T->tun.layer_groups;
  if (gpc == 0) {
    // about 6,000 workgroups: several rounds over the chip, so the last
    // round's tail is short (measured on the MI355X at n = 180,000). A
    // workgroup applies its groups one after another, a memory round trip
    // each, so small passes get one group per workgroup.
    const u32 want_chunks = std::max<u32>(1, 6144 / tiles);
    gpc = cdiv(ngroups, want_chunks);
  }
  gpc = std::max<u32>(gpc, cdiv(ngroups, kMaxChunks));
  return std::max<u32>(gpc, 1);
}

u32 rowsum_cpc(const sq_tableau *T) {
  const u32 tiles = cdiv(T->d.L, (u64)T->tun.rowsum_block * T->tun.rowsum_wpt);
  u32 cpc = T->tun.rowsum_cols;
  if (cpc == 0) {
    const u32 want_chunks = std::max<u32>(1, 2048 / tiles);
    cpc = std::max<u32>(16, cdiv(T->d.n, want_chunks));
  }
  cpc = std::max<u32>(cpc, cdiv(T->d.n, kMaxChunks));
  return std::max<u32>(cpc, 1);
}

u32 det_cpw(const sq_tableau *T) {
  if (T->tun.det_cols) return T->tun.det_cols;
  return std::max<u32>(4, cdiv(T->d.n, 2048));  // 2048 workgroups of 4 waves at most
}

hipEvent_t take_event(sq_tableau *T) {
  if (!T->pool.empty()) {
    hipEvent_t e = T->pool.back();
    T->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Launch `fn` (returning hipError_t), bracketed by events when profiling.
template <class F>
sq_status timed(sq_tableau *T, int kid, F &&fn) {
  hipEvent_t a = nullptr, b = nullptr;
  if (T->prof) {
    a = take_event(T);
    b = take_event(T);
    if (a && b) HIP_TRY(hipEventRecord(a, T->stream));
  }
  const hipError_t e = fn();
  if (e != hipSuccess) return fail(SQ_EDEVICE, "kernel %d launch: %s", kid, hipGetErrorString(e));
  if (T->prof && a && b) {
    HIP_TRY(hipEventRecord(b, T->stream));
    T->pending[kid].emplace_back(a, b);
  }
  return SQ_OK;
}

sq_status collect_profile(sq_tableau *T) {
  HIP_TRY(hipStreamSynchronize(T->stream));
  for (int k = 0; k < SQ_K_COUNT; ++k) {
    for (auto &pr : T->pending[k]) {
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, pr.first, pr.second));
      T->ms[k] += ms;
      T->launches[k] += 1;
      T->pool.push_back(pr.first);
      T->pool.push_back(pr.second);
    }
    T->pending[k].clear();
  }
  return SQ_OK;
}

#define SQ_TRY(expr)                 \
  do {                               \
    sq_status s_ = (expr);           \
    if (s_ != SQ_OK) return s_;      \
  } while (0)

// Operator-tableau gate pass (k_layer_op): a thread per position word, the
// workgroup size 64 for K <= 64 words, else 256; about 6,000 workgroups per
// pass as for k_layer; its per-wave phase counters (16 bytes per group and
// wave) live in the sign_part buffer, which bounds the groups per launch.
struct OpGeom {
  u32 block, gpc, max_groups;
};
OpGeom layer_op_geom(const sq_tableau *T, u32 ngroups) {
  OpGeom g;
  g.block = T->d.K <= 64 ? 64 : 256;
  const u32 tiles = cdiv(T->d.K, g.block);
  const u32 nw = tiles * (g.block / 64);
  g.gpc = T->tun.layer_groups ? T->tun.layer_groups : cdiv(ngroups, std::max<u32>(1, 6144 / tiles));
  g.gpc = std::max<u32>(g.gpc, 1);
  g.max_groups = (u32)std::min<size_t>((size_t)kMaxChunks * T->d.Ls / 2 / nw, 1u << 30);
  return g;
}

sq_status run_passes_on(sq_tableau *T, hipStream_t stream, const u32 *dev_words, const u32 *dev_offs,
                        const std::vector<PassRange> &passes, size_t first, size_t count) {
  if (T->collapse == SQ_COLLAPSE_INJECT) {
    for (size_t i = first; i < first + count; ++i) {
      const PassRange &p = passes[i];
      const u32 *offs = dev_offs + p.offset;
      SQ_TRY(timed(T, SQ_K_LAYER, [&] {
        const OpGeom g = layer_op_geom(T, p.count);
        return launch_layer_op(T->t, dev_words, offs, p.count, g.block, g.gpc, g.max_groups, T->sign_part,
                               &T->st->flags, stream);
      }));
    }
    return SQ_OK;
  }
  for (size_t i = first; i < first + count; ++i) {
    const PassRange &p = passes[i];
    const u32 gpc = layer_gpc(T, p.count);
    const u32 chunks = cdiv(p.count, gpc);
    const u32 *offs = dev_offs + p.offset;
    SQ_TRY(timed(T, SQ_K_LAYER, [&] {
      return launch_layer(T->t, dev_words, offs, p.count, T->tun.layer_block, T->tun.layer_wpt, gpc, T->sign_part,
                          stream);
    }));
    SQ_TRY(timed(T, SQ_K_SIGNS, [&] { return launch_sign_reduce(T->t, T->sign_part, chunks, stream); }));
  }
  return SQ_OK;
}

sq_status run_passes(sq_tableau *T, const u32 *dev_words, const u32 *dev_offs, const std::vector<PassRange> &passes,
                     size_t first, size_t count) {
  return run_passes_on(T, T->stream, dev_words, dev_offs, passes, first, count);
}

// Row blocks of the row layout's deterministic product (partial XORs in cnt0
// and cnt1, which hold kMaxChunks rows of Ls words).
constexpr u32 kRowDetBlocks = 64;
static_assert(kRowDetBlocks <= kMaxChunks, "row-layout block sums must fit the chunk buffers");

// Switch the layout (the transpose is its own inverse).
sq_status set_rows(sq_tableau *T, bool rows) {
  if (T->rows == rows) return SQ_OK;
  SQ_TRY(timed(T, SQ_K_TRANSPOSE, [&] { return launch_transpose(T->t, T->stream); }));
  if (rows) HIP_TRY(launch_row_begin(T->st, T->stream));
  T->rows = rows;
  return SQ_OK;
}

constexpr size_t kMaxSegGraphs = 32;

// A program's gate segment: kernel by kernel on its first run (or while
// kernels are timed), captured as a graph on a private stream on its second
// run (capturing runs nothing, so the order of T's stream is unaffected; the
// null stream, which cannot be captured, is fine to launch on), then launched
// as that graph. The graph holds T's buffers and the program's records, both
// fixed for their lifetimes, and the launch geometry of the capture.
sq_status run_gate_segment(sq_tableau *T, const sq_program *P, u64 first, u64 count) {
  if (count) SQ_TRY(set_rows(T, false));  // gate passes work on columns
  if (!T->use_graphs || T->prof || count == 0)
    return run_passes(T, P->dev_words, P->dev_offs, P->passes, first, count);
  const sq_tuning &tn = T->tun;
  size_t i = 0;
  for (; i < T->graphs.size(); ++i) {
    const auto &g = T->graphs[i];
    if (g.prog == P->uid && g.first == first && g.count == count && g.layer_block == tn.layer_block &&
        g.layer_wpt == tn.layer_wpt && g.layer_groups == tn.layer_groups && g.collapse == T->collapse)
      break;
  }
  if (i == T->graphs.size()) {  // first run: remember it, launch kernel by kernel
    if (T->graphs.size() >= kMaxSegGraphs) {
      if (T->graphs.front().exec) {
        HIP_TRY(hipStreamSynchronize(T->stream));  // its last launch may still be queued
        (void)hipGraphExecDestroy(T->graphs.front().exec);
      }
      T->graphs.erase(T->graphs.begin());
    }
    sq_tableau::SegGraph g;
    g.prog = P->uid;
    g.first = first;
    g.count = count;
    g.layer_block = tn.layer_block;
    g.layer_wpt = tn.layer_wpt;
    g.layer_groups = tn.layer_groups;
    g.collapse = T->collapse;
    T->graphs.push_back(g);
    return run_passes(T, P->dev_words, P->dev_offs, P->passes, first, count);
  }
  std::rotate(T->graphs.begin() + i, T->graphs.begin() + i + 1, T->graphs.end());  // most recently used last
  sq_tableau::SegGraph &g = T->graphs.back();
  if (!g.exec) {
    if (!T->cap_stream) {
      hipStream_t cs = nullptr;
      if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) == hipSuccess) T->cap_stream = cs;
    }
    const bool ready =
        T->cap_stream && hipStreamBeginCapture(T->cap_stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (!ready) {  // no capture: this segment stays kernel by kernel
      (void)hipGetLastError();
      T->graphs.pop_back();
      return run_passes(T, P->dev_words, P->dev_offs, P->passes, first, count);
    }
    const sq_status st = run_passes_on(T, T->cap_stream, P->dev_words, P->dev_offs, P->passes, first, count);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(T->cap_stream, &graph);
    hipGraphExec_t ex = nullptr;
    hipError_t ei = hipErrorUnknown;
    if (st == SQ_OK && e == hipSuccess && graph) ei = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (st != SQ_OK) return st;
    if (ei != hipSuccess || !ex) {  // no graph: this segment stays kernel by kernel
      (void)hipGetLastError();
      T->graphs.pop_back();
      return run_passes(T, P->dev_words, P->dev_offs, P->passes, first, count);
    }
    g.exec = ex;
    ++T->graph_captures;
  }
  HIP_TRY(hipGraphLaunch(g.exec, T->stream));
  ++T->graph_replays;
  return SQ_OK;
}

// A measurement sweep over a device-resident list, driven by the cursor in
// device memory (Cursor). Its kernels are queued in slots that read the list
// position from the cursor and advance it, so nothing is read back per block:
//   meas_block == 1: a slot is pivot, gather, rowsum, post for list[i];
//   meas_block >= 2: a slot is the blocked path on list[i .. i + kb) (pivot
//   step, masks and pivot rows, pass, signs and special rows), then pivot and
//   post for the deterministic measurement that ended the block, if any
//   (their kernels exit at once otherwise, as do the blocked ones once the
//   list is done).
// Every slot advances the cursor by at least one measurement until the list
// is done. The host queues one slot per kb measurements, reads the position
// back (one 4-byte copy), and only when deterministic measurements cut blocks
// short queues more, sized from the measurements per slot seen so far.
// Workspace of sq_sample (byte offsets, 256-byte aligned): X and Z copies,
// sign columns, affine forms, coin and outcome words, the compacted coin
// columns, per-measurement kind and constant, the blocked sweep's zeroed sign
// words and pivot coefficients, a byte-count sink, and the measured list.
struct SampleWs {
  u32 Ks, CW;
  size_t o_x, o_z, o_sg, o_fm, o_cw, o_out, o_sv, o_kind, o_fc, o_cvec, o_svt, o_stats, o_q;
};

size_t sample_ws(const Dims &d, u32 count, u32 shots, SampleWs *L) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t r = off;
    off += (bytes + 255) / 256 * 256;
    return r;
  };
  L->Ks = round_up(d.K, 16);
  L->CW = cdiv(count, 64);
  L->o_x = take((size_t)d.n * d.Ls * 8);
  L->o_z = take((size_t)d.n * d.Ls * 8);
  L->o_sg = take((size_t)(count + 1) * L->Ks * 8);
  L->o_fm = take((size_t)count * L->CW * 8);
  L->o_cw = take((size_t)shots * L->CW * 8);
  L->o_out = take((size_t)shots * L->CW * 8);
  L->o_sv = take((size_t)(count + 1) * 4);
  L->o_kind = take(count);
  L->o_fc = take(count);
  L->o_cvec = take((size_t)d.Ls * 8);
  L->o_svt = take((size_t)(count + 1) * 4);
  L->o_stats = take(sizeof(MeasStats));
  L->o_q = take((size_t)count * 4);
  return off;
}

struct SweepCtx {
  TabDev tab;             // tableau the single path works on
  TabDev tabb;            // tableau of the blocked path (the sampler's has zeroed signs, cvec)
  const SymCtx *sym;      // sampler's symbolic signs, or NULL
  MeasStats *bstats;      // byte counters of the blocked path
  u64 *cvec;              // sampler: the blocked path's zeroed sign words, cleared per slot
  u32 *svt;               // sampler: per sign column, its coefficients in the block's pivots
};

sq_status queue_slot(sq_tableau *T, const SweepCtx &c, u32 kb) {
  if (T->rows) {
    SQ_TRY(timed(T, SQ_K_RPREP, [&] { return launch_row_prep(c.tab, T->cur, T->st, T->pivx, T->pivz, T->stream); }));
    SQ_TRY(timed(T, SQ_K_RROWSUM, [&] { return launch_row_rowsum(c.tab, T->st, T->pivx, T->pivz, T->stream); }));
    SQ_TRY(timed(T, SQ_K_RDET, [&] {
      return launch_row_det(c.tab, T->st, T->cnt0, T->cnt1, kRowDetBlocks, T->stream);
    }));
    SQ_TRY(timed(T, SQ_K_RFINISH, [&] {
      return launch_row_finish(c.tab, T->cur, T->st, T->pivx, T->pivz, T->stats, T->stream);
    }));
    return SQ_OK;
  }
  if (T->collapse == SQ_COLLAPSE_INJECT) {
    SQ_TRY(timed(T, SQ_K_IPIVOT, [&] {
      return launch_inj_pivot(c.tab, T->cur, T->st, T->mask, T->cols, T->stats, T->stream);
    }));
    // the pair's bit changes are staged one byte per column in cnt0 (unused in this mode)
    SQ_TRY(timed(T, SQ_K_IAPPLY, [&] {
      return launch_inj_apply(c.tab, T->st, T->mask, T->cols, reinterpret_cast<uint8_t *>(T->cnt0), T->stats,
                              T->stream);
    }));
    return SQ_OK;
  }
  if (kb <= 1) {
    const u32 cpc = rowsum_cpc(T);
    const u32 max_chunks = cdiv(T->d.n, cpc);
    SQ_TRY(timed(T, SQ_K_PIVOT,
                 [&] { return launch_pivot(c.tab, T->cur, T->st, T->mask, T->cols, T->pivx, T->stream); }));
    SQ_TRY(timed(T, SQ_K_GATHER, [&] {
      return launch_gather(c.tab, T->st, T->pivx, T->pivz, T->cols, c.sym, T->stream);
    }));
    SQ_TRY(timed(T, SQ_K_ROWSUM, [&] {
      return launch_rowsum(c.tab, T->mask, T->cols, T->st, T->cnt0, T->cnt1, T->tun.rowsum_block, T->tun.rowsum_wpt,
                           cpc, max_chunks, c.sym, T->stream);
    }));
    SQ_TRY(timed(T, SQ_K_POST, [&] {
      return launch_post(c.tab, T->cur, T->mask, T->pivx, T->pivz, T->cnt0, T->cnt1, T->cols, T->st, T->stats, cpc,
                         det_cpw(T), c.sym, T->stream);
    }));
    return SQ_OK;
  }
  SQ_TRY(timed(T, SQ_K_BPIVOT, [&] {
    return launch_blk_pivots(c.tabb, T->cur, T->blk, T->tun.pivot_waves, c.cvec, c.cvec ? T->d.Ls : 0u, T->stream);
  }));
  SQ_TRY(timed(T, SQ_K_BPREP, [&] { return launch_blk_prep(c.tabb, T->blk, T->stream); }));
  SQ_TRY(timed(T, SQ_K_BPASS, [&] { return launch_blk_pass(c.tabb, T->blk, T->blk_cpc, T->stream); }));
  SQ_TRY(timed(T, SQ_K_BFINAL, [&] {
    return launch_blk_final(c.tabb, T->blk, T->st, c.bstats, T->blk_cpc, c.sym ? c.sym->sg : nullptr,
                            c.sym ? c.sym->Ks : 0u, c.sym ? c.sym->count : 0u, c.svt, T->stream);
  }));
  if (c.sym) HIP_TRY(launch_blk_sv(c.sym->sg, c.sym->Ks, c.sym->count, T->blk, c.svt, c.cvec, T->d.Ls, T->d.K,
                                   T->stream));
  // the deterministic measurement that ended the block: its product only
  // (pivot search, mask snapshot, then the ordered product in k_post)
  const u32 cpc = rowsum_cpc(T);
  SQ_TRY(timed(T, SQ_K_PIVOT,
               [&] { return launch_pivot(c.tab, T->cur, T->st, T->mask, T->cols, T->pivx, T->stream); }));
  SQ_TRY(timed(T, SQ_K_POST, [&] {
    return launch_post(c.tab, T->cur, T->mask, T->pivx, T->pivz, T->cnt0, T->cnt1, T->cols, T->st, T->stats, cpc,
                       det_cpw(T), c.sym, T->stream);
  }));
  return SQ_OK;
}

// Measurements offered per slot: the CX-injection collapse takes one at a time.
u32 sweep_kb(const sq_tableau *T) {
  return (T->collapse == SQ_COLLAPSE_INJECT || T->rows) ? 1u : std::min<u32>(T->tun.meas_block, KB);
}

// Queue the sweep of a list of `count` measurements whose cursor has been
// initialised on T's stream, and wait until it is done.
sq_status run_sweep(sq_tableau *T, const SweepCtx &c, u32 count) {
  if (count == 0) return SQ_OK;
  const u32 kb = sweep_kb(T);
  u64 queued = 0;
  u64 slots = kb <= 1 ? count : cdiv(count, kb);
  for (;;) {
    for (u64 k = 0; k < slots; ++k) SQ_TRY(queue_slot(T, c, kb));
    queued += slots;
    HIP_TRY(hipMemcpyAsync(T->cur_host, &T->cur->i, sizeof(u32), hipMemcpyDeviceToHost, T->stream));
    HIP_TRY(hipStreamSynchronize(T->stream));
    const u32 pos = *T->cur_host;
    if (pos == count) return SQ_OK;
    if (pos > count || pos < queued) return fail(SQ_ESTATE, "measurement sweep: cursor at %u of %u after %llu slots",
                                                 pos, count, (unsigned long long)queued);
    const double per = std::max(1.0, (double)pos / (double)queued);  // measurements per slot so far
    slots = std::max<u64>(1, (u64)((double)(count - pos) / per));
  }
}

// Grow a stream-ordered u32 device buffer of the handle to hold `need` words.
sq_status ensure_capacity(sq_tableau *T, u32 **buf, size_t *cap, size_t need) {
  if (need <= *cap) return SQ_OK;
  if (*buf) (void)hipFreeAsync(*buf, T->stream);
  *buf = nullptr;
  *cap = 0;
  const size_t want = std::max<size_t>(need + need / 4, 4096);
  if (hipMallocAsync((void **)buf, want * 4, T->stream) != hipSuccess) {
    (void)hipGetLastError();
    return fail(SQ_ENOMEM, "device allocation of %zu gate-pass words failed", want);
  }
  *cap = want;
  return SQ_OK;
}

sq_status reset_device(sq_tableau *T) {
  T->rows = false;
  size_t off[kLayoutSlots];
  const size_t words = layout_words(T->d, off);
  HIP_TRY(launch_fill_zero(T->base, words, T->stream));
  HIP_TRY(launch_init_diag(T->t, T->stream));
  return SQ_OK;
}

sq_status check_tuning(const sq_tuning &t) {
  auto ok_block = [](u32 b, u32 hi) { return b >= 64 && b <= hi && b % 64 == 0; };
  if (!ok_block(t.layer_block, 512) || !ok_block(t.rowsum_block, 1024))
    return fail(SQ_EINVAL, "block sizes must be multiples of 64 in [64, 512] (gate pass), [64, 1024] (rowsum)");
  if ((t.layer_wpt != 1 && t.layer_wpt != 2) || (t.rowsum_wpt != 1 && t.rowsum_wpt != 2))
    return fail(SQ_EINVAL, "words per thread must be 1 or 2");
  if (t.meas_block < 1 || t.meas_block > KB) return fail(SQ_EINVAL, "meas_block must be in [1, %u]", KB);
  if (t.pivot_waves != SQ_PIVOT_AUTO && (t.pivot_waves < 1 || t.pivot_waves > 16))
    return fail(SQ_EINVAL, "pivot_waves must be in [1, 16] or SQ_PIVOT_AUTO");
  return SQ_OK;
}

}  // namespace

// ============================================================================
extern "C" {

const char *sq_last_error(void) { return g_err.c_str(); }
const char *sq_version(void) { return "sq 0.1 (gfx950)"; }

size_t sq_bytes_required(uint32_t n) {
  if (n == 0 || n > SQ_MAX_QUBITS) return 0;
  size_t off[kLayoutSlots];
  return layout_words(dims_of(n), off) * 8;
}

}  // extern "C"

namespace {

// sq_create / sq_create_in: dev_buf NULL allocates the device block
// (stream-ordered), else the caller's block of `bytes` bytes is used and never
// freed by the library.
sq_status create_tableau(uint32_t n, void *hip_stream, void *dev_buf, size_t bytes, sq_tableau **out) {
  if (!out) return fail(SQ_EINVAL, "out is NULL");
  *out = nullptr;
  if (n == 0) return fail(SQ_EINVAL, "n must be >= 1");
  if (n > SQ_MAX_QUBITS) return fail(SQ_ERANGE, "n=%u above the limit %u", n, SQ_MAX_QUBITS);
  const Dims d = dims_of(n);
  size_t off[kLayoutSlots];
  const size_t words = layout_words(d, off);
  if (dev_buf) {
    if (bytes < words * 8)
      return fail(SQ_ERANGE, "device buffer of %zu bytes, n=%u needs %zu (sq_bytes_required)", bytes, n, words * 8);
    if ((uintptr_t)dev_buf % 256)
      return fail(SQ_EINVAL, "device buffer must be 256-byte aligned");
  }
  sq_tableau *T = new (std::nothrow) sq_tableau();
  if (!T) return fail(SQ_ENOMEM, "host allocation failed");
  if (hipGetDevice(&T->device) != hipSuccess) {
    delete T;
    return fail(SQ_EDEVICE, "no HIP device");
  }
  T->stream = (hipStream_t)hip_stream;
  T->d = d;
  if (hipHostMalloc((void **)&T->cur_host, sizeof(u32), hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    delete T;
    return fail(SQ_ENOMEM, "pinned host allocation failed");
  }
  if (dev_buf) {
    T->base = (u64 *)dev_buf;
    T->owns_base = false;
  } else if (hipMallocAsync((void **)&T->base, words * 8, T->stream) != hipSuccess) {
    // stream-ordered allocation: no device-wide synchronization, so handles can
    // be created and destroyed while other streams keep working
    (void)hipGetLastError();
    (void)hipHostFree(T->cur_host);
    delete T;
    return fail(SQ_ENOMEM, "device allocation of %zu bytes failed", words * 8);
  }
  u64 *b = T->base;
  T->t = TabDev{b + off[0], b + off[1], b + off[2], T->d.n, T->d.K, T->d.L, T->d.Ls};
  T->mask = b + off[3];
  T->pivx = b + off[4];
  T->pivz = b + off[5];
  T->cnt0 = b + off[6];
  T->cnt1 = b + off[7];
  T->sign_part = b + off[8];
  T->cols = reinterpret_cast<u32 *>(b + off[9]);
  T->st = reinterpret_cast<MeasState *>(b + off[10]);
  T->stats = reinterpret_cast<MeasStats *>(b + off[11]);
  T->blk = BlkBuffers{b + off[12], reinterpret_cast<u32 *>(b + off[13]), reinterpret_cast<u32 *>(b + off[14]),
                      reinterpret_cast<u32 *>(b + off[15]), b + off[16], reinterpret_cast<BlkState *>(b + off[17]), reinterpret_cast<u32 *>(b + off[19])};
  T->cur = reinterpret_cast<Cursor *>(b + off[18]);
  T->blk_cpc = blk_cpc_of(T->d);
  default_tuning(T->d, &T->tun);
  T->builder.init(n, T->d.L);
  sq_status s = reset_device(T);
  if (s == SQ_OK && hipStreamSynchronize(T->stream) != hipSuccess) s = fail(SQ_EDEVICE, "initialisation failed");
  if (s != SQ_OK) {
    if (T->owns_base) (void)hipFreeAsync(T->base, T->stream);
    (void)hipStreamSynchronize(T->stream);
    (void)hipHostFree(T->cur_host);
    delete T;
    return s;
  }
  *out = T;
  return SQ_OK;
}

}  // namespace

extern "C" {

sq_status sq_create(uint32_t n, void *hip_stream, sq_tableau **out) {
  return create_tableau(n, hip_stream, nullptr, 0, out);
}

sq_status sq_create_in(uint32_t n, void *dev_buf, size_t bytes, void *hip_stream, sq_tableau **out) {
  if (!dev_buf) return fail(SQ_EINVAL, "dev_buf is NULL");
  return create_tableau(n, hip_stream, dev_buf, bytes, out);
}

sq_status sq_layout(uint32_t n, sq_layout_info *out) {
  if (!out) return fail(SQ_EINVAL, "out is NULL");
  if (n == 0 || n > SQ_MAX_QUBITS) return fail(SQ_ERANGE, "bad n=%u", n);
  const Dims d = dims_of(n);
  size_t off[kLayoutSlots];
  const size_t words = layout_words(d, off);
  out->n = n;
  out->K = d.K;
  out->L = d.L;
  out->Ls = d.Ls;
  out->x_offset = off[0] * 8;
  out->z_offset = off[1] * 8;
  out->r_offset = off[2] * 8;
  out->bytes = words * 8;
  return SQ_OK;
}

sq_status sq_destroy(sq_tableau *T) {
  if (!T) return SQ_OK;
  (void)hipStreamSynchronize(T->stream);
  for (int k = 0; k < SQ_K_COUNT; ++k)
    for (auto &pr : T->pending[k]) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
  for (hipEvent_t e : T->pool) (void)hipEventDestroy(e);
  for (auto &g : T->graphs)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (T->cap_stream) (void)hipStreamDestroy(T->cap_stream);
  if (T->dev_out) (void)hipFreeAsync(T->dev_out, T->stream);
  if (T->dev_q) (void)hipFreeAsync(T->dev_q, T->stream);
  if (T->dev_words) (void)hipFreeAsync(T->dev_words, T->stream);
  if (T->dev_offs) (void)hipFreeAsync(T->dev_offs, T->stream);
  if (T->owns_base) (void)hipFreeAsync(T->base, T->stream);
  (void)hipStreamSynchronize(T->stream);
  (void)hipHostFree(T->cur_host);
  delete T;
  return SQ_OK;
}

sq_status sq_reset(sq_tableau *T) {
  if (!T) return fail(SQ_EINVAL, "tableau is NULL");
  return reset_device(T);
}

sq_status sq_set_collapse(sq_tableau *T, uint32_t mode) {
  if (!T) return fail(SQ_EINVAL, "tableau is NULL");
  if (mode != SQ_COLLAPSE_ROWSUM && mode != SQ_COLLAPSE_INJECT) return fail(SQ_EINVAL, "unknown collapse mode %u", mode);
  T->collapse = mode;
  return reset_device(T);
}

uint32_t sq_get_collapse(const sq_tableau *T) { return T ? T->collapse : 0u; }

sq_status sq_set_layout(sq_tableau *T, uint32_t layout) {
  if (!T) return fail(SQ_EINVAL, "tableau is NULL");
  if (layout != SQ_LAYOUT_COLUMNS && layout != SQ_LAYOUT_ROWS) return fail(SQ_EINVAL, "unknown layout %u", layout);
  if (layout == SQ_LAYOUT_ROWS && T->collapse != SQ_COLLAPSE_ROWSUM)
    return fail(SQ_EINVAL, "the row layout serves the rowsum collapse only");
  return set_rows(T, layout == SQ_LAYOUT_ROWS);
}

uint32_t sq_get_layout(const sq_tableau *T) { return T && T->rows ? (uint32_t)SQ_LAYOUT_ROWS : 0u; }

sq_status sq_sync(sq_tableau *T) {
  if (!T) return fail(SQ_EINVAL, "tableau is NULL");
  HIP_TRY(hipStreamSynchronize(T->stream));
  return SQ_OK;
}

uint32_t sq_num_qubits(const sq_tableau *T) { return T ? T->d.n : 0; }

sq_status sq_apply_gates(sq_tableau *T, const sq_op *ops, uint64_t count) {
  if (!T) return fail(SQ_EINVAL, "tableau is NULL");
  SQ_TRY(validate_ops(T->d.n, ops, count, false));
  if (count == 0) return SQ_OK;
  SQ_TRY(set_rows(T, false));  // gate passes work on columns
  WideBuilder &pb = T->builder;
  plan_gate_list(T->d.n, T->d.L, ops, count, pb);
  if (pb.offs.empty()) return SQ_OK;
  SQ_TRY(ensure_capacity(T, &T->dev_words, &T->dev_words_cap, pb.words.size()));
  SQ_TRY(ensure_capacity(T, &T->dev_offs, &T->dev_offs_cap, pb.offs.size()));
  HIP_TRY(hipMemcpyAsync(T->dev_words, pb.words.data(), pb.words.size() * 4, hipMemcpyHostToDevice, T->stream));
  HIP_TRY(hipMemcpyAsync(T->dev_offs, pb.offs.data(), pb.offs.size() * 4, hipMemcpyHostToDevice, T->stream));
  return run_passes(T, T->dev_words, T->dev_offs, pb.passes, 0, pb.passes.size());
}

}  // extern "C"

namespace {

// The measurement of a host list through device buffers the caller provides:
// dq (count words) for the list, dout (2 * count bytes) for outcomes and
// random flags. Copies the list in, sweeps, copies the results out, checks
// the device flags.
sq_status measure_list(sq_tableau *T, const uint32_t *qubits, uint32_t count, uint64_t seed, uint64_t shot,
                       uint64_t meas_base, uint8_t *out_bits, uint8_t *out_random, u32 *dq, uint8_t *dout) {
  MeasState before{}, after{};
  HIP_TRY(hipMemcpyAsync(&before, T->st, sizeof(MeasState), hipMemcpyDeviceToHost, T->stream));
  HIP_TRY(hipMemcpyAsync(dq, qubits, (size_t)count * 4, hipMemcpyHostToDevice, T->stream));
  HIP_TRY(launch_cursor_init(T->cur, count, sweep_kb(T), seed, shot, meas_base, dq, dout, dout + count, T->stream));
  SQ_TRY(run_sweep(T, SweepCtx{T->t, T->t, nullptr, T->stats, nullptr, nullptr}, count));
  HIP_TRY(hipMemcpyAsync(out_bits, dout, count, hipMemcpyDeviceToHost, T->stream));
  if (out_random) HIP_TRY(hipMemcpyAsync(out_random, dout + count, count, hipMemcpyDeviceToHost, T->stream));
  HIP_TRY(hipMemcpyAsync(&after, T->st, sizeof(MeasState), hipMemcpyDeviceToHost, T->stream));
  HIP_TRY(hipStreamSynchronize(T->stream));
  if (after.flags != before.flags)
    return fail(SQ_ESTATE, "device consistency check failed (flags 0x%x)", after.flags);
  return SQ_OK;
}

sq_status check_measure_args(sq_tableau *T, const uint32_t *qubits, uint32_t count, uint8_t *out_bits) {
  if (!T) return fail(SQ_EINVAL, "tableau is NULL");
  if (count == 0) return SQ_OK;
  if (!qubits || !out_bits) return fail(SQ_EINVAL, "qubits/out_bits is NULL");
  for (u32 i = 0; i < count; ++i)
    if (qubits[i] >= T->d.n) return fail(SQ_ERANGE, "qubit %u >= n=%u", qubits[i], T->d.n);
  return SQ_OK;
}

}  // namespace

extern "C" {

sq_status sq_measure(sq_tableau *T, const uint32_t *qubits, uint32_t count, uint64_t seed, uint64_t shot,
                     uint64_t meas_base, uint8_t *out_bits, uint8_t *out_random) {
  SQ_TRY(check_measure_args(T, qubits, count, out_bits));
  if (count == 0) return SQ_OK;
  const size_t need = 2 * (size_t)count;
  if (need > T->dev_out_cap) {
    if (T->dev_out) (void)hipFreeAsync(T->dev_out, T->stream);
    T->dev_out = nullptr;
    T->dev_out_cap = 0;
    if (hipMallocAsync((void **)&T->dev_out, need, T->stream) != hipSuccess) {
      (void)hipGetLastError();
      return fail(SQ_ENOMEM, "device allocation of %zu bytes failed", need);
    }
    T->dev_out_cap = need;
  }
  SQ_TRY(ensure_capacity(T, &T->dev_q, &T->dev_q_cap, count));
  return measure_list(T, qubits, count, seed, shot, meas_base, out_bits, out_random, T->dev_q, T->dev_out);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// sq_measure_noalloc: sq_measure with its staging (the measured list and the
// outcome and flag bytes) in a fixed device array instead of buffers the
// handle grows with hipMallocAsync. The array lives in the library's code
// object, one copy per device for the life of the process. In host code its
// name is only a stand-in, so its device address is looked up once per
// device (hipGetSymbolAddress with that device current) and only that
// address is used. Calls on one device share the array, so they are
// serialized by a per-device mutex (each call synchronizes its stream
// before returning, releasing the array).
static __device__ __align__(256) unsigned char scratch[(size_t)SQ_NOALLOC_MAX_MEAS * 6];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu[kMaxDevices];
unsigned char *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device `dev` (looked up on first use, with
// dev current; the caller's current device is restored). Caller holds
// g_scratch_mu[dev].
sq_status scratch_address(int dev, unsigned char **out) {
  if (g_scratch_ptr[dev]) {
    *out = g_scratch_ptr[dev];
    return SQ_OK;
  }
  int cur = 0;
  HIP_TRY(hipGetDevice(&cur));
  if (cur != dev) HIP_TRY(hipSetDevice(dev));
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (cur != dev) (void)hipSetDevice(cur);
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    return fail(SQ_EDEVICE, "hipGetSymbolAddress of the staging array failed: %s", hipGetErrorString(e));
  }
  g_scratch_ptr[dev] = static_cast<unsigned char *>(p);
  *out = g_scratch_ptr[dev];
  return SQ_OK;
}

}  // namespace

extern "C" {

sq_status sq_measure_noalloc(sq_tableau *T, const uint32_t *qubits, uint32_t count, uint64_t seed, uint64_t shot,
                             uint64_t meas_base, uint8_t *out_bits, uint8_t *out_random) {
  SQ_TRY(check_measure_args(T, qubits, count, out_bits));
  if (count == 0) return SQ_OK;
  if (count > SQ_NOALLOC_MAX_MEAS)
    return fail(SQ_ERANGE, "count=%u above SQ_NOALLOC_MAX_MEAS=%u", count, SQ_NOALLOC_MAX_MEAS);
  if (T->device < 0 || T->device >= kMaxDevices) return fail(SQ_EDEVICE, "device %d out of range", T->device);
  std::lock_guard<std::mutex> lk(g_scratch_mu[T->device]);
  unsigned char *base = nullptr;
  SQ_TRY(scratch_address(T->device, &base));
  u32 *dq = reinterpret_cast<u32 *>(base);
  uint8_t *dout = base + (size_t)SQ_NOALLOC_MAX_MEAS * 4;
  return measure_list(T, qubits, count, seed, shot, meas_base, out_bits, out_random, dq, dout);
}

sq_status sq_sample(sq_tableau *T, const uint32_t *qubits, uint32_t count, uint64_t seed, uint64_t shot_begin,
                    uint32_t shots, uint64_t meas_base, uint64_t *host_out) {
  const sq_shot_set one{seed, shot_begin, meas_base, shots, 0, host_out};
  return sq_sample_many(T, qubits, count, &one, 1);
}

size_t sq_sample_bytes(uint32_t n, uint32_t count, uint32_t shots) {
  if (n == 0 || n > SQ_MAX_QUBITS) return 0;
  SampleWs L;
  return sample_ws(dims_of(n), count, shots, &L);
}

sq_status sq_sample_many(sq_tableau *T, const uint32_t *qubits, uint32_t count, const sq_shot_set *sets,
                         uint32_t nsets) {
  if (!T) return fail(SQ_EINVAL, "tableau is NULL");
  if (T->collapse != SQ_COLLAPSE_ROWSUM)
    return fail(SQ_EINVAL, "shot sampling needs the rowsum collapse (generator signs); see sq_set_collapse");
  if (nsets && !sets) return fail(SQ_EINVAL, "sets is NULL");
  u32 shots = 0;  // the largest set sizes the coin and outcome buffers
  for (u32 k = 0; k < nsets; ++k) {
    if (sets[k].shots && !sets[k].out) return fail(SQ_EINVAL, "set %u: out is NULL", k);
    shots = std::max(shots, sets[k].shots);
  }
  if (count == 0 || shots == 0) return SQ_OK;
  SQ_TRY(set_rows(T, false));  // the sampling sweep works on a column-layout copy
  if (!qubits) return fail(SQ_EINVAL, "qubits is NULL");
  for (u32 i = 0; i < count; ++i)
    if (qubits[i] >= T->d.n) return fail(SQ_ERANGE, "qubit %u >= n=%u", qubits[i], T->d.n);
  const Dims &d = T->d;
  SampleWs L;
  const size_t ws_bytes = sample_ws(d, count, shots, &L);
  uint8_t *ws = nullptr;
  if (hipMallocAsync((void **)&ws, ws_bytes, T->stream) != hipSuccess) {
    (void)hipGetLastError();
    return fail(SQ_ENOMEM, "device allocation of %zu bytes for sampling failed", ws_bytes);
  }
  const u32 Ks = L.Ks, CW = L.CW;
  u64 *sg = (u64 *)(ws + L.o_sg), *fm = (u64 *)(ws + L.o_fm), *cw = (u64 *)(ws + L.o_cw), *dout = (u64 *)(ws + L.o_out);
  u32 *svlist = (u32 *)(ws + L.o_sv), *dq = (u32 *)(ws + L.o_q);
  uint8_t *kind = ws + L.o_kind, *fc = ws + L.o_fc;
  TabDev ts{(u64 *)(ws + L.o_x), (u64 *)(ws + L.o_z), T->t.R, d.n, d.K, d.L, d.Ls};
  // the blocked kernels run with a zeroed sign array (they then produce the
  // constants c(h)); the real signs live in the sign columns
  u64 *cvec = (u64 *)(ws + L.o_cvec);
  u32 *svt = (u32 *)(ws + L.o_svt);
  MeasStats *sstats = (MeasStats *)(ws + L.o_stats);
  TabDev tb{ts.X, ts.Z, cvec, d.n, d.K, d.L, d.Ls};
  const SymCtx sym{sg, svlist, kind, fm, fc, Ks, CW, count, 0};
  MeasState before{}, after{};
  sq_status s = SQ_OK;
  auto run = [&]() -> sq_status {
    HIP_TRY(hipMemcpyAsync(&before, T->st, sizeof(MeasState), hipMemcpyDeviceToHost, T->stream));
    HIP_TRY(hipMemcpyAsync(ts.X, T->t.X, (size_t)d.n * d.Ls * 8, hipMemcpyDeviceToDevice, T->stream));
    HIP_TRY(hipMemcpyAsync(ts.Z, T->t.Z, (size_t)d.n * d.Ls * 8, hipMemcpyDeviceToDevice, T->stream));
    HIP_TRY(hipMemcpyAsync(dq, qubits, (size_t)count * 4, hipMemcpyHostToDevice, T->stream));
    HIP_TRY(launch_sample_init(T->t, sg, Ks, count, T->stream));
    // the sweep: outcomes are not written (a random measurement's outcome is
    // its coin, a deterministic one an affine form), kind[] takes the flags
    HIP_TRY(launch_cursor_init(T->cur, count, std::min<u32>(T->tun.meas_block, KB), 0, 0, 0, dq, nullptr, kind,
                               T->stream));
    SQ_TRY(run_sweep(T, SweepCtx{ts, tb, &sym, sstats, cvec, svt}, count));
    // per shot set: its coins, its outcomes, its copy out (the sweep is shared)
    for (u32 k = 0; k < nsets; ++k) {
      const sq_shot_set &e = sets[k];
      if (e.shots == 0) continue;
      HIP_TRY(launch_coins(cw, e.seed, e.shot_begin, e.meas_base, e.shots, count, CW, T->stream));
      HIP_TRY(launch_eval(cw, kind, fm, fc, dout, e.shots, count, CW, T->stream));
      HIP_TRY(hipMemcpyAsync(e.out, dout, (size_t)e.shots * CW * 8, hipMemcpyDeviceToHost, T->stream));
    }
    HIP_TRY(hipMemcpyAsync(&after, T->st, sizeof(MeasState), hipMemcpyDeviceToHost, T->stream));
    HIP_TRY(hipStreamSynchronize(T->stream));
    return SQ_OK;
  };
  s = run();
  (void)hipFreeAsync(ws, T->stream);
  if (s != SQ_OK) (void)hipStreamSynchronize(T->stream);
  if (s == SQ_OK && after.flags != before.flags)
    s = fail(SQ_ESTATE, "device consistency check failed (flags 0x%x)", after.flags);
  return s;
}

namespace {
constexpr u32 kBatchMaxN = 16384;
constexpr u32 kBatchMaxCount = 32767;
// Automatic: one workgroup per circuit pays off up to about a thousand
// qubits; larger circuits finish sooner on the whole GPU (measured on the
// MI355X on the batched/served mix: 1024 qubits and 8 streams 2.2 s, 4096
// qubits 6.9 s).
constexpr u32 kBatchAutoMaxN = 1024;

// Whether sq_batch_sample runs an item in the persistent launch.
bool batched_item(u32 n, u32 count, u32 block, u32 max_n) {
  const u32 L = 2 * cdiv(n, 64);
  return n <= max_n && count <= kBatchMaxCount && L <= 2 * block;
}

// One item through the single-tableau path: create, gates, sample, destroy.
sq_status batch_item_plain(const sq_batch_item &it, hipStream_t stream) {
  sq_tableau *T = nullptr;
  SQ_TRY(sq_create(it.n, stream, &T));
  sq_status s = sq_apply_gates(T, it.ops, it.nops);
  if (s == SQ_OK) s = sq_sample(T, it.qubits, it.count, it.seed, it.shot_begin, it.shots, it.meas_base, it.out);
  sq_destroy(T);
  return s;
}
}  // namespace

size_t sq_batch_item_bytes(uint32_t n, uint64_t nops, uint32_t count, uint32_t shots, const sq_batch_opts *opts) {
  if (n == 0 || n > SQ_MAX_QUBITS || count == 0 || shots == 0) return 0;
  const u32 block = opts && opts->block ? opts->block : 256;
  const u32 max_n = std::min(opts && opts->max_batch_n ? opts->max_batch_n : kBatchAutoMaxN, kBatchMaxN);
  const Dims d = dims_of(n);
  auto r256 = [](size_t b) { return (b + 255) / 256 * 256; };
  if (batched_item(n, count, block, max_n)) {
    const size_t Ks = round_up(d.K, 16), CW = cdiv(count, 64);
    return 2 * r256((size_t)n * d.Ls * 8) + r256((count + 1) * Ks * 8) + r256(count * CW * 8) +
           2 * r256((size_t)shots * CW * 8) + 2 * r256(count) + 16 * nops + 4 * (size_t)count + sizeof(BatchItem) + 8;
  }
  SampleWs L;
  return sq_bytes_required(n) + sample_ws(d, count, shots, &L) + 20 * nops + 32768;
}

sq_status sq_batch_sample(const sq_batch_item *items, uint32_t nitems, const sq_batch_opts *opts, void *hip_stream) {
  if (nitems == 0) return SQ_OK;
  if (!items) return fail(SQ_EINVAL, "items is NULL");
  hipStream_t stream = (hipStream_t)hip_stream;
  u32 block = opts && opts->block ? opts->block : 256;
  u32 max_n = opts && opts->max_batch_n ? opts->max_batch_n : kBatchAutoMaxN;
  if (block % 64 || block < 64 || block > 512) return fail(SQ_EINVAL, "batch block must be a multiple of 64 in [64, 512]");
  max_n = std::min(max_n, kBatchMaxN);
  for (u32 k = 0; k < nitems; ++k) {
    const sq_batch_item &it = items[k];
    if (it.n == 0 || it.n > SQ_MAX_QUBITS) return fail(SQ_ERANGE, "item %u: bad n=%u", k, it.n);
    SQ_TRY(validate_ops(it.n, it.ops, it.nops, false));
    if (it.count && (!it.qubits || !it.out)) return fail(SQ_EINVAL, "item %u: NULL qubits/out", k);
    for (u32 i = 0; i < it.count; ++i)
      if (it.qubits[i] >= it.n) return fail(SQ_ERANGE, "item %u: qubit %u >= n=%u", k, it.qubits[i], it.n);
  }
  // split: batched (small) and single-tableau (large) items
  std::vector<u32> small, large;
  for (u32 k = 0; k < nitems; ++k) {
    const sq_batch_item &it = items[k];
    if (it.count == 0 || it.shots == 0) continue;
    if (batched_item(it.n, it.count, block, max_n)) small.push_back(k);
    else large.push_back(k);
  }
  // largest first: cost ~ n^2 * count (rowsum sweep) + gates
  auto cost = [&](u32 k) {
    const sq_batch_item &it = items[k];
    return (double)it.n * it.n * it.count + (double)it.nops * it.n;
  };
  std::sort(small.begin(), small.end(), [&](u32 a, u32 b) { return cost(a) > cost(b); });
  std::sort(large.begin(), large.end(), [&](u32 a, u32 b) { return cost(a) > cost(b); });
  // Large items: single-tableau path, several at once on worker threads with
  // their own (default-priority) streams, overlapping each other's launch
  // latency and the batched launch below.
  const u32 nworkers = std::min<u32>((u32)large.size(), opts && opts->streams ? opts->streams : 8);
  std::vector<sq_status> wstatus(nworkers, SQ_OK);
  std::vector<std::string> werr(nworkers);
  std::vector<std::thread> workers;
  // joins every worker on each way out of this function (a joinable thread
  // destroyed unjoined would terminate the process)
  struct JoinAll {
    std::vector<std::thread> &v;
    ~JoinAll() {
      for (std::thread &th : v)
        if (th.joinable()) th.join();
    }
  } join_all{workers};
  std::atomic<u32> next_large{0};
  int dev = 0;
  (void)hipGetDevice(&dev);
  for (u32 wk = 0; wk < nworkers; ++wk) {
    workers.emplace_back([&, wk]() {
      if (hipSetDevice(dev) != hipSuccess) {
        wstatus[wk] = SQ_EDEVICE;
        werr[wk] = "hipSetDevice failed in a batch worker";
        return;
      }
      hipStream_t ws = nullptr;
      if (hipStreamCreate(&ws) != hipSuccess) {
        wstatus[wk] = SQ_EDEVICE;
        werr[wk] = "hipStreamCreate failed in a batch worker";
        return;
      }
      for (;;) {
        const u32 idx = next_large.fetch_add(1);
        if (idx >= large.size()) break;
        const sq_status st = batch_item_plain(items[large[idx]], ws);
        if (st != SQ_OK) {
          wstatus[wk] = st;
          werr[wk] = g_err;
          break;
        }
      }
      (void)hipStreamSynchronize(ws);
      (void)hipStreamDestroy(ws);
    });
  }
  auto join_workers = [&]() -> sq_status {
    for (std::thread &th : workers) th.join();
    workers.clear();
    for (u32 wk = 0; wk < nworkers; ++wk)
      if (wstatus[wk] != SQ_OK) return fail(wstatus[wk], "%s", werr[wk].c_str());
    return SQ_OK;
  };
  if (!small.empty()) {
    // host-side compile and layout
    std::vector<Group> groups;
    std::vector<u32> pass_off, qubits;
    struct Off {
      size_t pass_off, groups, qubits, ws;
    };
    std::vector<Off> offs(small.size());
    size_t ws_bytes = 0;
    auto take = [&](size_t bytes) {
      size_t r = ws_bytes;
      ws_bytes += (bytes + 255) / 256 * 256;
      return r;
    };
    std::vector<BatchItem> bi(small.size());
    std::vector<size_t> o_x(small.size()), o_z(small.size()), o_sg(small.size()), o_fm(small.size()),
        o_cb(small.size()), o_out(small.size()), o_fc(small.size()), o_kind(small.size());
    PassBuilder pb;
    for (size_t s = 0; s < small.size(); ++s) {
      const sq_batch_item &it = items[small[s]];
      const Dims d = dims_of(it.n);
      pb.init(it.n, d.L);
      for (u64 i = 0; i < it.nops; ++i) pb.add(it.ops[i].type, it.ops[i].q0, it.ops[i].q1);
      pb.flush();
      offs[s].pass_off = pass_off.size();
      offs[s].groups = groups.size();
      for (const PassRange &r : pb.passes) pass_off.push_back((u32)r.offset);
      pass_off.push_back((u32)pb.groups.size());
      groups.insert(groups.end(), pb.groups.begin(), pb.groups.end());
      offs[s].qubits = qubits.size();
      qubits.insert(qubits.end(), it.qubits, it.qubits + it.count);
      const u32 Ks = round_up(d.K, 16), CW = cdiv(it.count, 64);
      BatchItem &b = bi[s];
      b.n = it.n;
      b.Ls = d.Ls;
      b.Ks = Ks;
      b.CW = CW;
      b.count = it.count;
      b.shots = it.shots;
      b.npasses = (u32)pb.passes.size();
      b.pad = 0;
      b.seed = it.seed;
      b.shot_begin = it.shot_begin;
      b.meas_base = it.meas_base;
      o_x[s] = take((size_t)it.n * d.Ls * 8);
      o_z[s] = take((size_t)it.n * d.Ls * 8);
      o_sg[s] = take((size_t)(it.count + 1) * Ks * 8);
      o_fm[s] = take((size_t)it.count * CW * 8);
      o_cb[s] = take((size_t)it.shots * CW * 8);
      o_out[s] = take((size_t)it.shots * CW * 8);
      o_fc[s] = take(it.count);
      o_kind[s] = take(it.count);
    }
    const size_t o_groups = take(groups.size() * sizeof(Group) + 16);
    const size_t o_poff = take(pass_off.size() * 4);
    const size_t o_q = take(qubits.size() * 4);
    const size_t o_items = take(bi.size() * sizeof(BatchItem));
    const size_t o_flags = take(bi.size() * 4);
    const size_t o_next = take(4);
    uint8_t *ws = nullptr;
    if (hipMallocAsync((void **)&ws, ws_bytes, stream) != hipSuccess) {
      (void)hipGetLastError();
      const sq_status ws_status = join_workers();  // the workers' own error, if any, comes first
      if (ws_status != SQ_OK) return ws_status;
      return fail(SQ_ENOMEM, "device allocation of %zu bytes for the batch failed", ws_bytes);
    }
    for (size_t s = 0; s < small.size(); ++s) {
      BatchItem &b = bi[s];
      b.X = (u64 *)(ws + o_x[s]);
      b.Z = (u64 *)(ws + o_z[s]);
      b.sg = (u64 *)(ws + o_sg[s]);
      b.fm = (u64 *)(ws + o_fm[s]);
      b.coinbuf = (u64 *)(ws + o_cb[s]);
      b.out = (u64 *)(ws + o_out[s]);
      b.fc = ws + o_fc[s];
      b.kind = ws + o_kind[s];
      b.groups = (const Group *)(ws + o_groups) + offs[s].groups;
      b.pass_off = (const u32 *)(ws + o_poff) + offs[s].pass_off;
      b.qubits = (const u32 *)(ws + o_q) + offs[s].qubits;
      b.flags = (u32 *)(ws + o_flags) + s;
    }
    // pass offsets are relative to each item's own groups
    std::vector<u32> flags(small.size(), 0);
    int ncu = 256;
    {
      int dev = 0;
      if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) ncu = prop.multiProcessorCount;
      }
    }
    u32 grid = opts && opts->grid ? opts->grid : (u32)ncu * std::max<u32>(1, 1024 / block);
    grid = std::min<u32>(grid, (u32)small.size());
    sq_status st = SQ_OK;
    auto run = [&]() -> sq_status {
      HIP_TRY(hipMemcpyAsync(ws + o_groups, groups.data(), groups.size() * sizeof(Group), hipMemcpyHostToDevice,
                             stream));
      HIP_TRY(hipMemcpyAsync(ws + o_poff, pass_off.data(), pass_off.size() * 4, hipMemcpyHostToDevice, stream));
      HIP_TRY(hipMemcpyAsync(ws + o_q, qubits.data(), qubits.size() * 4, hipMemcpyHostToDevice, stream));
      HIP_TRY(hipMemcpyAsync(ws + o_items, bi.data(), bi.size() * sizeof(BatchItem), hipMemcpyHostToDevice, stream));
      HIP_TRY(launch_fill_zero((u64 *)(ws + o_flags), (bi.size() * 4 + 4 + 7) / 8, stream));
      HIP_TRY(launch_fill_zero((u64 *)(ws + o_next), 1, stream));
      HIP_TRY(launch_batch((const BatchItem *)(ws + o_items), (u32)bi.size(), (u32 *)(ws + o_next), block, grid,
                           stream));
      for (size_t s = 0; s < small.size(); ++s) {
        const sq_batch_item &it = items[small[s]];
        HIP_TRY(hipMemcpyAsync(it.out, ws + o_out[s], (size_t)it.shots * bi[s].CW * 8, hipMemcpyDeviceToHost, stream));
      }
      HIP_TRY(hipMemcpyAsync(flags.data(), ws + o_flags, flags.size() * 4, hipMemcpyDeviceToHost, stream));
      HIP_TRY(hipStreamSynchronize(stream));
      return SQ_OK;
    };
    st = run();
    (void)hipFreeAsync(ws, stream);
    (void)hipStreamSynchronize(stream);
    if (st != SQ_OK) {
      (void)join_workers();
      return st;
    }
    for (size_t s = 0; s < small.size(); ++s)
      if (flags[s]) {
        (void)join_workers();
        return fail(SQ_ESTATE, "item %u: device consistency check failed (flags 0x%x)", small[s], flags[s]);
      }
  }
  SQ_TRY(join_workers());
  return SQ_OK;
}

sq_status sq_program_create(uint32_t n, const sq_op *ops, uint64_t count, sq_program **out) {
  if (!out) return fail(SQ_EINVAL, "out is NULL");
  *out = nullptr;
  if (n == 0 || n > SQ_MAX_QUBITS) return fail(SQ_ERANGE, "bad n=%u", n);
  SQ_TRY(validate_ops(n, ops, count, true));
  sq_program *P = new (std::nothrow) sq_program();
  if (!P) return fail(SQ_ENOMEM, "host allocation failed");
  static std::atomic<u64> next_uid{1};
  P->uid = next_uid.fetch_add(1);
  (void)hipGetDevice(&P->device);
  P->n = n;
  P->d = dims_of(n);
  WideBuilder pb;
  pb.init(n, P->d.L);
  u64 i = 0;
  while (i < count) {
    if (ops[i].type == SQ_MEASURE) {
      sq_program::Seg s{1, P->meas_qubits.size(), 0};
      while (i < count && ops[i].type == SQ_MEASURE) P->meas_qubits.push_back(ops[i++].q0);
      s.count = P->meas_qubits.size() - s.first;
      P->segs.push_back(s);
    } else {
      const size_t first = pb.passes.size();
      while (i < count && ops[i].type != SQ_MEASURE) {
        if (ops[i].type != SQ_I) P->ngates++;
        pb.add(ops[i].type, ops[i].q0, ops[i].q1);
        ++i;
      }
      pb.flush();
      if (pb.passes.size() > first) P->segs.push_back(sq_program::Seg{0, first, pb.passes.size() - first});
    }
  }
  P->passes = pb.passes;
  for (const PassRange &r : P->passes) P->gate_bytes += r.bytes;
  if (!P->meas_qubits.empty()) {
    if (P->meas_qubits.size() >= 0xFFFFFFFFull) {
      delete P;
      return fail(SQ_ERANGE, "a program holds at most 2^32 - 2 measurements");
    }
    if (hipMalloc((void **)&P->dev_meas, P->meas_qubits.size() * 4) != hipSuccess) {
      (void)hipGetLastError();
      delete P;
      return fail(SQ_ENOMEM, "device allocation of %zu measured qubits failed", P->meas_qubits.size());
    }
    if (hipMemcpy(P->dev_meas, P->meas_qubits.data(), P->meas_qubits.size() * 4, hipMemcpyHostToDevice) !=
        hipSuccess) {
      (void)hipFree(P->dev_meas);
      delete P;
      return fail(SQ_EDEVICE, "upload of the measured qubits failed");
    }
  }
  if (!pb.offs.empty()) {
    if (hipMalloc((void **)&P->dev_words, pb.words.size() * 4) != hipSuccess ||
        hipMalloc((void **)&P->dev_offs, pb.offs.size() * 4) != hipSuccess) {
      (void)hipGetLastError();
      (void)hipFree(P->dev_words);
      (void)hipFree(P->dev_meas);
      delete P;
      return fail(SQ_ENOMEM, "device allocation of %zu gate-pass words failed", pb.words.size() + pb.offs.size());
    }
    if (hipMemcpy(P->dev_words, pb.words.data(), pb.words.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(P->dev_offs, pb.offs.data(), pb.offs.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipFree(P->dev_words);
      (void)hipFree(P->dev_offs);
      (void)hipFree(P->dev_meas);
      delete P;
      return fail(SQ_EDEVICE, "upload of gate passes failed");
    }
  }
  *out = P;
  return SQ_OK;
}

sq_status sq_plan_gates(uint32_t n, const sq_op *ops, uint64_t count, uint64_t *out, uint64_t cap,
                        uint64_t *out_len) {
  if (!out_len || (cap && !out)) return fail(SQ_EINVAL, "NULL argument");
  if (n == 0 || n > SQ_MAX_QUBITS) return fail(SQ_ERANGE, "bad n=%u", n);
  SQ_TRY(validate_ops(n, ops, count, false));
  WideBuilder pb;
  plan_gate_list(n, dims_of(n).L, ops, count, pb);
  u64 k = 0;
  auto put = [&](u64 v) {
    if (k < cap) out[k] = v;
    ++k;
  };
  for (const PassRange &r : pb.passes) {
    put(r.count);
    for (u32 g = 0; g < r.count; ++g) {
      const u32 *rec = pb.words.data() + pb.offs[r.offset + g];
      const u32 nq = rec[0] & 15u, nops = (rec[0] >> WH_NOPS_SHIFT) & 63u;
      put(rec[0]);
      for (u32 q = 0; q < nq; ++q) put(rec[1 + q]);
      for (u32 j = 0; j < nops; ++j) put((rec[1 + nq + j / 2] >> ((j & 1u) * 16u)) & 0xFFFFu);
    }
  }
  *out_len = k;
  return SQ_OK;
}

sq_status sq_program_destroy(sq_program *P) {
  if (!P) return SQ_OK;
  (void)hipFree(P->dev_words);
  (void)hipFree(P->dev_offs);
  (void)hipFree(P->dev_meas);
  delete P;
  return SQ_OK;
}

uint64_t sq_program_num_measurements(const sq_program *P) { return P ? P->meas_qubits.size() : 0; }
uint64_t sq_program_num_gates(const sq_program *P) { return P ? P->ngates : 0; }
uint64_t sq_program_num_passes(const sq_program *P) { return P ? P->passes.size() : 0; }

sq_status sq_run(sq_tableau *T, const sq_program *P, uint64_t seed, uint64_t shot, uint64_t meas_base,
                 uint8_t *dev_out_bits, uint8_t *dev_out_random) {
  if (!T || !P) return fail(SQ_EINVAL, "tableau or program is NULL");
  if (P->n != T->d.n) return fail(SQ_EINVAL, "program has n=%u, tableau n=%u", P->n, T->d.n);
  if (!P->meas_qubits.empty() && !dev_out_bits) return fail(SQ_EINVAL, "dev_out_bits is NULL");
  const u32 kb = sweep_kb(T);
  for (const sq_program::Seg &s : P->segs) {
    if (s.kind == 0) {
      SQ_TRY(run_gate_segment(T, P, s.first, s.count));
    } else {
      HIP_TRY(launch_cursor_init(T->cur, (u32)s.count, kb, seed, shot, meas_base + s.first, P->dev_meas + s.first,
                                 dev_out_bits + s.first, dev_out_random ? dev_out_random + s.first : nullptr,
                                 T->stream));
      SQ_TRY(run_sweep(T, SweepCtx{T->t, T->t, nullptr, T->stats, nullptr, nullptr}, (u32)s.count));
    }
  }
  return SQ_OK;
}

sq_status sq_frame_sample(const sq_program *P, const uint8_t *host_ref, uint64_t seed, uint32_t shots,
                          uint64_t *host_out, void *hip_stream) {
  if (!P) return fail(SQ_EINVAL, "program is NULL");
  if (shots == 0) return SQ_OK;
  const u64 M = P->meas_qubits.size();
  if (M && (!host_ref || !host_out)) return fail(SQ_EINVAL, "host_ref/host_out is NULL");
  for (u64 i = 0; i < M; ++i)
    if (host_ref[i] > 1) return fail(SQ_EINVAL, "reference outcome %llu is %u, not 0 or 1", (unsigned long long)i,
                                     host_ref[i]);
  if (M == 0) return SQ_OK;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != P->device) return fail(SQ_EINVAL, "program lives on device %d, current device is %d", P->device, dev);
  hipStream_t st = (hipStream_t)hip_stream;
  const u32 n = P->n, Lf = cdiv(shots, 64), Ls = round_up(Lf, 16), W = cdiv(M, 64);
  const u32 block = Lf >= 1024 ? 256 : 64, wpt = Lf >= 512 ? 2 : 1;
  const u32 tiles = cdiv(Lf, (u64)block * wpt);
  // workspace: Fx | Fz | dummy signs | sign partials | records | output | qubits | reference
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t r = off;
    off += (bytes + 255) / 256 * 256;
    return r;
  };
  const size_t o_fx = take((size_t)n * Ls * 8), o_fz = take((size_t)n * Ls * 8), o_r = take((size_t)Ls * 8);
  const size_t o_sp = take((size_t)kMaxChunks * Ls * 8), o_rec = take((size_t)M * Lf * 8);
  const size_t o_out = take((size_t)shots * W * 8), o_q = take(M * 4), o_ref = take(M);
  char *ws = nullptr;
  if (hipMallocAsync((void **)&ws, off, st) != hipSuccess) {
    (void)hipGetLastError();
    return fail(SQ_ENOMEM, "device allocation of %zu bytes failed", off);
  }
  auto release = [&]() { (void)hipFreeAsync(ws, st); };
  u64 *Fx = (u64 *)(ws + o_fx), *Fz = (u64 *)(ws + o_fz), *rec = (u64 *)(ws + o_rec), *dout = (u64 *)(ws + o_out);
  u32 *dq = (u32 *)(ws + o_q);
  uint8_t *dref = (uint8_t *)(ws + o_ref);
  const TabDev ft{Fx, Fz, (u64 *)(ws + o_r), n, cdiv(Lf, 2), Lf, Ls};
  hipError_t e = hipMemcpyAsync(dq, P->meas_qubits.data(), M * 4, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(dref, host_ref, M, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = launch_frame_init(Fx, Fz, n, Lf, Ls, seed, st);
  for (const sq_program::Seg &sg : P->segs) {
    if (e != hipSuccess) break;
    if (sg.kind == 0) {
      for (u64 i = sg.first; i < sg.first + sg.count && e == hipSuccess; ++i) {
        const PassRange &p = P->passes[i];
        const u32 want = std::max<u32>(1, 6144 / tiles);
        const u32 gpc = std::max<u32>(std::max<u32>(16, cdiv(p.count, want)), cdiv(p.count, kMaxChunks));
        // frame signs are not used: the partials are written and left
        e = launch_layer(ft, P->dev_words, P->dev_offs + p.offset, p.count, block, wpt, gpc, (u64 *)(ws + o_sp), st);
      }
    } else {
      e = launch_frame_measure(Fx, Fz, dq, (u32)sg.count, sg.first, dref, rec, n, Lf, Ls, seed, st);
    }
  }
  if (e == hipSuccess) e = launch_frame_transpose(rec, dout, M, W, Lf, shots, st);
  if (e == hipSuccess) e = hipMemcpyAsync(host_out, dout, (size_t)shots * W * 8, hipMemcpyDeviceToHost, st);
  release();
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail(SQ_EDEVICE, "frame sampling: %s", hipGetErrorString(e));
  return SQ_OK;
}

sq_status sq_export_rows(sq_tableau *T, const uint32_t *rows, uint32_t nrows, uint64_t *hx, uint64_t *hz,
                         uint8_t *hr) {
  if (!T) return fail(SQ_EINVAL, "tableau is NULL");
  if (nrows == 0) return SQ_OK;
  if (!rows || !hx || !hz || !hr) return fail(SQ_EINVAL, "NULL buffer");
  for (u32 k = 0; k < nrows; ++k)
    if (rows[k] >= 2 * T->d.n) return fail(SQ_ERANGE, "row %u >= 2n=%u", rows[k], 2 * T->d.n);
  SQ_TRY(set_rows(T, false));
  const u32 W = T->d.K;
  const size_t xwords = (size_t)nrows * W;
  void *buf = nullptr;
  const size_t bytes = nrows * 4 + 2 * xwords * 8 + nrows + 256;
  if (hipMallocAsync(&buf, bytes, T->stream) != hipSuccess) {
    (void)hipGetLastError();
    return fail(SQ_ENOMEM, "device allocation of %zu bytes failed", bytes);
  }
  u64 *dx = (u64 *)buf;
  u64 *dz = dx + xwords;
  u32 *drows = (u32 *)(dz + xwords);
  uint8_t *dr = (uint8_t *)(drows + nrows);
  sq_status s = SQ_OK;
  if (hipMemcpyAsync(drows, rows, nrows * 4, hipMemcpyHostToDevice, T->stream) != hipSuccess ||
      launch_export_rows(T->t, drows, nrows, W, dx, dz, dr, T->stream) != hipSuccess ||
      hipMemcpyAsync(hx, dx, xwords * 8, hipMemcpyDeviceToHost, T->stream) != hipSuccess ||
      hipMemcpyAsync(hz, dz, xwords * 8, hipMemcpyDeviceToHost, T->stream) != hipSuccess ||
      hipMemcpyAsync(hr, dr, nrows, hipMemcpyDeviceToHost, T->stream) != hipSuccess ||
      hipStreamSynchronize(T->stream) != hipSuccess)
    s = fail(SQ_EDEVICE, "export failed: %s", hipGetErrorString(hipGetLastError()));
  (void)hipFreeAsync(buf, T->stream);
  (void)hipStreamSynchronize(T->stream);
  return s;
}

sq_status sq_export(sq_tableau *T, uint64_t *hx, uint64_t *hz, uint8_t *hr) {
  if (!T) return fail(SQ_EINVAL, "tableau is NULL");
  std::vector<u32> rows(2 * (size_t)T->d.n);
  for (u32 k = 0; k < rows.size(); ++k) rows[k] = k;
  return sq_export_rows(T, rows.data(), (u32)rows.size(), hx, hz, hr);
}

sq_status sq_import(sq_tableau *T, const uint64_t *hx, const uint64_t *hz, const uint8_t *hr) {
  if (!T) return fail(SQ_EINVAL, "tableau is NULL");
  if (!hx || !hz || !hr) return fail(SQ_EINVAL, "NULL buffer");
  const u32 n = T->d.n, W = T->d.K;
  const size_t rows = 2 * (size_t)n, xwords = rows * W;
  if (n % 64) {
    const u64 bad = ~0ULL << (n % 64);
    for (size_t g = 0; g < rows; ++g)
      if ((hx[g * W + W - 1] & bad) || (hz[g * W + W - 1] & bad))
        return fail(SQ_EINVAL, "row %zu has bits at qubit positions >= n", g);
  }
  SQ_TRY(set_rows(T, false));
  void *buf = nullptr;
  const size_t bytes = 2 * xwords * 8 + rows + 256;
  if (hipMallocAsync(&buf, bytes, T->stream) != hipSuccess) {
    (void)hipGetLastError();
    return fail(SQ_ENOMEM, "device allocation of %zu bytes failed", bytes);
  }
  u64 *dx = (u64 *)buf;
  u64 *dz = dx + xwords;
  uint8_t *dr = (uint8_t *)(dz + xwords);
  sq_status s = SQ_OK;
  if (hipMemcpyAsync(dx, hx, xwords * 8, hipMemcpyHostToDevice, T->stream) != hipSuccess ||
      hipMemcpyAsync(dz, hz, xwords * 8, hipMemcpyHostToDevice, T->stream) != hipSuccess ||
      hipMemcpyAsync(dr, hr, rows, hipMemcpyHostToDevice, T->stream) != hipSuccess ||
      launch_import(T->t, dx, dz, dr, W, T->stream) != hipSuccess || hipStreamSynchronize(T->stream) != hipSuccess)
    s = fail(SQ_EDEVICE, "import failed: %s", hipGetErrorString(hipGetLastError()));
  (void)hipFreeAsync(buf, T->stream);
  (void)hipStreamSynchronize(T->stream);
  return s;
}

sq_status sq_measure_stats(sq_tableau *T, sq_meas_stats *out) {
  if (!T || !out) return fail(SQ_EINVAL, "NULL argument");
  MeasStats s{};
  HIP_TRY(hipMemcpyAsync(&s, T->stats, sizeof(s), hipMemcpyDeviceToHost, T->stream));
  HIP_TRY(hipStreamSynchronize(T->stream));
  out->n_random = s.n_random;
  out->n_det = s.n_det;
  out->rowsum_bytes = s.rowsum_bytes;
  out->det_bytes = s.det_bytes;
  out->blocks = s.blocks;
  out->block_bytes = s.block_bytes;
  out->inject_bytes = s.inject_bytes;
  return SQ_OK;
}

uint64_t sq_program_gate_bytes(const sq_program *P) { return P ? P->gate_bytes : 0; }

sq_status sq_error_flags(sq_tableau *T, uint32_t *flags) {
  if (!T || !flags) return fail(SQ_EINVAL, "NULL argument");
  MeasState s{};
  HIP_TRY(hipMemcpyAsync(&s, T->st, sizeof(s), hipMemcpyDeviceToHost, T->stream));
  HIP_TRY(hipStreamSynchronize(T->stream));
  *flags = s.flags;
  return SQ_OK;
}

sq_status sq_get_tuning(const sq_tableau *T, sq_tuning *out) {
  if (!T || !out) return fail(SQ_EINVAL, "NULL argument");
  *out = T->tun;
  return SQ_OK;
}

sq_status sq_set_tuning(sq_tableau *T, const sq_tuning *in) {
  if (!T || !in) return fail(SQ_EINVAL, "NULL argument");
  sq_tuning t = T->tun;
  if (in->layer_block) t.layer_block = in->layer_block;
  if (in->layer_wpt) t.layer_wpt = in->layer_wpt;
  if (in->layer_groups) t.layer_groups = in->layer_groups;
  if (in->rowsum_block) t.rowsum_block = in->rowsum_block;
  if (in->rowsum_wpt) t.rowsum_wpt = in->rowsum_wpt;
  if (in->rowsum_cols) t.rowsum_cols = in->rowsum_cols;
  if (in->det_cols) t.det_cols = in->det_cols;
  if (in->meas_block) t.meas_block = in->meas_block;
  if (in->pivot_waves) t.pivot_waves = in->pivot_waves;
  SQ_TRY(check_tuning(t));
  T->tun = t;
  return SQ_OK;
}

sq_status sq_set_graphs(sq_tableau *T, int on) {
  if (!T) return fail(SQ_EINVAL, "tableau is NULL");
  T->use_graphs = on != 0;
  if (!T->use_graphs) {
    HIP_TRY(hipStreamSynchronize(T->stream));  // no launched graph may still be pending
    for (auto &g : T->graphs)
      if (g.exec) (void)hipGraphExecDestroy(g.exec);
    T->graphs.clear();
  }
  return SQ_OK;
}

sq_status sq_graph_stats(const sq_tableau *T, uint64_t *captures, uint64_t *replays) {
  if (!T || !captures || !replays) return fail(SQ_EINVAL, "NULL argument");
  *captures = T->graph_captures;
  *replays = T->graph_replays;
  return SQ_OK;
}

sq_status sq_profile_enable(sq_tableau *T, int on) {
  if (!T) return fail(SQ_EINVAL, "tableau is NULL");
  T->prof = on != 0;
  return SQ_OK;
}

sq_status sq_profile_read(sq_tableau *T, int kernel, double *total_ms, uint64_t *launches) {
  if (!T || kernel < 0 || kernel >= SQ_K_COUNT) return fail(SQ_EINVAL, "bad argument");
  SQ_TRY(collect_profile(T));
  if (total_ms) *total_ms = T->ms[kernel];
  if (launches) *launches = T->launches[kernel];
  return SQ_OK;
}

sq_status sq_profile_reset(sq_tableau *T) {
  if (!T) return fail(SQ_EINVAL, "tableau is NULL");
  SQ_TRY(collect_profile(T));
  for (int k = 0; k < SQ_K_COUNT; ++k) {
    T->ms[k] = 0;
    T->launches[k] = 0;
  }
  return SQ_OK;
}

}  // extern "C"
